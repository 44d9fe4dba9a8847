"""Reduced-precision wind storage, numpy reference -- TEST INFRASTRUCTURE ONLY.

Winds stored as BF16 or FP16 with one FP32 scale per (variable, level, time
level): s = max|f| over the level (1 when the level is all zero),
q = RNE_16(f * fl32(1/s)), decoded as fl32(q * s).  The decoded values are
what the FP64 oracle then interpolates.
"""
from __future__ import annotations

import numpy as np

BF16, F16 = 1, 2


def level_scales(f: np.ndarray) -> np.ndarray:
    """f: (nz, ny, nx) float32 -> (nz,) float32 max |f| per level (1 if 0)."""
    s = np.abs(f).reshape(f.shape[0], -1).max(axis=1).astype(np.float32)
    s[s == 0] = np.float32(1.0)
    return s


def bf16_rne_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (round to nearest, ties to even), as the
    upper 16 bits of the float32 pattern.  Inputs are finite."""
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = b + 0x7FFF + ((b >> 16) & 1)
    return (b >> 16).astype(np.uint16)


def bf16_bits_to_f32(q: np.ndarray) -> np.ndarray:
    return (q.astype(np.uint32) << 16).view(np.float32)


def encode_level(f: np.ndarray, kind: int) -> tuple[np.ndarray, np.ndarray]:
    """(nz, ny, nx) float32 -> (16-bit patterns, scales)."""
    s = level_scales(f)
    inv = (np.float32(1.0) / s).astype(np.float32)
    y = (f * inv[:, None, None]).astype(np.float32)
    if kind == BF16:
        q = bf16_rne_bits(y)
    elif kind == F16:
        q = y.astype(np.float16).view(np.uint16)
    else:
        raise ValueError(kind)
    return q, s


def decode_level(q: np.ndarray, s: np.ndarray, kind: int) -> np.ndarray:
    if kind == BF16:
        v = bf16_bits_to_f32(q)
    else:
        v = q.view(np.float16).astype(np.float32)
    return (v * s[:, None, None]).astype(np.float32)


def dequantized_met(met, kind: int):
    """A copy of an ``inputs.Met`` whose u, v, w (and temperature, when
    present: the fourth value of each record, with its own per-level scale)
    hold the decoded stored values (what a reduced-precision run actually
    interpolates).  The surface fields are stored in FP32 and stay as they
    are."""
    import dataclasses
    out = dataclasses.replace(met, u=np.empty_like(met.u), v=np.empty_like(met.v),
                              w=np.empty_like(met.w))
    names = ("u", "v", "w")
    if getattr(met, "temp", None) is not None:
        out.temp = np.empty_like(met.temp)
        names = names + ("temp",)
    for name in names:
        src, dst = getattr(met, name), getattr(out, name)
        for l in range(met.nt):
            q, s = encode_level(src[l], kind)
            dst[l] = decode_level(q, s, kind)
    return out
