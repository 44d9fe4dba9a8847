"""Surrogate MLP forward pass, numpy reference -- TEST INFRASTRUCTURE ONLY.

ReLU network 81 -> 128 -> 128 -> 128 -> 3 evaluated in float32 on the same
bfloat16-rounded weights, inputs and hidden activations the GPU uses (its
MFMA products are exact bf16 x bf16 products accumulated in FP32), with the
same flat parameter layout: per layer W[in][out] (padded 96x128, 128x128,
128x128, 128x16) followed by the bias.
"""
from __future__ import annotations

import numpy as np

from . import encode

SHAPES = [(96, 128), (128, 128), (128, 128), (128, 16)]
NIN, NOUT = 81, 3


def unpack(params: np.ndarray):
    params = np.asarray(params, np.float32)
    out, off = [], 0
    for fi, fo in SHAPES:
        w = params[off:off + fi * fo].reshape(fi, fo)
        off += fi * fo
        b = params[off:off + fo]
        off += fo
        out.append((w, b))
    assert off == params.size
    return out


def bf16(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    return encode.bf16_bits_to_f32(encode.bf16_rne_bits(x)).reshape(x.shape)


def normalize_inputs(x: np.ndarray, norm: np.ndarray) -> np.ndarray:
    x = np.asarray(x, np.float32)
    norm = np.asarray(norm, np.float32)
    var = np.arange(NIN) // 27
    xn = np.zeros((x.shape[0], 96), np.float32)
    xn[:, :NIN] = (x - norm[var]) / norm[3 + var]
    return bf16(xn)


def forward_normalized(params: np.ndarray, xn: np.ndarray) -> np.ndarray:
    layers = unpack(params)
    h = xn
    for li, (w, b) in enumerate(layers):
        z = h @ bf16(w) + b
        h = bf16(np.maximum(z, 0.0)) if li < 3 else z
    return h[:, :NOUT]


def forward(params: np.ndarray, x: np.ndarray, norm: np.ndarray) -> np.ndarray:
    """(n, 81) raw inputs -> (n, 3) displacements (east km, north km, dp hPa)."""
    norm = np.asarray(norm, np.float32)
    y = forward_normalized(params, normalize_inputs(x, norm))
    return norm[6:9] + norm[9:12] * y
