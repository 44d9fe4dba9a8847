"""Surrogate MLP, numpy reference -- TEST INFRASTRUCTURE ONLY.

The network is the plain ReLU MLP 81 -> 128 -> 128 -> 128 -> 3 (a project
addition; the paper has no surrogate).  It is evaluated in float32 on
bfloat16-rounded weights, inputs and hidden activations, the values the GPU
multiplies (its MFMA products are exact bf16 x bf16 products accumulated
in FP32).

The library passes the parameters as one flat FP32 array whose layout is
part of its C ABI: per layer W[in][out] then the bias, with the padded
shapes FLAT_SHAPES (layer 1 has 96 input rows, layer 4 has 16 output
columns; the padding is zero and takes no part in the network).  ``layers``
cuts the plain matrices out of that array; everything below works on the
plain shapes only.
"""
from __future__ import annotations

import numpy as np

from . import encode

NIN, NHID, NOUT = 81, 128, 3
SHAPES = [(NIN, NHID), (NHID, NHID), (NHID, NHID), (NHID, NOUT)]
FLAT_SHAPES = [(96, 128), (128, 128), (128, 128), (128, 16)]


def layers(params: np.ndarray):
    """[(W [in][out], b [out])] of the plain network, from the flat array."""
    params = np.asarray(params, np.float32)
    out, off = [], 0
    for (fi, fo), (pi, po) in zip(SHAPES, FLAT_SHAPES):
        w = params[off:off + pi * po].reshape(pi, po)[:fi, :fo]
        off += pi * po
        b = params[off:off + po][:fo]
        off += po
        out.append((w, b))
    assert off == params.size
    return out


def flat_offsets():
    """(offset of W, offset of b) of each layer in the flat array."""
    out, off = [], 0
    for pi, po in FLAT_SHAPES:
        out.append((off, off + pi * po))
        off += pi * po + po
    return out


def bf16(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    return encode.bf16_bits_to_f32(encode.bf16_rne_bits(x)).reshape(x.shape)


def normalize_inputs(x: np.ndarray, norm: np.ndarray) -> np.ndarray:
    """(n, 81) raw inputs -> normalized, rounded to bf16.  Inputs 27 v ..
    27 v + 26 belong to variable v (u, v, w)."""
    x = np.asarray(x, np.float32)
    norm = np.asarray(norm, np.float32)
    var = np.arange(NIN) // 27
    return bf16((x - norm[var]) / norm[3 + var])


def forward_normalized(params: np.ndarray, xn: np.ndarray, keep: bool = False):
    """Normalized outputs (n, 3); with keep, also the bf16 activations
    [xn, h1, h2, h3] each layer multiplies."""
    h = xn
    acts = [xn]
    L = layers(params)
    for li, (w, b) in enumerate(L):
        z = h @ bf16(w) + b
        if li < 3:
            h = bf16(np.maximum(z, 0.0))
            acts.append(h)
        else:
            h = z
    return (h, acts) if keep else h


def forward(params: np.ndarray, x: np.ndarray, norm: np.ndarray) -> np.ndarray:
    """(n, 81) raw inputs -> (n, 3) displacements (east km, north km, dp hPa)."""
    norm = np.asarray(norm, np.float32)
    y = forward_normalized(params, normalize_inputs(x, norm))
    return norm[6:9] + norm[9:12] * y


def grad(params: np.ndarray, x: np.ndarray, y: np.ndarray, norm: np.ndarray,
         round_bf16: bool = True):
    """Loss (mean over the batch and the 3 outputs of the squared error of
    the normalized outputs) and its gradient with respect to the plain
    parameters: [(dW, db)] per layer, float64.

    Backpropagation by the chain rule: dY = 2 (Y - T) / (3 B);
    dH3 = (dY W4^T) masked by H3 > 0; dH2 = (dH3 W3^T) masked by H2 > 0;
    dH1 = (dH2 W2^T) masked by H1 > 0; dW_l = A_l^T dH_l, db_l = sum of dH_l
    over the batch (A_l = the layer's input).  With round_bf16 the output
    gradient and the three hidden gradients are rounded to bf16 where they
    are formed, as the GPU keeps them (its products use those bf16 values);
    without, the same steps in float32 (for pinning against autograd)."""
    rnd = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float32))
    norm = np.asarray(norm, np.float32)
    y = np.asarray(y, np.float32)
    xn = normalize_inputs(x, norm)
    out, acts = forward_normalized(params, xn, keep=True)
    tn = (y - norm[6:9]) / norm[9:12]
    B = x.shape[0]
    e = out - tn
    loss = float(np.mean(np.asarray(e, np.float64) ** 2))
    L = layers(params)
    g = rnd(np.float32(2.0 / (NOUT * B)) * e)
    grads = [None] * 4
    for li in (3, 2, 1, 0):
        a = np.asarray(acts[li], np.float64)
        grads[li] = (a.T @ np.asarray(g, np.float64), np.asarray(g, np.float64).sum(axis=0))
        if li == 0:
            break
        back = g @ bf16(L[li][0]).T
        g = rnd(np.where(acts[li] > 0.0, back, 0.0))
    return loss, grads
