"""Pins of the numpy reference of the surrogate MLP (oracle/mlp.py): the
forward pass against torch's CPU float32 network built here from the flat
parameter array, and the backward pass against torch's CPU autograd (a
wrong transpose, a missing ReLU mask or a wrong loss scale fails these)."""
import numpy as np
import torch

from oracle import mlp


def torch_net(P, xn):
    """The plain network 81 -> 128 -> 128 -> 128 -> 3 from the flat array
    (W[in][out] then bias per layer, padded shapes 96x128, 128x128,
    128x128, 128x16), written without oracle.mlp's slicing."""
    h, off, out = xn, 0, []
    dims = [(81, 128, 96, 128), (128, 128, 128, 128), (128, 128, 128, 128), (128, 3, 128, 16)]
    for li, (fi, fo, pi, po) in enumerate(dims):
        w = P[off:off + pi * po].reshape(pi, po)[:fi, :fo]
        off += pi * po
        b = P[off:off + fo]
        off += po
        out.append((w, b))
        z = h @ w + b
        h = torch.relu(z) if li < 3 else z
    return h, out


def case(rng, n=257):
    P = (rng.standard_normal(47504) * 0.1).astype(np.float32)
    x = rng.standard_normal((n, 81)).astype(np.float32) * 5 + 1
    y = rng.standard_normal((n, 3)).astype(np.float32) * 20
    norm = np.array([1.0, 0.5, -0.2, 5.0, 4.0, 0.01, 0.3, -0.1, 2.0, 30.0, 20.0, 5.0], np.float32)
    return P, x, y, norm


def test_forward_matches_torch(rng):
    P, x, _, norm = case(rng)
    got = mlp.forward(P, x, norm)
    xn = torch.from_numpy(mlp.normalize_inputs(x, norm))
    # bf16 weights; hidden activations rounded to bf16 after each ReLU
    h, off = xn, 0
    dims = [(81, 128, 96, 128), (128, 128, 128, 128), (128, 128, 128, 128), (128, 3, 128, 16)]
    for li, (fi, fo, pi, po) in enumerate(dims):
        w = torch.from_numpy(mlp.bf16(P[off:off + pi * po].reshape(pi, po)[:fi, :fo]))
        off += pi * po
        b = torch.from_numpy(P[off:off + fo])
        off += po
        z = h @ w + b
        h = torch.from_numpy(mlp.bf16(torch.relu(z).numpy())) if li < 3 else z
    want = norm[6:9] + norm[9:12] * h.numpy()
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-5 * np.abs(want).max())


def test_padding_is_inert(rng):
    """Layer-1 rows >= 81 and layer-4 columns >= 3 of the flat array are
    padding: changing them changes nothing."""
    P = (rng.standard_normal(47504) * 0.1).astype(np.float32)
    x = rng.standard_normal((64, 81)).astype(np.float32)
    norm = np.array([0, 0, 0, 1, 1, 1, 0, 0, 0, 1, 1, 1], np.float32)
    a = mlp.forward(P, x, norm)
    Q = P.copy()
    Q[81 * 128:96 * 128] = 7.0                     # layer-1 rows 81..95
    off4 = 96 * 128 + 128 + 2 * (128 * 128 + 128)
    w4 = Q[off4:off4 + 128 * 16].reshape(128, 16)
    w4[:, 3:] = -3.0                               # layer-4 columns 3..15
    Q[off4 + 128 * 16 + 3:off4 + 128 * 16 + 16] = 9.0   # layer-4 bias 3..15
    np.testing.assert_array_equal(a, mlp.forward(Q, x, norm))


def test_backward_matches_autograd(rng):
    """Unrounded backward (float32 gradients) against autograd through the
    same bf16 weights and bf16 activations, element by element."""
    P, x, y, norm = case(rng, 512)
    loss, g = mlp.grad(P, x, y, norm, round_bf16=False)
    Pb = torch.from_numpy(P.copy())
    # autograd on the bf16-rounded weights; the forward keeps the GPU's
    # bf16 activations (rounding treated as identity in the backward)
    layers = []
    off = 0
    dims = [(81, 128, 96, 128), (128, 128, 128, 128), (128, 128, 128, 128), (128, 3, 128, 16)]
    for fi, fo, pi, po in dims:
        w = torch.from_numpy(mlp.bf16(P[off:off + pi * po].reshape(pi, po)[:fi, :fo])).requires_grad_(True)
        off += pi * po
        b = torch.from_numpy(P[off:off + fo].copy()).requires_grad_(True)
        off += po
        layers.append((w, b))
    h = torch.from_numpy(mlp.normalize_inputs(x, norm))
    for li, (w, b) in enumerate(layers):
        z = h @ w + b
        if li < 3:
            r = torch.relu(z)
            h = r + (torch.from_numpy(mlp.bf16(r.detach().numpy())) - r).detach()
        else:
            h = z
    tn = torch.from_numpy(((y - norm[6:9]) / norm[9:12]).astype(np.float32))
    L = ((h - tn) ** 2).mean()
    L.backward()
    assert abs(loss - L.item()) <= 1e-5 * L.item()
    for li, (w, b) in enumerate(layers):
        for mine, ref in ((g[li][0], w.grad.numpy()), (g[li][1], b.grad.numpy())):
            assert mine.shape == ref.shape
            np.testing.assert_allclose(mine, ref, rtol=2e-4, atol=2e-5 * np.abs(ref).max())


def test_rounded_backward_is_near_the_exact_one(rng):
    """Rounding the four gradient layers to bf16 moves each weight gradient
    by a few bf16 ulps of the layer's scale, no more."""
    P, x, y, norm = case(rng, 512)
    _, ga = mlp.grad(P, x, y, norm, round_bf16=True)
    _, gb = mlp.grad(P, x, y, norm, round_bf16=False)
    for li in range(4):
        for a, b in zip(ga[li], gb[li]):
            assert np.abs(a - b).max() <= 2e-2 * np.abs(b).max()
