"""Pins of the numpy reference of the surrogate MLP (oracle/mlp.py) against
torch's CPU float32 network on the same bf16-rounded weights and inputs."""
import numpy as np
import torch

from oracle import mlp


def test_forward_matches_torch(rng):
    P = (rng.standard_normal(47504) * 0.1).astype(np.float32)
    x = rng.standard_normal((257, 81)).astype(np.float32) * 5 + 1
    norm = np.array([1.0, 0.5, -0.2, 5.0, 4.0, 0.01, 0.3, -0.1, 2.0, 30.0, 20.0, 5.0], np.float32)
    got = mlp.forward(P, x, norm)
    xn = torch.from_numpy(mlp.normalize_inputs(x, norm))
    h, off = xn, 0
    for li, (fi, fo) in enumerate(mlp.SHAPES):
        w = torch.from_numpy(mlp.bf16(P[off:off + fi * fo].reshape(fi, fo)))
        off += fi * fo
        b = torch.from_numpy(P[off:off + fo])
        off += fo
        z = h @ w + b
        h = torch.from_numpy(mlp.bf16(torch.relu(z).numpy())) if li < 3 else z
    want = norm[6:9] + norm[9:12] * h[:, :3].numpy()
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-5 * np.abs(want).max())


def test_padding_is_inert(rng):
    """Inputs beyond 81 and outputs beyond 3 are padding: changing padded
    weights of layer 1 rows >= 81 or layer 4 columns >= 3 changes nothing."""
    P = (rng.standard_normal(47504) * 0.1).astype(np.float32)
    x = rng.standard_normal((64, 81)).astype(np.float32)
    norm = np.array([0, 0, 0, 1, 1, 1, 0, 0, 0, 1, 1, 1], np.float32)
    a = mlp.forward(P, x, norm)
    Q = P.copy()
    Q[81 * 128:96 * 128] = 7.0                     # layer-1 rows 81..95
    off4 = 96 * 128 + 128 + 2 * (128 * 128 + 128)
    w4 = Q[off4:off4 + 128 * 16].reshape(128, 16)
    w4[:, 3:] = -3.0                               # layer-4 columns 3..15
    np.testing.assert_array_equal(a, mlp.forward(Q, x, norm))
