"""Pins of the reduced-precision encoding reference (oracle/encode.py):
its bfloat16 rounding against torch's own float32 -> bfloat16 conversion,
its float16 rounding against numpy's, ties to even, and exact decoding."""
import numpy as np
import torch

from oracle import encode


def test_bf16_matches_torch(rng):
    x = (rng.standard_normal(200_000) * 10.0 ** rng.uniform(-6, 3, 200_000)).astype(np.float32)
    ours = encode.bf16_rne_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, ref)


def test_bf16_ties_to_even():
    # 1 + 2^-8 lies halfway between bf16 neighbours 1 and 1 + 2^-7: ties to 1
    x = np.array([1 + 2.0**-8, 1 + 3 * 2.0**-8, -(1 + 2.0**-8)], np.float32)
    got = encode.bf16_bits_to_f32(encode.bf16_rne_bits(x))
    np.testing.assert_array_equal(got, np.array([1.0, 1 + 2.0**-6, -1.0], np.float32))


def test_scales_and_roundtrip(rng):
    f = rng.standard_normal((5, 7, 9)).astype(np.float32) * np.array([1, 10, 0, 1e-4, 50],
                                                                      np.float32)[:, None, None]
    for kind, rel in ((encode.BF16, 2.0**-8), (encode.F16, 2.0**-11)):
        q, s = encode.encode_level(f, kind)
        assert s[2] == 1.0 and np.all((q[2] & 0x7FFF) == 0)     # all-zero level: +-0
        np.testing.assert_array_equal(s[[0, 1, 3, 4]], np.abs(f[[0, 1, 3, 4]]).reshape(4, -1).max(1))
        d = encode.decode_level(q, s, kind)
        err = np.abs(d - f) / s[:, None, None]
        assert err.max() <= rel
        # decoding is exact: q * s equals the float32 product
        v = (encode.bf16_bits_to_f32(q) if kind == encode.BF16 else q.view(np.float16).astype(np.float32))
        np.testing.assert_array_equal(d, v * s[:, None, None])
