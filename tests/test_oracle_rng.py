"""Pins of the oracle's random numbers.

The paper draws three normals per parcel and step for turbulent and three for
mesoscale diffusion (Sec. 4.3, Listing 6, randoms_t).  Here they come from a
counter-based Philox4x32-10 (Salmon et al., SC'11) keyed by (id, step,
purpose) and a Box-Muller transform; these tests pin the generator against an
independent implementation (rocRAND's header, run on the host) and pin the
normals by their distribution.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("pin") / "rocrand_philox")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "pins", "rocrand_philox.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(ctr: np.ndarray, key) -> np.ndarray:
        ctr = np.asarray(ctr, np.uint64).reshape(-1, 4)
        lines = "\n".join(f"{a} {b} {c} {d} {key[0]} {key[1]}" for a, b, c, d in ctr) + "\n"
        out = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout
        return np.array([[int(x) for x in ln.split()] for ln in out.strip().splitlines()], np.uint32)

    return run


def test_philox_zero_block_matches_rocrand(rocrand_philox):
    ctr = np.zeros((1, 4), np.uint32)
    np.testing.assert_array_equal(oracle.philox(ctr, [0, 0]), rocrand_philox(ctr, [0, 0]))


def test_philox_random_blocks_match_rocrand(rocrand_philox, rng):
    n = 400
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] &= (1 << 30) - 1          # rocRAND offset must fit in 64 bits
    for key in ([0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [221112616, 0], [0x9ABCDEF0, 0x12345678]):
        np.testing.assert_array_equal(oracle.philox(ctr, key), rocrand_philox(ctr, key))


def test_philox_parcel_counters_match_rocrand(rocrand_philox):
    """The counters the step actually uses: (id, step, purpose, 0), key = seed."""
    ids = np.array([0, 1, 2, 12345, 99_999_999, 2**32 - 1], np.uint64)
    ctr = []
    for i in ids:
        for step in (0, 1, 239, 479):
            for purpose in (0, 1):
                ctr.append([i, step, purpose, 0])
    ctr = np.array(ctr, np.uint64)
    seed = oracle.SEED
    key = [seed & 0xFFFFFFFF, seed >> 32]
    np.testing.assert_array_equal(oracle.philox(ctr, key), rocrand_philox(ctr, key))


def test_uniform_map_endpoints():
    # ((x >> 8) + 1/2) / 2^24: strictly inside (0, 1), symmetric about 1/2
    assert oracle.uniform(0) == 2.0**-25
    assert oracle.uniform(0xFFFFFFFF) == 1.0 - 2.0**-25
    assert oracle.uniform(0x80000000) == 0.5 + 2.0**-25
    assert oracle.uniform(0x000000FF) == 2.0**-25          # low byte ignored


def test_box_muller_polar_invariants(rng):
    """xi0, xi1 are the Cartesian coordinates of radius sqrt(-2 ln u0) at
    angle 2 pi u1; xi2 has |xi2| <= sqrt(-2 ln u2)."""
    ids = rng.integers(0, 2**32, 2000, dtype=np.uint64).astype(np.uint32)
    seed = oracle.SEED
    xi = oracle.normals(seed, ids, 17, 1)
    ctr = np.stack([ids, np.full_like(ids, 17), np.full_like(ids, 1), np.zeros_like(ids)], 1)
    x = oracle.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32]).astype(np.float64)
    u = (np.floor(x / 256.0) + 0.5) / 2.0**24
    r2 = xi[:, 0] ** 2 + xi[:, 1] ** 2
    np.testing.assert_allclose(r2, -2.0 * np.log(u[:, 0]), rtol=1e-12)
    ang = np.mod(np.arctan2(xi[:, 1], xi[:, 0]), 2 * np.pi)
    d = np.abs(ang - 2 * np.pi * u[:, 1])
    d = np.minimum(d, 2 * np.pi - d)
    assert d.max() < 1e-9
    assert np.all(np.abs(xi[:, 2]) <= np.sqrt(-2.0 * np.log(u[:, 2])) * (1 + 1e-14))


def test_normals_distribution():
    """Mean 0, variance 1, Kolmogorov-Smirnov against N(0,1), no correlation
    between the three components or between purposes."""
    n = 400_000
    ids = np.arange(n, dtype=np.uint32)
    a = oracle.normals(oracle.SEED, ids, 5, 0)
    b = oracle.normals(oracle.SEED, ids, 5, 1)
    for q in range(3):
        col = a[:, q]
        assert abs(col.mean()) < 5 / np.sqrt(n)
        assert abs(col.var() - 1.0) < 5 * np.sqrt(2.0 / n)
        assert stats.kstest(col, "norm").pvalue > 1e-4
    c = np.corrcoef(np.concatenate([a, b], 1).T)
    off = c[~np.eye(6, dtype=bool)]
    assert np.abs(off).max() < 5 / np.sqrt(n)
    assert np.abs(a).max() <= np.sqrt(-2 * np.log(2.0**-25)) + 1e-12


def test_counter_fields_change_the_stream():
    ids = np.arange(64, dtype=np.uint32)
    base = oracle.normals(oracle.SEED, ids, 3, 0)
    assert not np.any(base == oracle.normals(oracle.SEED, ids, 4, 0))
    assert not np.any(base == oracle.normals(oracle.SEED, ids, 3, 1))
    assert not np.any(base == oracle.normals(oracle.SEED + 1, ids, 3, 0))
