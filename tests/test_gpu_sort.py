"""The sort by grid-box tile (Sec. 6, sorting modules) on inputs built to
exercise how ranks are counted: runs of one key that are longer than a wave
and cross the groups of parcels a thread handles, ragged totals (1 parcel, a
partial wave, a partial block), non-finite positions, and a second sort of
already sorted parcels.  After each sort: the ids are a permutation, the
tile keys of the oracle never decrease along the array, and every field
(position, FP64 or FP32 mesoscale state) moved with its parcel."""
import numpy as np
import pytest

import inputs
import oracle
from gpu_common import require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpt():
    return require_gpu()


@pytest.fixture(scope="module")
def met3():
    return inputs.make_met_c1(seed=11, nt=3)


def clustered(met, n, seed):
    """Parcels in three boxes of a few tiles each (long runs of equal keys),
    2 % of them with a non-finite coordinate, mesoscale state random."""
    rng = np.random.default_rng(seed)
    part = inputs.make_particles(n, seed)
    box = rng.integers(0, 3, n)
    lon_c = np.array([10.0, 200.0, 355.0])[box]
    lat_c = np.array([-40.0, 0.0, 60.0])[box]
    p_c = np.array([850.0, 300.0, 50.0])[box]
    part.lon = lon_c + rng.uniform(0.0, 3.0 * met.dlon * 8, n)
    part.lat = lat_c + rng.uniform(0.0, 2.0 * met.dlat * 8, n)
    part.p = p_c * np.exp(rng.uniform(-0.15, 0.15, n))
    bad = rng.random(n) < 0.02
    which = rng.integers(0, 3, n)
    part.lon[bad & (which == 0)] = np.nan
    part.lat[bad & (which == 1)] = np.inf
    part.p[bad & (which == 2)] = np.nan
    part.up, part.vp, part.wp = (rng.normal(size=n) for _ in range(3))
    return part


def check_sorted(met, h, ref, math):
    n = ref.n
    np.testing.assert_array_equal(np.sort(h.id), np.arange(n, dtype=np.uint32))
    for f in ("lon", "lat", "p"):
        np.testing.assert_array_equal(getattr(h, f), getattr(ref, f)[h.id])
    for f in ("up", "vp", "wp"):
        want = getattr(ref, f)[h.id]
        if math == 1:
            want = want.astype(np.float32).astype(np.float64)
        np.testing.assert_array_equal(getattr(h, f), want)
    keys = oracle.tile_keys(oracle.Met(met), h.lon, h.lat, h.p).astype(np.int64)
    assert np.all(np.diff(keys) >= 0)


@pytest.mark.parametrize("math", [0, 1])
@pytest.mark.parametrize("n", [1, 63, 65, 1023, 1025, 20011])
def test_sort_runs_ragged_and_resorted(mpt, met3, n, math):
    import torch
    say(f"[sort] clustered n={n} math={math}")
    part = clustered(met3, n, 500 + n)
    ctx = mpt.Context(met3, mpt.make_params(math=math, sort_interval=1), n_max=n)
    ctx.upload_met(met3)
    P = mpt.DeviceParticles.from_host(part, math=math)
    for _ in range(2):
        ctx.sort(P)
        torch.cuda.synchronize()
        check_sorted(met3, P.to_host(), part, math)
