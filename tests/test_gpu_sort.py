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
from gpu_common import by_id, oracle_run, require_gpu, say

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


def sorted_by_oracle_keys(met, h, frac=0.0):
    """The tile keys of the oracle never decrease along the array, except for
    at most frac of the places (positions within rounding of a boundary)."""
    keys = oracle.tile_keys(oracle.Met(met), h.lon, h.lat, h.p).astype(np.int64)
    bad = int(np.sum(np.diff(keys) < 0))
    assert bad <= frac * len(keys), bad
    return keys


@pytest.mark.parametrize("form", [(0, 0), (1, 0), (1, 1)])
def test_presort_keys_from_the_step(mpt, met3, form):
    """presort: the step's last launch leaves the keys of the final positions;
    the sort that follows uses them instead of its key pass and orders the
    parcels as that pass would (and moves the whole state with them)."""
    import torch
    math, dtype = form
    say(f"[sort] presort math={math} dtype={dtype}")
    part = inputs.make_particles(20_011, 61)
    out = []
    for presort in (1, 0):
        ctx = mpt.Context(met3, mpt.make_params(math=math, fuse=10, presort=presort), n_max=part.n, dtype=dtype)
        ctx.upload_met(met3)
        P = mpt.DeviceParticles.from_host(part, math=math)
        ctx.step(P, 0, 10)
        ctx.sort(P)
        torch.cuda.synchronize()
        h = P.to_host()
        np.testing.assert_array_equal(np.sort(h.id), np.arange(part.n, dtype=np.uint32))
        out.append((sorted_by_oracle_keys(met3, h), by_id(h)))
    np.testing.assert_array_equal(out[0][0], out[1][0])        # the same key sequence
    for f in ("lon", "lat", "p", "up", "vp", "wp"):
        np.testing.assert_array_equal(getattr(out[0][1], f), getattr(out[1][1], f))


def test_sorts_inside_a_call_use_the_launch_keys(mpt, met3):
    """mpt_step with sort_interval 10: the sort at step 10 takes its keys from
    the launch that ends there; the parcels leave the call in the order of
    their cells at step 10 (by the oracle's positions at step 10)."""
    import torch
    part = inputs.make_particles(20_000, 62)
    ctx = mpt.Context(met3, mpt.make_params(math=0, sort_interval=10, fuse=10), n_max=part.n)
    ctx.upload_met(met3)
    P = mpt.DeviceParticles.from_host(part, math=0)
    ctx.step(P, 0, 20)
    torch.cuda.synchronize()
    h = P.to_host()
    at10 = oracle_run(met3, part, 0, 10)                        # ordered by id
    order10 = at10.subset(h.id.astype(np.int64))
    sorted_by_oracle_keys(met3, order10, frac=1e-3)


def test_presort_keys_of_changed_positions_still_permute(mpt, met3):
    """Positions changed by the caller between the step and the sort: the sort
    follows the stale keys, but every parcel's whole state moves together."""
    import torch
    part = inputs.make_particles(5_000, 63)
    ctx = mpt.Context(met3, mpt.make_params(math=0, fuse=10, presort=1), n_max=part.n)
    ctx.upload_met(met3)
    P = mpt.DeviceParticles.from_host(part, math=0)
    ctx.step(P, 0, 10)
    torch.cuda.synchronize()
    P.lat.mul_(-1.0)                                            # the caller moves the parcels
    before = by_id(P.to_host())
    ctx.sort(P)
    torch.cuda.synchronize()
    h = P.to_host()
    np.testing.assert_array_equal(np.sort(h.id), np.arange(part.n, dtype=np.uint32))
    for f in ("lon", "lat", "p", "up", "vp", "wp"):
        np.testing.assert_array_equal(getattr(by_id(h), f), getattr(before, f))


def test_presort_keys_dropped_by_other_calls(mpt, met3):
    """A call that moves the parcels without keys (mpt_advect) drops them:
    the next sort orders by the current positions."""
    import torch
    part = inputs.make_particles(20_000, 64)
    ctx = mpt.Context(met3, mpt.make_params(math=0, fuse=10, presort=1), n_max=part.n)
    ctx.upload_met(met3)
    P = mpt.DeviceParticles.from_host(part, math=0)
    ctx.step(P, 0, 10)
    for s in range(10, 40):
        ctx.advect(P, s)
    ctx.sort(P)
    torch.cuda.synchronize()
    sorted_by_oracle_keys(met3, P.to_host())


@pytest.mark.parametrize("form", [(0, 0), (1, 0), (1, 1)])
def test_deferred_sort_equals_sort_then_step(mpt, met3, form):
    """mpt_sort_particles_deferred + mpt_step: the launch reads the parcels
    through the sort's order and writes them sorted.  Final states by id
    equal those of mpt_sort_particles + mpt_step bit for bit (parcels are
    independent); the order left is the order of the oracle's keys of the
    positions at the sort; every field moved with its parcel, non-finite
    parcels included (the clustered set has 2 % of them)."""
    import torch
    math, dtype = form
    say(f"[sort] deferred math={math} dtype={dtype}")
    part = clustered(met3, 50_003, 71)
    out = []
    for deferred in (False, True):
        ctx = mpt.Context(met3, mpt.make_params(math=math, fuse=10), n_max=part.n, dtype=dtype)
        ctx.upload_met(met3)
        P = mpt.DeviceParticles.from_host(part, math=math)
        (ctx.sort_deferred if deferred else ctx.sort)(P)
        ctx.step(P, 0, 10)
        torch.cuda.synchronize()
        h = P.to_host()
        np.testing.assert_array_equal(np.sort(h.id), np.arange(part.n, dtype=np.uint32))
        keys = oracle.tile_keys(oracle.Met(met3), part.lon, part.lat, part.p).astype(np.int64)[h.id]
        assert np.all(np.diff(keys) >= 0)
        out.append(by_id(h))
    for f in ("lon", "lat", "p", "up", "vp", "wp"):
        np.testing.assert_array_equal(getattr(out[0], f), getattr(out[1], f))


def test_deferred_sort_dropped_by_other_calls(mpt, met3):
    """A deferred order is dropped, unused, by a sort in between, and by a
    step on other parcels; nothing moves until a step consumes it."""
    import torch
    part = clustered(met3, 20_000, 72)
    ctx = mpt.Context(met3, mpt.make_params(math=0, fuse=10), n_max=part.n)
    ctx.upload_met(met3)
    P = mpt.DeviceParticles.from_host(part, math=0)
    ctx.sort_deferred(P)
    torch.cuda.synchronize()
    h0 = P.to_host()
    np.testing.assert_array_equal(h0.id, part.id)               # nothing moved yet
    ctx.sort(P)                                                  # drops the order
    Q = mpt.DeviceParticles.from_host(part, math=0)
    ctx.sort_deferred(Q)
    ctx.step(P, 0, 10)                                           # other parcels: Q's order unused
    ctx.step(Q, 0, 10)                                           # dropped by the step on P
    torch.cuda.synchronize()
    hq = Q.to_host()
    np.testing.assert_array_equal(hq.id, part.id)               # Q kept its order
    a, b = by_id(P.to_host()), by_id(hq)
    for f in ("lon", "lat", "p", "up", "vp", "wp"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))


def test_sorts_inside_a_call_equal_explicit_sorts(mpt, met3):
    """mpt_step with sort_interval 10 (each sort deferred into the launch
    after it) against explicit sorts and steps of 10: the same final states
    by id, bit for bit, over 30 steps with all modules."""
    import torch
    part = clustered(met3, 30_001, 73)
    res = []
    for internal in (True, False):
        ctx = mpt.Context(met3, mpt.make_params(math=1, sort_interval=10 if internal else 0, fuse=10),
                          n_max=part.n)
        ctx.upload_met(met3)
        P = mpt.DeviceParticles.from_host(part, math=1)
        if internal:
            ctx.step(P, 0, 30)
        else:
            for s0 in (0, 10, 20):
                ctx.sort(P)
                ctx.step(P, s0, 10)
        torch.cuda.synchronize()
        res.append(by_id(P.to_host()))
    for f in ("lon", "lat", "p", "up", "vp", "wp"):
        np.testing.assert_array_equal(getattr(res[0], f), getattr(res[1], f))
