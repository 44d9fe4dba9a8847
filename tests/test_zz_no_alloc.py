"""mpt_sort_particles_noalloc, the sort whose scratch is the library's fixed
per-device array instead of the context's workspace, against
mpt_sort_particles on the same parcels: two calls in a row on the same
contexts, the second with fewer parcels (the fixed array keeps the first
call's contents).  Order inside a tile is not unique (atomics), so the test
compares what is: the sequence of tile keys along the array, the set of
parcel ids under each key, and every field of every parcel (by id)."""
import ctypes

import numpy as np
import pytest

import inputs
import oracle
from gpu_common import by_id, require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpt():
    return require_gpu()


@pytest.fixture(scope="module")
def met3():
    return inputs.make_met_c1(seed=11, nt=3)


def clustered(met, n, seed):
    """Uniform parcels plus a third of them packed into a few tiles (runs of
    equal keys longer than a wave), 1 % with a non-finite coordinate."""
    rng = np.random.default_rng(seed)
    part = inputs.make_particles(n, seed)
    m = n // 3
    part.lon[:m] = 200.0 + rng.uniform(0.0, 2.0 * met.dlon * 8, m)
    part.lat[:m] = -30.0 + rng.uniform(0.0, met.dlat * 8, m)
    part.p[:m] = 300.0 * np.exp(rng.uniform(-0.1, 0.1, m))
    bad = rng.random(n) < 0.01
    part.lat[bad] = np.nan
    part.up, part.vp, part.wp = (rng.normal(size=n) for _ in range(3))
    return part


def keys_and_groups(met, h):
    keys = oracle.tile_keys(oracle.Met(met), h.lon, h.lat, h.p).astype(np.int64)
    assert np.all(np.diff(keys) >= 0)
    cuts = np.flatnonzero(np.diff(keys)) + 1
    groups = [np.sort(g) for g in np.split(h.id.astype(np.int64), cuts)]
    return keys, groups


def test_noalloc_sort_equals_workspace_sort_on_two_calls(mpt, met3):
    import torch
    math = 1
    ctx_ref = mpt.Context(met3, mpt.make_params(math=math, sort_interval=10), n_max=300_000)
    ctx_ref.upload_met(met3)
    # n_max = 0: the context holds no sort scratch; the fixed array serves
    ctx_na = mpt.Context(met3, mpt.make_params(math=math, sort_interval=10), n_max=0)
    ctx_na.upload_met(met3)
    for call, n in enumerate((300_000, 20_011)):
        say(f"[noalloc] call {call}: n={n}")
        part = clustered(met3, n, 900 + call)
        A = mpt.DeviceParticles.from_host(part, math=math)
        B = mpt.DeviceParticles.from_host(part, math=math)
        ctx_ref.sort(A)
        ctx_na.sort_noalloc(B)
        torch.cuda.synchronize()
        ha, hb = A.to_host(), B.to_host()
        np.testing.assert_array_equal(np.sort(hb.id), np.arange(n, dtype=np.uint32))
        ka, ga = keys_and_groups(met3, ha)
        kb, gb = keys_and_groups(met3, hb)
        np.testing.assert_array_equal(ka, kb)
        assert len(ga) == len(gb)
        for x, y in zip(ga, gb):
            np.testing.assert_array_equal(x, y)
        oa, ob = by_id(ha), by_id(hb)
        for f in ("lon", "lat", "p", "up", "vp", "wp", "id"):
            np.testing.assert_array_equal(getattr(oa, f), getattr(ob, f), err_msg=f)
        np.testing.assert_array_equal(ob.lon, part.lon)


def test_noalloc_sort_with_scenarios(mpt, met3):
    """Parcels of scenarios not yet released go behind the tiles in release
    order, as with the workspace sort."""
    import torch
    n = 50_000
    part = inputs.make_particles(n, 905)
    scen = (np.arange(n) % 5).astype(np.uint16)
    release = np.array([0, 30, 10, 0, 20], np.int32)
    hs = []
    for use_na in (False, True):
        ctx = mpt.Context(met3, mpt.make_params(math=0, sort_interval=10), n_max=n if not use_na else 0)
        ctx.upload_met(met3)
        ctx.set_release(release)
        P = mpt.DeviceParticles.from_host(part, math=0, scen=scen)
        (ctx.sort_noalloc if use_na else ctx.sort)(P)
        torch.cuda.synchronize()
        hs.append((P.to_host(), P.scen.cpu().numpy().view(np.uint16)))
    (ha, sa), (hb, sb) = hs
    m = int(np.sum(release[scen] <= 0))                  # released parcels come first, by tile
    assert np.all(release[sa[:m]] <= 0) and np.all(release[sb[:m]] <= 0)
    np.testing.assert_array_equal(sa[m:], sb[m:])         # then the pending ones, in release order
    ka, ga = keys_and_groups(met3, ha.subset(np.arange(m)))
    kb, gb = keys_and_groups(met3, hb.subset(np.arange(m)))
    np.testing.assert_array_equal(ka, kb)
    for x, y in zip(ga, gb):
        np.testing.assert_array_equal(x, y)
    for f in ("lon", "lat", "p", "id"):
        np.testing.assert_array_equal(getattr(by_id(ha), f), getattr(by_id(hb), f))


def test_noalloc_sort_limits(mpt, met3):
    """Beyond the fixed array's size the call fails with MPT_ERR_WORKSPACE and
    enqueues nothing; an empty set is a no-op."""
    ctx = mpt.Context(met3, mpt.make_params(math=0, sort_interval=10), n_max=0)
    s = mpt.ParticlesC(n=mpt.NOALLOC_SORT_MAX_N + 1)
    assert mpt.lib().mpt_sort_particles_noalloc(ctx.h, ctypes.byref(s), None) == -4
    s = mpt.ParticlesC(n=0)
    assert mpt.lib().mpt_sort_particles_noalloc(ctx.h, ctypes.byref(s), None) == 0
    assert mpt.lib().mpt_sort_particles_noalloc(None, ctypes.byref(s), None) == -1
