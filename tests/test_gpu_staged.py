"""The LDS-staged winds of the step kernels against the per-parcel gathers.

Dense parcels in two small regions (one across the longitude seam, one near
a pole), sorted every 10 steps: every block's parcels then fit the staged
box, which the test checks on the host from the sorted positions.  The same
parcels interleaved with decoys half a circle away and left unsorted make
every block's box span the globe, so those blocks gather each parcel's 16
records from global memory instead.  Both paths weight each corner in time
first and then interpolate with the same operations: the original parcels'
final states must be equal bit for bit (the decoys do not change them:
parcels are independent).  A sample of ids is compared with the oracle."""
import numpy as np
import pytest

import inputs
import oracle
from gpu_common import (TOL_F64_DEG, TOL_F64_HPA, TOL_R32_DEG, TOL_R32_HPA, assert_bitwise, by_id,
                        compare, oracle_run, require_gpu, say)
from oracle import encode

pytestmark = pytest.mark.gpu

# capacity of the staged box in grid points: FP32-arithmetic and FP64 forms
BOX_CAP = {0: 1536, 1: 1280}


@pytest.fixture(scope="module")
def mpt():
    return require_gpu()


@pytest.fixture(scope="module")
def met3():
    return inputs.make_met_c1(seed=11, nt=3)


def dense(n, seed):
    """Half the parcels in lon 352..368 (across the seam), lat -10..6,
    p 420..560 hPa; half in lon 40..56, lat 72..88, p 200..260 hPa."""
    rng = np.random.default_rng(seed)
    part = inputs.make_particles(n, seed)
    h = n // 2
    part.lon[:h] = np.mod(rng.uniform(352.0, 368.0, h), 360.0)
    part.lat[:h] = rng.uniform(-10.0, 6.0, h)
    part.p[:h] = rng.uniform(420.0, 560.0, h)
    part.lon[h:] = rng.uniform(40.0, 56.0, n - h)
    part.lat[h:] = rng.uniform(72.0, 88.0, n - h)
    part.p[h:] = rng.uniform(200.0, 260.0, n - h)
    return part


def boxes_fit(met, part, cap):
    """Host check: the fraction of blocks of 256 parcels, after the sort by
    tile, whose cell bounding box (corners included, longitude taken the
    short way round) has at most cap grid points."""
    m = oracle.Met(met)
    keys = oracle.tile_keys(m, part.lon, part.lat, part.p)
    o = np.argsort(keys, kind="stable")
    i0, j, k = (a[o] for a in cells(met, part))
    fit = []
    for b in range(0, part.n, 256):
        ii, jj, kk = i0[b:b + 256], j[b:b + 256], k[b:b + 256]
        ext = min(np.ptp(ii), np.ptp((ii + met.nx // 2) % met.nx))
        fit.append((ext + 2) * (np.ptp(jj) + 2) * (np.ptp(kk) + 2) <= cap)
    return float(np.mean(fit))


def cells(met, part):
    i0 = np.floor(np.mod(part.lon - met.lon0, 360.0) / met.dlon).astype(np.int64) % met.nx
    j = np.clip(np.floor((np.clip(part.lat, -90, 90) - met.lat0) / met.dlat).astype(np.int64), 0, met.ny - 2)
    asc = np.asarray(met.plev)[::-1]
    pc = np.clip(part.p, met.plev[-1], met.plev[0])
    k = np.clip(met.nz - 1 - np.searchsorted(asc, pc, side="left"), 0, met.nz - 2)
    return i0, j, k


def run(mpt, met, part, math, dtype, sort_interval, nsteps, flags=7, dt=180.0):
    import torch
    ctx = mpt.Context(met, mpt.make_params(dt=dt, math=math, sort_interval=sort_interval, fuse=10, flags=flags),
                      n_max=part.n, dtype=dtype)
    ctx.upload_met(met)
    P = mpt.DeviceParticles.from_host(part, math=math, pingpong=sort_interval > 0)
    ctx.step(P, 0, nsteps)
    torch.cuda.synchronize()
    return by_id(P.to_host())


@pytest.mark.parametrize("form", [(0, 0), (1, 0), (1, 1), (1, 2)])
def test_staged_equals_gathered_bitwise(mpt, met3, form):
    math, dtype = form
    n = 200_000
    part = dense(n, 31)
    frac = boxes_fit(met3, part, BOX_CAP[math])
    say(f"[staged] form {form}: {frac:.4f} of the sorted blocks fit the box")
    assert frac >= 0.99
    a = run(mpt, met3, part, math, dtype, 10, 60)
    # decoys half a circle away, interleaved, unsorted: every box spans the globe
    rng = np.random.default_rng(5)
    dec = part.copy()
    dec.lon = np.mod(part.lon + 180.0, 360.0)
    dec.id = part.id + np.uint32(n)
    both = inputs.Particles(*(np.concatenate([getattr(part, f), getattr(dec, f)])
                              for f in ("lon", "lat", "p", "id", "up", "vp", "wp")))
    both = both.subset(rng.permutation(2 * n))
    b = run(mpt, met3, both, math, dtype, 0, 60)
    b = b.subset(np.arange(n))                       # ids 0 .. n-1, by id
    assert_bitwise(a, b)


@pytest.mark.parametrize("form", [(0, 0), (1, 0)])
def test_one_staging_with_midpoints_off_the_box(mpt, met3, form):
    """The F64 and F32 forms stage each step's box once, for the start
    cells, and the lanes whose midpoint cell leaves it (or whose midpoint
    falls in the next time-level pair) gather.  A step of 1500 s sends many
    more midpoints off the box than the 180 s of the workload, and the step
    from 21000 s has its midpoint past the time level at 21600 s; the result
    must still equal the all-gather run bit for bit."""
    math, dtype = form
    n = 100_000
    part = dense(n, 33)
    a = run(mpt, met3, part, math, dtype, 10, 20, dt=1500.0)
    rng = np.random.default_rng(6)
    dec = part.copy()
    dec.lon = np.mod(part.lon + 180.0, 360.0)
    dec.id = part.id + np.uint32(n)
    both = inputs.Particles(*(np.concatenate([getattr(part, f), getattr(dec, f)])
                              for f in ("lon", "lat", "p", "id", "up", "vp", "wp")))
    both = both.subset(rng.permutation(2 * n))
    b = run(mpt, met3, both, math, dtype, 0, 20, dt=1500.0)
    b = b.subset(np.arange(n))
    assert_bitwise(a, b)
    moved = oracle.chord_deg(part.lon, part.lat, a.lon, a.lat)
    say(f"[one staging] form {form}: median distance after 20 steps of 1500 s {np.median(moved):.2f} deg")


@pytest.mark.parametrize("form", [(0, 0), (1, 0), (1, 1)])
def test_staged_against_the_oracle(mpt, met3, form):
    """Sampled ids of the dense sorted run against the oracle: FP64 over 60
    steps with all modules; the FP32-arithmetic forms over one step with all
    modules and 60 steps of advection and turbulence (continuous in the
    position), on the stored values."""
    math, dtype = form
    n = 200_000
    part = dense(n, 32)
    ids = np.random.default_rng(9).choice(n, 3000, replace=False)
    sub = part.subset(np.sort(ids))
    met_o = met3 if dtype == 0 else encode.dequantized_met(met3, dtype)
    runs = [(7, 60)] if math == 0 else [(7, 1), (3, 60)]
    for flags, nsteps in runs:
        g = run(mpt, met3, part, math, dtype, 10, nsteps, flags=flags).subset(np.sort(ids))
        r = oracle_run(met_o, sub, 0, nsteps, flags=flags)
        if math == 0:
            compare(g, r, TOL_F64_DEG, TOL_F64_HPA, f"staged F64 flags {flags}")
        else:
            compare(g, r, TOL_R32_DEG, TOL_R32_HPA, f"staged form {form} flags {flags} steps {nsteps}")
