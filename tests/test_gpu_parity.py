"""GPU parity on the tiny workload (2 deg grid, 30 levels): the HIP path
through the C ABI against the FP64 oracle, element by element by parcel id,
plus the invariants the method guarantees (step = advect then diffuse,
sort neutrality, restart, fusion, repeatability, activity gating)."""
import numpy as np
import pytest

import inputs
import oracle
from gpu_common import (TOL_F64_DEG, TOL_F64_HPA, TOL_R32_DEG, TOL_R32_HPA, assert_bitwise,
                        by_id, compare, compare_flips, gpu_run, oracle_run, require_gpu, say)
from oracle import encode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpt():
    return require_gpu()


@pytest.fixture(scope="module")
def met2():
    return inputs.make_met_c1(seed=11, nt=2)


@pytest.fixture(scope="module")
def met3():
    return inputs.make_met_c1(seed=11, nt=3)


def test_tiny_workload_advection_f64(mpt, met2):
    """Config: 1e4 parcels, 60 midpoint steps of 180 s, no diffusion, FP64."""
    say("tiny advection-only F64, n=10000, 60 steps")
    part = inputs.make_particles(10_000, 21)
    g = gpu_run(met2, part, 0, 60, flags=oracle.ADVECT)
    r = oracle_run(met2, part, 0, 60, flags=oracle.ADVECT)
    compare(g, r, TOL_F64_DEG, TOL_F64_HPA, "c1 advect F64")


def test_tiny_full_step_sorted_fused_f64(mpt, met3):
    say("tiny all modules F64, n=10000, 240 steps, sort/10, fuse 10")
    part = inputs.make_particles(10_000, 22)
    g = gpu_run(met3, part, 0, 240, sort_interval=10, fuse=10)
    r = oracle_run(met3, part, 0, 240)
    compare(g, r, TOL_F64_DEG, TOL_F64_HPA, "c1 full F64")
    np.testing.assert_allclose(g.up, r.up, atol=1e-9)
    np.testing.assert_allclose(g.vp, r.vp, atol=1e-9)
    np.testing.assert_allclose(g.wp, r.wp, atol=1e-11)


@pytest.mark.parametrize("n", [1, 63, 255, 257, 1000, 4097])
def test_ragged_sizes(mpt, met3, n):
    say(f"ragged n={n}")
    part = inputs.make_particles(n, 100 + n)
    g = gpu_run(met3, part, 5, 20, sort_interval=4, fuse=3)
    r = oracle_run(met3, part, 5, 20)
    compare(g, r, TOL_F64_DEG, TOL_F64_HPA, f"ragged {n}")


def test_empty(mpt, met3):
    import torch
    part = inputs.make_particles(0, 1)
    ctx = mpt.Context(met3, mpt.make_params(sort_interval=10), n_max=16)
    ctx.upload_met(met3)
    P = mpt.DeviceParticles.from_host(part)
    ctx.step(P, 0, 20)
    ctx.sort(P)
    torch.cuda.synchronize()
    assert P.n == 0


@pytest.mark.parametrize("form", [(0, 0), (1, 0), (1, 1)])
def test_empty_every_entry_point(mpt, met3, form):
    """An empty set through every call that moves or orders parcels (with the
    in-step sort keys, the graph-replayed loop, convection and sedimentation,
    and the surrogate): each returns success and touches nothing; the
    surrogate adds no fallbacks."""
    import torch
    math, dtype = form
    part = inputs.make_particles(0, 1)
    phys = inputs.add_phys_fields(inputs.make_met_c1(seed=11, nt=3), seed=31)
    flags = oracle.ADVECT | oracle.TURB | oracle.MESO | oracle.CONV | oracle.SEDI
    for met, fl in ((met3, None), (phys, flags)):
        kw = {} if fl is None else {"flags": fl}
        ctx = mpt.Context(met, mpt.make_params(math=math, sort_interval=10, fuse=10, presort=1, **kw),
                          n_max=16, dtype=dtype)
        ctx.upload_met(met)
        P = mpt.DeviceParticles.from_host(part, math=math)
        ctx.advect(P, 3)
        ctx.diffuse(P, 3)
        ctx.step(P, 0, 20)
        ctx.sort(P)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            ctx.step_graph(P, 20, 20, s)
        torch.cuda.synchronize()
        assert P.n == 0
    if form != (1, 0):
        return
    ctx = mpt.Context(met3, mpt.make_params(math=1, sort_interval=16), n_max=4096)
    ctx.upload_met(met3)
    rng = np.random.default_rng(7)
    x, y = ctx.surrogate_datagen(*(torch.from_numpy(a).cuda() for a in (
        rng.uniform(0, 360, 1024), rng.uniform(-60, 60, 1024), rng.uniform(100, 900, 1024),
        rng.integers(0, 200, 1024).astype(np.int32))))
    ctx.surrogate_load(ctx.surrogate_init(3), ctx.surrogate_stats(x, y), 1.0)
    P = mpt.DeviceParticles.from_host(part, math=1)
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.step_surrogate(P, 0, 64, fb)
    torch.cuda.synchronize()
    assert fb.item() == 0 and P.n == 0


def test_step_equals_advect_then_diffuse(mpt, met3):
    import torch
    say("step == advect;diffuse bitwise")
    part = inputs.make_particles(3000, 23)
    params = mpt.make_params()
    ctx = mpt.Context(met3, params, n_max=part.n)
    ctx.upload_met(met3)
    A = mpt.DeviceParticles.from_host(part, pingpong=False)
    B = mpt.DeviceParticles.from_host(part, pingpong=False)
    for s in range(12):
        ctx.step(A, s, 1)
        ctx.advect(B, s)
        ctx.diffuse(B, s)
    torch.cuda.synchronize()
    assert_bitwise(A.to_host(), B.to_host())


def test_sort_neutral_and_valid(mpt, met3):
    say("sort neutrality + validity")
    part = inputs.make_particles(20_000, 24)
    a = gpu_run(met3, part, 0, 60, sort_interval=10, fuse=10)
    b = gpu_run(met3, part, 0, 60, sort_interval=0, fuse=10)
    assert_bitwise(a, b)
    # one explicit sort: permutation of ids, keys non-decreasing
    import torch
    ctx = mpt.Context(met3, mpt.make_params(sort_interval=1), n_max=part.n)
    ctx.upload_met(met3)
    P = mpt.DeviceParticles.from_host(part)
    ctx.sort(P)
    torch.cuda.synchronize()
    h = P.to_host()
    np.testing.assert_array_equal(np.sort(h.id), np.arange(part.n, dtype=np.uint32))
    keys = oracle.tile_keys(oracle.Met(met3), h.lon, h.lat, h.p)
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)
    np.testing.assert_array_equal(h.lon, part.lon[h.id])


def test_restart_fusion_repeat_bitwise(mpt, met3):
    say("restart / fuse / repeat bitwise")
    part = inputs.make_particles(5000, 25)
    a = gpu_run(met3, part, 0, 50, fuse=1)
    b = gpu_run(met3, part, 0, 50, fuse=7)
    c = gpu_run(met3, part, 0, 50, fuse=7)
    assert_bitwise(a, b)
    assert_bitwise(b, c)
    half = gpu_run(met3, part, 0, 23, fuse=5)
    rest = gpu_run(met3, half, 23, 27, fuse=5)
    assert_bitwise(a, rest)


def test_subset_independence(mpt, met3):
    part = inputs.make_particles(6000, 26)
    idx = np.arange(1000, 1800)
    full = gpu_run(met3, part, 0, 40, sort_interval=10, fuse=10)
    sub = gpu_run(met3, part.subset(idx), 0, 40, sort_interval=10, fuse=10)
    assert_bitwise(full.subset(idx), sub)


def test_release_gating(mpt, met3):
    say("scenario release gating")
    part = inputs.make_particles(4000, 27)
    scen = (np.arange(4000) % 5).astype(np.uint16)
    rel_s = np.array([0, 3, 17, 30, 1000], np.int32)
    g = gpu_run(met3, part, 0, 40, scen=scen, release=rel_s, sort_interval=10, fuse=10)
    r = oracle_run(met3, part, 0, 40, release=rel_s[scen])
    compare(g, r, TOL_F64_DEG, TOL_F64_HPA, "release")
    never = np.where(scen == 4)[0]
    np.testing.assert_array_equal(g.lon[never], part.lon[never])


def test_nonfinite_parcels_untouched(mpt, met3):
    part = inputs.make_particles(700, 28)
    part.lon[5] = np.nan
    part.p[9] = np.inf
    g = gpu_run(met3, part, 0, 15, sort_interval=5, fuse=5)
    r = oracle_run(met3, part, 0, 15)
    assert np.isnan(g.lon[5]) and np.isinf(g.p[9])
    ok = np.isfinite(r.lon) & np.isfinite(r.p)
    d = oracle.chord_deg(g.lon[ok], g.lat[ok], r.lon[ok], r.lat[ok])
    assert d.max() <= TOL_F64_DEG


CONT = oracle.ADVECT | oracle.TURB       # the continuous part of the step


def reduced_precision_checks(met_gpu, met_ref, part, math, dtype, label):
    """(1) advection + turbulent diffusion trajectories (continuous in the
    position): every parcel within tolerance; (2) single full steps from
    identical states at several step indices: every parcel within tolerance;
    (3) full-physics trajectories: within tolerance except parcels whose
    mesoscale cell differed at some step (bounded fraction)."""
    g = gpu_run(met_gpu, part, 0, 240, math=math, dtype=dtype, flags=CONT, sort_interval=10, fuse=10)
    r = oracle_run(met_ref, part, 0, 240, flags=CONT)
    compare(g, r, TOL_R32_DEG, TOL_R32_HPA, f"{label} advect+turb 240")
    state = part.copy()
    for s0 in (0, 60, 119, 200):
        g1 = gpu_run(met_gpu, state, s0, 1, math=math, dtype=dtype)
        r1 = oracle_run(met_ref, state, s0, 1)
        compare(g1, r1, TOL_R32_DEG, TOL_R32_HPA, f"{label} one full step at {s0}")
        state = oracle_run(met_ref, state, s0, 40)
    g = gpu_run(met_gpu, part, 0, 240, math=math, dtype=dtype, sort_interval=10, fuse=10)
    r = oracle_run(met_ref, part, 0, 240)
    compare_flips(g, r, TOL_R32_DEG, TOL_R32_HPA, 5e-3, f"{label} full 240")


def test_f32_form(mpt, met3):
    say("F32 form vs oracle")
    part = inputs.make_particles(10_000, 29)
    reduced_precision_checks(met3, met3, part, 1, 0, "c1 F32")


@pytest.mark.parametrize("kind", [encode.BF16, encode.F16])
def test_r16_encoding_bitwise(mpt, met3, kind):
    import torch
    ctx = mpt.Context(met3, mpt.make_params(math=1), dtype=kind)
    ctx.upload_met(met3)
    for l in range(met3.nt):
        packed, sc = ctx.copy_met_level(l)
        torch.cuda.synchronize()
        rec = packed.cpu().numpy().view(np.uint16).reshape(met3.nz, met3.ny, met3.nx, 4)
        scales = sc.cpu().numpy().reshape(3, met3.nz)
        for q, name in enumerate(("u", "v", "w")):
            want_q, want_s = encode.encode_level(getattr(met3, name)[l], kind)
            np.testing.assert_array_equal(scales[q], want_s)
            np.testing.assert_array_equal(rec[..., q], want_q)
        assert np.all(rec[..., 3] == 0)


@pytest.mark.parametrize("kind", [encode.BF16, encode.F16])
def test_r16_form(mpt, met3, kind):
    say(f"R16 form kind={kind} vs oracle on decoded fields")
    part = inputs.make_particles(10_000, 30)
    deq = encode.dequantized_met(met3, kind)
    reduced_precision_checks(met3, deq, part, 1, kind, f"c1 R16 {kind}")


@pytest.mark.parametrize("kind", [encode.BF16, encode.F16])
def test_r16_launches_across_met_levels(mpt, met3, kind):
    """16-bit storage: the step kernels read the per-level scales of the met
    levels a launch touches from LDS.  Launches that cross a met level (fuse
    7: steps 117..123 cross the level at step 120) and long launches cut to
    fit the window (fuse 200: 120 steps from step 5) equal one-step launches
    bit for bit."""
    say(f"[r16] launches across met levels, storage {kind}")
    part = inputs.make_particles(3000, 29)
    base = gpu_run(met3, part, 5, 235, math=1, dtype=kind, fuse=1)
    for fuse in (7, 200):
        assert_bitwise(base, gpu_run(met3, part, 5, 235, math=1, dtype=kind, fuse=fuse))


def test_r16_graph_with_launches_cut_at_the_window(mpt):
    """The graph-replayed loop with 16-bit storage and a sort interval longer
    than the launch limit (150 > 120 steps): the captured launches are cut
    the same way and the replays equal the eager loop bit for bit."""
    import torch
    say("[r16] graph, sort interval 150, launches cut to 120 steps")
    met = inputs.make_met_c1(seed=11, nt=4)
    part = inputs.make_particles(3000, 30)
    out = []
    for graph in (False, True):
        ctx = mpt.Context(met, mpt.make_params(math=1, sort_interval=150, fuse=150), n_max=part.n,
                          dtype=encode.BF16)
        ctx.upload_met(met)
        P = mpt.DeviceParticles.from_host(part, math=1)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            if graph:
                ctx.step_graph(P, 0, 300, s)
            else:
                ctx.step(P, 0, 300, s)
        torch.cuda.synchronize()
        out.append(by_id(P.to_host()))
    assert_bitwise(out[0], out[1])


def test_errors_on_gpu(mpt, met3):
    part = inputs.make_particles(100, 31)
    ctx = mpt.Context(met3, mpt.make_params(sort_interval=10), n_max=100)
    P = mpt.DeviceParticles.from_host(part)
    with pytest.raises(mpt.MptError) as e:
        ctx.step(P, 0, 1)                         # met not stored yet
    assert e.value.code == -2
    ctx.upload_met(met3)
    with pytest.raises(mpt.MptError) as e:
        ctx.step(P, 230, 20)                      # beyond the last met level
    assert e.value.code == -3
    small = mpt.Context(met3, mpt.make_params(sort_interval=10), n_max=50)
    small.upload_met(met3)
    with pytest.raises(mpt.MptError) as e:
        small.step(P, 0, 5)                       # sorts, but n > n_max
    assert e.value.code == -4
    ctx2 = mpt.Context(met3, mpt.make_params(), n_max=100)
    ctx2.upload_met(met3)
    Q = mpt.DeviceParticles.from_host(part, scen=np.zeros(100, np.uint16), pingpong=False)
    with pytest.raises(mpt.MptError) as e:
        ctx2.step(Q, 0, 1)                        # scenarios without a release table
    assert e.value.code == -2


@pytest.mark.parametrize("math", [0, 1])
def test_long_launches_equal_short_ones(mpt, met3, math):
    """Launches of 40 fused steps (the step's time locations are formed 32
    steps at a time, so a launch crosses that boundary) starting at an
    unaligned step and crossing a met level (step 120) equal launches of 10,
    bit for bit, with all modules."""
    say(f"long launches math={math}")
    part = inputs.make_particles(20_000, 91)
    a = gpu_run(met3, part, 97, 80, math=math, fuse=40)
    b = gpu_run(met3, part, 97, 80, math=math, fuse=10)
    assert_bitwise(a, b)
