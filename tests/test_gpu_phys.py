"""Convection and sedimentation on the GPU (module_convection, module_sedi,
Sec. 3.2) against the FP64 oracle on the 2 deg grid with seeded fields:
all modules plus both, 240 steps with sorting and fused launches.  F64
within the FP64 tolerance; F32 and BF16 / F16 storage (the oracle on the
decoded fields) within the reduced-precision tolerance, except a bounded
fraction of parcels whose discrete decisions (mesoscale cell, convective
threshold) differ.  Also: the plain kernels are untouched when the flags
are off, the graph-replayed loop equals the eager one, and the fields are
required."""
import numpy as np
import pytest

import inputs
import oracle
from gpu_common import (TOL_F64_DEG, TOL_F64_HPA, TOL_R32_DEG, TOL_R32_HPA, assert_bitwise, by_id,
                        compare, compare_flips, gpu_run, oracle_run, require_gpu, say)
from oracle import encode

pytestmark = pytest.mark.gpu

ALL = oracle.ADVECT | oracle.TURB | oracle.MESO | oracle.CONV | oracle.SEDI
KW = dict(conv_cape=800.0)                      # a threshold inside the CAPE range
R_BIG = 25e-6                                   # radius: ~1.4 hPa per step near the ground


@pytest.fixture(scope="module")
def mpt():
    return require_gpu()


@pytest.fixture(scope="module")
def met3():
    return inputs.add_phys_fields(inputs.make_met_c1(seed=11, nt=3), seed=31)


def run_pair(met_gpu, met_ref, part, nsteps, math, dtype, flags=ALL, r=R_BIG):
    g = gpu_run(met_gpu, part, 0, nsteps, math=math, dtype=dtype, flags=flags, sort_interval=10,
                fuse=10, sedi_radius=r, **KW)
    ref = oracle_run(met_ref, part, 0, nsteps, flags=flags, sedi_r=r, **KW)
    return g, ref


def test_phys_f64_matches_oracle(mpt, met3):
    say("[phys] F64 all modules + convection + sedimentation, 240 steps")
    part = inputs.make_particles(10_000, 41, p_lo=100.0, p_hi=990.0)
    g, r = run_pair(met3, met3, part, 240, 0, 0)
    compare(g, r, TOL_F64_DEG, TOL_F64_HPA, "phys F64 240")
    moved = np.abs(g.p - part.subset(np.argsort(part.id)).p) > 50.0
    say(f"[phys] parcels moved by more than 50 hPa: {moved.mean():.3f}")
    assert moved.mean() > 0.05


@pytest.mark.parametrize("flags", [oracle.CONV, oracle.SEDI, oracle.ADVECT | oracle.SEDI])
def test_phys_modules_alone_f64(mpt, met3, flags):
    say(f"[phys] F64 flags {flags}, 60 steps")
    part = inputs.make_particles(5_000, 42, p_lo=100.0, p_hi=990.0)
    g, r = run_pair(met3, met3, part, 60, 0, 0, flags=flags)
    compare(g, r, TOL_F64_DEG, TOL_F64_HPA, f"phys F64 flags {flags}")


@pytest.mark.parametrize("dtype", [0, encode.BF16, encode.F16])
def test_phys_reduced_precision(mpt, met3, dtype):
    say(f"[phys] F32 math, storage {dtype}, 240 steps")
    part = inputs.make_particles(10_000, 43, p_lo=100.0, p_hi=990.0)
    ref_met = met3 if dtype == 0 else encode.dequantized_met(met3, dtype)
    # sedimentation alone from identical states: continuous, every parcel
    g, r = run_pair(met3, ref_met, part, 40, 1, dtype, flags=oracle.SEDI)
    compare(g, r, TOL_R32_DEG, TOL_R32_HPA, f"phys sedi F32/{dtype} 40")
    g, r = run_pair(met3, ref_met, part, 240, 1, dtype)
    compare_flips(g, r, TOL_R32_DEG, TOL_R32_HPA, 2e-2, f"phys all F32/{dtype} 240")


def test_plain_kernels_ignore_the_fields(mpt, met3):
    """With the flags off the step does not read the new fields: a run on
    met with them equals a run on met without them, bit for bit."""
    import dataclasses
    part = inputs.make_particles(5_000, 44)
    bare = dataclasses.replace(met3, temp=None, cape=None, pel=None, ps=None)
    a = gpu_run(met3, part, 0, 40, sort_interval=10, fuse=10)
    b = gpu_run(bare, part, 0, 40, sort_interval=10, fuse=10)
    assert_bitwise(a, b)


def test_phys_graph_equals_eager(mpt, met3):
    import torch
    part = inputs.make_particles(5_000, 45)
    out = []
    for graph in (False, True):
        params = mpt.make_params(math=0, flags=ALL, sort_interval=10, fuse=10, sedi_radius=R_BIG, **KW)
        ctx = mpt.Context(met3, params, n_max=part.n)
        ctx.upload_met(met3)
        P = mpt.DeviceParticles.from_host(part, math=0)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            if graph:
                for b in range(3):
                    ctx.step_graph(P, 20 * b, 20, s)
            else:
                ctx.step(P, 0, 60, s)
        torch.cuda.synchronize()
        out.append(by_id(P.to_host()))
    assert_bitwise(out[0], out[1])


def test_phys_fields_required(mpt, met3):
    import dataclasses
    import torch
    part = inputs.make_particles(100, 46)
    bare = dataclasses.replace(met3, temp=None, cape=None, pel=None, ps=None)
    ctx = mpt.Context(bare, mpt.make_params(math=0, flags=ALL, **KW), n_max=part.n)
    ctx.upload_met(bare)
    P = mpt.DeviceParticles.from_host(part, math=0, pingpong=False)
    with pytest.raises(mpt.MptError, match="STATE"):
        ctx.step(P, 0, 1)
    f = [torch.from_numpy(np.ascontiguousarray(a[0])).cuda()
         for a in (met3.temp, met3.cape, met3.pel, met3.ps)]
    for l in range(met3.nt):
        ctx.set_met_phys(l, *f)
    ctx.step(P, 0, 1)
    ctx.init_met(1, *(torch.from_numpy(a[1]).cuda() for a in (met3.u, met3.v, met3.w)))
    with pytest.raises(mpt.MptError, match="STATE"):              # storing u, v, w clears them
        ctx.step(P, 1, 1)
    torch.cuda.synchronize()


def test_phys_scenarios_vs_oracle(mpt, met3):
    """Batched releases take the persistent launch shape of the physics
    kernel (it walks the released prefix after each sort)."""
    say("[phys] scenarios, persistent kernel, 120 steps")
    sc = inputs.Scenarios(sizes=np.array([800, 3000, 1, 1200]),
                          release_step=np.array([0, 17, 40, 90], np.int32),
                          lon=np.array([10.0, 100.0, 200.0, 300.0]),
                          lat=np.array([0.0, 25.0, -30.0, 60.0]),
                          p=np.array([700.0, 850.0, 500.0, 900.0]),
                          kind=np.array([0, 1, 0, 1], np.int32))
    part, scen = inputs.make_scenario_particles(sc, seed=47)
    g = gpu_run(met3, part, 0, 120, scen=scen, release=sc.release_step, sort_interval=10, fuse=10,
                flags=ALL, sedi_radius=R_BIG, **KW)
    r = oracle_run(met3, part, 0, 120, flags=ALL, release=sc.release_step[scen], sedi_r=R_BIG, **KW)
    compare(g, r, TOL_F64_DEG, TOL_F64_HPA, "phys scenarios F64 120")


def test_phys_streamed_equals_all_resident(mpt):
    """Streamed levels: after each push the newest level's fields are stored
    again; the run equals the one with every level resident, bit for bit."""
    import torch
    met = inputs.add_phys_fields(inputs.make_met_c1(seed=11, nt=4), seed=31)
    part = inputs.make_particles(5_000, 48, p_lo=100.0, p_hi=990.0)
    per = 120
    prm = mpt.make_params(math=0, flags=ALL, sort_interval=10, fuse=10, sedi_radius=R_BIG, **KW)
    a_ctx = mpt.Context(met, prm, n_max=part.n)
    a_ctx.upload_met(met)
    A = mpt.DeviceParticles.from_host(part, math=0)
    a_ctx.step(A, 0, 3 * per)
    b_ctx = mpt.Context(met, prm, n_max=part.n, resident=2)
    b_ctx.upload_met(met)
    B = mpt.DeviceParticles.from_host(part, math=0)
    for b in range(3):
        b_ctx.step(B, per * b, per)
        if b + 2 < met.nt:
            lvl = b + 2
            b_ctx.push_met(*(torch.from_numpy(x[lvl]).cuda() for x in (met.u, met.v, met.w)))
            with pytest.raises(mpt.MptError, match="STATE"):
                b_ctx.step(B, per * (b + 1), 1)          # the new level lacks its fields
            b_ctx.set_met_phys(1, *(torch.from_numpy(np.ascontiguousarray(x[lvl])).cuda()
                                    for x in (met.temp, met.cape, met.pel, met.ps)))
    torch.cuda.synchronize()
    assert_bitwise(by_id(A.to_host()), by_id(B.to_host()))


def test_phys_r16_launches_across_met_levels(mpt, met3):
    """16-bit storage with convection and sedimentation: launches that cross
    a met level (fuse 7 from step 5: steps 117..123 cross the level at step
    120) read the scales of three levels from LDS and equal one-step
    launches bit for bit."""
    say("[phys] BF16 launches across met levels")
    part = inputs.make_particles(3000, 49, p_lo=100.0, p_hi=990.0)
    kw = dict(math=1, dtype=encode.BF16, flags=ALL, sedi_radius=R_BIG, **KW)
    base = gpu_run(met3, part, 5, 235, fuse=1, **kw)
    assert_bitwise(base, gpu_run(met3, part, 5, 235, fuse=7, **kw))
