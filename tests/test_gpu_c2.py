"""GPU parity on the realistic workload: 0.3 deg grid (1200 x 601) x 137
levels, jet + perturbation winds, 240 steps of 180 s with all modules and a
grid-box sort every 10 steps.

* 1e5 parcels, every parcel compared with the FP64 oracle (F64, F32, and
  BF16 / FP16 storage against the oracle run on the decoded fields); the
  reduced-precision runs also report their distance to the FP64 oracle on
  the original FP32 fields (precision loss, not parity);
* 1e7 parcels (the config's own size) and 1e8 parcels (the benchmark's
  launch configuration): a seeded sample of ids is recomputed by the oracle
  one by one -- parcels are independent and their random numbers are keyed
  by id, so a subset run is exact.
"""
import numpy as np
import pytest

import inputs
import oracle
from gpu_common import (TOL_F64_DEG, TOL_F64_HPA, TOL_R32_DEG, TOL_R32_HPA, by_id, compare,
                        compare_flips, gpu_run, oracle_run, require_gpu, say)
from oracle import encode

pytestmark = pytest.mark.gpu
KM_PER_DEG = np.pi * 6371.0 / 180.0


@pytest.fixture(scope="module")
def mpt():
    return require_gpu()


@pytest.fixture(scope="module")
def met(mpt):
    say("generating 0.3 deg fields, nt=3")
    return inputs.make_met_c2(seed=12, nt=3)


@pytest.fixture(scope="module")
def part_1e5():
    return inputs.make_particles(100_000, 22)


@pytest.fixture(scope="module")
def ref_1e5(met, part_1e5):
    say("oracle: 1e5 parcels x 240 steps on the 0.3 deg grid")
    return oracle_run(met, part_1e5, 0, 240)


def test_c2_f64_full_compare(mpt, met, part_1e5, ref_1e5):
    say("c2 F64 1e5 x 240, sort/10, fuse 10")
    g = gpu_run(met, part_1e5, 0, 240, math=0, sort_interval=10, fuse=10)
    compare(g, ref_1e5, TOL_F64_DEG, TOL_F64_HPA, "c2 F64 1e5")


CONT = oracle.ADVECT | oracle.TURB


def test_c2_f32_full_compare(mpt, met, part_1e5, ref_1e5):
    say("c2 F32 1e5 x 240")
    g = gpu_run(met, part_1e5, 0, 240, math=1, flags=CONT, sort_interval=10, fuse=10)
    r = oracle_run(met, part_1e5, 0, 240, flags=CONT)
    compare(g, r, TOL_R32_DEG, TOL_R32_HPA, "c2 F32 1e5 advect+turb")
    g = gpu_run(met, part_1e5, 0, 240, math=1, sort_interval=10, fuse=10)
    compare_flips(g, ref_1e5, TOL_R32_DEG, TOL_R32_HPA, 0.05, "c2 F32 1e5 full")


@pytest.mark.parametrize("kind", [encode.BF16, encode.F16])
def test_c2_r16_full_compare(mpt, met, part_1e5, ref_1e5, kind):
    say(f"c2 R16 kind={kind} 1e5 x 240")
    deq = encode.dequantized_met(met, kind)
    g = gpu_run(met, part_1e5, 0, 240, math=1, dtype=kind, flags=CONT, sort_interval=10, fuse=10)
    r = oracle_run(deq, part_1e5, 0, 240, flags=CONT)
    compare(g, r, TOL_R32_DEG, TOL_R32_HPA, f"c2 R16 {kind} advect+turb vs oracle on decoded fields")
    g = gpu_run(met, part_1e5, 0, 240, math=1, dtype=kind, sort_interval=10, fuse=10)
    r = oracle_run(deq, part_1e5, 0, 240)
    compare_flips(g, r, TOL_R32_DEG, TOL_R32_HPA, 0.05, f"c2 R16 {kind} full vs decoded")
    km = oracle.chord_deg(g.lon, g.lat, ref_1e5.lon, ref_1e5.lat) * KM_PER_DEG
    say(f"[c2 R16 {kind}] precision loss vs FP64 oracle on FP32 fields after 240 steps: "
        f"mean {km.mean():.3f} km, p99 {np.percentile(km, 99):.3f} km, max {km.max():.3f} km")


def sampled_check(mpt, met, n, seed, nsample, label):
    import torch
    part = inputs.make_particles(n, seed)
    params = mpt.make_params(math=0, sort_interval=10, fuse=10)
    ctx = mpt.Context(met, params, n_max=n)
    ctx.upload_met(met)
    P = mpt.DeviceParticles.from_host(part)
    say(f"{label}: GPU {n} x 240")
    ctx.step(P, 0, 240)
    torch.cuda.synchronize()
    ids = P.id.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(np.bincount(ids, minlength=n), 1)    # a permutation
    where = np.empty(n, np.int64)
    where[ids] = np.arange(n)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    sample = np.sort(rng.choice(n, nsample, replace=False))
    loc = torch.from_numpy(where[sample]).cuda()
    g = inputs.Particles(lon=P.lon[loc].cpu().numpy(), lat=P.lat[loc].cpu().numpy(),
                         p=P.p[loc].cpu().numpy(), id=sample.astype(np.uint32),
                         up=P.up[loc].cpu().numpy(), vp=P.vp[loc].cpu().numpy(),
                         wp=P.wp[loc].cpu().numpy())
    del P, ctx
    torch.cuda.empty_cache()
    say(f"{label}: oracle on {nsample} sampled ids")
    r = oracle_run(met, part.subset(sample), 0, 240)
    compare(g, r, TOL_F64_DEG, TOL_F64_HPA, label)


def test_c2_1e7_sampled(mpt, met):
    sampled_check(mpt, met, 10_000_000, 22, 3000, "c2 F64 1e7 sampled")


def test_bench_config_1e8_sampled(mpt, met):
    sampled_check(mpt, met, 100_000_000, 23, 2000, "1e8 F64 sampled")
