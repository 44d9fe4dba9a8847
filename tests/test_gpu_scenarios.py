"""GPU tests of batched release scenarios and of the graph-replayed step
loop: parcels of uneven scenarios released at different steps
(module_timesteps), the persistent launch that walks only released parcels,
and mpt_step_graph against mpt_step bit for bit."""
import numpy as np
import pytest

import inputs
import oracle
from gpu_common import (TOL_F64_DEG, TOL_F64_HPA, TOL_R32_DEG, TOL_R32_HPA, assert_bitwise, by_id,
                        compare, gpu_run, oracle_run, require_gpu, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpt():
    return require_gpu()


@pytest.fixture(scope="module")
def met3():
    return inputs.make_met_c1(seed=11, nt=3)


def scenario_set():
    sc = inputs.Scenarios(sizes=np.array([50, 3000, 700, 1, 256, 2000, 999]),
                          release_step=np.array([0, 37, 5, 120, 60, 239, 37], np.int32),
                          lon=np.array([10.0, 100.0, 200.0, 300.0, 359.9, 45.0, 270.0]),
                          lat=np.array([0.0, 45.0, -30.0, 80.0, -85.0, 10.0, 60.0]),
                          p=np.array([500.0, 250.0, 850.0, 150.0, 700.0, 300.0, 400.0]),
                          kind=np.array([0, 1, 0, 1, 1, 0, 1], np.int32))
    part, scen = inputs.make_scenario_particles(sc, seed=24)
    # scramble the memory order: scenarios interleave
    perm = np.random.Generator(np.random.PCG64(5)).permutation(part.n)
    return sc, part.subset(perm), scen[perm]


def run_graph(mpt, met, part, scen, release, step0, nsteps, math=0, **kw):
    import torch
    params = mpt.make_params(math=math, sort_interval=10, fuse=10, **kw)
    ctx = mpt.Context(met, params, n_max=part.n)
    ctx.upload_met(met)
    if release is not None:
        ctx.set_release(release)
    P = mpt.DeviceParticles.from_host(part, math=math, scen=scen)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx.step_graph(P, step0, nsteps, s)
    s.synchronize()
    return by_id(P.to_host())


def test_scenarios_vs_oracle(mpt, met3):
    sc, part, scen = scenario_set()
    say(f"scenarios: {part.n} parcels in {len(sc.sizes)} scenarios, 240 steps")
    g = gpu_run(met3, part, 0, 240, scen=scen, release=sc.release_step, sort_interval=10, fuse=10)
    r = oracle_run(met3, part, 0, 240, release=sc.release_step[scen])
    compare(g, r, TOL_F64_DEG, TOL_F64_HPA, "scenarios F64")
    # never-released parcels keep their start state bit for bit
    late = by_id(part)
    ids_late = np.where(sc.release_step[scen[np.argsort(part.id)]] >= 240)[0]
    np.testing.assert_array_equal(g.lon[ids_late], late.lon[ids_late])


def test_scenarios_sorted_equals_unsorted(mpt, met3):
    sc, part, scen = scenario_set()
    a = gpu_run(met3, part, 0, 120, scen=scen, release=sc.release_step, sort_interval=10, fuse=10)
    b = gpu_run(met3, part, 0, 120, scen=scen, release=sc.release_step, sort_interval=0, fuse=10)
    c = gpu_run(met3, part, 0, 120, scen=scen, release=sc.release_step, sort_interval=10, fuse=3)
    assert_bitwise(a, b)
    assert_bitwise(a, c)


def test_graph_equals_step_scenarios(mpt, met3):
    sc, part, scen = scenario_set()
    say("graph replay vs step, scenarios, 240 steps")
    a = gpu_run(met3, part, 0, 240, scen=scen, release=sc.release_step, sort_interval=10, fuse=10)
    b = run_graph(mpt, met3, part, scen, sc.release_step, 0, 240)
    assert_bitwise(a, b)


def test_graph_equals_step_plain(mpt, met3):
    part = inputs.make_particles(7000, 41)
    a = gpu_run(met3, part, 20, 200, sort_interval=10, fuse=10)
    b = run_graph(mpt, met3, part, None, None, 20, 200)
    assert_bitwise(a, b)
    f = gpu_run(met3, part, 20, 200, math=1, sort_interval=10, fuse=10)
    g = run_graph(mpt, met3, part, None, None, 20, 200, math=1)
    assert_bitwise(f, g)


def test_graph_argument_checks(mpt, met3):
    import torch
    part = inputs.make_particles(100, 42)
    ctx = mpt.Context(met3, mpt.make_params(sort_interval=10, fuse=10), n_max=100)
    ctx.upload_met(met3)
    P = mpt.DeviceParticles.from_host(part)
    s = torch.cuda.Stream()
    for step0, nsteps in ((5, 20), (0, 30)):
        with pytest.raises(mpt.MptError) as e:
            ctx.step_graph(P, step0, nsteps, s)
        assert e.value.code == -1
    with pytest.raises(mpt.MptError) as e:
        ctx.step_graph(P, 0, 20, torch.cuda.default_stream())   # null stream: cannot capture
    assert e.value.code == -1
