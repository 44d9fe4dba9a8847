"""Streamed met levels (mpt_push_met): a run over 5 time levels (24 h) with
only 2 or 3 of them resident, the next one pushed whenever the steps reach
the end of the window, must equal the run with all 5 resident bit for bit
(same kernels, same level pair for every evaluation; the ring's slot order
differs), in the F64, F32 and BF16 forms, and the F64 form must match the
oracle.  The window's errors: a step outside it, a push before every
resident level is stored."""
import numpy as np
import pytest

import inputs
from gpu_common import TOL_F64_DEG, TOL_F64_HPA, assert_bitwise, by_id, compare, oracle_run, require_gpu, say

pytestmark = pytest.mark.gpu
PER = 120                                   # steps per 6 h level interval (dt = 180 s)


@pytest.fixture(scope="module")
def mpt():
    return require_gpu()


@pytest.fixture(scope="module")
def met5():
    return inputs.make_met_c1(seed=11, nt=5)


def streamed(mpt, met, part, resident, math, dtype):
    import torch
    c = mpt.Context(met, mpt.make_params(math=math, sort_interval=10, fuse=10), n_max=part.n, dtype=dtype,
                    resident=resident)
    c.upload_met(met)
    P = mpt.DeviceParticles.from_host(part, math=math)
    nxt = resident
    for b in range(4):
        c.step(P, PER * b, PER)
        # the window must advance before the next interval's last step
        while nxt < met.nt and nxt <= b + 2:
            c.push_met(*(torch.from_numpy(a[nxt]).cuda() for a in (met.u, met.v, met.w)))
            nxt += 1
    torch.cuda.synchronize()
    return by_id(P.to_host())


def resident_all(mpt, met, part, math, dtype):
    import torch
    c = mpt.Context(met, mpt.make_params(math=math, sort_interval=10, fuse=10), n_max=part.n, dtype=dtype)
    c.upload_met(met)
    P = mpt.DeviceParticles.from_host(part, math=math)
    c.step(P, 0, 4 * PER)
    torch.cuda.synchronize()
    return by_id(P.to_host())


@pytest.mark.parametrize("resident", [2, 3])
@pytest.mark.parametrize("form", [(0, 0), (1, 0), (1, 1)])
def test_streamed_equals_all_resident(mpt, met5, resident, form):
    math, dtype = form
    say(f"[stream] resident {resident}, math {math}, dtype {dtype}")
    part = inputs.make_particles(20_000, 81)
    a = streamed(mpt, met5, part, resident, math, dtype)
    b = resident_all(mpt, met5, part, math, dtype)
    assert_bitwise(a, b)


def test_streamed_f64_matches_oracle(mpt, met5):
    part = inputs.make_particles(5_000, 82)
    g = streamed(mpt, met5, part, 2, 0, 0)
    r = oracle_run(met5, part, 0, 4 * PER)
    compare(g, r, TOL_F64_DEG, TOL_F64_HPA, "streamed F64 vs oracle, 480 steps over 5 levels")


def test_window_errors(mpt, met5):
    import torch
    part = inputs.make_particles(1000, 83)
    c = mpt.Context(met5, mpt.make_params(math=0), n_max=part.n, resident=2)
    u, v, w = (torch.from_numpy(a[0]).cuda() for a in (met5.u, met5.v, met5.w))
    with pytest.raises(mpt.MptError, match="STATE"):
        c.push_met(u, v, w)                       # resident levels not stored yet
    c.upload_met(met5)
    P = mpt.DeviceParticles.from_host(part, math=0, pingpong=False)
    with pytest.raises(mpt.MptError, match="TIME"):
        c.step(P, PER - 1, 2)                     # ends beyond level 1
    c.step(P, 0, PER)
    c.push_met(*(torch.from_numpy(a[2]).cuda() for a in (met5.u, met5.v, met5.w)))
    with pytest.raises(mpt.MptError, match="TIME"):
        c.step(P, PER - 1, 1)                     # before the new window
    c.step(P, PER, PER)
    torch.cuda.synchronize()
    assert np.isfinite(P.lon.cpu().numpy()).all()
