"""GPU parity of the model-level -> pressure-level regridding (read_met,
Sec. 3.1; reading in include/mpt.h) against the oracle: both interpolate in
FP64 and round to float, so they agree to the rounding of the result (the
logarithms may differ in their last bit), here held to 2 ulp of the result
plus 1e-14 of the field's magnitude for results that cancel.  Then the
pipeline: two converted time levels stored with mpt_init_met and stepped in
the F64 form match the oracle run on the same converted fields.  Errors:
conversion before the levels are set, non-monotone levels."""
import numpy as np
import pytest

import inputs
import oracle
from gpu_common import TOL_F64_DEG, TOL_F64_HPA, by_id, compare, require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpt():
    return require_gpu()


@pytest.fixture(scope="module")
def setup():
    met = inputs.make_met_c1(seed=11, nt=2)
    p_ref = inputs.levels_log(45, p_bot=1010.0, p_top=0.8)
    a, b = inputs.hybrid_levels(p_ref)
    levels = []
    for l in range(2):
        ps = inputs.make_surface_pressure(30 + l, met.nx, met.ny)
        levels.append((ps, inputs.make_model_level_fields(40 + l, p_ref, met.nx, met.ny)))
    return met, a, b, levels


def gpu_convert(mpt, ctx, ps, f):
    import torch
    out = ctx.ml_to_pl(*(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (ps, *f)))
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def test_matches_oracle(mpt, setup):
    met, a, b, levels = setup
    c = mpt.Context(met, mpt.make_params(math=0), n_max=16)
    c.set_hybrid(a, b)
    for ps, f in levels:
        g = gpu_convert(mpt, c, ps, f)
        for q in range(3):
            o = oracle.ml_to_pl(met.plev, a, b, ps, f[q])
            tol = 2.0 * np.spacing(np.maximum(np.abs(g[q]), np.abs(o))) + 1e-14 * np.abs(f[q]).max()
            d = np.abs(g[q].astype(np.float64) - o)
            say(f"[ml2pl] var {q}: max |gpu - oracle| {d.max():.3e}, exact {np.mean(d == 0) * 100:.2f} %")
            assert np.all(d <= tol)


def test_converted_levels_step_like_the_oracle(mpt, setup):
    import torch
    met, a, b, levels = setup
    c = mpt.Context(met, mpt.make_params(math=0, sort_interval=10, fuse=10), n_max=5000)
    c.set_hybrid(a, b)
    conv = inputs.empty_met(met.nx, met.ny, met.plev, 2)
    for l, (ps, f) in enumerate(levels):
        u, v, w = gpu_convert(mpt, c, ps, f)
        conv.u[l], conv.v[l], conv.w[l] = u, v, w
        c.init_met(l, *(torch.from_numpy(x).cuda() for x in (u, v, w)))
    part = inputs.make_particles(5000, 91)
    P = mpt.DeviceParticles.from_host(part, math=0)
    c.step(P, 0, 60)
    torch.cuda.synchronize()
    g = by_id(P.to_host())
    from gpu_common import oracle_run
    r = oracle_run(conv, part, 0, 60)
    compare(g, r, TOL_F64_DEG, TOL_F64_HPA, "converted levels, F64, 60 steps")


def test_errors(mpt, setup):
    import torch
    met, a, b, levels = setup
    c = mpt.Context(met, mpt.make_params(math=0), n_max=16)
    ps, f = levels[0]
    with pytest.raises(mpt.MptError, match="STATE"):
        c.ml_to_pl(*(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (ps, *f)))
    with pytest.raises(mpt.MptError, match="ARG"):      # pressure rises with the level index
        c.set_hybrid(np.array([1000.0, 800.0, 850.0, 400.0]), np.zeros(4))
    with pytest.raises(mpt.MptError, match="ARG"):      # negative pressure at ps = 500 hPa
        c.set_hybrid(np.array([-600.0, -700.0]), np.array([1.0, 0.9]))
