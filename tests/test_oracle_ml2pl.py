"""Pins of the oracle's model-level -> pressure-level regridding (read_met,
Sec. 3.1; the reading is stated in include/mpt.h):

* a field linear in ln p in every column is reproduced exactly (up to the
  float rounding of the result) at every target inside the column;
* pure pressure levels (b = 0) reduce to numpy's 1-D interpolation in ln p;
* targets below the lowest or above the highest model level of a column
  take that level's value, and a target on a model level takes its value;
* the hybrid coefficients put the model levels on their reference
  pressures where ps equals the reference surface pressure.
"""
import numpy as np

import inputs
import oracle


def test_linear_in_ln_p_is_exact():
    rng = np.random.default_rng(1)
    nx, ny = 16, 9
    p_ref = inputs.levels_log(40)
    a, b = inputs.hybrid_levels(p_ref)
    ps = inputs.make_surface_pressure(2, nx, ny)
    pk = a[:, None, None] + b[:, None, None] * ps[None].astype(np.float64)
    alpha = rng.uniform(-5, 5, (ny, nx))
    beta = rng.uniform(-3, 3, (ny, nx))
    f = (alpha[None] + beta[None] * np.log(pk)).astype(np.float32)
    # the node values are the line rounded to float: the bound allows that
    # rounding and the rounding of the result
    plev = inputs.levels_log(30, p_bot=990.0, p_top=2.0)
    out = oracle.ml_to_pl(plev, a, b, ps, f)
    want = alpha[None] + beta[None] * np.log(plev)[:, None, None]
    inside = (plev[:, None, None] < pk[0][None]) & (plev[:, None, None] > pk[-1][None])
    err = np.abs(out.astype(np.float64) - want)[inside]
    scale = (np.abs(alpha) + np.abs(beta) * 8)[None].repeat(len(plev), 0)[inside]
    assert err.max() <= 4e-7 * scale.max()


def test_pure_pressure_levels_reduce_to_numpy_interp():
    rng = np.random.default_rng(2)
    nx, ny = 7, 5
    a = np.sort(rng.uniform(5.0, 1000.0, 25))[::-1].copy()
    b = np.zeros_like(a)
    ps = rng.uniform(900, 1100, (ny, nx)).astype(np.float32)
    f = rng.normal(size=(len(a), ny, nx)).astype(np.float32)
    plev = np.linspace(1050.0, 2.0, 33)
    out = oracle.ml_to_pl(plev, a, b, ps, f)
    for j in range(ny):
        for i in range(nx):
            want = np.interp(np.log(plev), np.log(a[::-1]), f[::-1, j, i].astype(np.float64))
            np.testing.assert_allclose(out[:, j, i], want.astype(np.float32), rtol=1e-6, atol=1e-6)


def test_outside_and_on_model_levels():
    p_ref = np.array([1000.0, 700.0, 400.0, 100.0, 10.0])
    a, b = inputs.hybrid_levels(p_ref)
    ps = np.full((2, 3), 1013.25, np.float32)
    f = np.arange(5, dtype=np.float32)[:, None, None] * np.ones((5, 2, 3), np.float32)
    plev = np.array([1050.0, 1000.0, 700.0, 100.0, 10.0, 5.0])
    out = oracle.ml_to_pl(plev, a, b, ps, f)
    np.testing.assert_array_equal(out[:, 0, 0], [0.0, 0.0, 1.0, 3.0, 4.0, 4.0])


def test_hybrid_levels_sit_on_the_reference_pressures():
    p_ref = inputs.levels_hybrid137()
    a, b = inputs.hybrid_levels(p_ref)
    np.testing.assert_allclose(a + b * 1013.25, p_ref, rtol=1e-14)
    assert np.all(b[p_ref <= 100.0] == 0.0) and np.all(np.diff(b) <= 0.0)
