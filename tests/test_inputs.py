"""Pins of the synthetic input generators (their stated bounds and moments)."""
import numpy as np

import inputs


def test_levels():
    p = inputs.levels_log(30)
    assert p[0] == 1000.0 and abs(p[-1] - 1.0) < 1e-12 and np.all(np.diff(p) < 0)
    q = inputs.levels_hybrid137()
    assert q[0] == 1013.25 and abs(q[-1] - 0.01) < 1e-14 and np.all(np.diff(q) < 0)
    assert 40 <= np.count_nonzero((q >= 100) & (q <= 900)) <= 55


def test_c1_bounds(met_c1):
    assert met_c1.u.shape == (2, 30, 91, 180)
    assert np.abs(met_c1.u).max() <= 50.0 and np.abs(met_c1.v).max() <= 50.0
    assert np.abs(met_c1.w).max() <= 0.005
    assert np.abs(met_c1.u).max() > 10.0
    assert met_c1.u.dtype == np.float32


def test_c1_deterministic():
    a = inputs.make_met_c1(seed=11)
    b = inputs.make_met_c1(seed=11)
    np.testing.assert_array_equal(a.u, b.u)
    c = inputs.make_met_c1(seed=12)
    assert not np.array_equal(a.u, c.u)


def test_c2_jet_and_perturbations_small_grid():
    met = inputs.make_met_c2(seed=12, nt=2, nx=240, ny=121, nz=137)
    jet = inputs.jet_profile(met.lat_axis(), met.plev, met.jet_lat_c)
    for l in range(2):
        pert = met.u[l].astype(np.float64) - jet[:, :, None]
        assert abs(pert.std() - 5.0) < 1e-3 and abs(pert.mean()) < 1e-3
        assert abs(met.v[l].std(dtype=np.float64) - 5.0) < 1e-3
        assert abs(met.w[l].std(dtype=np.float64) - 0.0005) < 1e-7
    assert not np.array_equal(met.v[0], met.v[1])       # independent per time level
    # jet maximum is exactly 60 m/s at 200 hPa, lat_c
    jmax = inputs.jet_profile(np.array([met.jet_lat_c]), np.array([200.0]), met.jet_lat_c)
    assert jmax[0, 0] == 60.0
    assert 30 <= met.jet_lat_c <= 45


def test_particles():
    part = inputs.make_particles(10000, 21)
    assert part.lon.min() >= 0 and part.lon.max() < 360
    assert part.lat.min() >= -90 and part.lat.max() <= 90
    assert part.p.min() >= 100 and part.p.max() <= 900
    np.testing.assert_array_equal(part.id, np.arange(10000))


def test_scenarios():
    sc = inputs.make_scenarios()
    assert len(sc.sizes) == 16
    assert sc.sizes.min() >= 1e4 and sc.sizes.max() <= 2e7
    small = inputs.scale_scenarios(sc, 1e-3)
    part, scen = inputs.make_scenario_particles(small)
    assert part.n == small.sizes.sum() and scen.max() == 15
