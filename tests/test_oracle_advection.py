"""Pins of the oracle's midpoint advection and position handling.

Advection computes kinematic trajectories from the winds (Sec. 3.2,
module_advection); here as the explicit midpoint scheme.  Position handling
keeps parcels in the model domain (Sec. 3.2, module_position).  Pins: exact
displacement in uniform wind, return after one revolution of a gridded
solid-body rotation within the interpolation bound, second-order convergence
against the exact tilted solid-body rotation (Williamson et al. 1992, test 1),
pole reflection and longitude wrap that leave the point on the sphere
unchanged.
"""
import math

import numpy as np
import pytest

import inputs
import oracle

R = 6371000.0
DT = 180.0


def steady_met(nx, ny, plev, u=0.0, v=0.0, w=0.0, dt_met=1e7):
    met = inputs.empty_met(nx, ny, plev, 2, dt_met=dt_met)
    return inputs.fill_uniform(met, u, v, w)


def xyz(lon, lat):
    d = np.pi / 180
    return np.stack([np.cos(lat * d) * np.cos(lon * d), np.cos(lat * d) * np.sin(lon * d),
                     np.sin(lat * d)], -1)


def test_uniform_zonal_wind_exact_displacement(rng):
    U, W = 17.0, -0.0025               # m/s, hPa/s
    met = steady_met(180, 91, inputs.levels_log(30), u=U, w=W)
    m = oracle.Met(met)
    n, steps = 200, 120
    part = inputs.make_particles(n, 3, p_lo=300, p_hi=900, lat_lo=-70, lat_hi=70)
    lon0, lat0, p0 = part.lon.copy(), part.lat.copy(), part.p.copy()
    oracle.run(m, oracle.ctl(flags=oracle.ADVECT), part, 0, steps)
    dlon = steps * U * DT * 180 / (math.pi * R * np.cos(np.deg2rad(lat0)))
    want = np.mod(lon0 + dlon, 360)
    d = np.abs(part.lon - want)
    d = np.minimum(d, 360 - d)
    assert d.max() < 1e-9
    np.testing.assert_array_equal(part.lat, lat0)
    np.testing.assert_allclose(part.p, p0 + steps * W * DT, atol=1e-9)


def test_uniform_meridional_wind_exact_displacement():
    V = 9.0
    met = steady_met(180, 91, inputs.levels_log(30), v=V)
    m = oracle.Met(met)
    part = inputs.make_particles(100, 4, lat_lo=-60, lat_hi=40)
    lon0, lat0 = part.lon.copy(), part.lat.copy()
    steps = 200
    oracle.run(m, oracle.ctl(flags=oracle.ADVECT), part, 0, steps)
    np.testing.assert_allclose(part.lat, lat0 + steps * V * DT * 180 / (math.pi * R), atol=1e-9)
    np.testing.assert_array_equal(part.lon, lon0)


def test_gridded_solid_body_rotation_returns():
    """u = U0 cos(lat) on the tiny grid, U0 chosen so that nsteps * dt * U0
    = 2 pi R: each parcel keeps its latitude and returns to its longitude
    within 360 deg * dlat_rad^2 / 8 (linear interpolation of cos in lat,
    relative error of the angular speed at most h^2/8 * cos''/cos = h^2/8 for
    a row-centred parcel, up to the cos ratio across the cell)."""
    nx, ny = 180, 91
    plev = inputs.levels_log(30)
    nsteps = 1000
    U0 = 2 * math.pi * R / (nsteps * DT)
    met = inputs.empty_met(nx, ny, plev, 2, dt_met=1e7)
    coslat = np.cos(np.deg2rad(met.lat_axis())).astype(np.float32)
    met.u[...] = (U0 * coslat)[None, None, :, None]
    m = oracle.Met(met)
    lat = np.array([-60.0, -45.0, -31.0, 0.0, 1.0, 20.0, 45.0, 60.0, 59.0])
    n = len(lat)
    part = inputs.Particles(lon=np.linspace(3, 300, n), lat=lat.copy(), p=np.full(n, 500.0),
                            id=np.arange(n, dtype=np.uint32), up=np.zeros(n), vp=np.zeros(n),
                            wp=np.zeros(n))
    lon0 = part.lon.copy()
    oracle.run(m, oracle.ctl(flags=oracle.ADVECT), part, 0, nsteps)
    np.testing.assert_array_equal(part.lat, lat)
    d = np.abs(part.lon - lon0)
    d = np.minimum(d, 360 - d)
    h = np.deg2rad(met.dlat)
    ratio = np.cos(np.deg2rad(np.abs(lat) - met.dlat)) / np.cos(np.deg2rad(lat))
    bound = 360.0 * h * h / 8 * ratio + 360 * 2.0**-22      # + float32 storage of cos
    assert np.all(d <= bound), (d, bound)
    on_row = np.isin(lat, met.lat_axis())
    assert np.all(d[on_row] < 360 * 2.0**-21)               # rows interpolate exactly


def rotate(v, axis, ang):
    """Rodrigues rotation of vectors v (n,3) about a unit axis by ang."""
    k = np.asarray(axis, np.float64)
    c, s = math.cos(ang), math.sin(ang)
    return v * c + np.cross(k, v) * s + np.outer(v @ k, k) * (1 - c)


def test_midpoint_second_order_on_tilted_rotation():
    alpha = math.pi / 4
    U0 = 40.0
    met = steady_met(180, 91, inputs.levels_log(30))
    m = oracle.Met(met, analytic=True, an_u0=U0, an_alpha=alpha)
    axis = np.array([-math.sin(alpha), 0.0, math.cos(alpha)])
    rng = np.random.Generator(np.random.PCG64(8))
    lon0 = rng.uniform(0, 360, 400)
    lat0 = np.rad2deg(np.arcsin(rng.uniform(-0.95, 0.95, 400)))
    theta = np.rad2deg(np.arccos(np.clip(xyz(lon0, lat0) @ axis, -1, 1)))
    keep = (np.abs(theta - 45) > 12) & (np.abs(theta - 135) > 12)
    lon0, lat0 = lon0[keep][:40], lat0[keep][:40]
    n = len(lon0)
    T = 2 * 86400.0
    exact = rotate(xyz(lon0, lat0), axis, U0 / R * T)
    errs = []
    for dt in (3600.0, 1800.0, 900.0):
        part = inputs.Particles(lon=lon0.copy(), lat=lat0.copy(), p=np.full(n, 500.0),
                                id=np.arange(n, dtype=np.uint32), up=np.zeros(n),
                                vp=np.zeros(n), wp=np.zeros(n))
        oracle.run(m, oracle.ctl(dt=dt, flags=oracle.ADVECT), part, 0, int(T / dt))
        got = xyz(part.lon, part.lat)
        errs.append(np.linalg.norm(got - exact, axis=1).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs
    assert errs[-1] < 1e-4


def test_position_wrap_and_reflection(met_c1, orc_c1):
    lon = np.array([360.0, -1e-300, 725.0, -0.5, 10.0, 359.999, 10.0, 200.0])
    lat = np.array([0.0, 0.0, 10.0, 10.0, 90.5, -90.25, 45.0, 90.0])
    p = np.array([500.0, 500.0, 1500.0, 0.2, 500.0, 500.0, 500.0, 500.0])
    lo, la, pp = oracle.position(orc_c1, lon, lat, p)
    assert np.all((lo >= 0) & (lo < 360))
    assert np.all((la >= -90) & (la <= 90))
    np.testing.assert_array_equal(lo[[0, 1, 2, 3]], [0.0, 0.0, 5.0, 359.5])
    assert la[4] == 89.5 and lo[4] == 190.0
    assert la[5] == -89.75 and abs(lo[5] - 179.999) < 1e-12
    assert pp[2] == met_c1.plev[0] and pp[3] == met_c1.plev[-1]
    # the point on the sphere does not move
    np.testing.assert_allclose(xyz(lo, la), xyz(lon, lat), atol=1e-13)


def test_position_property(orc_c1, met_c1):
    hyp = pytest.importorskip("hypothesis")
    st = pytest.importorskip("hypothesis.strategies")

    @hyp.settings(max_examples=300, deadline=None)
    @hyp.given(st.floats(-1000, 1000), st.floats(-179.9, 179.9), st.floats(0.001, 2000))
    def prop(lon, lat, p):
        lo, la, pp = oracle.position(orc_c1, [lon], [lat], [p])
        assert 0 <= lo[0] < 360 and -90 <= la[0] <= 90
        assert met_c1.plev[-1] <= pp[0] <= met_c1.plev[0]
        np.testing.assert_allclose(xyz(lo, la), xyz(np.array([lon]), np.array([lat])), atol=1e-11)

    prop()
