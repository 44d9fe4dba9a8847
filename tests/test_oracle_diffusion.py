"""Pins of the oracle's turbulent and mesoscale diffusion.

Turbulent diffusion adds stochastic perturbations to the trajectories and
mesoscale diffusion adds sub-grid wind fluctuations (Sec. 3.2,
module_diffusion_turb / module_diffusion_meso), both fed by per-parcel
random numbers (Sec. 4.3, Listing 6).  Pins: the variance of a Fickian
random walk grows as 2 K t; a uniform field has no sub-grid variance, so the
mesoscale state stays exactly zero; on a checkerboard every cell has
standard deviation a, so the AR(1) state has the closed-form variance
f^2 a^2 (1 - r^(2n)).
"""
import math

import numpy as np

import inputs
import oracle

R = 6371000.0
H0 = 7000.0
DT = 180.0


def zero_met(nt=3):
    return inputs.empty_met(180, 91, inputs.levels_log(30), nt)


def start_at(n, lat=0.0, p=500.0, lon=180.0):
    z = np.zeros(n)
    return inputs.Particles(lon=np.full(n, lon), lat=np.full(n, lat), p=np.full(n, p),
                            id=np.arange(n, dtype=np.uint32), up=z, vp=z.copy(), wp=z.copy())


def test_turbulent_variance_grows_as_2Kt():
    Dx, Dz = 50.0, 0.1
    n, steps = 200_000, 240
    m = oracle.Met(zero_met())
    part = start_at(n)
    oracle.run(m, oracle.ctl(turb_dx=Dx, turb_dz=Dz, flags=oracle.TURB), part, 0, steps)
    t = steps * DT
    tol = 5 * math.sqrt(2.0 / n)
    y = part.lat * math.pi * R / 180.0
    x = (part.lon - 180.0) * math.pi * R / 180.0       # cos(lat) ~ 1 - 1e-10 here
    z = H0 * np.log(part.p / 500.0)
    for arr, D in ((x, Dx), (y, Dx), (z, Dz)):
        assert abs(arr.var() / (2 * D * t) - 1) < tol, (arr.var(), 2 * D * t)
        assert abs(arr.mean()) < 5 * math.sqrt(2 * D * t / n)
    np.testing.assert_array_equal(part.up, 0.0)          # no meso state touched


def test_meso_uniform_field_keeps_state_zero():
    met = zero_met()
    inputs.fill_uniform(met, 12.0, -7.0, 0.001)
    m = oracle.Met(met)
    part = inputs.make_particles(2000, 9)
    ref = part.copy()
    oracle.run(m, oracle.ctl(flags=oracle.MESO), part, 0, 50)
    for name in ("up", "vp", "wp"):
        np.testing.assert_array_equal(getattr(part, name), 0.0)
    np.testing.assert_array_equal(part.lon, ref.lon)
    np.testing.assert_array_equal(part.lat, ref.lat)
    np.testing.assert_array_equal(part.p, ref.p)


def test_meso_checkerboard_ar1_variance():
    a, fh, fv = 2.0, 0.16, 0.3
    met = zero_met()
    inputs.fill_checkerboard(met, a)
    m = oracle.Met(met)
    sig = oracle.cell_sigma(m, np.array([10.0, 200.0]), np.array([-50.0, 33.0]),
                            np.array([700.0, 20.0]), 1000.0)
    np.testing.assert_allclose(sig, a, rtol=1e-15)
    n = 100_000
    part = inputs.make_particles(n, 10, lat_lo=-60, lat_hi=60)
    r = 1 - 2 * DT / met.dt_met
    tol = 5 * math.sqrt(2.0 / n)
    done = 0
    for steps in (5, 55):
        oracle.run(m, oracle.ctl(meso_fh=fh, meso_fv=fv, flags=oracle.MESO), part, done, steps)
        done += steps
        for name, f in (("up", fh), ("vp", fh), ("wp", fv)):
            want = f * f * a * a * (1 - r ** (2 * done))
            got = getattr(part, name).var()
            assert abs(got / want - 1) < tol, (name, done, got, want)


def test_meso_displacement_uses_state():
    """With a checkerboard, after one step the displacement equals the new
    state times dt (converted to degrees / hPa)."""
    met = zero_met()
    inputs.fill_checkerboard(met, 1.5)
    m = oracle.Met(met)
    part = inputs.make_particles(500, 11, lat_lo=-50, lat_hi=50, p_lo=300, p_hi=700)
    ref = part.copy()
    oracle.run(m, oracle.ctl(flags=oracle.MESO), part, 7, 1)
    dlon = part.up * DT * 180 / (math.pi * R * np.cos(np.deg2rad(ref.lat)))
    d = np.mod(part.lon - ref.lon + 180, 360) - 180
    np.testing.assert_allclose(d, dlon, rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(part.lat - ref.lat, part.vp * DT * 180 / (math.pi * R), rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(part.p - ref.p, part.wp * DT, rtol=1e-9, atol=1e-12)
    # first step from zero state: u' = sqrt(1 - r^2) f a xi, xi from purpose 1
    r = 1 - 2 * DT / met.dt_met
    xi = oracle.normals(oracle.SEED, ref.id, 7, 1)
    np.testing.assert_allclose(part.up, math.sqrt(1 - r * r) * 0.16 * 1.5 * xi[:, 0], rtol=1e-13)
