"""Pins of the oracle's convection and sedimentation (module_convection,
module_sedi, Sec. 3.2; the paper names the modules only, the readings are
stated in include/mpt.h and the oracle's header).

Sedimentation, against what the physics fixes independently of the code:
* Sutherland's law with (1.458e-6, 110.4 K) gives the reference viscosity of
  air, 1.716e-5 Pa s at 273.15 K; recovered from the settling velocity of a
  centimetre sphere, where the slip correction is 1 to 1e-5;
* continuum regime (radius >> mean free path): v grows as r^2 and does not
  depend on the pressure;
* free-molecular regime (radius << mean free path): v grows as r and as
  1/p (Cc -> 1.657 Kn);
* standard aerosol tables (Hinds, Aerosol Technology, 2nd ed., 1999,
  terminal settling velocities of unit-density spheres at 293 K, 1 atm):
  1 um diameter 3.5e-5 m/s, 10 um 3.06e-3 m/s; within 3 % (the tables use
  slightly different slip-correction constants).

Convection, on fields where the answer is known:
* below the equilibrium level with CAPE over the threshold the new pressure
  is uniform between surface and equilibrium level (Kolmogorov-Smirnov);
* above the equilibrium level, or with CAPE below the threshold, nothing
  moves; the threshold is crossed where the bilinear CAPE (a linear field,
  reproduced exactly) equals it.
"""
import numpy as np
import pytest
from scipy import stats

import inputs
import oracle


def test_sutherland_reference_viscosity():
    r, rho_p, p, T = 1e-2, 1e6, 1013.25, 273.15
    v = oracle.settling_velocity(r, rho_p, p, T)
    rho_air = 100.0 * p / (287.058 * T)
    eta = 2.0 * r * r * (rho_p - rho_air) * 9.80665 / (9.0 * v)
    assert abs(eta / 1.716e-5 - 1.0) < 1e-3


def test_continuum_regime_scales_as_r_squared_and_ignores_pressure():
    v1 = oracle.settling_velocity(1e-3, 2000.0, 1000.0, 280.0)
    v2 = oracle.settling_velocity(2e-3, 2000.0, 1000.0, 280.0)
    assert abs(v2 / v1 - 4.0) < 4e-4
    v_low = oracle.settling_velocity(1e-3, 2000.0, 500.0, 280.0)
    rho = lambda p: 100.0 * p / (287.058 * 280.0)
    # only the buoyancy term differs
    assert abs(v_low / v1 - (2000.0 - rho(500.0)) / (2000.0 - rho(1000.0))) < 1e-3


def test_free_molecular_regime_scales_as_r_and_inverse_pressure():
    v1 = oracle.settling_velocity(1e-10, 1000.0, 1000.0, 250.0)
    v2 = oracle.settling_velocity(2e-10, 1000.0, 1000.0, 250.0)
    assert abs(v2 / v1 - 2.0) < 5e-3
    v_half = oracle.settling_velocity(1e-10, 1000.0, 500.0, 250.0)
    assert abs(v_half / v1 - 2.0) < 5e-3


@pytest.mark.parametrize("d, v_table", [(1e-6, 3.5e-5), (10e-6, 3.06e-3)])
def test_standard_settling_table(d, v_table):
    v = oracle.settling_velocity(d / 2, 1000.0, 1013.25, 293.15)
    assert abs(v / v_table - 1.0) < 0.03


def small_met(nt=2):
    met = inputs.empty_met(36, 19, inputs.levels_log(10, 1000.0, 10.0), nt)
    shape2 = (nt, met.ny, met.nx)
    met.temp = np.full(met.u.shape, 250.0, np.float32)
    met.cape = np.full(shape2, 1000.0, np.float32)
    met.pel = np.full(shape2, 200.0, np.float32)
    met.ps = np.full(shape2, 1000.0, np.float32)
    return met


def parcels(n, lon, lat, p, seed=5):
    part = inputs.make_particles(n, seed)
    part.lon[:] = lon
    part.lat[:] = lat
    part.p[:] = p
    return part


def test_convection_mixes_uniformly_between_surface_and_equilibrium_level():
    met = small_met()
    part = parcels(40_000, 33.0, 12.0, 800.0)
    c = oracle.ctl(flags=oracle.CONV)
    oracle.run(oracle.Met(met), c, part, 3, 1)
    assert np.all((part.p >= 200.0) & (part.p <= 1000.0))
    ks = stats.kstest((part.p - 200.0) / 800.0, "uniform")
    assert ks.pvalue > 1e-3
    # the draw is the first word of Philox (id, step, 5, 0)
    x = oracle.philox(np.stack([part.id, np.full(part.n, 3, np.uint32), np.full(part.n, 5, np.uint32),
                                np.zeros(part.n, np.uint32)], 1).astype(np.uint32),
                      (oracle.SEED & 0xFFFFFFFF, oracle.SEED >> 32))
    u = ((x[:, 0] >> 8).astype(np.float64) + 0.5) / 2.0 ** 24
    np.testing.assert_allclose(part.p, 1000.0 + (200.0 - 1000.0) * u, rtol=0, atol=1e-12)


def test_convection_leaves_parcels_above_the_equilibrium_level_or_below_threshold():
    met = small_met()
    part = parcels(1000, 100.0, -30.0, 150.0)
    oracle.run(oracle.Met(met), oracle.ctl(flags=oracle.CONV), part, 0, 5)
    assert np.all(part.p == 150.0)
    part = parcels(1000, 100.0, -30.0, 800.0)
    oracle.run(oracle.Met(met), oracle.ctl(flags=oracle.CONV, conv_cape=1000.5), part, 0, 5)
    assert np.all(part.p == 800.0)


def test_convection_threshold_follows_bilinear_cape():
    met = small_met()
    lat = met.lat_axis()
    met.cape[:] = (20.0 * (lat + 90.0)).astype(np.float32)[None, :, None]   # linear in lat
    lat_star = 500.0 / 20.0 - 90.0                                         # CAPE = 500 here
    lats = np.concatenate([np.full(500, lat_star - 0.01), np.full(500, lat_star + 0.01)])
    part = parcels(1000, 77.0, 0.0, 900.0)
    part.lat[:] = lats
    oracle.run(oracle.Met(met), oracle.ctl(flags=oracle.CONV), part, 0, 1)
    assert np.all(part.p[:500] == 900.0)
    assert np.all(part.p[500:] != 900.0)


def test_sedimentation_step_matches_settling_velocity():
    met = small_met()
    part = parcels(10, 50.0, 20.0, 600.0)
    r, rho = 20e-6, 1500.0
    oracle.run(oracle.Met(met), oracle.ctl(flags=oracle.SEDI, sedi_r=r, sedi_rho=rho), part, 0, 1)
    v = oracle.settling_velocity(r, rho, 600.0, 250.0)
    np.testing.assert_allclose(part.p, 600.0 + 600.0 * v * 180.0 / 7000.0, rtol=1e-14)
    assert np.all(part.p > 600.0)
