"""Pins of the oracle's full time step (advection, position, turbulent and
mesoscale diffusion, position) and its activity gating.

Parcels are independent (Sec. 3.4: no communication between them), so a
parcel's trajectory may not depend on which other parcels are run with it;
random numbers are keyed by parcel id and step (Sec. 4.3 decouples them from
the modules), so splitting a run, reordering parcels or running a subset
must reproduce the same trajectories bit for bit.  Parcels not yet
released or with non-finite positions are skipped (Sec. 4.3,
module_timesteps).  The last test pins the parity tolerance: it measures how
much the flow amplifies a 1e-12 deg perturbation.
"""
import numpy as np
import pytest

import inputs
import oracle

FIELDS = ("lon", "lat", "p", "up", "vp", "wp")


def assert_same(a, b):
    for f in FIELDS:
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f), err_msg=f)


@pytest.fixture(scope="module")
def met_nt3():
    return inputs.make_met_c1(seed=11, nt=3)


def test_step_is_advect_then_diffuse(met_nt3):
    m = oracle.Met(met_nt3)
    a = inputs.make_particles(3000, 21)
    b = a.copy()
    for s in range(10):
        oracle.run(m, oracle.ctl(), a, s, 1)
        oracle.run(m, oracle.ctl(flags=oracle.ADVECT), b, s, 1)
        oracle.run(m, oracle.ctl(flags=oracle.TURB | oracle.MESO), b, s, 1)
    assert_same(a, b)


def test_restart_is_bitwise(met_nt3):
    m = oracle.Met(met_nt3)
    a = inputs.make_particles(2000, 22)
    b = a.copy()
    oracle.run(m, oracle.ctl(), a, 0, 60)
    oracle.run(m, oracle.ctl(), b, 0, 25)
    oracle.run(m, oracle.ctl(), b, 25, 35)
    assert_same(a, b)


def test_subset_and_order_independence(met_nt3):
    m = oracle.Met(met_nt3)
    full = inputs.make_particles(4000, 23)
    rng = np.random.Generator(np.random.PCG64(2))
    idx = rng.permutation(4000)[:700]
    sub = full.subset(idx)
    oracle.run(m, oracle.ctl(), full, 0, 40, nthreads=3)
    oracle.run(m, oracle.ctl(), sub, 0, 40, nthreads=1)
    assert_same(full.subset(idx), sub)


def test_nonfinite_parcels_untouched(met_nt3):
    m = oracle.Met(met_nt3)
    a = inputs.make_particles(100, 24)
    a.lon[3] = np.nan
    a.lat[7] = np.inf
    a.p[11] = -np.inf
    ref = a.copy()
    oracle.run(m, oracle.ctl(), a, 0, 20)
    for i in (3, 7, 11):
        for f in FIELDS:
            x, y = getattr(a, f)[i], getattr(ref, f)[i]
            assert (x == y) or (np.isnan(x) and np.isnan(y))
    assert not np.any(a.lon[[0, 1, 2]] == ref.lon[[0, 1, 2]])


def test_release_gating(met_nt3):
    m = oracle.Met(met_nt3)
    a = inputs.make_particles(500, 25)
    ref = a.copy()
    rel = np.where(np.arange(500) % 2 == 0, 10, 0).astype(np.int32)
    oracle.run(m, oracle.ctl(), a, 0, 10, release=rel)
    even = np.arange(0, 500, 2)
    assert_same(a.subset(even), ref.subset(even))              # not yet released
    oracle.run(m, oracle.ctl(), a, 10, 20, release=rel)
    late = ref.subset(even)
    oracle.run(m, oracle.ctl(), late, 10, 20)                  # released at step 10
    assert_same(a.subset(even), late)


def test_met_time_levels_advance(met_nt3):
    """Runs across the 6 h level boundary use the next level pair (the
    met0/met1 pair advances); a run of 240 steps spans three levels."""
    m = oracle.Met(met_nt3)
    a = inputs.make_particles(200, 26)
    oracle.run(m, oracle.ctl(), a, 0, 240)
    assert np.all(np.isfinite(a.lon)) and np.all((a.lon >= 0) & (a.lon < 360))


def test_tolerance_from_perturbation_growth(met_nt3):
    """Parity tolerance pin: FP64 rounding differences are about one ulp of
    a longitude (~4e-14 deg); the flow amplifies a perturbation by the factor
    measured here.  The F64 tolerance of 1e-9 deg must exceed that product
    by a wide margin."""
    m = oracle.Met(met_nt3)
    a = inputs.make_particles(2000, 27)
    b = a.copy()
    b.lon = b.lon + 1e-12
    b.lat = np.clip(b.lat + 1e-12, -90, 90)
    oracle.run(m, oracle.ctl(), a, 0, 240)
    oracle.run(m, oracle.ctl(), b, 0, 240)
    d = oracle.chord_deg(a.lon, a.lat, b.lon, b.lat)
    growth = d.max() / 1e-12
    assert growth < 1e3, growth
    assert 4e-14 * growth < 1e-9 / 10


def test_tolerance_growth_realistic_fields():
    """The same pin on jet + perturbation fields (0.9 deg version of the
    0.3 deg workload): horizontal growth stays small and a 1e-12 deg
    horizontal perturbation moves pressure by far less than the 1e-7 hPa
    pressure tolerance allows for ulp-level differences."""
    met = inputs.make_met_c2(seed=12, nt=3, nx=400, ny=201)
    m = oracle.Met(met)
    a = inputs.make_particles(3000, 22)
    b = a.copy()
    b.lon = b.lon + 1e-12
    oracle.run(m, oracle.ctl(), a, 0, 240)
    oracle.run(m, oracle.ctl(), b, 0, 240)
    d = oracle.chord_deg(a.lon, a.lat, b.lon, b.lat)
    growth = d.max() / 1e-12
    assert growth < 1e3, growth
    # ulp-level start (4e-14 deg) scaled by the observed pressure response
    assert np.abs(a.p - b.p).max() * (4e-14 / 1e-12) < 1e-7 / 10
