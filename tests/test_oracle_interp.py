"""Pins of the oracle's locate + 4D interpolation (lon, lat, pressure, time).

The paper reads winds on a grid (Sec. 3.1, read_met and its periodic
extension read_met_periodic) and samples them along trajectories (Sec. 3.2);
the interpolation here is quadrilinear with periodic longitude, clamped
latitude and pressure, and a weight linear in p.  Pins: exactness on
multilinear fields built from integers, brute force with independently
computed indices and product weights, continuity across cells, levels, the
seam and time levels.
"""
import numpy as np
import pytest

import inputs
import oracle


def multilinear_met(nt=3):
    """Tiny grid whose stored values f = (1 + lon/45)(2 + (lat+90)/45)
    (3 + p/100)(1 + l) are integers, hence exact in float32."""
    plev = np.array([1000.0, 700.0, 400.0, 100.0])
    met = inputs.empty_met(nx=8, ny=5, plev=plev, nt=nt, dt_met=3600.0)
    lon = met.lon_axis()
    lat = met.lat_axis()
    f = ((1 + lon / 45)[None, None, :] * (2 + (lat + 90) / 45)[None, :, None]
         * (3 + plev / 100)[:, None, None])
    for l in range(nt):
        met.u[l] = f * (1 + l)
        met.v[l] = 2 * f * (1 + l)
        met.w[l] = -f * (1 + l)
    return met


def f_exact(lon, lat, p, t, dt_met):
    return (1 + lon / 45) * (2 + (lat + 90) / 45) * (3 + p / 100) * (1 + t / dt_met)


def test_exact_on_multilinear_fields(rng):
    met = multilinear_met()
    m = oracle.Met(met)
    n = 5000
    lon = rng.uniform(0, 315, n)                  # away from the seam cell
    lat = rng.uniform(-90, 90, n)
    p = rng.uniform(100, 1000, n)
    for t in (0.0, 1234.5, 3600.0, 5000.0, 7200.0):
        got = oracle.interp(m, lon, lat, p, t)
        want = f_exact(lon, lat, p, t, met.dt_met)
        np.testing.assert_allclose(got[:, 0], want, rtol=1e-13)
        np.testing.assert_allclose(got[:, 1], 2 * want, rtol=1e-13)
        np.testing.assert_allclose(got[:, 2], -want, rtol=1e-13)


def test_exact_on_constants(met_c1, rng):
    met = inputs.empty_met(met_c1.nx, met_c1.ny, met_c1.plev, 2)
    inputs.fill_uniform(met, 12.5, -3.25, 0.0078125)
    m = oracle.Met(met)
    n = 2000
    got = oracle.interp(m, rng.uniform(-720, 720, n), rng.uniform(-95, 95, n),
                        rng.uniform(0.5, 1100, n), 1000.0)
    np.testing.assert_allclose(got, np.tile([12.5, -3.25, 0.0078125], (n, 1)), rtol=1e-15)


def brute_force(met, lon, lat, p, t):
    """Direct weighted sum over the 16 corners, with indices found by
    searchsorted and weights as products -- written independently of the
    oracle's nested lerps."""
    out = np.zeros((len(lon), 3))
    lons = np.mod(lon - met.lon0, 360.0)
    x = lons / met.dlon
    i0 = np.floor(x).astype(np.int64)
    fx = x - i0
    i0 %= met.nx
    i1 = (i0 + 1) % met.nx
    latc = np.clip(lat, -90, 90)
    y = (latc - met.lat0) / met.dlat
    j0 = np.minimum(np.floor(y).astype(np.int64), met.ny - 2)
    fy = y - j0
    pc = np.clip(p, met.plev[-1], met.plev[0])
    # ascending copy of the levels: index of the first level >= pc from the top
    asc = met.plev[::-1]
    kk = met.nz - 1 - np.searchsorted(asc, pc, side="left")
    k0 = np.clip(kk, 0, met.nz - 2)
    fz = (met.plev[k0] - pc) / (met.plev[k0] - met.plev[k0 + 1])
    l0 = int(min(max(np.floor((t - met.t_met0) / met.dt_met), 0), met.nt - 2))
    ft = (t - (met.t_met0 + l0 * met.dt_met)) / met.dt_met
    for dl, wl in ((0, 1 - ft), (1, ft)):
        for dk in (0, 1):
            wk = (1 - fz) if dk == 0 else fz
            for dj in (0, 1):
                wj = (1 - fy) if dj == 0 else fy
                for ii, wi in ((i0, 1 - fx), (i1, fx)):
                    w = wl * wk * wj * wi
                    for q, arr in enumerate((met.u, met.v, met.w)):
                        out[:, q] += w * arr[l0 + dl, k0 + dk, j0 + dj, ii]
    return out


def test_brute_force_random_field(met_c1, orc_c1, rng):
    n = 4000
    lon = rng.uniform(-10, 370, n)
    lat = rng.uniform(-90, 90, n)
    lat[:50] = rng.choice([-90.0, 90.0], 50)
    p = rng.uniform(0.9, 1010, n)
    p[:30] = met_c1.plev[rng.integers(0, met_c1.nz, 30)]
    for t in (0.0, 777.0, 21600.0):
        got = oracle.interp(orc_c1, lon, lat, p, t)
        want = brute_force(met_c1, lon, lat, p, t)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_periodic_in_longitude(orc_c1, rng):
    n = 1000
    lon = rng.uniform(0, 360, n)
    lat = rng.uniform(-89, 89, n)
    p = rng.uniform(100, 900, n)
    a = oracle.interp(orc_c1, lon, lat, p, 100.0)
    for shift in (360.0, -360.0, 720.0, -1080.0):
        b = oracle.interp(orc_c1, lon + shift, lat, p, 100.0)
        np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-10)


def test_seam_cell_is_average_of_last_and_first_columns(met_c1, orc_c1):
    lon = np.array([met_c1.lon0 + (met_c1.nx - 0.5) * met_c1.dlon])
    lat = np.array([met_c1.lat_axis()[40]])
    p = np.array([met_c1.plev[7]])
    got = oracle.interp(orc_c1, lon, lat, p, 0.0)[0]
    want = 0.5 * (met_c1.u[0, 7, 40, -1].astype(np.float64) + met_c1.u[0, 7, 40, 0])
    assert abs(got[0] - want) < 1e-12


@pytest.mark.parametrize("which", ["lon", "lat", "p", "t", "seam"])
def test_continuity_across_boundaries(met_c1, which, rng):
    met = met_c1
    nt3 = inputs.make_met_c1(seed=5, nt=3)
    m = oracle.Met(nt3)
    n = 200
    eps = 1e-9
    lon = rng.uniform(0, 350, n)
    lat = rng.uniform(-80, 80, n)
    p = rng.uniform(150, 850, n)
    t = 15000.0
    if which == "lon":
        lon = met.lon0 + rng.integers(1, met.nx - 1, n) * met.dlon
        a, b = oracle.interp(m, lon - eps, lat, p, t), oracle.interp(m, lon + eps, lat, p, t)
    elif which == "seam":
        a, b = oracle.interp(m, np.full(n, 360 - eps), lat, p, t), oracle.interp(m, np.full(n, eps), lat, p, t)
    elif which == "lat":
        lat = met.lat_axis()[rng.integers(1, met.ny - 1, n)]
        a, b = oracle.interp(m, lon, lat - eps, p, t), oracle.interp(m, lon, lat + eps, p, t)
    elif which == "p":
        p = met.plev[rng.integers(1, met.nz - 1, n)]
        a, b = oracle.interp(m, lon, lat, p * (1 - eps), t), oracle.interp(m, lon, lat, p * (1 + eps), t)
    else:
        tl = nt3.t_met0 + nt3.dt_met
        a, b = oracle.interp(m, lon, lat, p, tl - 1e-6), oracle.interp(m, lon, lat, p, tl + 1e-6)
    assert np.abs(a - b).max() < 1e-5


def test_clamping_outside_domain(met_c1, orc_c1, rng):
    n = 300
    lon = rng.uniform(0, 360, n)
    lat = rng.uniform(-80, 80, n)
    for p_out, p_in in ((1200.0, met_c1.plev[0]), (0.1, met_c1.plev[-1])):
        a = oracle.interp(orc_c1, lon, lat, np.full(n, p_out), 0.0)
        b = oracle.interp(orc_c1, lon, lat, np.full(n, p_in), 0.0)
        np.testing.assert_array_equal(a, b)
    a = oracle.interp(orc_c1, lon, np.full(n, 95.0), np.full(n, 500.0), 0.0)
    b = oracle.interp(orc_c1, lon, np.full(n, 90.0), np.full(n, 500.0), 0.0)
    np.testing.assert_array_equal(a, b)


def test_locate_brackets(met_c1, orc_c1, rng):
    n = 3000
    lon = rng.uniform(0, 360, n)
    lat = rng.uniform(-90, 90, n)
    p = rng.uniform(1, 1000, n)
    idx, frac = oracle.locate(orc_c1, lon, lat, p, 0.0)
    i, j, k = idx[:, 0], idx[:, 1], idx[:, 2]
    assert np.all((frac[:, :3] >= 0) & (frac[:, :3] <= 1))
    assert np.all((0 <= i) & (i < met_c1.nx))
    np.testing.assert_allclose(met_c1.lon0 + (i + frac[:, 0]) * met_c1.dlon, lon, atol=1e-10)
    np.testing.assert_allclose(met_c1.lat0 + (j + frac[:, 1]) * met_c1.dlat, lat, atol=1e-10)
    assert np.all(met_c1.plev[k] >= p) and np.all(met_c1.plev[k + 1] <= p)
    pl = met_c1.plev[k] + frac[:, 2] * (met_c1.plev[k + 1] - met_c1.plev[k])
    np.testing.assert_allclose(pl, p, rtol=1e-12)


def test_cell_sigma_brute_force(met_c1, orc_c1, rng):
    n = 500
    lon = rng.uniform(0, 360, n)
    lat = rng.uniform(-90, 90, n)
    p = rng.uniform(1, 1000, n)
    t = 5000.0
    got = oracle.cell_sigma(orc_c1, lon, lat, p, t)
    idx, _ = oracle.locate(orc_c1, lon, lat, p, t)
    for q, arr in enumerate((met_c1.u, met_c1.v, met_c1.w)):
        for r in range(n):
            i, j, k, l = idx[r]
            ii = [i, (i + 1) % met_c1.nx]
            vals = arr[l:l + 2, k:k + 2, j:j + 2][:, :, :, ii].astype(np.float64).ravel()
            assert vals.size == 16
            assert abs(got[r, q] - vals.std()) <= 1e-12 * max(1.0, vals.std())
