"""Pins of three oracle functions against closed forms and brute force.

* ``stencil81`` (surrogate inputs, row A14; the oracle's C12 reading):
  on a field that is a product of integer-valued linear factors in lon,
  lat, p and t, a quadrilinear interpolation with product weights is the
  product of four 1-D linear interpolations, so the value in the cell
  shifted by (a, b, c) with the parcel's own weights has a closed form --
  written here factor by factor, with the shifted columns wrapping over
  the periodic seam and the shifted rows and levels clamped to the grid.
* ``displacement`` (surrogate targets, row A15): under a uniform wind the
  8-step midpoint displacement is exact: east 8 U dt along the start
  latitude, north 8 V dt, dp 8 W dt (advection, Sec. 3.2).
* ``tile_keys`` (the sort by grid box of Sec. 6, row A11; tile then half-tile): brute force
  with the cell found by ``searchsorted`` on the level table, the tile
  numbered lon fastest, non-finite positions on the last key.
"""
import numpy as np
import pytest

import inputs
import oracle


# ---- stencil81 --------------------------------------------------------------

def product_met(nx=8, ny=7, nt=3):
    """Stored values (1 + i)(2 + j)(3 + k)(1 + l) times 1, 2, -1 for u, v, w:
    integers, exact in float32, and a product of one factor per axis that
    is not periodic in i (so a wrong seam shows)."""
    plev = np.array([1000.0, 850.0, 700.0, 500.0, 300.0, 100.0])
    met = inputs.empty_met(nx=nx, ny=ny, plev=plev, nt=nt, dt_met=3600.0)
    gi = 1.0 + np.arange(nx)
    gj = 2.0 + np.arange(ny)
    gk = 3.0 + np.arange(len(plev))
    f = gk[:, None, None] * gj[None, :, None] * gi[None, None, :]
    for l in range(nt):
        met.u[l] = f * (1 + l)
        met.v[l] = 2 * f * (1 + l)
        met.w[l] = -f * (1 + l)
    return met, gi, gj, gk


def cell_of(met, lon, lat, p):
    """Cell and weights found independently: mod / floor in lon, clamped
    floor in lat, searchsorted on the ascending level table in p."""
    x = np.mod(lon - met.lon0, 360.0) / met.dlon
    i0 = np.floor(x).astype(np.int64)
    fx = x - i0
    i0 %= met.nx
    y = (np.clip(lat, -90.0, 90.0) - met.lat0) / met.dlat
    j = np.minimum(np.floor(y).astype(np.int64), met.ny - 2)
    fy = y - j
    pc = np.clip(p, met.plev[-1], met.plev[0])
    k = np.clip(met.nz - 1 - np.searchsorted(met.plev[::-1], pc, side="left"), 0, met.nz - 2)
    fz = (met.plev[k] - pc) / (met.plev[k] - met.plev[k + 1])
    return i0, j, k, fx, fy, fz


def expected_stencil(met, gi, gj, gk, lon, lat, p, t):
    i0, j, k, fx, fy, fz = cell_of(met, lon, lat, p)
    l0 = int(min(max(np.floor((t - met.t_met0) / met.dt_met), 0), met.nt - 2))
    ft = (t - (met.t_met0 + l0 * met.dt_met)) / met.dt_met
    gt = (1.0 + l0) * (1 - ft) + (2.0 + l0) * ft
    out = np.empty((len(lon), 81))
    for c in (-1, 0, 1):
        kc = np.clip(k + c, 0, met.nz - 2)
        zf = gk[kc] * (1 - fz) + gk[kc + 1] * fz
        for b in (-1, 0, 1):
            jb = np.clip(j + b, 0, met.ny - 2)
            yf = gj[jb] * (1 - fy) + gj[jb + 1] * fy
            for a in (-1, 0, 1):
                ia = (i0 + a) % met.nx
                xf = gi[ia] * (1 - fx) + gi[(ia + 1) % met.nx] * fx
                val = xf * yf * zf * gt
                col = (c + 1) * 9 + (b + 1) * 3 + (a + 1)
                out[:, col] = val
                out[:, 27 + col] = 2 * val
                out[:, 54 + col] = -val
    return out


def test_stencil81_closed_form(rng):
    met, gi, gj, gk = product_met()
    m = oracle.Met(met)
    n = 3000
    lon = rng.uniform(-30, 390, n)
    lat = rng.uniform(-90, 90, n)
    p = rng.uniform(100, 1000, n)
    # the seam column (i0 = nx - 1 and shifts across it), the first column,
    # the polar rows (clamped shifts), the bottom and top levels
    lon[:200] = rng.uniform(315, 360, 200)
    lon[200:300] = rng.uniform(0, 45, 100)
    lat[300:400] = rng.uniform(-90, -60, 100)
    lat[400:500] = rng.uniform(60, 90, 100)
    lat[500:520] = 90.0
    lat[520:540] = -90.0
    p[540:640] = rng.uniform(850, 1000, 100)
    p[640:740] = rng.uniform(100, 300, 100)
    p[740:760] = 1000.0
    p[760:780] = 100.0
    for t in (0.0, 1800.0, 3600.0, 6000.0):
        got = oracle.stencil81(m, lon, lat, p, t)
        want = expected_stencil(met, gi, gj, gk, lon, lat, p, t)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)


def test_stencil81_centre_is_the_interpolation(rng):
    """The (0, 0, 0) entries are the plain interpolation of each variable."""
    met = inputs.make_met_c1(seed=11, nt=2)
    m = oracle.Met(met)
    n = 500
    lon, lat, p = rng.uniform(0, 360, n), rng.uniform(-89, 89, n), rng.uniform(100, 900, n)
    s = oracle.stencil81(m, lon, lat, p, 900.0)
    w = oracle.interp(m, lon, lat, p, 900.0)
    for q in range(3):
        np.testing.assert_array_equal(s[:, 27 * q + 13], w[:, q])


def test_stencil81_order_of_offsets(rng):
    """A field varying along one axis only shows the offset order: columns
    a = -1, 0, 1 are fastest, then rows b, then levels c."""
    met, gi, gj, gk = product_met()
    for axis in range(3):
        m2 = inputs.empty_met(nx=met.nx, ny=met.ny, plev=met.plev, nt=2, dt_met=3600.0)
        shape = (met.nz, met.ny, met.nx)
        f = np.broadcast_to(np.arange(shape[2 - axis], dtype=np.float32).reshape(
            [-1 if d == 2 - axis else 1 for d in range(3)]), shape)
        for l in range(2):
            m2.u[l] = f
            m2.v[l] = 0
            m2.w[l] = 0
        m = oracle.Met(m2)
        # a cell in the interior, with weights 0 so values are grid values
        lon = np.array([3 * met.dlon])
        lat = np.array([-90 + 3 * met.dlat])
        p = np.array([met.plev[2]])
        s = oracle.stencil81(m, lon, lat, p, 0.0)[0, :27].reshape(3, 3, 3)   # [c][b][a]
        idx = np.indices((3, 3, 3))[2 - axis] - 1
        np.testing.assert_array_equal(s, idx + (2 if axis == 2 else 3))


# ---- displacement -------------------------------------------------------------

def f32(x):
    """The value as stored (fields are float32)."""
    return float(np.float32(x))


def uniform_met(u, v, w_hpa):
    met = inputs.empty_met(nx=36, ny=19, plev=np.geomspace(1000.0, 10.0, 12), nt=2, dt_met=21600.0)
    inputs.fill_uniform(met, u, v, w_hpa)
    return met


@pytest.mark.parametrize("U,W", [(20.0, 0.0), (-35.0, 0.002), (7.5, -0.001)])
def test_displacement_uniform_zonal(rng, U, W):
    met = uniform_met(U, 0.0, W)
    m = oracle.Met(met)
    c = oracle.ctl(dt=180.0)
    n = 400
    lon = rng.uniform(0, 360, n)
    lon[:50] = rng.uniform(355, 360, 50)            # across the seam
    lat = rng.uniform(-80, 80, n)
    p = rng.uniform(300, 700, n)
    d = oracle.displacement(m, c, lon, lat, p, 3, 8)
    np.testing.assert_allclose(d[:, 0], 8 * f32(U) * 180.0 / 1000.0, rtol=1e-11)
    np.testing.assert_allclose(d[:, 1], 0.0, atol=1e-12)
    np.testing.assert_allclose(d[:, 2], 8 * f32(W) * 180.0, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("V,W", [(15.0, 0.0), (-25.0, -0.003)])
def test_displacement_uniform_meridional(rng, V, W):
    met = uniform_met(0.0, V, W)
    m = oracle.Met(met)
    c = oracle.ctl(dt=180.0)
    n = 400
    lon = rng.uniform(0, 360, n)
    lat = rng.uniform(-70, 70, n)
    p = rng.uniform(300, 700, n)
    d = oracle.displacement(m, c, lon, lat, p, 0, 8)
    np.testing.assert_allclose(d[:, 0], 0.0, atol=1e-12)
    np.testing.assert_allclose(d[:, 1], 8 * f32(V) * 180.0 / 1000.0, rtol=1e-11)
    np.testing.assert_allclose(d[:, 2], 8 * f32(W) * 180.0, rtol=1e-11, atol=1e-12)


def test_displacement_is_k_advection_steps(met_c1, orc_c1, rng):
    """Against k plain steps of the oracle's own run (advection only): the
    displacement converts the difference of positions to km."""
    n = 300
    part = inputs.make_particles(n, 5)
    d = oracle.displacement(orc_c1, oracle.ctl(), part.lon, part.lat, part.p, 4, 8)
    q = part.copy()
    oracle.run(orc_c1, oracle.ctl(flags=oracle.ADVECT), q, 4, 8)
    km = np.pi * 6371.0 / 180.0
    dl = (q.lon - part.lon + 540.0) % 360.0 - 180.0
    c0 = np.maximum(np.cos(np.deg2rad(part.lat)), np.cos(np.deg2rad(89.999)))
    np.testing.assert_allclose(d[:, 0], dl * c0 * km, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(d[:, 1], (q.lat - part.lat) * km, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(d[:, 2], q.p - part.p, rtol=1e-12, atol=1e-12)


# ---- tile keys ---------------------------------------------------------------------

def brute_keys(met, lon, lat, p):
    """8 x tile + half-tile: the tile of the cell, lon fastest, then the
    half of the tile it lies in along level (4), lat (2) and lon (1)."""
    ntx = -(-met.nx // 8)
    nty = -(-(met.ny - 1) // 8)
    ntz = -(-(met.nz - 1) // 4)
    out = np.full(len(lon), 8 * ntx * nty * ntz, np.int64)
    ok = np.isfinite(lon) & np.isfinite(lat) & np.isfinite(p)
    i0, j, k, _, _, _ = cell_of(met, lon[ok], lat[ok], p[ok])
    tile = ((k // 4) * nty + j // 8) * ntx + i0 // 8
    half = 4 * (k - 4 * (k // 4) >= 2) + 2 * (j - 8 * (j // 8) >= 4) + (i0 - 8 * (i0 // 8) >= 4)
    out[ok] = 8 * tile + half
    return out


@pytest.mark.parametrize("grid", ["c1", "odd"])
def test_tile_keys_brute_force(met_c1, rng, grid):
    if grid == "c1":
        met = met_c1
    else:                                      # sizes that are not multiples of the tile
        met = inputs.empty_met(nx=45, ny=23, plev=np.geomspace(1000.0, 1.0, 14), nt=2)
    m = oracle.Met(met)
    n = 20000
    lon = rng.uniform(-400, 760, n)
    lat = rng.uniform(-95, 95, n)
    p = rng.uniform(0.1, 1200, n)
    # grid lines, poles, the level values and the ends of the table exactly
    lon[:200] = met.dlon * rng.integers(-met.nx, 2 * met.nx, 200)
    lat[200:400] = -90.0 + met.dlat * rng.integers(0, met.ny, 200)
    p[400:600] = met.plev[rng.integers(0, met.nz, 200)]
    p[600:620] = met.plev[0]
    p[620:640] = met.plev[-1]
    lat[640:660] = 90.0
    lon[660:670] = np.nan
    lat[670:680] = np.inf
    p[680:690] = -np.inf
    got = oracle.tile_keys(m, lon, lat, p).astype(np.int64)
    want = brute_keys(met, lon, lat, p)
    np.testing.assert_array_equal(got, want)
    ntiles = (-(-met.nx // 8)) * (-(-(met.ny - 1) // 8)) * (-(-(met.nz - 1) // 4))
    assert np.all(got[660:690] == 8 * ntiles)
    assert got[np.isfinite(lon) & np.isfinite(lat) & np.isfinite(p)].max() < 8 * ntiles


def test_tile_keys_walk_the_halves_of_a_tile(met_c1):
    """The cell centres of one tile: keys 8t .. 8t + 7, each half-tile of
    4 x 4 x 2 cells one key, in the order (level, lat, lon) halves."""
    met = met_c1
    m = oracle.Met(met)
    ti, tj, tk = 3, 2, 1                       # a tile away from the grid edges
    ii, jj, kk = np.meshgrid(np.arange(8), np.arange(8), np.arange(4), indexing="ij")
    i0, j, k = 8 * ti + ii.ravel(), 8 * tj + jj.ravel(), 4 * tk + kk.ravel()
    lon = met.lon0 + (i0 + 0.5) * met.dlon
    lat = met.lat0 + (j + 0.5) * met.dlat
    p = np.sqrt(np.asarray(met.plev)[k] * np.asarray(met.plev)[k + 1])
    got = oracle.tile_keys(m, lon, lat, p).astype(np.int64)
    ntx, nty = -(-met.nx // 8), -(-(met.ny - 1) // 8)
    t = (tk * nty + tj) * ntx + ti
    assert set(np.unique(got)) == set(range(8 * t, 8 * t + 8))
    for key in range(8 * t, 8 * t + 8):
        h = key - 8 * t
        sel = got == key
        assert sel.sum() == 32
        assert np.all((ii.ravel()[sel] >= 4) == bool(h & 1))
        assert np.all((jj.ravel()[sel] >= 4) == bool(h & 2))
        assert np.all((kk.ravel()[sel] >= 2) == bool(h & 4))
