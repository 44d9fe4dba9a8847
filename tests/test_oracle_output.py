"""Pins of the oracle's gridded output (write_grid, Sec. 3.3; the box
assignment and air mass are a reading stated in include/mpt.h):

* the air mass of all boxes of a global grid sums to the closed form
  4 pi R^2 (p_bottom - p_top) 100 / g;
* one parcel at the centre of every box gives count 1 and its own mass;
* brute force on tiny inputs: box membership by interval tests on each
  coordinate (not by the floor division the oracle uses);
* conservation: counts and masses of the parcels inside the grid volume;
* edges: a layer owns its upper-pressure edge, the grid's north edge falls
  in the last row, non-finite parcels and parcels outside are not counted.
"""
import math

import numpy as np

import oracle

R, G = 6371e3, 9.80665


def centres(nx, ny, lon0, lat0, dlat, pe):
    k, j, i = np.meshgrid(np.arange(len(pe) - 1), np.arange(ny), np.arange(nx), indexing="ij")
    lon = (lon0 + (i + 0.5) * 360.0 / nx) % 360.0
    lat = lat0 + (j + 0.5) * dlat
    p = 0.5 * (pe[k] + pe[k + 1])
    return lon.ravel(), lat.ravel(), p.ravel()


def test_air_mass_of_a_global_grid_is_the_closed_form():
    pe = np.array([1000.0, 850.0, 500.0, 200.0, 50.0, 10.0])
    for nx, ny in ((36, 18), (7, 5), (360, 180)):
        lon, lat, p = centres(nx, ny, 3.0, -90.0, 180.0 / ny, pe)
        _, _, mmr = oracle.grid_output(lon, lat, p, None, nx, ny, 3.0, -90.0, 180.0 / ny, pe)
        total = (1.0 / mmr).sum()
        assert abs(total / (4 * math.pi * R * R * (pe[0] - pe[-1]) * 100.0 / G) - 1.0) < 1e-12


def test_one_parcel_per_box_centre():
    pe = np.array([900.0, 700.0, 300.0])
    nx, ny, lon0, lat0, dlat = 12, 6, -7.5, -60.0, 20.0
    lon, lat, p = centres(nx, ny, lon0, lat0, dlat, pe)
    mass = np.arange(1, len(lon) + 1, dtype=np.float64)
    c, m, _ = oracle.grid_output(lon, lat, p, mass, nx, ny, lon0, lat0, dlat, pe)
    np.testing.assert_array_equal(c.ravel(), 1)
    np.testing.assert_array_equal(m.ravel(), mass)


def test_brute_force_membership_on_tiny_inputs():
    rng = np.random.default_rng(3)
    pe = np.array([1000.0, 800.0, 450.0, 120.0])
    nx, ny, lon0, lat0, dlat = 5, 4, 17.0, -50.0, 30.0
    n = 600
    lon = rng.uniform(0, 360, n)
    lat = rng.uniform(-90, 90, n)
    p = rng.uniform(50, 1050, n)
    mass = rng.uniform(0.5, 2.0, n)
    c, m, _ = oracle.grid_output(lon, lat, p, mass, nx, ny, lon0, lat0, dlat, pe)
    dlon = 360.0 / nx
    want_c = np.zeros((len(pe) - 1, ny, nx), np.int64)
    want_m = np.zeros((len(pe) - 1, ny, nx))
    for q in range(n):
        for k in range(len(pe) - 1):
            if not (pe[k] >= p[q] > pe[k + 1]):
                continue
            for j in range(ny):
                if not (lat0 + j * dlat <= lat[q] < lat0 + (j + 1) * dlat):
                    continue
                for i in range(nx):
                    if math.fmod(lon[q] - (lon0 + i * dlon) + 720.0, 360.0) < dlon:
                        want_c[k, j, i] += 1
                        want_m[k, j, i] += mass[q]
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_allclose(m, want_m, rtol=1e-14, atol=0)
    assert c.sum() > 100


def test_conservation_inside_the_grid_volume():
    rng = np.random.default_rng(4)
    pe = np.linspace(1000.0, 100.0, 10)
    nx, ny, lon0, lat0, dlat = 72, 30, 0.0, -60.0, 4.0
    n = 200_000
    lon = rng.uniform(0, 360, n)
    lat = rng.uniform(-90, 90, n)
    p = rng.uniform(0, 1100, n)
    mass = rng.uniform(0, 1, n)
    c, m, _ = oracle.grid_output(lon, lat, p, mass, nx, ny, lon0, lat0, dlat, pe)
    inside = (lat >= -60.0) & (lat < 60.0) & (p <= 1000.0) & (p > 100.0)
    assert c.sum() == inside.sum()
    assert abs(m.sum() - mass[inside].sum()) < 1e-9 * mass.sum()


def test_edges():
    pe = np.array([1000.0, 500.0, 100.0])
    nx, ny, lon0, lat0, dlat = 4, 3, 0.0, -90.0, 60.0
    lon = np.array([0.0, 359.999, 90.0, 45.0, 45.0, 45.0, 45.0, np.nan, 45.0, 45.0])
    lat = np.array([0.0, 0.0, 90.0, -90.0, 10.0, 10.0, 10.0, 0.0, 10.0, np.inf])
    p = np.array([500.0, 500.0, 300.0, 300.0, 1000.0, 100.0, 1000.0001, 300.0, 99.999, 300.0])
    c, _, _ = oracle.grid_output(lon, lat, p, None, nx, ny, lon0, lat0, dlat, pe)
    got = {tuple(b) for b in np.argwhere(c)}
    # p = 500 is the upper-pressure edge of layer 0 (1000 >= p > 500 fails) -> layer 1
    assert (1, 1, 0) in got and (1, 1, 3) in got
    assert (1, 2, 1) in got                          # the north edge -> last row
    assert (1, 0, 0) in got                          # lat = lat0 -> row 0
    assert (0, 1, 0) in got                          # p = pedges[0] -> layer 0
    assert c.sum() == 5                              # p = pedges[2], p > 1000, NaN, inf not counted
    assert c[1, 1, 0] == 1 and c[0, 1, 0] == 1
