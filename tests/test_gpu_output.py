"""GPU parity of the gridded output (write_grid, Sec. 3.3; reading in
include/mpt.h) against the oracle.  Counts must agree bit for bit: both
sides assign boxes with the same FP64 divisions and comparisons.  Mass sums
are accumulated in no fixed order on the GPU, so each box is held to the
error bound of an FP64 sum of n terms in any order, 2 gamma_n sum|m|
(gamma_n = n u / (1 - n u), u = 2^-53); mixing ratios to that bound plus the
rounding of the air mass.  Cases: parcels exactly on every box edge and one
ulp either side; random parcels with masses after sorted stepping (runs of
equal boxes within a wave) and the same parcels shuffled; 1e7 parcels; an
empty set; the state error before a grid is set."""
import numpy as np
import pytest

import inputs
import oracle
from gpu_common import require_gpu, say

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
PE = np.linspace(1000.0, 100.0, 11)
NX, NY, LON0, LAT0, DLAT = 360, 180, -0.5, -90.0, 1.0


@pytest.fixture(scope="module")
def mpt():
    return require_gpu()


@pytest.fixture(scope="module")
def met():
    return inputs.make_met_c1(seed=11, nt=3)


@pytest.fixture(scope="module")
def ctx(mpt, met):
    c = mpt.Context(met, mpt.make_params(math=1, sort_interval=10, fuse=10), n_max=10_000_000)
    c.upload_met(met)
    c.set_outgrid(NX, NY, LON0, LAT0, DLAT, PE)
    return c


def gpu_output(mpt, ctx, lon, lat, p, mass):
    import torch
    part = inputs.Particles(lon=lon, lat=lat, p=p, id=np.arange(len(lon), dtype=np.uint32),
                            up=np.zeros(len(lon)), vp=np.zeros(len(lon)), wp=np.zeros(len(lon)))
    P = mpt.DeviceParticles.from_host(part, math=1, pingpong=False)
    m = torch.from_numpy(mass).cuda() if mass is not None else None
    c, s, r = ctx.grid_output(P, m)
    torch.cuda.synchronize()
    return c.cpu().numpy().view(np.uint32), s.cpu().numpy(), r.cpu().numpy()


def compare(g, o, mass, label):
    gc, gs, gr = g
    oc, os_, or_ = o
    np.testing.assert_array_equal(gc, oc)
    n = oc.astype(np.float64)
    gam = n * U / (1.0 - n * U)
    absum = os_ if mass is None or np.all(mass >= 0) else None
    assert absum is not None
    bound = 2.0 * gam * absum
    assert np.all(np.abs(gs - os_) <= bound)
    nz = os_ > 0
    rel = np.abs(gr[nz] - or_[nz]) / np.abs(or_[nz])
    assert np.all(rel <= 2.0 * gam[nz] + 1e-13)
    assert np.all(gr[~nz] == 0.0)
    say(f"[{label}] {int(oc.sum())} parcels in {int((oc > 0).sum())} boxes; max |dsum| / bound "
        f"{(np.abs(gs - os_)[nz] / np.maximum(bound[nz], 1e-300)).max():.3f}, max rel dmmr {rel.max():.2e}")


def test_parcels_on_every_box_edge(mpt, ctx):
    i = np.arange(NX)
    j = np.arange(NY + 1)
    lon_e = (LON0 + i * 360.0 / NX) % 360.0
    lat_e = LAT0 + j * DLAT
    rng = np.random.default_rng(5)
    lon, lat, p = [], [], []
    for d in (-1, 0, 1):
        lo = np.nextafter(lon_e, lon_e + d) if d else lon_e
        la = np.nextafter(lat_e, lat_e + d) if d else lat_e
        pp = np.nextafter(PE, PE + d) if d else PE
        lon.append(rng.permutation(np.resize(lo, 20000)))
        lat.append(rng.permutation(np.resize(la, 20000)))
        p.append(rng.permutation(np.resize(pp, 20000)))
    lon, lat, p = (np.concatenate(a) for a in (lon, lat, p))
    lon = np.where(lon >= 360.0, lon - 360.0, np.where(lon < 0.0, lon + 360.0, lon))
    lat = np.clip(lat, -90.0, 90.0)
    g = gpu_output(mpt, ctx, lon, lat, p, None)
    o = oracle.grid_output(lon, lat, p, None, NX, NY, LON0, LAT0, DLAT, PE)
    compare(g, o, None, "edges")


def test_sorted_and_shuffled_parcels_with_masses(mpt, ctx, met):
    import torch
    part = inputs.make_particles(100_003, 71)
    P = mpt.DeviceParticles.from_host(part, math=1)
    ctx.step(P, 0, 20)                               # sorted by tile every 10 steps
    torch.cuda.synchronize()
    h = P.to_host()
    mass = np.random.default_rng(7).uniform(0.1, 3.0, part.n)
    for label, order in (("sorted", np.arange(part.n)), ("shuffled", np.random.default_rng(8).permutation(part.n))):
        lon, lat, p, m = h.lon[order], h.lat[order], h.p[order], mass[order]
        g = gpu_output(mpt, ctx, lon, lat, p, m)
        o = oracle.grid_output(lon, lat, p, m, NX, NY, LON0, LAT0, DLAT, PE)
        compare(g, o, m, label)


def test_ten_million_parcels(mpt, ctx):
    part = inputs.make_particles(10_000_000, 72)
    g = gpu_output(mpt, ctx, part.lon, part.lat, part.p, None)
    o = oracle.grid_output(part.lon, part.lat, part.p, None, NX, NY, LON0, LAT0, DLAT, PE)
    compare(g, o, None, "1e7")
    np.testing.assert_array_equal(g[1], g[0].astype(np.float64))     # unit masses


def test_empty_set_and_state_error(mpt, met):
    import torch
    c = mpt.Context(met, mpt.make_params(math=1), n_max=10)
    c.upload_met(met)
    empty = mpt.DeviceParticles.from_host(inputs.make_particles(0, 1), math=1, pingpong=False)
    with pytest.raises(RuntimeError, match="STATE|state"):
        c._outgrid = (2, 2, 1)
        c.grid_output(empty)
    c.set_outgrid(8, 4, 0.0, -90.0, 45.0, np.array([1000.0, 500.0]))
    counts, msum, mmr = c.grid_output(empty)
    torch.cuda.synchronize()
    assert counts.abs().sum().item() == 0 and msum.abs().sum().item() == 0.0
    assert mmr.abs().sum().item() == 0.0


@pytest.mark.parametrize("bad", ["nx360", "lat", "edges", "nz"])
def test_bad_output_grid_is_rejected(mpt, met, bad):
    c = mpt.Context(met, mpt.make_params(math=1), n_max=10)
    args = dict(nx=8, ny=4, lon0=0.0, lat0=-90.0, dlat=45.0, pedges=np.array([1000.0, 500.0]))
    if bad == "nx360":
        import ctypes
        pe = np.array([1000.0, 500.0])
        g = mpt.OutGrid(nx=8, ny=4, nz=1, lon0=0.0, dlon=40.0, lat0=-90.0, dlat=45.0, pedges=pe.ctypes.data)
        assert mpt.lib().mpt_set_outgrid(c.h, ctypes.byref(g), None) == -1
        return
    if bad == "lat":
        args["dlat"] = 50.0                       # lat0 + ny * dlat > 90
    elif bad == "edges":
        args["pedges"] = np.array([500.0, 1000.0])
    else:
        args["pedges"] = np.linspace(1000.0, 1.0, 514)
    with pytest.raises(RuntimeError):
        c.set_outgrid(**args)
