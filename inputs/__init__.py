"""Seeded synthetic inputs for the particle time step.

This module only produces input data: meteorological wind fields on a
regular lon-lat grid with fixed pressure levels, and particle sets.  It holds
none of the method's arithmetic (no interpolation, no advection, no random
numbers that the method itself draws) and it is the one piece of code that
both the CPU oracle and the GPU path consume.

The paper reads its winds from reanalysis files (Sec. 3.1, ``read_met``) and
its particles from a file (``read_atm``); neither is available, so seeded
fields with the shapes of the workloads stand in for them:

* tiny case: 2 deg grid (180 x 91), 30 log-spaced levels 1000..1 hPa, two
  time levels 6 h apart, each wind a sum of 8 low-wavenumber sinusoids;
* realistic case: 0.3 deg grid (1200 x 601), 137 levels, a zonal jet band
  (60 m/s at 200 hPa) plus smoothed random perturbations of std 5 m/s.

Units handed to the step: u, v in m/s, w (omega) in hPa/s, pressure in hPa,
longitude / latitude in degrees, time in seconds.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Optional

import numpy as np

# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------

DT_MET = 21600.0          # 6 h between meteorological time levels [s]


def levels_log(nz: int = 30, p_bot: float = 1000.0, p_top: float = 1.0) -> np.ndarray:
    """Pressure levels equally spaced in ln p from p_bot down to p_top [hPa]."""
    k = np.arange(nz, dtype=np.float64)
    return p_bot * (p_top / p_bot) ** (k / (nz - 1))


def levels_hybrid137(nz: int = 137, p_bot: float = 1013.25, p_top: float = 0.01) -> np.ndarray:
    """137 fixed levels standing in for hybrid levels without a surface
    pressure field: ln p is quadratic in the level index, dense near the
    ground and sparse aloft (p_0 = 1013.25 hPa, p_136 = 0.01 hPa)."""
    k = np.arange(nz, dtype=np.float64)
    return p_bot * (p_top / p_bot) ** ((k / (nz - 1)) ** 2)


@dataclasses.dataclass
class Met:
    """Gridded winds at ``nt`` time levels.

    ``u``, ``v``, ``w`` are float32 arrays of shape (nt, nz, ny, nx) with
    longitude fastest.  Longitude i sits at lon0 + i*dlon (periodic,
    nx*dlon = 360), latitude j at lat0 + j*dlat (lat0 = -90, last row at
    +90), level k at plev[k] (strictly decreasing, hPa), time level l at
    t_met0 + l*dt_met.
    """
    nx: int
    ny: int
    nz: int
    nt: int
    lon0: float
    dlon: float
    lat0: float
    dlat: float
    plev: np.ndarray
    t_met0: float
    dt_met: float
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    # convection / sedimentation fields (optional): temperature [K] shaped
    # like u; CAPE [J/kg], equilibrium-level and surface pressure [hPa]
    # shaped (nt, ny, nx)
    temp: Optional[np.ndarray] = None
    cape: Optional[np.ndarray] = None
    pel: Optional[np.ndarray] = None
    ps: Optional[np.ndarray] = None

    @property
    def t_end(self) -> float:
        return self.t_met0 + (self.nt - 1) * self.dt_met

    def lon_axis(self) -> np.ndarray:
        return self.lon0 + self.dlon * np.arange(self.nx)

    def lat_axis(self) -> np.ndarray:
        return self.lat0 + self.dlat * np.arange(self.ny)


def empty_met(nx: int, ny: int, plev: np.ndarray, nt: int, dt_met: float = DT_MET,
              t_met0: float = 0.0) -> Met:
    nz = len(plev)
    shape = (nt, nz, ny, nx)
    return Met(nx=nx, ny=ny, nz=nz, nt=nt, lon0=0.0, dlon=360.0 / nx,
               lat0=-90.0, dlat=180.0 / (ny - 1), plev=np.asarray(plev, np.float64),
               t_met0=t_met0, dt_met=dt_met,
               u=np.zeros(shape, np.float32), v=np.zeros(shape, np.float32),
               w=np.zeros(shape, np.float32))


# --------------------------------------------------------------------------
# tiny case: sums of 8 low-wavenumber sinusoids
# --------------------------------------------------------------------------

def make_met_c1(seed: int = 11, nt: int = 2, nx: int = 180, ny: int = 91, nz: int = 30) -> Met:
    """Each wind X = A_X * g_X * sum_m a_m cos(s_m lon + l_m lat
    + n_m ln(p/1000) + om_m t + th_m) with lon, lat in radians, a_m >= 0
    summing to 1 (so |X| <= A_X), s_m in {0..3} (periodic in lon),
    l_m in {1,2,3}, n_m ~ U(0.5, 2), th_m ~ U(0, 2pi),
    om_m ~ U(-1, 1) * 2pi / 2 days; A_u = A_v = 50 m/s,
    A_w = 0.5 Pa/s = 0.005 hPa/s.

    Taper g_X: cos(lat) for u and v, p / 1000 hPa for w.  Without it the
    horizontal wind would take many values at a pole and omega would not
    vanish toward the model top; parcels near either would follow chaotic
    paths that no two correct implementations can reproduce to 1e-9 deg."""
    met = empty_met(nx, ny, levels_log(nz), nt)
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = np.deg2rad(met.lon_axis())[None, None, :]
    phi = np.deg2rad(met.lat_axis())[None, :, None]
    lnp = np.log(met.plev / 1000.0)[:, None, None]
    taper_h = np.cos(phi)
    taper_w = (met.plev / 1000.0)[:, None, None]
    for name, amp in (("u", 50.0), ("v", 50.0), ("w", 0.5 / 100.0)):
        taper = taper_w if name == "w" else taper_h
        a = rng.uniform(0.0, 1.0, 8)
        a /= a.sum()
        s = rng.integers(0, 4, 8)
        lm = rng.integers(1, 4, 8)
        nm = rng.uniform(0.5, 2.0, 8)
        th = rng.uniform(0.0, 2 * math.pi, 8)
        om = rng.uniform(-1.0, 1.0, 8) * 2 * math.pi / (2 * 86400.0)
        arr = getattr(met, name)
        for l in range(nt):
            t = met.t_met0 + l * met.dt_met
            acc = np.zeros((nz, ny, nx), np.float64)
            for m in range(8):
                acc += a[m] * np.cos(s[m] * lam + lm[m] * phi + nm[m] * lnp + om[m] * t + th[m])
            arr[l] = (amp * taper * acc).astype(np.float32)
    return met


# --------------------------------------------------------------------------
# hybrid model levels (input for the model-level -> pressure-level step)
# --------------------------------------------------------------------------
def hybrid_levels(p_ref: np.ndarray, p_pure: float = 100.0, ps_ref: float = 1013.25):
    """Coefficients (a [hPa], b) of model levels at the pressures p_ref
    (decreasing) where the surface pressure is ps_ref: terrain following
    below p_pure, b = ((p - p_pure) / (ps_ref - p_pure))^1.5, pure pressure
    above (b = 0); a = p - b ps_ref.  Column pressures a + b ps decrease
    with the level index for every ps in [500, 1100] hPa."""
    p_ref = np.asarray(p_ref, np.float64)
    b = np.clip((p_ref - p_pure) / (ps_ref - p_pure), 0.0, None) ** 1.5
    return p_ref - b * ps_ref, b


def make_surface_pressure(seed: int, nx: int, ny: int, mean: float = 1013.25,
                          amp: float = 40.0) -> np.ndarray:
    """ps [ny, nx] float32 hPa: mean + amp * a smooth sum of 4 sinusoids in
    lon / lat with amplitudes summing to 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = np.deg2rad(np.arange(nx) * 360.0 / nx)[None, :]
    phi = np.deg2rad(-90.0 + np.arange(ny) * 180.0 / (ny - 1))[:, None]
    a = rng.uniform(0.0, 1.0, 4)
    a /= a.sum()
    acc = np.zeros((ny, nx))
    for m in range(4):
        acc += a[m] * np.cos(rng.integers(0, 4) * lam + rng.integers(1, 4) * phi + rng.uniform(0, 2 * math.pi))
    return (mean + amp * acc).astype(np.float32)


def make_model_level_fields(seed: int, p_ref: np.ndarray, nx: int, ny: int) -> tuple:
    """u, v, w [nml, ny, nx] float32 on model levels: smooth sinusoids of lon,
    lat and ln(p_ref / 1000) as in the tiny workload (winds 50 m/s, omega
    0.005 hPa/s), with its taper (cos lat on u and v, p_ref / 1000 on omega)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = np.deg2rad(np.arange(nx) * 360.0 / nx)[None, None, :]
    phi = np.deg2rad(-90.0 + np.arange(ny) * 180.0 / (ny - 1))[None, :, None]
    lnp = np.log(np.asarray(p_ref, np.float64) / 1000.0)[:, None, None]
    taper_h = np.cos(phi)
    taper_w = (np.asarray(p_ref, np.float64) / 1000.0)[:, None, None]
    out = []
    for amp, taper in ((50.0, taper_h), (50.0, taper_h), (0.005, taper_w)):
        a = rng.uniform(0.0, 1.0, 6)
        a /= a.sum()
        acc = np.zeros((len(p_ref), ny, nx))
        for m in range(6):
            acc += a[m] * np.cos(rng.integers(0, 4) * lam + rng.integers(1, 4) * phi
                                 + rng.uniform(0.5, 2.0) * lnp + rng.uniform(0, 2 * math.pi))
        out.append((amp * taper * acc).astype(np.float32))
    return tuple(out)


# --------------------------------------------------------------------------
# realistic case: jet band + smoothed perturbations
# --------------------------------------------------------------------------

def _nthreads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _smooth_slab(x: np.ndarray) -> None:
    """Two passes of the binomial filter [1,2,1]/4 in longitude (periodic)
    and in latitude (edge rows replicated), in place, on a (ny, nx) slab."""
    tmp = np.empty_like(x)
    for _ in range(2):
        # longitude, periodic
        tmp[:, 1:-1] = x[:, :-2] + x[:, 2:]
        tmp[:, 0] = x[:, -1] + x[:, 1]
        tmp[:, -1] = x[:, -2] + x[:, 0]
        tmp *= 0.25
        x *= 0.5
        x += tmp
        # latitude, edges replicated
        tmp[1:-1] = x[:-2] + x[2:]
        tmp[0] = x[0] + x[1]
        tmp[-1] = x[-2] + x[-1]
        tmp *= 0.25
        x *= 0.5
        x += tmp


def _perturbation(out: np.ndarray, seed: int, l: int, var: int, std: float,
                  taper_lat: np.ndarray, taper_lev: np.ndarray) -> None:
    """Fill out[(nz, ny, nx)] with white noise smoothed per level, multiply
    by taper_lev[k] * taper_lat[j], then scale the whole array (about its
    mean) to the requested std."""
    nz = out.shape[0]

    def gen(k: int):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, l, var, k])))
        rng.standard_normal(out=out[k], dtype=np.float32)
        _smooth_slab(out[k])
        out[k] *= (taper_lat * taper_lev[k]).astype(np.float32)[:, None]
        x = out[k].astype(np.float64)
        return float(x.sum()), float((x * x).sum())

    with ThreadPoolExecutor(_nthreads()) as ex:
        sums = list(ex.map(gen, range(nz)))
    n = out.size
    mean = sum(s for s, _ in sums) / n
    var_ = sum(q for _, q in sums) / n - mean * mean
    scale = std / math.sqrt(var_)

    def fix(k: int):
        out[k] -= np.float32(mean)
        out[k] *= np.float32(scale)

    with ThreadPoolExecutor(_nthreads()) as ex:
        list(ex.map(fix, range(nz)))


def jet_profile(lat_deg: np.ndarray, plev: np.ndarray, lat_c: float) -> np.ndarray:
    """Zonal jet u_jet(lat, p) = 60 exp(-((|lat|-lat_c)/10)^2)
    * exp(-ln(p/200)^2 / (2*0.6^2)) [m/s], shape (nz, ny)."""
    a = np.exp(-((np.abs(lat_deg) - lat_c) / 10.0) ** 2)
    b = np.exp(-np.log(plev / 200.0) ** 2 / (2 * 0.6 ** 2))
    return 60.0 * b[:, None] * a[None, :]


def make_met_c2(seed: int = 12, nt: int = 3, nx: int = 1200, ny: int = 601, nz: int = 137,
                pert_std: float = 5.0, w_std_pa: float = 0.05) -> Met:
    """Jet-like zonal band peaking at exactly 60 m/s at 200 hPa plus
    mesoscale perturbations: u_p, v_p, w_p are N(0,1) white noise per grid
    point, smoothed twice by [1,2,1]/4 in lon and lat, tapered (u_p, v_p by
    cos(lat) so the wind is single-valued at the poles, w_p by p / p_bot so
    omega vanishes toward the model top) and rescaled per (time level,
    variable) to std 5 m/s (u, v) and 0.05 Pa/s (w).  Perturbations are
    drawn independently per time level.  The jet centre latitude is
    U(30, 45) deg, drawn from ``seed``."""
    plev = levels_hybrid137(nz) if nz == 137 else levels_log(nz, 1013.25, 0.01)
    met = empty_met(nx, ny, plev, nt)
    rng = np.random.Generator(np.random.PCG64(seed))
    lat_c = float(rng.uniform(30.0, 45.0))
    jet = jet_profile(met.lat_axis(), met.plev, lat_c).astype(np.float32)
    coslat = np.cos(np.deg2rad(met.lat_axis()))
    ones_lat = np.ones(ny)
    ones_lev = np.ones(nz)
    plev_rel = met.plev / met.plev[0]
    for l in range(nt):
        _perturbation(met.u[l], seed, l, 0, pert_std, coslat, ones_lev)
        _perturbation(met.v[l], seed, l, 1, pert_std, coslat, ones_lev)
        _perturbation(met.w[l], seed, l, 2, w_std_pa / 100.0, ones_lat, plev_rel)

        def addjet(k: int, l=l):
            met.u[l, k] += jet[k][:, None]

        with ThreadPoolExecutor(_nthreads()) as ex:
            list(ex.map(addjet, range(nz)))
    met.jet_lat_c = lat_c  # type: ignore[attr-defined]
    return met


# --------------------------------------------------------------------------
# particles
# --------------------------------------------------------------------------

def add_phys_fields(met: Met, seed: int = 31, cape_max: float = 2500.0) -> Met:
    """Seeded convection / sedimentation fields on met's grid (in place):

    * temperature: the standard-atmosphere troposphere 288.15 (p/1013.25)^0.1903
      K floored at 216.65 K, minus 25 sin^2(lat) K below 200 hPa, plus a
      smooth +-3 K wave moving in time;
    * CAPE: cape_max * max(0, cos(2 lat)) * (1/2 + 1/2 sin(2 lon + om t + th)),
      so about half of the tropics and mid-latitudes exceed a few hundred J/kg
      at any time and the rest is below;
    * equilibrium level: 150 + 150 |lat| / 90 hPa plus a +-30 hPa wave;
    * surface pressure: 1013.25 - 60 max(0, sin(3 lon) cos(lat))^2 + a +-5 hPa
      wave (orography-like lows down to about 950 hPa)."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, 2.0 * np.pi, 4)
    om = rng.uniform(-1.0, 1.0, 4) * 2.0 * np.pi / (2.0 * 86400.0)
    lon = np.deg2rad(met.lon_axis())[None, :]
    lat = np.deg2rad(met.lat_axis())[:, None]
    p = met.plev[:, None, None]
    base = np.maximum(216.65, 288.15 * (p / 1013.25) ** 0.190263)
    base = base - 25.0 * np.sin(lat)[None] ** 2 * (p > 200.0)
    shape3, shape2 = (met.nt, met.nz, met.ny, met.nx), (met.nt, met.ny, met.nx)
    met.temp = np.empty(shape3, np.float32)
    met.cape = np.empty(shape2, np.float32)
    met.pel = np.empty(shape2, np.float32)
    met.ps = np.empty(shape2, np.float32)
    for l in range(met.nt):
        t = met.t_met0 + l * met.dt_met
        wave = 3.0 * np.sin(lon + 2.0 * lat + om[0] * t + th[0])
        met.temp[l] = (base + wave[None]).astype(np.float32)
        met.cape[l] = (cape_max * np.maximum(0.0, np.cos(2.0 * lat))
                       * (0.5 + 0.5 * np.sin(2.0 * lon + om[1] * t + th[1]))).astype(np.float32)
        met.pel[l] = (150.0 + 150.0 * np.abs(lat) / (0.5 * np.pi)
                      + 30.0 * np.sin(3.0 * lon - lat + om[2] * t + th[2])).astype(np.float32)
        met.ps[l] = (1013.25 - 60.0 * np.maximum(0.0, np.sin(3.0 * lon) * np.cos(lat)) ** 2
                     + 5.0 * np.sin(lon + lat + om[3] * t + th[3])).astype(np.float32)
    return met


@dataclasses.dataclass
class Particles:
    """Particle state on the host: positions (FP64), ids, mesoscale wind
    perturbation state (starts at zero)."""
    lon: np.ndarray
    lat: np.ndarray
    p: np.ndarray
    id: np.ndarray
    up: np.ndarray
    vp: np.ndarray
    wp: np.ndarray

    @property
    def n(self) -> int:
        return len(self.lon)

    def subset(self, idx: np.ndarray) -> "Particles":
        return Particles(*(getattr(self, f.name)[idx].copy() for f in dataclasses.fields(self)))

    def copy(self) -> "Particles":
        return Particles(*(getattr(self, f.name).copy() for f in dataclasses.fields(self)))


def make_particles(n: int, seed: int, p_lo: float = 100.0, p_hi: float = 900.0,
                   lat_lo: float = -90.0, lat_hi: float = 90.0) -> Particles:
    """n particles uniform in longitude [0, 360), latitude [lat_lo, lat_hi]
    (equal-angle) and pressure [p_lo, p_hi] hPa; ids 0..n-1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lon = rng.uniform(0.0, 360.0, n)
    lat = rng.uniform(lat_lo, lat_hi, n)
    p = rng.uniform(p_lo, p_hi, n)
    z = np.zeros(n, np.float64)
    return Particles(lon=lon, lat=lat, p=p, id=np.arange(n, dtype=np.uint32),
                     up=z, vp=z.copy(), wp=z.copy())


# --------------------------------------------------------------------------
# batched release scenarios
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Scenarios:
    """Independent release scenarios: sizes, release step, location, kind
    (0 = point release, 1 = column release with p ~ U[100, 900] hPa)."""
    sizes: np.ndarray
    release_step: np.ndarray
    lon: np.ndarray
    lat: np.ndarray
    p: np.ndarray
    kind: np.ndarray


def make_scenarios(seed: int = 24, nscen: int = 16, n_lo: float = 1e4, n_hi: float = 2e7,
                   release_max: int = 240) -> Scenarios:
    """Sizes exp(U[ln n_lo, ln n_hi]); lon ~ U[0, 360), lat ~ U[-80, 80],
    release step ~ U{0..release_max-1}; point or column with prob. 1/2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), nscen)).astype(np.int64)
    rel = rng.integers(0, release_max, nscen).astype(np.int32)
    lon = rng.uniform(0.0, 360.0, nscen)
    lat = rng.uniform(-80.0, 80.0, nscen)
    p = rng.uniform(100.0, 900.0, nscen)
    kind = rng.integers(0, 2, nscen).astype(np.int32)
    return Scenarios(sizes=sizes, release_step=rel, lon=lon, lat=lat, p=p, kind=kind)


def scale_scenarios(sc: Scenarios, factor: float, n_min: int = 1) -> Scenarios:
    """The same scenarios with every size multiplied by ``factor``."""
    sizes = np.maximum(n_min, (sc.sizes * factor).astype(np.int64))
    return dataclasses.replace(sc, sizes=sizes)


def make_scenario_particles(sc: Scenarios, seed: int = 24) -> tuple[Particles, np.ndarray]:
    """Particles of all scenarios, concatenated in scenario order, and the
    scenario index (uint16) of every particle."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1])))
    lons, lats, ps, scen = [], [], [], []
    for s, n in enumerate(sc.sizes):
        n = int(n)
        lons.append(np.full(n, sc.lon[s]))
        lats.append(np.full(n, sc.lat[s]))
        if sc.kind[s] == 0:
            ps.append(np.full(n, sc.p[s]))
        else:
            ps.append(rng.uniform(100.0, 900.0, n))
        scen.append(np.full(n, s, np.uint16))
    lon = np.concatenate(lons)
    n = len(lon)
    z = np.zeros(n, np.float64)
    part = Particles(lon=lon, lat=np.concatenate(lats), p=np.concatenate(ps),
                     id=np.arange(n, dtype=np.uint32), up=z, vp=z.copy(), wp=z.copy())
    return part, np.concatenate(scen)


# --------------------------------------------------------------------------
# structured test fields
# --------------------------------------------------------------------------

def fill_uniform(met: Met, u: float, v: float, w: float) -> Met:
    met.u[...] = u
    met.v[...] = v
    met.w[...] = w
    return met


def fill_checkerboard(met: Met, a: float) -> Met:
    """u = v = w = +a or -a on alternate grid points ((i+j+k) parity),
    identical at every time level.  Needs even nx for periodic parity."""
    k, j, i = np.meshgrid(np.arange(met.nz), np.arange(met.ny), np.arange(met.nx), indexing="ij")
    cb = np.where((i + j + k) % 2 == 0, a, -a).astype(np.float32)
    for arr in (met.u, met.v, met.w):
        arr[...] = cb[None]
    return met
