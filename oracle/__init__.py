"""CPU oracle of the particle time step -- TEST INFRASTRUCTURE ONLY.

Plain FP64 C (``mpt_oracle.c``, OpenMP over parcels) behind ctypes, plus the
numpy reference of the reduced-precision field encoding (``encode.py``) and
of the surrogate's forward pass (``mlp.py``).  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import this package; the GPU
library neither imports it nor shares any code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpt_oracle.c")
_LIB = os.path.join(_HERE, "libmpt_oracle.so")

ADVECT, TURB, MESO, CONV, SEDI = 1, 2, 4, 8, 16
SEED = 221112616


def build() -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no FMA contraction,
    no fast-math)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
           "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class OrcMet(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("lon0", ctypes.c_double), ("dlon", ctypes.c_double),
                ("lat0", ctypes.c_double), ("dlat", ctypes.c_double),
                ("plev", ctypes.POINTER(ctypes.c_double)), ("t_met0", ctypes.c_double),
                ("dt_met", ctypes.c_double), ("u", ctypes.POINTER(ctypes.c_float)),
                ("v", ctypes.POINTER(ctypes.c_float)), ("w", ctypes.POINTER(ctypes.c_float)),
                ("analytic", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("an_u0", ctypes.c_double), ("an_alpha", ctypes.c_double),
                ("temp", ctypes.POINTER(ctypes.c_float)), ("cape", ctypes.POINTER(ctypes.c_float)),
                ("pel", ctypes.POINTER(ctypes.c_float)), ("ps", ctypes.POINTER(ctypes.c_float))]


class OrcCtl(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("t_start", ctypes.c_double),
                ("turb_dx", ctypes.c_double), ("turb_dz", ctypes.c_double),
                ("meso_fh", ctypes.c_double), ("meso_fv", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("conv_cape", ctypes.c_double), ("sedi_r", ctypes.c_double),
                ("sedi_rho", ctypes.c_double)]


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_run.argtypes = [P, P, ctypes.c_int64, P, P, P, P, P, P, P, P,
                              ctypes.c_uint32, ctypes.c_int32, ctypes.c_int32]
        L.orc_interp_many.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_double, P]
        L.orc_cell_sigma_many.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_double, P]
        L.orc_locate_many.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_double, P, P]
        L.orc_position_many.argtypes = [P, ctypes.c_int64, P, P, P]
        L.orc_ml_to_pl.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, P, P, P]
        L.orc_grid_output.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      P, P, P, P]
        L.orc_philox_many.argtypes = [ctypes.c_int64, P, P, P]
        L.orc_normals_many.argtypes = [ctypes.c_uint64, ctypes.c_int64, P, ctypes.c_uint32,
                                       ctypes.c_uint32, P]
        L.orc_tile_keys.argtypes = [P, ctypes.c_int64, P, P, P, P]
        L.orc_stencil81_many.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_double, P]
        L.orc_displacement_many.argtypes = [P, P, ctypes.c_int64, P, P, P, ctypes.c_uint32,
                                            ctypes.c_int32, P, ctypes.c_int32]
        L.orc_settling_velocity.argtypes = [ctypes.c_double] * 4
        L.orc_settling_velocity.restype = ctypes.c_double
        L.orc_uniform.argtypes = [ctypes.c_uint32]
        L.orc_uniform.restype = ctypes.c_double
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


class Met:
    """Oracle view of met fields.  Holds references to C-contiguous copies
    of the stored values (float32) and the level table."""

    def __init__(self, met, analytic: bool = False, an_u0: float = 0.0, an_alpha: float = 0.0):
        self.plev = np.ascontiguousarray(met.plev, np.float64)
        self.u = np.ascontiguousarray(met.u, np.float32)
        self.v = np.ascontiguousarray(met.v, np.float32)
        self.w = np.ascontiguousarray(met.w, np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        # convection / sedimentation fields (absent: null pointers)
        self.temp = self.cape = self.pel = self.ps = None
        if getattr(met, "temp", None) is not None:
            self.temp = np.ascontiguousarray(met.temp, np.float32)
            self.cape = np.ascontiguousarray(met.cape, np.float32)
            self.pel = np.ascontiguousarray(met.pel, np.float32)
            self.ps = np.ascontiguousarray(met.ps, np.float32)

        def opt(a):
            return a.ctypes.data_as(fp) if a is not None else None

        self.s = OrcMet(nx=met.nx, ny=met.ny, nz=met.nz, nt=met.nt, lon0=met.lon0,
                        dlon=met.dlon, lat0=met.lat0, dlat=met.dlat,
                        plev=self.plev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        t_met0=met.t_met0, dt_met=met.dt_met,
                        u=self.u.ctypes.data_as(fp), v=self.v.ctypes.data_as(fp),
                        w=self.w.ctypes.data_as(fp), analytic=int(analytic), pad_=0,
                        an_u0=an_u0, an_alpha=an_alpha, temp=opt(self.temp),
                        cape=opt(self.cape), pel=opt(self.pel), ps=opt(self.ps))

    @property
    def ref(self):
        return ctypes.byref(self.s)


def ctl(dt: float = 180.0, t_start: float = 0.0, turb_dx: float = 50.0, turb_dz: float = 0.1,
        meso_fh: float = 0.16, meso_fv: float = 0.16, seed: int = SEED,
        flags: int = ADVECT | TURB | MESO, conv_cape: float = 500.0, sedi_r: float = 5e-6,
        sedi_rho: float = 1000.0) -> OrcCtl:
    return OrcCtl(dt=dt, t_start=t_start, turb_dx=turb_dx, turb_dz=turb_dz, meso_fh=meso_fh,
                  meso_fv=meso_fv, seed=seed, flags=flags, pad_=0, conv_cape=conv_cape,
                  sedi_r=sedi_r, sedi_rho=sedi_rho)


def settling_velocity(r: float, rho_p: float, p: float, T: float) -> float:
    """Settling velocity [m/s] of a sphere (radius r [m], density rho_p
    [kg/m^3]) in air at p [hPa], T [K] (module_sedi reading)."""
    return lib().orc_settling_velocity(r, rho_p, p, T)


def run(m: Met, c: OrcCtl, part, step0: int, nsteps: int, release: Optional[np.ndarray] = None,
        nthreads: Optional[int] = None):
    """Advance ``part`` (an ``inputs.Particles``; arrays float64 / uint32)
    in place by ``nsteps`` steps starting at step index ``step0``."""
    for name in ("lon", "lat", "p", "up", "vp", "wp"):
        a = getattr(part, name)
        assert a.dtype == np.float64 and a.flags.c_contiguous, name
    assert part.id.dtype == np.uint32 and part.id.flags.c_contiguous
    rel = None
    if release is not None:
        rel = np.ascontiguousarray(release, np.int32)
        assert len(rel) == part.n
    nt = nthreads if nthreads else lib().orc_max_threads()
    lib().orc_run(m.ref, ctypes.byref(c), part.n, _ptr(part.lon), _ptr(part.lat), _ptr(part.p),
                  _ptr(part.id), _ptr(part.up), _ptr(part.vp), _ptr(part.wp),
                  _ptr(rel) if rel is not None else None, step0, nsteps, nt)
    return part


def interp(m: Met, lon, lat, p, t: float) -> np.ndarray:
    lon, lat, p = (np.ascontiguousarray(a, np.float64) for a in (lon, lat, p))
    out = np.empty((len(lon), 3), np.float64)
    lib().orc_interp_many(m.ref, len(lon), _ptr(lon), _ptr(lat), _ptr(p), t, _ptr(out))
    return out


def cell_sigma(m: Met, lon, lat, p, t: float) -> np.ndarray:
    lon, lat, p = (np.ascontiguousarray(a, np.float64) for a in (lon, lat, p))
    out = np.empty((len(lon), 3), np.float64)
    lib().orc_cell_sigma_many(m.ref, len(lon), _ptr(lon), _ptr(lat), _ptr(p), t, _ptr(out))
    return out


def locate(m: Met, lon, lat, p, t: float):
    lon, lat, p = (np.ascontiguousarray(a, np.float64) for a in (lon, lat, p))
    idx = np.empty((len(lon), 4), np.int32)
    frac = np.empty((len(lon), 4), np.float64)
    lib().orc_locate_many(m.ref, len(lon), _ptr(lon), _ptr(lat), _ptr(p), t, _ptr(idx), _ptr(frac))
    return idx, frac


def position(m: Met, lon, lat, p):
    lon, lat, p = (np.array(a, np.float64) for a in (lon, lat, p))
    lib().orc_position_many(m.ref, len(lon), _ptr(lon), _ptr(lat), _ptr(p))
    return lon, lat, p


def philox(ctr: np.ndarray, key) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.empty_like(ctr)
    lib().orc_philox_many(len(ctr), _ptr(ctr), _ptr(k), _ptr(out))
    return out


def normals(seed: int, ids, step: int, purpose: int) -> np.ndarray:
    ids = np.ascontiguousarray(ids, np.uint32)
    out = np.empty((len(ids), 3), np.float64)
    lib().orc_normals_many(seed, len(ids), _ptr(ids), step, purpose, _ptr(out))
    return out


def uniform(x: int) -> float:
    return lib().orc_uniform(x)


def tile_keys(m: Met, lon, lat, p) -> np.ndarray:
    lon, lat, p = (np.ascontiguousarray(a, np.float64) for a in (lon, lat, p))
    out = np.empty(len(lon), np.uint32)
    lib().orc_tile_keys(m.ref, len(lon), _ptr(lon), _ptr(lat), _ptr(p), _ptr(out))
    return out


def ml_to_pl(plev, a, b, ps, f) -> np.ndarray:
    """Model-level field f [nml, ny, nx] with surface pressure ps [ny, nx] to
    the pressure levels plev: [nz, ny, nx] float32."""
    plev, a, b = (np.ascontiguousarray(x, np.float64) for x in (plev, a, b))
    ps = np.ascontiguousarray(ps, np.float32)
    f = np.ascontiguousarray(f, np.float32)
    ny, nx = ps.shape
    out = np.empty((len(plev), ny, nx), np.float32)
    lib().orc_ml_to_pl(nx, ny, len(plev), _ptr(plev), len(a), _ptr(a), _ptr(b), _ptr(ps), _ptr(f), _ptr(out))
    return out


def grid_output(lon, lat, p, mass, nx: int, ny: int, lon0: float, lat0: float, dlat: float,
                pedges) -> tuple:
    """Gridded output: (counts, mass sums, mass mixing ratios), each [nz, ny, nx]."""
    lon, lat, p = (np.ascontiguousarray(a, np.float64) for a in (lon, lat, p))
    pe = np.ascontiguousarray(pedges, np.float64)
    nz = len(pe) - 1
    m = None if mass is None else np.ascontiguousarray(mass, np.float64)
    counts = np.empty((nz, ny, nx), np.uint32)
    msum = np.empty((nz, ny, nx), np.float64)
    mmr = np.empty((nz, ny, nx), np.float64)
    lib().orc_grid_output(len(lon), _ptr(lon), _ptr(lat), _ptr(p), _ptr(m) if m is not None else None,
                          nx, ny, nz, lon0, 360.0 / nx, lat0, dlat, _ptr(pe), _ptr(counts), _ptr(msum),
                          _ptr(mmr))
    return counts, msum, mmr


def stencil81(m: Met, lon, lat, p, t: float) -> np.ndarray:
    """Surrogate inputs: (n, 81) = u, v, w on the 3x3x3 cell stencil."""
    lon, lat, p = (np.ascontiguousarray(a, np.float64) for a in (lon, lat, p))
    out = np.empty((len(lon), 81), np.float64)
    lib().orc_stencil81_many(m.ref, len(lon), _ptr(lon), _ptr(lat), _ptr(p), t, _ptr(out))
    return out


def displacement(m: Met, c: OrcCtl, lon, lat, p, step0: int, k: int,
                 nthreads: Optional[int] = None) -> np.ndarray:
    """(n, 3) k-step plain-advection displacement: east km, north km, dp hPa."""
    lon, lat, p = (np.ascontiguousarray(a, np.float64) for a in (lon, lat, p))
    out = np.empty((len(lon), 3), np.float64)
    nt = nthreads if nthreads else lib().orc_max_threads()
    lib().orc_displacement_many(m.ref, ctypes.byref(c), len(lon), _ptr(lon), _ptr(lat), _ptr(p),
                                step0, k, _ptr(out), nt)
    return out


def max_threads() -> int:
    return lib().orc_max_threads()


# ---------------------------------------------------------------------------
# parity metric
# ---------------------------------------------------------------------------

def chord_deg(lon1, lat1, lon2, lat2) -> np.ndarray:
    """Great-circle chord between two sets of positions, expressed as the
    central angle in degrees: 2 asin(|x1 - x2| / 2).  Robust at the poles
    and across the longitude seam."""
    d = np.pi / 180.0

    def xyz(lon, lat):
        lon = np.asarray(lon, np.float64) * d
        lat = np.asarray(lat, np.float64) * d
        return np.stack([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)])

    c = np.linalg.norm(xyz(lon1, lat1) - xyz(lon2, lat2), axis=0)
    return 2.0 * np.arcsin(np.minimum(c / 2.0, 1.0)) / d
