"""Python binding of libmpt (include/mpt.h): argument marshalling only.

Every step of the particle time step runs in the HIP kernels of libmpt.so;
PyTorch provides device memory and streams.  There is no fallback: loading
fails loudly when the library has not been built.

    ctx = Context(grid_of(met), Params(...), n_max)
    ctx.init_met(level, u, v, w)            # torch float32 cuda tensors
    P = DeviceParticles.from_host(part)     # torch tensors on the GPU
    ctx.step(P, step0, nsteps)
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpt.so")

MPT_OK = 0
STATUS = {0: "MPT_OK", -1: "MPT_ERR_ARG", -2: "MPT_ERR_STATE", -3: "MPT_ERR_TIME",
          -4: "MPT_ERR_WORKSPACE", -5: "MPT_ERR_HIP", -6: "MPT_ERR_UNSUPPORTED"}
MATH_F64, MATH_F32 = 0, 1
DT_F32, DT_BF16, DT_F16 = 0, 1, 2
ADVECT, TURB, MESO, CONV, SEDI = 1, 2, 4, 8, 16
SEED = 221112616


class MptError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {STATUS.get(code, code)}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("lon0", ctypes.c_double), ("dlon", ctypes.c_double),
                ("lat0", ctypes.c_double), ("dlat", ctypes.c_double),
                ("plev", ctypes.POINTER(ctypes.c_double)), ("t_met0", ctypes.c_double),
                ("dt_met", ctypes.c_double), ("dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class OutGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lon0", ctypes.c_double), ("dlon", ctypes.c_double), ("lat0", ctypes.c_double),
                ("dlat", ctypes.c_double), ("pedges", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("t_start", ctypes.c_double),
                ("turb_dx", ctypes.c_double), ("turb_dz", ctypes.c_double),
                ("meso_fh", ctypes.c_double), ("meso_fv", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("sort_interval", ctypes.c_int32),
                ("math", ctypes.c_int32), ("flags", ctypes.c_uint32), ("fuse", ctypes.c_int32),
                ("conv_cape", ctypes.c_double), ("sedi_radius", ctypes.c_double),
                ("sedi_density", ctypes.c_double), ("presort", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ParticlesC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [
        (name, ctypes.c_void_p) for name in
        ("lon", "lat", "p", "id", "up", "vp", "wp", "scen",
         "lon2", "lat2", "p2", "id2", "up2", "vp2", "wp2", "scen2")]


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """Load libmpt.so (build it with ``python -m paper_2211_12616_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: the HIP library has not been built")
        # torch carries its own HIP runtime under the same soname as the
        # system's.  Loaded first, it is the one the library binds to; loaded
        # after the library, it would be a second runtime in the process that
        # does not know the library's allocations, nor the library its
        # tensors (device copies into a torch workspace then fail).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P, S = ctypes.c_void_p, ctypes.c_int
        L.mpt_workspace_bytes.argtypes = [P, P, ctypes.c_int64]
        L.mpt_workspace_bytes.restype = ctypes.c_size_t
        L.mpt_create.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_size_t, ctypes.POINTER(P)]
        L.mpt_init_met.argtypes = [P, ctypes.c_int32, P, P, P, P]
        L.mpt_copy_met_level.argtypes = [P, ctypes.c_int32, P, P, P]
        L.mpt_met_level_bytes.argtypes = [P]
        L.mpt_met_level_bytes.restype = ctypes.c_size_t
        L.mpt_set_release.argtypes = [P, ctypes.c_int32, P, P]
        L.mpt_advect.argtypes = [P, P, ctypes.c_uint32, P]
        L.mpt_diffuse.argtypes = [P, P, ctypes.c_uint32, P]
        L.mpt_sort_particles.argtypes = [P, P, P]
        L.mpt_sort_particles_noalloc.argtypes = [P, P, P]
        L.mpt_sort_particles_deferred.argtypes = [P, P, P]
        L.mpt_step.argtypes = [P, P, ctypes.c_uint32, ctypes.c_int32, P]
        L.mpt_step_graph.argtypes = [P, P, ctypes.c_uint32, ctypes.c_int32, P]
        L.mpt_surrogate_datagen.argtypes = [P, ctypes.c_int64, P, P, P, P, P, P, P]
        L.mpt_surrogate_stats.argtypes = [P, ctypes.c_int64, P, P, P, P]
        L.mpt_surrogate_init.argtypes = [P, P, ctypes.c_uint64, P]
        L.mpt_surrogate_train_step.argtypes = [P, P, P, ctypes.c_int32, P, P, P, P, ctypes.c_int32,
                                               ctypes.c_float, P, P]
        L.mpt_surrogate_grad.argtypes = [P, P, P, ctypes.c_int32, P, P, P, P, P]
        L.mpt_surrogate_load.argtypes = [P, P, P, ctypes.c_float, P]
        L.mpt_surrogate_forward.argtypes = [P, ctypes.c_int64, P, P, P]
        L.mpt_step_surrogate.argtypes = [P, P, ctypes.c_uint32, ctypes.c_int32, P, P, P]
        L.mpt_push_met.argtypes = [P, P, P, P, P]
        L.mpt_set_met_phys.argtypes = [P, ctypes.c_int32, P, P, P, P, P]
        L.mpt_set_hybrid.argtypes = [P, ctypes.c_int32, P, P, P]
        L.mpt_ml_to_pl.argtypes = [P, P, P, P, P, P, P, P, P]
        L.mpt_set_outgrid.argtypes = [P, P, P]
        L.mpt_grid_output.argtypes = [P, P, P, P, P, P, P]
        L.mpt_destroy.argtypes = [P]
        L.mpt_status_string.argtypes = [S]
        L.mpt_status_string.restype = ctypes.c_char_p
        for fn in ("mpt_create", "mpt_init_met", "mpt_copy_met_level", "mpt_set_release",
                   "mpt_advect", "mpt_diffuse", "mpt_sort_particles", "mpt_sort_particles_noalloc",
                   "mpt_sort_particles_deferred", "mpt_step", "mpt_step_graph",
                   "mpt_destroy", "mpt_surrogate_datagen", "mpt_surrogate_stats",
                   "mpt_surrogate_init", "mpt_surrogate_train_step", "mpt_surrogate_grad",
                   "mpt_surrogate_load", "mpt_surrogate_forward", "mpt_step_surrogate",
                   "mpt_set_outgrid", "mpt_grid_output", "mpt_push_met", "mpt_set_hybrid",
                   "mpt_ml_to_pl", "mpt_set_met_phys"):
            getattr(L, fn).restype = S
        _lib = L
    return _lib


def exported_symbols():
    return ["mpt_workspace_bytes", "mpt_create", "mpt_init_met", "mpt_copy_met_level",
            "mpt_met_level_bytes", "mpt_set_release", "mpt_advect", "mpt_diffuse",
            "mpt_sort_particles", "mpt_sort_particles_noalloc", "mpt_sort_particles_deferred",
            "mpt_step", "mpt_step_graph", "mpt_destroy",
            "mpt_status_string", "mpt_surrogate_datagen", "mpt_surrogate_stats",
            "mpt_surrogate_init", "mpt_surrogate_train_step", "mpt_surrogate_grad",
            "mpt_surrogate_load", "mpt_surrogate_forward", "mpt_step_surrogate",
            "mpt_set_outgrid", "mpt_grid_output", "mpt_push_met", "mpt_set_hybrid", "mpt_ml_to_pl",
            "mpt_set_met_phys"]

SURR_K, SURR_NIN, SURR_NOUT, SURR_NPARAM, SURR_MAX_BATCH = 8, 81, 3, 47504, 8192
NOALLOC_SORT_MAX_N, NOALLOC_SORT_MAX_KEYS = 1 << 22, 1 << 20


def _check(fn: str, code: int):
    if code != MPT_OK:
        raise MptError(fn, code)


def make_grid(met, dtype: int = DT_F32) -> tuple[Grid, np.ndarray]:
    """mpt_grid for an ``inputs.Met``-like object; returns the struct and the
    level array it points to (keep both alive while the struct is used)."""
    plev = np.ascontiguousarray(met.plev, np.float64)
    g = Grid(nx=met.nx, ny=met.ny, nz=met.nz, nt=met.nt, lon0=met.lon0, dlon=met.dlon,
             lat0=met.lat0, dlat=met.dlat,
             plev=plev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
             t_met0=met.t_met0, dt_met=met.dt_met, dtype=dtype, reserved=0)
    return g, plev


def make_params(dt=180.0, t_start=0.0, turb_dx=50.0, turb_dz=0.1, meso_fh=0.16, meso_fv=0.16,
                seed=SEED, sort_interval=0, math=MATH_F64, flags=ADVECT | TURB | MESO,
                fuse=1, conv_cape=500.0, sedi_radius=5e-6, sedi_density=1000.0,
                presort=0) -> Params:
    return Params(dt=dt, t_start=t_start, turb_dx=turb_dx, turb_dz=turb_dz, meso_fh=meso_fh,
                  meso_fv=meso_fv, seed=seed, sort_interval=sort_interval, math=math,
                  flags=flags, fuse=fuse, conv_cape=conv_cape, sedi_radius=sedi_radius,
                  sedi_density=sedi_density, presort=presort, reserved=0)


def _stream_handle(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


@dataclasses.dataclass
class DeviceParticles:
    """Parcel state in device memory (torch tensors), plus the second set
    that sorting scatters into.  ``id`` holds uint32 bit patterns in an
    int32 tensor; ``scen`` holds uint16 bit patterns in an int16 tensor."""
    lon: "torch.Tensor"
    lat: "torch.Tensor"
    p: "torch.Tensor"
    id: "torch.Tensor"
    up: "torch.Tensor"
    vp: "torch.Tensor"
    wp: "torch.Tensor"
    scen: Optional["torch.Tensor"] = None
    second: Optional["DeviceParticles"] = None

    FIELDS = ("lon", "lat", "p", "id", "up", "vp", "wp", "scen")

    @property
    def n(self) -> int:
        return int(self.lon.numel())

    @staticmethod
    def from_host(part, math: int = MATH_F64, scen: Optional[np.ndarray] = None,
                  pingpong: bool = True, device: str = "cuda") -> "DeviceParticles":
        import torch
        mt = torch.float64 if math == MATH_F64 else torch.float32

        def dev(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)

        P = DeviceParticles(
            lon=dev(part.lon, torch.float64), lat=dev(part.lat, torch.float64),
            p=dev(part.p, torch.float64),
            id=torch.from_numpy(np.ascontiguousarray(part.id).view(np.int32)).to(device),
            up=dev(part.up, mt), vp=dev(part.vp, mt), wp=dev(part.wp, mt),
            scen=(torch.from_numpy(np.ascontiguousarray(scen, np.uint16).view(np.int16)).to(device)
                  if scen is not None else None))
        if pingpong:
            P.second = DeviceParticles(**{f: (torch.empty_like(getattr(P, f))
                                              if getattr(P, f) is not None else None)
                                          for f in DeviceParticles.FIELDS})
        return P

    def to_host(self):
        """Copy back to an ``inputs.Particles`` (meso state as float64)."""
        import inputs
        return inputs.Particles(
            lon=self.lon.cpu().numpy(), lat=self.lat.cpu().numpy(), p=self.p.cpu().numpy(),
            id=self.id.cpu().numpy().view(np.uint32),
            up=self.up.double().cpu().numpy(), vp=self.vp.double().cpu().numpy(),
            wp=self.wp.double().cpu().numpy())

    def cstruct(self) -> ParticlesC:
        def ptr(t):
            return t.data_ptr() if t is not None else None

        s = ParticlesC(n=self.n)
        for f in self.FIELDS:
            setattr(s, f, ptr(getattr(self, f)))
        if self.second is not None:
            for f in self.FIELDS:
                setattr(s, f + "2", ptr(getattr(self.second, f)))
        return s

    def adopt(self, s: ParticlesC):
        """After a sort the library swapped the sets inside the struct:
        mirror that on the tensors."""
        if self.second is None or (s.lon or 0) == self.lon.data_ptr():
            return
        assert (s.lon or 0) == self.second.lon.data_ptr()
        for f in self.FIELDS:
            a, b = getattr(self, f), getattr(self.second, f)
            setattr(self, f, b)
            setattr(self.second, f, a)


class Context:
    """One mpt_ctx with its workspace (a torch uint8 tensor on the GPU)."""

    def __init__(self, met_meta, params: Params, n_max: int = 0, dtype: int = DT_F32,
                 device: str = "cuda", resident: Optional[int] = None):
        """``resident``: number of met time levels held on the device (default:
        all of ``met_meta``); later levels arrive with push_met."""
        import torch
        self.grid, self._plev = make_grid(met_meta, dtype)
        if resident is not None:
            self.grid.nt = resident
        self.params = params
        L = lib()
        nbytes = L.mpt_workspace_bytes(ctypes.byref(self.grid), ctypes.byref(params), n_max)
        if nbytes == 0:
            raise MptError("mpt_workspace_bytes", -1)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check("mpt_create", L.mpt_create(ctypes.byref(self.grid), ctypes.byref(params), n_max,
                                          self.workspace.data_ptr(), nbytes, ctypes.byref(h)))
        self.h = h

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        if getattr(self, "h", None) and _lib is not None:
            _lib.mpt_destroy(self.h)
            self.h = None

    def init_met(self, level: int, u, v, w, stream=None):
        for t in (u, v, w):
            assert t.is_cuda and t.dtype.itemsize == 4 and t.is_contiguous()
        _check("mpt_init_met", lib().mpt_init_met(self.h, level, u.data_ptr(), v.data_ptr(),
                                                  w.data_ptr(), _stream_handle(stream)))

    def set_hybrid(self, a: np.ndarray, b: np.ndarray, stream=None):
        """Hybrid model levels p_k = a_k + b_k ps [hPa], k = 0 lowest."""
        a = np.ascontiguousarray(a, np.float64)
        b = np.ascontiguousarray(b, np.float64)
        _check("mpt_set_hybrid", lib().mpt_set_hybrid(self.h, len(a), a.ctypes.data, b.ctypes.data,
                                                      _stream_handle(stream)))

    def ml_to_pl(self, ps, u, v, w, stream=None):
        """Model-level u, v, w [nml, ny, nx] (torch float32 cuda) with surface
        pressure ps [ny, nx] -> the context's pressure levels, [nz, ny, nx]."""
        import torch
        g = self.grid
        out = [torch.empty((g.nz, g.ny, g.nx), dtype=torch.float32, device="cuda") for _ in range(3)]
        for t in (ps, u, v, w):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        _check("mpt_ml_to_pl", lib().mpt_ml_to_pl(self.h, ps.data_ptr(), u.data_ptr(), v.data_ptr(),
                                                  w.data_ptr(), *(o.data_ptr() for o in out),
                                                  _stream_handle(stream)))
        return out

    def push_met(self, u, v, w, stream=None):
        """mpt_push_met: the next time level replaces the oldest resident one."""
        for t in (u, v, w):
            assert t.is_cuda and t.dtype.itemsize == 4 and t.is_contiguous()
        _check("mpt_push_met", lib().mpt_push_met(self.h, u.data_ptr(), v.data_ptr(), w.data_ptr(),
                                                  _stream_handle(stream)))

    def set_met_phys(self, level: int, temp, cape, pel, ps, stream=None):
        """mpt_set_met_phys: temperature [nz, ny, nx] and CAPE, equilibrium-level
        and surface pressure [ny, nx] (torch float32 cuda) of a resident level."""
        for t in (temp, cape, pel, ps):
            assert t.is_cuda and t.dtype.itemsize == 4 and t.is_contiguous()
        _check("mpt_set_met_phys", lib().mpt_set_met_phys(self.h, level, temp.data_ptr(),
                                                          cape.data_ptr(), pel.data_ptr(),
                                                          ps.data_ptr(), _stream_handle(stream)))

    def upload_met(self, met, stream=None):
        """Store the first grid.nt time levels of an ``inputs.Met`` (host float32),
        with its convection / sedimentation fields when it has them."""
        import torch
        for l in range(self.grid.nt):
            u = torch.from_numpy(met.u[l]).cuda()
            v = torch.from_numpy(met.v[l]).cuda()
            w = torch.from_numpy(met.w[l]).cuda()
            self.init_met(l, u, v, w, stream)
            torch.cuda.current_stream().synchronize()
            del u, v, w
            if getattr(met, "temp", None) is not None:
                f = [torch.from_numpy(np.ascontiguousarray(a[l])).cuda()
                     for a in (met.temp, met.cape, met.pel, met.ps)]
                self.set_met_phys(l, *f, stream=stream)
                torch.cuda.current_stream().synchronize()
                del f

    def met_level_bytes(self) -> int:
        return lib().mpt_met_level_bytes(self.h)

    def copy_met_level(self, level: int, stream=None):
        import torch
        dst = torch.empty(self.met_level_bytes(), dtype=torch.uint8, device="cuda")
        sc = torch.empty(3 * self.grid.nz, dtype=torch.float32, device="cuda")
        _check("mpt_copy_met_level", lib().mpt_copy_met_level(self.h, level, dst.data_ptr(),
                                                              sc.data_ptr(), _stream_handle(stream)))
        return dst, sc

    def set_release(self, release_step: np.ndarray, stream=None):
        rel = np.ascontiguousarray(release_step, np.int32)
        _check("mpt_set_release", lib().mpt_set_release(self.h, len(rel), rel.ctypes.data,
                                                        _stream_handle(stream)))

    def set_outgrid(self, nx: int, ny: int, lon0: float, lat0: float, dlat: float,
                    pedges: np.ndarray, stream=None):
        """Output grid: nx boxes over 360 deg of longitude from lon0, ny rows of
        dlat from lat0, layers between the decreasing pressure edges [hPa]."""
        pe = np.ascontiguousarray(pedges, np.float64)
        g = OutGrid(nx=nx, ny=ny, nz=len(pe) - 1, lon0=lon0, dlon=360.0 / nx, lat0=lat0, dlat=dlat,
                    pedges=pe.ctypes.data)
        _check("mpt_set_outgrid", lib().mpt_set_outgrid(self.h, ctypes.byref(g), _stream_handle(stream)))
        self._outgrid = (nx, ny, len(pe) - 1)

    def grid_output(self, P: DeviceParticles, mass=None, mmr: bool = True, stream=None):
        """(counts [nz, ny, nx] uint32 as int32, mass sums, mass mixing ratios or None)."""
        import torch
        nx, ny, nz = self._outgrid
        counts = torch.empty((nz, ny, nx), dtype=torch.int32, device="cuda")
        msum = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
        m = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda") if mmr else None
        s = P.cstruct()
        _check("mpt_grid_output", lib().mpt_grid_output(
            self.h, ctypes.byref(s), mass.data_ptr() if mass is not None else None, counts.data_ptr(),
            msum.data_ptr(), m.data_ptr() if m is not None else None, _stream_handle(stream)))
        return counts, msum, m

    def advect(self, P: DeviceParticles, step: int, stream=None):
        s = P.cstruct()
        _check("mpt_advect", lib().mpt_advect(self.h, ctypes.byref(s), step, _stream_handle(stream)))

    def diffuse(self, P: DeviceParticles, step: int, stream=None):
        s = P.cstruct()
        _check("mpt_diffuse", lib().mpt_diffuse(self.h, ctypes.byref(s), step, _stream_handle(stream)))

    def sort(self, P: DeviceParticles, stream=None):
        s = P.cstruct()
        _check("mpt_sort_particles", lib().mpt_sort_particles(self.h, ctypes.byref(s),
                                                              _stream_handle(stream)))
        P.adopt(s)

    def sort_noalloc(self, P: DeviceParticles, stream=None):
        """mpt_sort_particles_noalloc: the same sort with the library's fixed
        per-device scratch (no workspace, n <= NOALLOC_SORT_MAX_N)."""
        s = P.cstruct()
        _check("mpt_sort_particles_noalloc", lib().mpt_sort_particles_noalloc(self.h, ctypes.byref(s),
                                                                              _stream_handle(stream)))
        P.adopt(s)

    def sort_deferred(self, P: DeviceParticles, stream=None):
        """mpt_sort_particles_deferred: the sort's order only; the parcels move
        in the next step() on them (the particle sets then swap)."""
        s = P.cstruct()
        _check("mpt_sort_particles_deferred", lib().mpt_sort_particles_deferred(self.h, ctypes.byref(s),
                                                                                _stream_handle(stream)))
        P.adopt(s)

    def step(self, P: DeviceParticles, step0: int, nsteps: int, stream=None):
        s = P.cstruct()
        _check("mpt_step", lib().mpt_step(self.h, ctypes.byref(s), step0, nsteps,
                                          _stream_handle(stream)))
        P.adopt(s)

    # ---- surrogate ----------------------------------------------------------
    def surrogate_datagen(self, lon, lat, p, step, stream=None):
        """Training samples at the given starts (torch cuda tensors: lon, lat,
        p float64, step int32 holding uint32): returns (x [n, 81], y [n, 3])."""
        import torch
        n = lon.numel()
        x = torch.empty((n, SURR_NIN), dtype=torch.float32, device="cuda")
        y = torch.empty((n, SURR_NOUT), dtype=torch.float32, device="cuda")
        _check("mpt_surrogate_datagen", lib().mpt_surrogate_datagen(
            self.h, n, lon.data_ptr(), lat.data_ptr(), p.data_ptr(), step.data_ptr(),
            x.data_ptr(), y.data_ptr(), _stream_handle(stream)))
        return x, y

    def surrogate_stats(self, x, y, stream=None):
        import torch
        norm = torch.empty(12, dtype=torch.float32, device="cuda")
        _check("mpt_surrogate_stats", lib().mpt_surrogate_stats(
            self.h, x.shape[0], x.data_ptr(), y.data_ptr(), norm.data_ptr(), _stream_handle(stream)))
        return norm

    def surrogate_init(self, seed: int, stream=None):
        import torch
        params = torch.empty(SURR_NPARAM, dtype=torch.float32, device="cuda")
        _check("mpt_surrogate_init", lib().mpt_surrogate_init(self.h, params.data_ptr(), seed,
                                                              _stream_handle(stream)))
        return params

    def surrogate_train_step(self, x, y, norm, params, m, v, t: int, lr: float, loss, stream=None):
        _check("mpt_surrogate_train_step", lib().mpt_surrogate_train_step(
            self.h, x.data_ptr(), y.data_ptr(), x.shape[0], norm.data_ptr(), params.data_ptr(),
            m.data_ptr(), v.data_ptr(), t, lr, loss.data_ptr(), _stream_handle(stream)))

    def surrogate_grad(self, x, y, norm, params, stream=None):
        import torch
        grad = torch.zeros(SURR_NPARAM, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        _check("mpt_surrogate_grad", lib().mpt_surrogate_grad(
            self.h, x.data_ptr(), y.data_ptr(), x.shape[0], norm.data_ptr(), params.data_ptr(),
            grad.data_ptr(), loss.data_ptr(), _stream_handle(stream)))
        return grad, loss

    def surrogate_load(self, params, norm, tau_km: float, stream=None):
        _check("mpt_surrogate_load", lib().mpt_surrogate_load(self.h, params.data_ptr(), norm.data_ptr(),
                                                              tau_km, _stream_handle(stream)))

    def surrogate_forward(self, x, stream=None):
        import torch
        y = torch.empty((x.shape[0], SURR_NOUT), dtype=torch.float32, device="cuda")
        _check("mpt_surrogate_forward", lib().mpt_surrogate_forward(self.h, x.shape[0], x.data_ptr(),
                                                                    y.data_ptr(), _stream_handle(stream)))
        return y

    def step_surrogate(self, P: DeviceParticles, step0: int, nsteps: int, fallbacks, err=None,
                       stream=None):
        s = P.cstruct()
        _check("mpt_step_surrogate", lib().mpt_step_surrogate(
            self.h, ctypes.byref(s), step0, nsteps, fallbacks.data_ptr(),
            err.data_ptr() if err is not None else None, _stream_handle(stream)))
        P.adopt(s)

    def step_graph(self, P: DeviceParticles, step0: int, nsteps: int, stream):
        """mpt_step_graph on ``stream`` (a created torch.cuda.Stream, not the
        null stream); the caller orders it with its other work."""
        s = P.cstruct()
        _check("mpt_step_graph", lib().mpt_step_graph(self.h, ctypes.byref(s), step0, nsteps,
                                                      _stream_handle(stream)))
        P.adopt(s)
