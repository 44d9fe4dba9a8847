"""Host-side checks of the C ABI (no GPU needed): the library loads,
exports every entry point include/mpt.h declares, and rejects bad
arguments synchronously, before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

import inputs
import paper_2211_12616_amd as mpt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "mpt.h")).read()
    return sorted(set(re.findall(r"\b(mpt_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    L = mpt.lib()
    names = declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert sorted(mpt.exported_symbols()) == names


def grid_params(dtype=mpt.DT_F32, math=mpt.MATH_F64, **kw):
    met = inputs.empty_met(180, 91, inputs.levels_log(30), 3)
    g, plev = mpt.make_grid(met, dtype)
    return g, plev, mpt.make_params(math=math, **kw)


def ws_bytes(g, p, n=0):
    return mpt.lib().mpt_workspace_bytes(ctypes.byref(g), ctypes.byref(p), n)


def create(g, p, n_max=0, ws=0x100000, nbytes=None):
    h = ctypes.c_void_p()
    nb = ws_bytes(g, p, n_max) if nbytes is None else nbytes
    return mpt.lib().mpt_create(ctypes.byref(g), ctypes.byref(p), n_max, ws, nb, ctypes.byref(h))


def test_workspace_bytes():
    g, plev, p = grid_params()
    nb = ws_bytes(g, p, 1000)
    assert nb >= 180 * 91 * 30 * 16 * 3 + 4000
    assert ws_bytes(g, p, 2000) > nb
    g2, plev2, p2 = grid_params(dtype=mpt.DT_BF16, math=mpt.MATH_F32)
    assert ws_bytes(g2, p2, 1000) < nb


@pytest.mark.parametrize("case", ["nz", "nt", "plev", "dlon", "lat0", "dtype", "reserved"])
def test_bad_grid_is_rejected(case):
    g, plev, p = grid_params()
    if case == "nz":
        g.nz = 1
    elif case == "nt":
        g.nt = 1
    elif case == "plev":
        plev[5] = plev[4] + 1.0                   # not strictly decreasing
    elif case == "dlon":
        g.dlon = 2.5
    elif case == "lat0":
        g.lat0 = -80.0
    elif case == "dtype":
        g.dtype = 7
    else:
        g.reserved = 1
    assert ws_bytes(g, p) == 0
    assert create(g, p, nbytes=1 << 30) == -1


@pytest.mark.parametrize("case", ["dt", "turb", "sort", "fuse", "flags", "math", "conv_cape",
                                  "sedi_radius", "sedi_density", "presort", "reserved"])
def test_bad_params_are_rejected(case):
    g, plev, p = grid_params()
    if case == "dt":
        p.dt = 0.0
    elif case == "turb":
        p.turb_dx = -1.0
    elif case == "sort":
        p.sort_interval = -1
    elif case == "fuse":
        p.fuse = 0
    elif case == "flags":
        p.flags = 32
    elif case == "conv_cape":
        p.flags |= mpt.CONV
        p.conv_cape = float("nan")
    elif case == "sedi_radius":
        p.flags |= mpt.SEDI
        p.sedi_radius = 0.0
    elif case == "sedi_density":
        p.flags |= mpt.SEDI
        p.sedi_density = -1.0
    elif case == "presort":
        p.presort = 2
    elif case == "reserved":
        p.reserved = 1
    else:
        p.math = 3
    assert ws_bytes(g, p) == 0
    assert create(g, p, nbytes=1 << 30) == -1


def test_f64_with_16bit_storage_unsupported():
    g, plev, p = grid_params(dtype=mpt.DT_BF16, math=mpt.MATH_F64)
    assert create(g, p, nbytes=1 << 30) == -6


@pytest.mark.parametrize("dtype", [mpt.DT_BF16, mpt.DT_F16])
def test_16bit_storage_needs_half_a_step_inside_a_met_interval(dtype):
    """16-bit storage keeps the scales of at most three met levels per
    launch: a step whose half spans a whole met interval is unsupported."""
    g, plev, p = grid_params(dtype=dtype, math=mpt.MATH_F32)
    p.dt = 2.0 * g.dt_met
    assert ws_bytes(g, p) == 0
    assert create(g, p, nbytes=1 << 30) == -6
    p.dt = 1.9 * g.dt_met
    assert ws_bytes(g, p) > 0
    g32, _, p32 = grid_params(math=mpt.MATH_F32, dt=2.0 * g.dt_met)
    assert ws_bytes(g32, p32) > 0                       # FP32 storage: no limit


def test_workspace_checks():
    g, plev, p = grid_params()
    assert create(g, p, ws=0) == -1                                   # null
    assert create(g, p, ws=0x100010) == -1                            # misaligned
    assert create(g, p, nbytes=ws_bytes(g, p) - 1) == -4              # too small
    h = ctypes.c_void_p()
    assert mpt.lib().mpt_create(ctypes.byref(g), ctypes.byref(p), -1, 0x100000, 1 << 30,
                                ctypes.byref(h)) == -1                # n_max < 0
    assert ws_bytes(g, p, 1 << 32) == 0                               # 32-bit sort positions
    assert mpt.lib().mpt_create(ctypes.byref(g), ctypes.byref(p), 1 << 32, 0x100000, 1 << 30,
                                ctypes.byref(h)) == -6


def test_no_gpu_gives_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    g, plev, p = grid_params()
    assert create(g, p) == -5


def test_null_context_calls():
    L = mpt.lib()
    s = mpt.ParticlesC(n=0)
    assert L.mpt_advect(None, ctypes.byref(s), 0, None) == -1
    assert L.mpt_diffuse(None, ctypes.byref(s), 0, None) == -1
    assert L.mpt_step(None, ctypes.byref(s), 0, 1, None) == -1
    assert L.mpt_sort_particles(None, ctypes.byref(s), None) == -1
    assert L.mpt_init_met(None, 0, None, None, None, None) == -1
    assert L.mpt_set_release(None, 1, None, None) == -1
    assert L.mpt_destroy(None) == -1
    assert L.mpt_met_level_bytes(None) == 0
    assert L.mpt_status_string(-3) == b"step outside the resident met time levels"


def test_null_context_newer_entry_points():
    L = mpt.lib()
    s = mpt.ParticlesC(n=0)
    assert L.mpt_step_graph(None, ctypes.byref(s), 0, 20, None) == -1
    assert L.mpt_surrogate_datagen(None, 1, None, None, None, None, None, None, None) == -1
    assert L.mpt_surrogate_stats(None, 1, None, None, None, None) == -1
    assert L.mpt_surrogate_init(None, None, 0, None) == -1
    assert L.mpt_surrogate_train_step(None, None, None, 64, None, None, None, None, 1, 1e-3, None,
                                      None) == -1
    assert L.mpt_surrogate_grad(None, None, None, 64, None, None, None, None, None) == -1
    assert L.mpt_surrogate_load(None, None, None, 1.0, None) == -1
    assert L.mpt_surrogate_forward(None, 1, None, None, None) == -1
    assert L.mpt_step_surrogate(None, ctypes.byref(s), 0, 8, None, None, None) == -1
    pe = (ctypes.c_double * 2)(1000.0, 500.0)
    og = mpt.OutGrid(nx=8, ny=4, nz=1, lon0=0.0, dlon=45.0, lat0=-90.0, dlat=45.0,
                     pedges=ctypes.cast(pe, ctypes.c_void_p))
    assert L.mpt_set_outgrid(None, ctypes.byref(og), None) == -1
    assert L.mpt_grid_output(None, ctypes.byref(s), None, None, None, None, None) == -1
    assert L.mpt_push_met(None, None, None, None, None) == -1
    assert L.mpt_set_hybrid(None, 2, None, None, None) == -1
    assert L.mpt_ml_to_pl(None, None, None, None, None, None, None, None, None) == -1
    assert L.mpt_set_met_phys(None, 0, None, None, None, None, None) == -1


def test_physics_flags_are_accepted():
    g, plev, p = grid_params()
    p.flags |= mpt.CONV | mpt.SEDI
    assert ws_bytes(g, p) > 0


def test_surrogate_constants_match_header():
    txt = open(os.path.join(ROOT, "include", "mpt.h")).read()
    for name, val in (("MPT_SURR_K", mpt.SURR_K), ("MPT_SURR_NIN", mpt.SURR_NIN),
                      ("MPT_SURR_NOUT", mpt.SURR_NOUT), ("MPT_SURR_NPARAM", mpt.SURR_NPARAM),
                      ("MPT_SURR_MAX_BATCH", mpt.SURR_MAX_BATCH)):
        m = re.search(name + r"\s*=\s*(\d+)", txt)
        assert m and int(m.group(1)) == val, name
    # the flat parameter layout: per layer W[in][out] + bias with padded shapes
    from oracle import mlp
    assert sum(fi * fo + fo for fi, fo in mlp.FLAT_SHAPES) == mpt.SURR_NPARAM


def test_workspace_includes_surrogate_scratch():
    g, plev, p = grid_params(dtype=mpt.DT_F32, math=mpt.MATH_F32)
    assert ws_bytes(g, p, 0) > 16 * 1024 * 1024
