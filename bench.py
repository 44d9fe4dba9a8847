#!/usr/bin/env python3
"""Benchmark of the particle time step on one MI355X.

Workload: 0.3 deg global grid (1200 x 601) x 137 levels, synthetic jet +
perturbation winds, 1e8 parcels uniform in lon/lat and 100..900 hPa,
dt = 180 s, advection + turbulent + mesoscale diffusion, parcels sorted by
grid box every 10 steps.  One "step" advances every parcel by one time step
(all modules; the sorts that fall into the timed steps are included).

Prints one JSON line (particle-steps/s), with the step kernel's roofline
figures measured live with HIP events on the library's stream and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# Algorithmic FLOP of one parcel-step (all modules): the operations the
# method itself needs -- two locates, two 16-corner quadrilinear
# interpolations of three winds, the spread of 16 values per wind, two
# Philox blocks with Box-Muller, cos(lat) three times -- counted at 1,000
# and used for every arithmetic form.  The kernels execute fewer (the F64
# form 810 FP64 FLOP per parcel-step by counter): a grid point's time
# interpolation is shared by the parcels of a block and the spreads are
# tabulated per cell, so `achieved` credits work the kernel avoids, as an
# algorithmic roofline does; the executed rate is in the profiles.
FLOP_PER_PS = 1000.0
# HBM bytes per 10-step launch of 1e8 parcels = 2 x FETCH_SIZE + WRITE_SIZE
# (KiB x 1024; a 1 GiB copy reads FETCH_SIZE = 512 MiB and WRITE_SIZE =
# 1 GiB) from rocprofv3 --pmc runs of this workload on the current step
# kernels (profiles/k_step_<form>_1e8_0p3deg.md; the timed launches, each
# after a sort whose order it applies as it reads the parcels); None where
# not measured.
TRAFFIC_BYTES_PER_LAUNCH = {"f64": 19.244e9, "f32": 16.072e9, "bf16": 17.416e9, "f16": 14.588e9}
TRAFFIC_STEPS_PER_LAUNCH = 10
# The convection / sedimentation kernel, F64 form, same workload
# (profiles/k_step_phys_1e8_0p3deg.md): FP64 FLOP per parcel-step and HBM
# bytes per 10-step launch (2 x FETCH_SIZE + WRITE_SIZE), with sedimentation
# alone and with both modules.
FLOP_PER_PS_PHYS = {"f64_sedi": 947.0, "f64_phys": 1026.0}
TRAFFIC_BYTES_PER_LAUNCH_PHYS = {"f64_sedi": 64.262e9, "f64_phys": 176.239e9}
METRIC = "particle-steps/s (advect+diffuse, 1e8 particles, 0.3° grid); surrogate vs plain"
FORMS = {"f64": (0, 0), "f32": (1, 0), "bf16": (1, 1), "f16": (1, 2)}   # (math, dtype)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=240)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=float, default=1e8)
    ap.add_argument("--form", default="f64", choices=list(FORMS))
    ap.add_argument("--extra-forms", default="f32,bf16,f16",
                    help="comma list of other forms timed on the same workload ('' = none)")
    ap.add_argument("--sort-interval", type=int, default=10)
    ap.add_argument("--fuse", type=int, default=10)
    ap.add_argument("--nx", type=int, default=1200)
    ap.add_argument("--ny", type=int, default=601)
    ap.add_argument("--nz", type=int, default=137)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target wall time of the CPU-oracle sample (0 = skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    ap.add_argument("--scenarios", action="store_true",
                    help="also run the batched release workload (16 scenarios, 480 steps)")
    ap.add_argument("--no-surrogate", dest="surrogate", action="store_false",
                    help="skip the learned 8-step surrogate leg (trained here, then 480 steps against plain)")
    ap.add_argument("--no-c3", dest="c3", action="store_false",
                    help="skip the 16-bit storage precision report (240 steps, sampled ids vs the FP64 oracle)")
    ap.add_argument("--hbm-steps", type=int, default=10,
                    help="one-step launches of the F64 form timed against the HBM roofline (0 = skip)")
    ap.add_argument("--ml2pl", action="store_true",
                    help="also time the model-level -> pressure-level regridding of one time level")
    ap.add_argument("--stream-met", action="store_true",
                    help="also run 480 steps over 5 met levels with 2 resident, the next level "
                         "copied on a second stream while stepping, against all 5 resident")
    ap.add_argument("--grid-output", action="store_true",
                    help="also time the gridded output on 1e8 parcels (random and sorted order)")
    ap.add_argument("--physics", action="store_true",
                    help="also run all modules plus convection and sedimentation (F64 and F32 "
                         "forms, 60 timed steps) against the same run without them")
    ap.add_argument("--surr-train", type=float, default=5e7, help="surrogate training segments")
    ap.add_argument("--surr-epochs", type=int, default=2)
    ap.add_argument("--surr-bound-km", type=float, default=1.0,
                    help="p99 bound on the accepted 8-step advection error used to set tau")
    return ap.parse_args()


def run_scenarios(met, mpt, inputs, torch, nsteps=480):
    """Batched releases: 16 scenarios of 1e4..2e7 parcels (log-uniform), each
    a point or column release at a random place and step, FP32 fields,
    advection + diffusion for 480 steps through the graph-replayed loop."""
    sc = inputs.make_scenarios(seed=24)
    part, scen = inputs.make_scenario_particles(sc, seed=24)
    n = part.n
    ctx = mpt.Context(met, mpt.make_params(math=1, sort_interval=10, fuse=10), n_max=n)
    ctx.upload_met(met)
    ctx.set_release(sc.release_step)
    P = mpt.DeviceParticles.from_host(part, math=1, scen=scen)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        ctx.step_graph(P, 0, nsteps, s)
    s.synchronize()
    elapsed = time.perf_counter() - t0
    active = int(np.sum(sc.sizes * np.maximum(0, nsteps - np.minimum(sc.release_step, nsteps))))
    lon = P.lon.cpu().numpy()
    return {"workload": "16 release scenarios (1e4..2e7 parcels, log-uniform), 0.3deg grid, "
                        "480 steps, FP32, graph-replayed loop, persistent launches",
            "n_particles": int(n), "steps": nsteps, "active_particle_steps": active,
            "active_particle_steps_per_s": active / elapsed, "seconds": elapsed,
            "finite": bool(np.isfinite(lon).all())}


def run_surrogate(met, mpt, inputs, torch, args, nsteps=480):
    """Learned 8-step surrogate: train on plain-scheme segments, set tau on
    held-out parcels, then run 1e8 parcels for 480 steps and compare with the
    plain FP32 run (time and distance)."""
    K = mpt.SURR_K
    rng = np.random.Generator(np.random.PCG64(25))
    ntr = int(args.surr_train)
    ctx = mpt.Context(met, mpt.make_params(math=1, sort_interval=0, fuse=10), n_max=200_000)
    ctx.upload_met(met)
    steps_max = nsteps - K
    xs, ys = [], []
    t0 = time.perf_counter()
    chunk = 5_000_000
    for c0 in range(0, ntr, chunk):
        m = min(chunk, ntr - c0)
        lon = torch.from_numpy(rng.uniform(0, 360, m)).cuda()
        lat = torch.from_numpy(np.rad2deg(np.arcsin(rng.uniform(-0.985, 0.985, m)))).cuda()
        p = torch.from_numpy(rng.uniform(100, 900, m)).cuda()
        st = torch.from_numpy((rng.integers(0, steps_max // K + 1, m) * K).astype(np.int32)).cuda()
        x, y = ctx.surrogate_datagen(lon, lat, p, st)
        xs.append(x)
        ys.append(y)
    x = torch.cat(xs)
    y = torch.cat(ys)
    del xs, ys
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    norm = ctx.surrogate_stats(x, y)
    params = ctx.surrogate_init(26)
    mom = torch.zeros_like(params)
    var = torch.zeros_like(params)
    B = 4096
    t = 0
    losses = []
    t0 = time.perf_counter()
    for ep in range(args.surr_epochs):
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        nb = 0
        for b0 in range(0, ntr - B + 1, B):
            t += 1
            nb += 1
            ctx.surrogate_train_step(x[b0:b0 + B], y[b0:b0 + B], norm, params, mom, var, t, 1e-3, loss)
        losses.append(loss.item() / nb)
        log(f"surrogate epoch {ep}: mean batch loss {losses[-1]:.5f}")
    t_train = time.perf_counter() - t0
    del x, y
    torch.cuda.empty_cache()

    # tau: held-out parcels, advection only, one block from several starts
    ncal = 200_000
    cal = inputs.make_particles(ncal, 27)
    ctxc = mpt.Context(met, mpt.make_params(math=1, sort_interval=0, flags=mpt.ADVECT), n_max=ncal)
    ctxc.upload_met(met)
    ctxc.surrogate_load(params, norm, float("inf"))
    errs, trues = [], []
    for s0 in (0, 120, 240, 360):
        A = mpt.DeviceParticles.from_host(cal, math=1, pingpong=False)
        Bp = mpt.DeviceParticles.from_host(cal, math=1, pingpong=False)
        fb = torch.zeros(1, dtype=torch.int32, device="cuda")
        e = torch.empty(ncal, dtype=torch.float32, device="cuda")
        ctxc.step_surrogate(A, s0, K, fb, e)
        ctxc.step(Bp, s0, K)
        torch.cuda.synchronize()
        a, bq = A.to_host(), Bp.to_host()
        d = _chord_km(a.lon, a.lat, bq.lon, bq.lat)
        errs.append(e.cpu().numpy())
        trues.append(d)
    est = np.concatenate(errs)
    true = np.concatenate(trues)
    order = np.argsort(est)
    tau = 0.0
    lo = 0
    for q in np.linspace(0.05, 1.0, 96):
        k = int(q * len(order))
        if k < 100:
            continue
        if np.percentile(true[order[:k]], 99) <= args.surr_bound_km:
            tau = float(est[order[k - 1]])
            lo = k
    accepted_frac_cal = lo / len(order)
    log(f"surrogate tau = {tau:.4f} km (accepts {accepted_frac_cal:.3f} of held-out blocks)")

    # production run vs plain, 1e8 parcels (the benchmark's parcels), all modules
    n = int(args.n)
    part = inputs.make_particles(n, 23)
    ctxs = mpt.Context(met, mpt.make_params(math=1, sort_interval=16, fuse=8), n_max=n)
    ctxs.upload_met(met)
    ctxs.surrogate_load(params, norm, tau)
    S = mpt.DeviceParticles.from_host(part, math=1)
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctxs.step_surrogate(S, 0, nsteps, fb)
    torch.cuda.synchronize()
    t_surr = time.perf_counter() - t0
    ids_s, pos_s = _by_id_gpu(S, torch)
    del S
    torch.cuda.empty_cache()
    ctxp = mpt.Context(met, mpt.make_params(math=1, sort_interval=16, fuse=8), n_max=n)
    ctxp.upload_met(met)
    Pp = mpt.DeviceParticles.from_host(part, math=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctxp.step(Pp, 0, nsteps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    ids_p, pos_p = _by_id_gpu(Pp, torch)
    del Pp, ctxp, ctxs
    torch.cuda.empty_cache()
    d = _chord_km_gpu(pos_s, pos_p, torch)
    del pos_s, pos_p
    # the learned part alone: advection only, same parcels and steps
    adv = {}
    for name in ("surr", "plain"):
        ctxa = mpt.Context(met, mpt.make_params(math=1, sort_interval=16, fuse=8, flags=mpt.ADVECT), n_max=n)
        ctxa.upload_met(met)
        A = mpt.DeviceParticles.from_host(part, math=1)
        if name == "surr":
            ctxa.surrogate_load(params, norm, tau)
            fba = torch.zeros(1, dtype=torch.int32, device="cuda")
            ctxa.step_surrogate(A, 0, nsteps, fba)
            adv_fb = fba.item() / (n * (nsteps // K))
        else:
            ctxa.step(A, 0, nsteps)
        torch.cuda.synchronize()
        adv[name] = _by_id_gpu(A, torch)[1]
        del A, ctxa
        torch.cuda.empty_cache()
    da = _chord_km_gpu(adv["surr"], adv["plain"], torch)
    del adv
    blocks = n * (nsteps // K)
    return {"workload": "learned 8-step surrogate, 1e8 parcels, 0.3deg grid, 480 steps, FP32 fields, "
                        "advect+turb+meso; fallback to plain midpoint",
            "train_segments": ntr, "epochs": args.surr_epochs, "loss_by_epoch": losses,
            "datagen_s": t_data, "train_s": t_train, "tau_km": tau,
            "accept_bound_p99_km": args.surr_bound_km, "heldout_accept_frac": accepted_frac_cal,
            "fallback_rate": fb.item() / blocks,
            "surrogate_particle_steps_per_s": n * nsteps / t_surr,
            "plain_f32_particle_steps_per_s": n * nsteps / t_plain,
            "speedup_vs_plain_f32": t_plain / t_surr,
            "error_vs_plain_km": {"p50": d[0], "p99": d[1], "max": d[2],
                                  "note": "all modules; accepted blocks run the plain steps' diffusion "
                                          "draws with the spread of the block's first cell"},
            "advect_only": {"fallback_rate": adv_fb,
                            "error_vs_plain_km": {"p50": da[0], "p99": da[1], "max": da[2]}}}


def _by_id_gpu(P, torch):
    """(ids, positions [n, 3] lon, lat, p) of a device particle set, ordered by id."""
    o = torch.argsort(P.id.to(torch.int64) & 0xFFFFFFFF)
    return P.id[o], torch.stack([P.lon[o], P.lat[o], P.p[o]], 1)


def _chord_km_gpu(a, b, torch):
    """p50, p99, max of the great-circle chord distance [km] between two
    position sets ordered by id (FP64 on the GPU)."""
    r = math.pi / 180.0

    def xyz(x):
        lo, la = x[:, 0] * r, x[:, 1] * r
        return torch.stack([torch.cos(la) * torch.cos(lo), torch.cos(la) * torch.sin(lo), torch.sin(la)], 1)

    c = torch.linalg.norm(xyz(a) - xyz(b), dim=1)
    d = 2.0 * torch.arcsin(torch.clamp(c / 2.0, max=1.0)) * 6371.0
    q = torch.quantile(d[torch.randperm(len(d), device=d.device)[:(1 << 24) - 1]].float(),
                       torch.tensor([0.5, 0.99], device=d.device))
    return float(q[0]), float(q[1]), float(d.max())


def run_ml2pl(met, mpt, inputs, torch, args, reps=5):
    """Regridding of one time level from 137 hybrid model levels (terrain
    following below 100 hPa) to the 137 pressure levels of the grid, with a
    smooth surface pressure field; the stored pressure-level fields stand in
    for the model-level data (the values do not change the work)."""
    a, b = inputs.hybrid_levels(met.plev)
    ctx = mpt.Context(met, mpt.make_params(math=0), n_max=16)
    ctx.set_hybrid(a, b)
    ps = torch.from_numpy(inputs.make_surface_pressure(31, met.nx, met.ny)).cuda()
    u, v, w = (torch.from_numpy(x[0]).cuda() for x in (met.u, met.v, met.w))
    ctx.ml_to_pl(ps, u, v, w)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = ctx.ml_to_pl(ps, u, v, w)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = float(np.median(ms))
    ncol = met.nx * met.ny
    nbytes = 3 * 4 * ncol * (len(a) + met.nz) + 4 * ncol
    del out, ctx
    torch.cuda.empty_cache()
    return {"workload": f"one time level, {len(a)} hybrid model levels -> {met.nz} pressure levels, "
                        f"{met.nx}x{met.ny} columns, u, v, w",
            "ms_per_level": t, "algorithmic_GBps": nbytes / (t * 1e-3) / 1e9,
            "hbm_frac": nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}


def run_stream_met(met, mpt, inputs, torch, args, nsteps=480):
    """A run longer than the resident window: 5 time levels (24 h), 2 on the
    device; while the steps of one 6 h interval run, the next level goes
    host -> pinned staging (CPU) -> device (second stream), and is pushed
    into the ring on the compute stream once copied.  Timed against the same
    run with all 5 levels resident; the final states must be identical."""
    math_, dtype = FORMS[args.form]
    n = int(args.n)
    per = int(round(met.dt_met / 180.0))
    part = inputs.make_particles(n, 23)
    prm = mpt.make_params(math=math_, sort_interval=args.sort_interval, fuse=args.fuse)
    out = {"workload": f"{n} parcels, {nsteps} steps over {met.nt} met levels (6 h apart), "
                       f"form {args.form.upper()}; streamed: 2 levels resident"}
    ctx = mpt.Context(met, prm, n_max=n, dtype=dtype)
    ctx.upload_met(met)
    A = mpt.DeviceParticles.from_host(part, math=math_)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(A, 0, nsteps)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    del ctx
    torch.cuda.empty_cache()
    ctx = mpt.Context(met, prm, n_max=n, dtype=dtype, resident=2)
    ctx.upload_met(met)
    B = mpt.DeviceParticles.from_host(part, math=math_)
    shape = met.u[0].shape
    pinned = [[torch.empty(shape, dtype=torch.float32, pin_memory=True) for _ in range(3)] for _ in range(2)]
    dev = [[torch.empty(shape, dtype=torch.float32, device="cuda") for _ in range(3)] for _ in range(2)]
    copy = torch.cuda.Stream()
    comp = torch.cuda.current_stream()
    copied, pushed = [None, None], [None, None]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt = 2
    for b in range(nsteps // per):
        ctx.step(B, per * b, per)                      # async on the compute stream
        if nxt < met.nt:
            k = nxt % 2
            if copied[k] is not None:
                copied[k].synchronize()                # staging buffer k free again
            for h, a in zip(pinned[k], (met.u, met.v, met.w)):
                h.numpy()[...] = a[nxt]
            with torch.cuda.stream(copy):
                if pushed[k] is not None:
                    copy.wait_event(pushed[k])         # device buffer k consumed
                for d, h in zip(dev[k], pinned[k]):
                    d.copy_(h, non_blocking=True)
                copied[k] = torch.cuda.Event()
                copied[k].record(copy)
            comp.wait_event(copied[k])
            ctx.push_met(*dev[k])
            pushed[k] = torch.cuda.Event()
            pushed[k].record(comp)
            nxt += 1
    torch.cuda.synchronize()
    t_stream = time.perf_counter() - t0
    # the order within a tile follows the sort's atomics: compare by parcel id
    oa, ob = torch.argsort(A.id), torch.argsort(B.id)
    same = all(bool(torch.equal(getattr(A, f)[oa], getattr(B, f)[ob])) for f in ("lon", "lat", "p", "id"))
    del oa, ob
    out.update({"all_resident_particle_steps_per_s": n * nsteps / t_all,
                "streamed_particle_steps_per_s": n * nsteps / t_stream,
                "streamed_over_all_resident": t_all / t_stream,
                "level_bytes_copied": 3 * int(np.prod(shape)) * 4,
                "identical_final_state": same})
    del A, B, ctx, dev, pinned
    torch.cuda.empty_cache()
    if not same:
        raise RuntimeError("streamed run differs from the all-resident run")
    return out


def run_physics(met, mpt, inputs, torch, args, nsteps=60, warm=10):
    """All modules plus convection (CAPE threshold 800 J/kg) and
    sedimentation (radius 5 um, density 1000 kg/m^3) on the headline
    workload, F64 and F32 forms, against the same runs without the two
    modules (F64 also with sedimentation alone); launches of 10 steps timed
    with events, sort every 10 steps."""
    inputs.add_phys_fields(met, seed=31)
    n = int(args.n)
    part = inputs.make_particles(n, 23)
    out = {"workload": f"{n} parcels, 0.3deg grid {met.nx}x{met.ny}x{met.nz}, advect+turb+meso"
                       f"+convection+sedimentation, {nsteps} timed steps"}
    S = args.sort_interval
    base = mpt.ADVECT | mpt.TURB | mpt.MESO
    for form in ("f64", "f32"):
        math_, dtype = FORMS[form]
        runs = [("plain", base), ("phys", base | mpt.CONV | mpt.SEDI)]
        if form == "f64":
            runs.insert(1, ("sedi", base | mpt.SEDI))
        for tag, flags in runs:
            prm = mpt.make_params(math=math_, flags=flags, fuse=args.fuse, conv_cape=800.0,
                                  sedi_radius=5e-6, sedi_density=1000.0)
            ctx = mpt.Context(met, prm, n_max=n, dtype=dtype)
            ctx.upload_met(met)
            P = mpt.DeviceParticles.from_host(part, math=math_)
            stream = torch.cuda.current_stream()
            ev = []

            def run(s0, k, timed):
                s = s0
                while s < s0 + k:
                    if S > 0 and (s - s0) % S == 0:            # cadence from the run's first step
                        ctx.sort_deferred(P)
                    stop = min(s0 + k, s0 + ((s - s0) // S + 1) * S if S > 0 else s0 + k, s + args.fuse)
                    if timed:
                        ev.append([torch.cuda.Event(enable_timing=True) for _ in range(2)])
                        ev[-1][0].record(stream)
                    ctx.step(P, s, stop - s)
                    if timed:
                        ev[-1][1].record(stream)
                    s = stop

            run(0, warm, False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run(warm, nsteps, True)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            key = f"{form}_{tag}"
            ms = [a.elapsed_time(b) for a, b in ev]
            out[key] = {"particle_steps_per_s": n * nsteps / el,
                        "step_kernel_ms_avg": float(np.mean(ms)),
                        "finite": bool(torch.isfinite(P.lon).all().item())}
            if key in FLOP_PER_PS_PHYS and args.fuse == 10 and n == 100_000_000 and met.nz == 137:
                # per launch of 10 steps, as the headline kernel's roofline
                tf = FLOP_PER_PS_PHYS[key] * n * 10 / (np.mean(ms) * 1e-3) / 1e12
                gbs = TRAFFIC_BYTES_PER_LAUNCH_PHYS[key] / (np.mean(ms) * 1e-3) / 1e9
                out[key]["roofline"] = {"flop_per_particle_step": FLOP_PER_PS_PHYS[key],
                                        "achieved_TFLOPs": tf, "frac_fp64_peak": tf / FP64_PEAK_TFLOPS,
                                        "traffic_bytes_per_launch": TRAFFIC_BYTES_PER_LAUNCH_PHYS[key],
                                        "hbm_GBps": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS}
            log(f"physics leg {key}: {n * nsteps / el:.3e} particle-steps/s")
            del ctx, P
            torch.cuda.empty_cache()
        out[f"{form}_phys_over_plain_time"] = (out[f"{form}_plain"]["particle_steps_per_s"]
                                               / out[f"{form}_phys"]["particle_steps_per_s"])
    met.temp = met.cape = met.pel = met.ps = None
    return out


def run_grid_output(met, mpt, inputs, torch, args, reps=5):
    """Gridded output of 1e8 parcels on a 1 x 1 deg grid with 18 layers
    (1000 .. 100 hPa): per call, count and FP64 mass sum per box plus the
    mass mixing ratio.  Timed with HIP events on the library's stream, for
    parcels in random order and after a sort by tile."""
    n = int(args.n)
    pe = np.linspace(1000.0, 100.0, 19)
    nx, ny = 360, 180
    ctx = mpt.Context(met, mpt.make_params(math=1, sort_interval=10), n_max=n)
    ctx.upload_met(met)
    ctx.set_outgrid(nx, ny, -0.5, -90.0, 1.0, pe)
    part = inputs.make_particles(n, 23)
    P = mpt.DeviceParticles.from_host(part, math=1)
    mass = torch.rand(n, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    inside = int(((P.p <= 1000.0) & (P.p > 100.0)).sum().item())
    out = {"workload": f"gridded output, {n} parcels, 360x180x18 boxes (1 deg, 1000..100 hPa), FP64 masses",
           "boxes": nx * ny * (len(pe) - 1)}
    nbox = nx * ny * (len(pe) - 1)
    bytes_call = n * (3 * 8 + 8) + nbox * (4 + 8) * 2 + nbox * 8
    for label in ("random", "sorted"):
        if label == "sorted":
            ctx.sort(P)
        ctx.grid_output(P, mass)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            counts, msum, mmr = ctx.grid_output(P, mass)
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        got = int(counts.sum().item())
        if got != inside:
            raise RuntimeError(f"grid output lost parcels: {got} != {inside}")
        t = float(np.median(ms))
        out[label] = {"ms_per_call": t, "parcels_per_s": n / (t * 1e-3),
                      "algorithmic_GBps": bytes_call / (t * 1e-3) / 1e9,
                      "hbm_frac": bytes_call / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
    out["algorithmic_bytes_per_call"] = bytes_call
    del P, ctx
    torch.cuda.empty_cache()
    return out


def _chord_km(lon1, lat1, lon2, lat2):
    r = np.pi / 180.0

    def xyz(lo, la):
        return np.stack([np.cos(la * r) * np.cos(lo * r), np.cos(la * r) * np.sin(lo * r), np.sin(la * r)])

    c = np.linalg.norm(xyz(lon1, lat1) - xyz(lon2, lat2), axis=0)
    return 2.0 * np.arcsin(np.minimum(c / 2.0, 1.0)) * 6371.0


def unique_points_per_step(P, met, torch):
    """Algorithmic field traffic: grid points that are corners of any
    parcel's cell (8 corners of the cell holding the parcel), counted with a
    bitmap over the grid; each such point is read at 2 time levels."""
    nx, ny, nz = met.nx, met.ny, met.nz
    plev = torch.tensor(met.plev, dtype=torch.float64, device="cuda")
    asc = torch.flip(plev, [0]).contiguous()
    bitmap = torch.zeros(nx * ny * nz, dtype=torch.bool, device="cuda")
    n = P.n
    chunk = 1 << 24
    for s in range(0, n, chunk):
        lon = P.lon[s:s + chunk]
        lat = P.lat[s:s + chunk]
        p = P.p[s:s + chunk]
        i0 = torch.floor(lon / met.dlon).long() % nx
        j0 = torch.clamp(torch.floor((lat + 90.0) / met.dlat).long(), 0, ny - 2)
        pc = torch.clamp(p, met.plev[-1], met.plev[0])
        k0 = torch.clamp(nz - 1 - torch.searchsorted(asc, pc, right=False), 0, nz - 2)
        for dk in (0, 1):
            for dj in (0, 1):
                for di in (0, 1):
                    idx = ((k0 + dk) * ny + (j0 + dj)) * nx + (i0 + di) % nx
                    bitmap[idx] = True
    return int(bitmap.sum().item())


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_c3(met, mpt, inputs, torch, part, form, nsample=2000, nsteps=240):
    """Config 3: 16-bit storage of the headline workload over 240 steps (all
    modules, sort every 10, 10 steps per launch), position error of a seeded
    id sample against the FP64 oracle on the original FP32 fields."""
    import oracle
    math_, dtype = FORMS[form]
    n = part.n
    ctx = mpt.Context(met, mpt.make_params(math=math_, sort_interval=10, fuse=10), n_max=n, dtype=dtype,
                      resident=3)
    ctx.upload_met(met)
    P = mpt.DeviceParticles.from_host(part, math=math_)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(P, 0, nsteps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rng = np.random.Generator(np.random.PCG64(323))
    sample = np.sort(rng.choice(n, nsample, replace=False))
    ids = P.id.to(torch.int64) & 0xFFFFFFFF
    where = torch.empty(n, dtype=torch.int64, device="cuda")
    where[ids] = torch.arange(n, device="cuda")
    loc = where[torch.from_numpy(sample).cuda()]
    lon, lat = P.lon[loc].cpu().numpy(), P.lat[loc].cpu().numpy()
    level_bytes = ctx.met_level_bytes()
    del P, ctx, where, ids, loc
    torch.cuda.empty_cache()
    r = part.subset(sample)
    oracle.run(oracle.Met(met), oracle.ctl(dt=180.0), r, 0, nsteps)
    km = oracle.chord_deg(lon, lat, r.lon, r.lat) * math.pi * 6371.0 / 180.0
    return {"steps": nsteps, "sample": f"{nsample} seeded ids of the {n} parcels",
            "km_vs_fp64_oracle_on_fp32_fields": {"mean": float(km.mean()), "p99": float(np.percentile(km, 99)),
                                                  "max": float(km.max())},
            "met_level_bytes": level_bytes, "particle_steps_per_s_240": n * nsteps / el}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; use --gpus 1"}))
        sys.stderr.write("bench.py: only --gpus 1 is supported (the library runs on one GPU)\n")
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        sys.stderr.write("bench.py: no GPU visible\n")
        sys.exit(1)
    import inputs
    import paper_2211_12616_amd as mpt
    mpt.lib()

    n = int(args.n)
    W, K = args.warmup, args.steps
    dt = 180.0
    total = W + K + max(0, args.hbm_steps)
    nt_timed = int(math.ceil(total * dt / inputs.DT_MET)) + 1
    nt = nt_timed
    if args.c3:
        nt = max(nt, 3)
    if args.scenarios or args.surrogate or args.stream_met:
        nt = max(nt, int(math.ceil(480 * dt / inputs.DT_MET)) + 1)
    t0 = time.time()
    log(f"generating fields {args.nx}x{args.ny}x{args.nz}, nt={nt}")
    met = inputs.make_met_c2(seed=12, nt=nt, nx=args.nx, ny=args.ny, nz=args.nz)
    log(f"fields done in {time.time() - t0:.1f} s; generating {n} parcels")
    part = inputs.make_particles(n, 23)
    log(f"parcels done at {time.time() - t0:.1f} s")

    forms = [args.form] + [f for f in args.extra_forms.split(",") if f and f != args.form]
    results = {}
    hbm_leg = None
    for form in forms:
        math_, dtype = FORMS[form]
        log(f"form {form}: upload")
        params = mpt.make_params(math=math_, sort_interval=0, fuse=args.fuse, presort=1)
        ctx = mpt.Context(met, params, n_max=n, dtype=dtype, resident=nt_timed)
        ctx.upload_met(met)
        P = mpt.DeviceParticles.from_host(part, math=math_)
        stream = torch.cuda.current_stream()
        S = args.sort_interval

        def run(step0, nsteps, ev=None, fuse=args.fuse):
            # sorts every S steps counted from the run's first step, so a
            # timed run is whole sort intervals (a sort, then S steps) and
            # no launch is cut short by where the warm-up ended
            s = step0
            end = step0 + nsteps
            while s < end:
                if S > 0 and (s - step0) % S == 0:
                    if ev is not None:
                        ev["sort"].append([torch.cuda.Event(enable_timing=True) for _ in range(2)])
                        ev["sort"][-1][0].record(stream)
                    # the order only; the step launch that follows moves the parcels
                    ctx.sort_deferred(P)
                    if ev is not None:
                        ev["sort"][-1][1].record(stream)
                stop = min(end, step0 + ((s - step0) // S + 1) * S) if S > 0 else end
                stop = min(stop, s + fuse)
                if ev is not None:
                    ev["step"].append(([torch.cuda.Event(enable_timing=True) for _ in range(2)],
                                       stop - s))
                    ev["step"][-1][0][0].record(stream)
                ctx.step(P, s, stop - s)
                if ev is not None:
                    ev["step"][-1][0][1].record(stream)
                s = stop

        log(f"form {form}: warmup {W} steps")
        run(0, W)
        torch.cuda.synchronize()
        pts = unique_points_per_step(P, met, torch)
        torch.cuda.synchronize()
        ev = {"sort": [], "step": []}
        log(f"form {form}: timing {K} steps")
        t_start = time.perf_counter()
        run(W, K, ev)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        step_ms = [a.elapsed_time(b) for (a, b), _ in ev["step"]]
        step_steps = [k for _, k in ev["step"]]
        sort_ms = [a.elapsed_time(b) for a, b in ev["sort"]]
        ok = bool(torch.isfinite(P.lon).all().item())
        results[form] = dict(elapsed=elapsed, step_ms=step_ms, step_steps=step_steps,
                             sort_ms=sort_ms, unique_pts=pts, ok=ok)
        log(f"form {form}: {n * K / elapsed:.3e} particle-steps/s, {1e3 * elapsed / K:.3f} ms/step")
        if form == "f64" and args.hbm_steps > 0:
            # one step per launch: the state is read and written every step,
            # the per-step form priced against HBM
            ev1 = {"sort": [], "step": []}
            run(W + K, args.hbm_steps, ev1, fuse=1)
            torch.cuda.synchronize()
            ms1 = [a.elapsed_time(b) for (a, b), _ in ev1["step"]]
            field_b = pts * 2 * 12 / n
            gbs = n * (100.0 + field_b) / (float(np.mean(ms1)) * 1e-3) / 1e9
            hbm_leg = {"form": "F64", "steps_per_launch": 1, "launches": len(ms1),
                       "avg_launch_ms": float(np.mean(ms1)),
                       "algorithmic_bytes_per_particle_step": 100.0 + field_b,
                       "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                       "particle_steps_per_s": n / (float(np.mean(ms1)) * 1e-3)}
            log(f"form f64, one step per launch: {np.mean(ms1):.3f} ms, {gbs:.0f} GB/s algorithmic")
        del ctx, P
        torch.cuda.empty_cache()

    main_r = results[args.form]
    math_, dtype = FORMS[args.form]
    # state bytes a launch reads and writes per parcel: read lon, lat, p,
    # id and the mesoscale state, write them all (the launch after a sort
    # moves the whole state into sorted order)
    state_b = 104 if math_ == 0 else 80
    rec_b = 12 if dtype == 0 else 6
    field_b = main_r["unique_pts"] * 2 * rec_b / n
    durations = main_r["step_ms"]
    ksteps = main_r["step_steps"]
    avg_ms = float(np.mean(durations))
    # the dominant kernel is bound by its vector ALU: algorithmic FLOP per
    # launch = FLOP per parcel-step x parcel-steps of that launch
    peak = FP64_PEAK_TFLOPS if math_ == 0 else FP32_PEAK_TFLOPS
    achieved_tf = float(np.mean([FLOP_PER_PS * n * k / (d * 1e-3) / 1e12 for k, d in zip(ksteps, durations)]))
    hbm_gbs = float(np.mean([n * (state_b + field_b * k) / (d * 1e-3) / 1e9 for k, d in zip(ksteps, durations)]))
    traffic = TRAFFIC_BYTES_PER_LAUNCH.get(args.form) if (n == 100_000_000 and args.nz == 137) else None
    value = n * K / main_r["elapsed"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * main_r["elapsed"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if math_ == 0 else "f32",
        "data": "synthetic",
        "config": {"workload": "0.3deg grid 1200x601x137, 1e8 parcels, advect+turb+meso, "
                               "dt=180s, sort every 10 steps",
                   "n_particles": n, "grid": f"{args.nx}x{args.ny}x{args.nz}",
                   "form": args.form.upper(), "sort_interval": args.sort_interval,
                   "fuse": args.fuse, "met_levels": nt_timed},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved_tf / peak, "traffic": traffic,
                     "traffic_steps_per_launch": TRAFFIC_STEPS_PER_LAUNCH if traffic else None,
                     "kernel": "k_step_f64<0>" if math_ == 0 else f"k_step_f32<0, {dtype}>",
                     "avg_launch_ms": avg_ms, "launches": len(durations),
                     "flop_per_particle_step": FLOP_PER_PS,
                     "steps_per_launch": ksteps,
                     "hbm_algorithmic_GBps": hbm_gbs,
                     "hbm_frac": hbm_gbs / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_particle_step": state_b * len(ksteps) / sum(ksteps) + field_b},
        "sort_ms_avg": float(np.mean(main_r["sort_ms"])) if main_r["sort_ms"] else None,
        "forms": {f: {"particle_steps_per_s": n * K / r["elapsed"],
                      "step_kernel_ms_avg": float(np.mean(r["step_ms"])),
                      "steps_per_launch": r["step_steps"],
                      "sort_ms_avg": float(np.mean(r["sort_ms"])) if r["sort_ms"] else None,
                      "finite": r["ok"]} for f, r in results.items()},
    }
    if hbm_leg is not None:
        line["hbm_per_step_form"] = hbm_leg

    if args.c3:
        c3 = {}
        for form in ("bf16", "f16"):
            log(f"c3: {form} storage, 240 steps, sampled ids vs the FP64 oracle")
            c3[form] = run_c3(met, mpt, inputs, torch, part, form)
            if form in results and "f32" in results:
                c3[form]["speedup_vs_f32_timed"] = results["f32"]["elapsed"] / results[form]["elapsed"]
        c3["f32_met_level_bytes"] = 16 * args.nx * args.ny * args.nz
        line["c3"] = c3

    if args.cpu_seconds > 0:
        import oracle
        log("CPU oracle baseline")
        m = oracle.Met(met)
        c = oracle.ctl(dt=dt)
        nthreads = oracle.max_threads()
        probe = part.subset(np.arange(0, 2000))
        tp = time.perf_counter()
        oracle.run(m, c, probe, 0, 10, nthreads=nthreads)
        rate_est = 2000 * 10 / (time.perf_counter() - tp)
        steps_cpu = 20
        m_cpu = int(min(n, max(1000, rate_est * args.cpu_seconds / steps_cpu)))
        sample = part.subset(np.arange(0, m_cpu))
        tc = time.perf_counter()
        oracle.run(m, c, sample, 0, steps_cpu, nthreads=nthreads)
        tcpu = time.perf_counter() - tc
        # one thread, a sample sized for about a fifth of the time
        m1 = int(max(200, m_cpu / max(1, nthreads) / 5))
        s1 = part.subset(np.arange(0, m1))
        t1 = time.perf_counter()
        oracle.run(m, c, s1, 0, steps_cpu, nthreads=1)
        t1 = time.perf_counter() - t1
        line["cpu_baseline"] = {"value": m_cpu * steps_cpu / tcpu, "unit": "particle-steps/s",
                                "cores": nthreads, "kind": "oracle",
                                "sample": f"ids 0..{m_cpu - 1} of the same workload, steps 0..{steps_cpu - 1} "
                                          f"(all modules, FP64), {tcpu:.1f} s wall",
                                "single_thread": {"value": m1 * steps_cpu / t1, "sample": f"ids 0..{m1 - 1}, "
                                                  f"steps 0..{steps_cpu - 1}, {t1:.1f} s wall"},
                                "cpu_model": cpu_model()}
    extras = {}
    if args.scenarios:
        log("scenario workload")
        extras["scenarios"] = run_scenarios(met, mpt, inputs, torch)
        torch.cuda.empty_cache()
    if args.ml2pl:
        log("model levels to pressure levels")
        extras["ml2pl"] = run_ml2pl(met, mpt, inputs, torch, args)
        torch.cuda.empty_cache()
    if args.stream_met:
        log("streamed met levels")
        extras["stream_met"] = run_stream_met(met, mpt, inputs, torch, args)
        torch.cuda.empty_cache()
    if args.grid_output:
        log("gridded output")
        extras["grid_output"] = run_grid_output(met, mpt, inputs, torch, args)
        torch.cuda.empty_cache()
    if args.physics:
        log("convection and sedimentation")
        extras["physics"] = run_physics(met, mpt, inputs, torch, args)
        torch.cuda.empty_cache()
    if args.surrogate:
        log("surrogate workload")
        line["surrogate"] = run_surrogate(met, mpt, inputs, torch, args)
        torch.cuda.empty_cache()
    if extras:
        line["extras"] = extras
    if args.copy_probe:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = 1 << 30
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
