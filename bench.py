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
    ap.add_argument("--extra-forms", default="f32,bf16",
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
    return ap.parse_args()


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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.stderr.write("bench.py: only --gpus 1 is supported (single-GPU build)\n")
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
    total = W + K
    nt = int(math.ceil(total * dt / inputs.DT_MET)) + 1
    t0 = time.time()
    log(f"generating fields {args.nx}x{args.ny}x{args.nz}, nt={nt}")
    met = inputs.make_met_c2(seed=12, nt=nt, nx=args.nx, ny=args.ny, nz=args.nz)
    log(f"fields done in {time.time() - t0:.1f} s; generating {n} parcels")
    part = inputs.make_particles(n, 23)
    log(f"parcels done at {time.time() - t0:.1f} s")

    forms = [args.form] + [f for f in args.extra_forms.split(",") if f and f != args.form]
    results = {}
    for form in forms:
        math_, dtype = FORMS[form]
        log(f"form {form}: upload")
        params = mpt.make_params(math=math_, sort_interval=0, fuse=args.fuse)
        ctx = mpt.Context(met, params, n_max=n, dtype=dtype)
        ctx.upload_met(met)
        P = mpt.DeviceParticles.from_host(part, math=math_)
        stream = torch.cuda.current_stream()
        S = args.sort_interval

        def run(step0, nsteps, ev=None):
            s = step0
            end = step0 + nsteps
            while s < end:
                if S > 0 and s % S == 0:
                    if ev is not None:
                        ev["sort"].append([torch.cuda.Event(enable_timing=True) for _ in range(2)])
                        ev["sort"][-1][0].record(stream)
                    ctx.sort(P)
                    if ev is not None:
                        ev["sort"][-1][1].record(stream)
                stop = min(end, (s // S + 1) * S) if S > 0 else end
                stop = min(stop, s + args.fuse)
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
        h = P.to_host() if form == args.form else None
        ok = bool(np.all(np.isfinite(P.lon.cpu().numpy())))
        results[form] = dict(elapsed=elapsed, step_ms=step_ms, step_steps=step_steps,
                             sort_ms=sort_ms, unique_pts=pts, ok=ok, host=h)
        log(f"form {form}: {n * K / elapsed:.3e} particle-steps/s, {1e3 * elapsed / K:.3f} ms/step")
        del ctx, P
        torch.cuda.empty_cache()

    main_r = results[args.form]
    math_, dtype = FORMS[args.form]
    state_b = 100 if math_ == 0 else 76
    rec_b = 12 if dtype == 0 else 6
    field_b = main_r["unique_pts"] * 2 * rec_b / n
    # dominant kernel: the fused step kernel; algorithmic bytes per launch =
    # N * (state read+write once per launch + field bytes per step * steps)
    launch_bytes = [n * (state_b + field_b * k) for k in main_r["step_steps"]]
    durations = main_r["step_ms"]
    avg_ms = float(np.mean(durations))
    achieved_gbs = float(np.mean([b / (d * 1e-3) / 1e9 for b, d in zip(launch_bytes, durations)]))
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
                   "fuse": args.fuse, "met_levels": nt},
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_step", "avg_launch_ms": avg_ms,
                     "algorithmic_bytes_per_particle_step": state_b / args.fuse + field_b,
                     "field_bytes_per_particle_step": field_b},
        "sort_ms_avg": float(np.mean(main_r["sort_ms"])) if main_r["sort_ms"] else None,
        "forms": {f: {"particle_steps_per_s": n * K / r["elapsed"],
                      "step_kernel_ms_avg": float(np.mean(r["step_ms"])),
                      "sort_ms_avg": float(np.mean(r["sort_ms"])) if r["sort_ms"] else None,
                      "finite": r["ok"]} for f, r in results.items()},
    }

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
        line["cpu_baseline"] = {"value": m_cpu * steps_cpu / tcpu, "unit": "particle-steps/s",
                                "cores": nthreads, "kind": "oracle",
                                "sample": f"ids 0..{m_cpu - 1} of the same workload, steps 0..{steps_cpu - 1} "
                                          f"(all modules, FP64), {tcpu:.1f} s wall"}
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
