"""Benchmark: RK3-step cell-updates/s of the IIM hot path on one MI355X.

Workload: impulsively started cylinder in free space, D = 1, 1024 x 512 nodes
(h = D/64), u_inf = (1, 0), Re 100 (nu = 0.01), dt = 0.0025, from rest;
zero-padded lattice-Green's-function FFT Poisson solve on a 2048 x 1024 torus.
One step = the three RK3 stages, each with the full IIM velocity
reconstruction, boundary vorticity, transport and Kelvin update.

Headline path (`value`): FP64 with the dense Schur inverse (bodies are fixed)
and the step replayed as a HIP graph.  The paper's iterative path (GMRES with
the FFT matrix-vector product, previous-stage initial guess) is timed too and
reported under "paths".

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def _parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    p.add_argument("--solver", choices=["krylov", "direct"], default="direct")
    p.add_argument("--krylov-steps", type=int, default=5, help="steps of the GMRES path timed for 'paths'")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=10)
    return p.parse_args()


def _run_path(iim, w, torch, np, precision, solver, guess, warmup, steps, profile_kernels=None):
    g = w.grid
    ctx = iim.Context(g, w.bodies, precision=precision, tol=1e-13, guess=guess, solver=solver)
    omega = torch.zeros((g.ny, g.nx), dtype=torch.float64, device="cuda:0")
    Gamma = np.zeros(ctx.n_circ)
    pre = {}
    # warm-up: all but the last two steps with every kernel timed by events (to
    # find the dominant kernel); the last two without instrumentation, so that a
    # step graph is captured before the timed region
    n_prof = max(0, warmup - 2) if profile_kernels else 0
    if n_prof:
        ctx.profile(profile_kernels)
        Gamma, _ = ctx.rk3_steps(omega, Gamma, w.dt, n_prof)
        torch.cuda.synchronize()
        pre = ctx.profile_read()
        ctx.profile(0)
    if warmup - n_prof:
        Gamma, _ = ctx.rk3_steps(omega, Gamma, w.dt, warmup - n_prof)
    torch.cuda.synchronize()
    s0, m0 = ctx.krylov_totals()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Gamma, stats = ctx.rk3_steps(omega, Gamma, w.dt, steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    s1, m1 = ctx.krylov_totals()
    res = {"value": g.nx * g.ny * steps / secs, "ms_per_step": 1e3 * secs / steps, "steps": steps,
           "krylov": {"solves": s1 - s0, "matvecs": m1 - m0, "matvecs_per_solve": (m1 - m0) / max(1, s1 - s0),
                      "last_step": stats}}
    return ctx, omega, Gamma, res, pre


def main():
    args = _parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as wl
    import paper_2109_13628_amd as iim

    w = wl.cylinder()
    g = w.grid
    prec = iim.PREC_FP64 if args.precision == "fp64" else iim.PREC_MIXED
    solver = iim.SOLVER_KRYLOV if args.solver == "krylov" else iim.SOLVER_DIRECT
    all_kernels = (1 << len(iim.KERNEL_NAMES)) - 1
    tag = "fp64" if prec == iim.PREC_FP64 else "mixed"

    # headline path: warm-up (kernels timed with events only to find the dominant
    # one), then exactly `steps` timed steps without instrumentation
    ctx, omega, Gamma, head, pre = _run_path(iim, w, torch, np, prec, solver, iim.GUESS_PREVIOUS,
                                             args.warmup, args.steps, profile_kernels=all_kernels)
    dominant = max(pre, key=lambda k: pre[k]["total_ms"]) if pre else "fft_cols_conv"
    total = sum(x["total_ms"] for x in pre.values()) or 1.0
    shares = {n: round(v["total_ms"] / total, 4) for n, v in pre.items()}

    # roofline of the dominant kernel: HIP events around each of its launches on
    # the context stream, over the same number of steps continuing the run
    ctx.profile(1 << iim.KERNEL_NAMES.index(dominant))
    Gamma, _ = ctx.rk3_steps(omega, Gamma, w.dt, args.steps)
    torch.cuda.synchronize()
    prof = ctx.profile_read().get(dominant, {})
    ctx.profile(0)
    achieved = prof.get("GBps")
    roof = {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
            "frac": (achieved / 8000.0) if achieved else None, "traffic": None,
            "avg_us": prof.get("avg_us"), "launches": prof.get("launches"),
            "algorithmic_bytes_per_launch": prof.get("bytes_per_launch"),
            "timing": "HIP events around every launch of this kernel over %d eager steps continuing the "
                      "timed run" % args.steps}

    paths = {tag + "_" + args.solver: head}
    if args.krylov_steps and solver != iim.SOLVER_KRYLOV:
        _, _, _, kry, _ = _run_path(iim, w, torch, np, prec, iim.SOLVER_KRYLOV, iim.GUESS_PREVIOUS,
                                    args.warmup, args.krylov_steps)
        paths[tag + "_krylov_plain"] = kry

    out = {
        "metric": "RK3 step cell-updates/s at 1e-8 rel. error; FP64 plain vs mixed+learned warm-start",
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == iim.PREC_FP64 else "f32+f64",
        "data": "synthetic (impulsively started flow from rest)",
        "config": {"workload": w.name, "nx": g.nx, "ny": g.ny, "h": g.h,
                   "fft": [ctx.info["fft_mx"], ctx.info["fft_my"]], "Re": 100, "dt": w.dt,
                   "precision": args.precision, "solver": args.solver, "guess": "previous-stage",
                   "krylov_tol": 1e-13, "t_start": args.warmup * w.dt},
        "paths": paths,
        "roofline": roof,
        "kernel_time_share_warmup": shares,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out))


def _cpu_baseline(w, steps):
    """The FP64 oracle, timed on this host's cores over a bounded sample of the
    same workload (a few RK3 steps from rest; set-up excluded)."""
    import numpy as np
    import scipy.fft as sfft
    from oracle import geometry as OG, ns as ONS
    cores = len(os.sched_getaffinity(0))
    cores = max(1, min(cores, 16))
    geo = OG.Geometry(w.grid, w.bodies)
    st = ONS.Stepper(geo)
    om = np.zeros((w.grid.ny, w.grid.nx))
    G = np.zeros(geo.nbc)
    with sfft.set_workers(cores):
        om, G = st.step(om, G, w.dt)           # builds and factorises the Schur matrix (set-up)
        t0 = time.perf_counter()
        for _ in range(steps):
            om, G = st.step(om, G, w.dt)
        secs = time.perf_counter() - t0
    return {"value": w.grid.nx * w.grid.ny * steps / secs, "unit": "cell-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d RK3 steps of the same 1024x512 cylinder workload after one set-up step from rest "
                      "(FP64 NumPy/SciPy, dense Schur LU, scipy.fft workers=%d)" % (steps, cores)}


if __name__ == "__main__":
    main()
