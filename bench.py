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
    p.add_argument("--krylov-steps", type=int, default=20, help="timed steps of each GMRES path in 'paths' (0: none)")
    p.add_argument("--krylov-tol", type=float, default=1e-10, help="relative residual of the GMRES paths")
    p.add_argument("--train-runs", type=int, default=7,
                   help="recorded runs at distinct Re for the network, one of them for validation (0: no network path)")
    p.add_argument("--train-steps", type=int, default=1000, help="RK3 steps per recorded run (3 solves each)")
    p.add_argument("--train-iters", type=int, default=2000)
    p.add_argument("--eval-start", type=int, default=400,
                   help="steps of the held-out run (direct solver) before the GMRES paths take over")
    p.add_argument("--batch-sims", type=int, default=64, help="simulations of the batched-serving measurement (0: none)")
    p.add_argument("--batch-steps", type=int, default=20)
    p.add_argument("--no-autotune", action="store_true", help="keep the default FFT tile shapes on the headline path")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=20)
    p.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "OUT"),
                   help="write the text summary of a rocprofv3 --kernel-trace --stats run and exit")
    p.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"),
                   help="write the HBM traffic summary of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) and exit")
    p.add_argument("--summarize-mfma", nargs=2, metavar=("PMC_DIR", "OUT"),
                   help="write the matrix-core counter summary of a --net-only counter run and exit")
    p.add_argument("--command", default="", help="command line recorded in a summary")
    p.add_argument("--copy-probe", action="store_true",
                   help="end with one plain device copy of 256 MiB (scale reference for HBM byte counters)")
    p.add_argument("--workload", choices=sorted(WORKLOADS), default="cylinder_1024x512",
                   help="the headline workload; multi_body_2048 serves the kernel profiles at the 2048 x 2048 "
                        "four-body configuration")
    p.add_argument("--net-only", action="store_true",
                   help="only the network's matrix-core timing (forward and training steps at the training "
                        "batch shape); for counter runs")
    p.add_argument("--batch-only", action="store_true",
                   help="run only the batched-serving leg and print its JSON object (the benchmark runs this "
                        "in a child process)")
    p.add_argument("--batch-timeout", type=float, default=420.0, help="seconds allowed for the batch child process")
    p.add_argument("--no-extra-workloads", action="store_true",
                   help="skip the Taylor-Couette box and four-body outflow legs (profiling runs of the headline)")
    p.add_argument("--cpu-single-steps", type=int, default=3,
                   help="oracle steps timed on one core beside the multi-core CPU baseline (0: none)")
    return p.parse_args()


def _say(msg):
    """One progress line on stderr, flushed at once: it names the leg that is
    about to run, so a run that dies shows where."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def _run_path(iim, w, torch, np, precision, solver, guess, warmup, steps, profile_kernels=None, tol=1e-13,
              net=None, per_step=False, tiles=None, start=None):
    g = w.grid
    ctx = iim.Context(g, w.bodies, precision=precision, tol=tol, guess=guess, solver=solver)
    if net is not None:
        ctx.set_warm_start(iim.GUESS_NETWORK, net)
    if tiles is not None:
        ctx.set_fft_shape(tiles["row_per"], tiles["col_per"])
    if start is None:
        omega = torch.zeros((g.ny, g.nx), dtype=torch.float64, device="cuda:0")
        Gamma = np.zeros(ctx.n_circ)
    else:
        omega, Gamma = start[0].clone(), np.array(start[1], dtype=np.float64)
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
    c0 = ctx.counters()
    iters, rounds, res0 = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if per_step:
        # Krylov paths synchronise inside every solve anyway: one call per step
        # to collect the statistics of every stage
        for _ in range(steps):
            Gamma, st = ctx.rk3_steps(omega, Gamma, w.dt, 1)
            iters += st["iters"]
            rounds += st["refine_rounds"]
            res0 += st["res0"]
    else:
        Gamma, st = ctx.rk3_steps(omega, Gamma, w.dt, steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    c1 = ctx.counters()
    d = {k: c1[k] - c0[k] for k in c1}
    res = {"value": g.nx * g.ny * steps / secs, "ms_per_step": 1e3 * secs / steps, "steps": steps,
           "krylov": {"tol": tol, "solves": d["solves"], "iterations": d["krylov_iterations"],
                      "iterations_per_solve": d["krylov_iterations"] / max(1, d["solves"]),
                      "fp32_products": d["fp32_products"],
                      "initial_residual_matvecs": d["initial_residual_matvecs"]}}
    if per_step:
        res["krylov"]["refine_rounds_per_solve"] = float(np.mean(rounds)) if rounds else 0.0
        res["krylov"]["median_initial_residual"] = float(np.median(res0)) if res0 else None
        if net is not None:
            res["krylov"]["network_guesses_kept"] = d["network_kept"]
            res["krylov"]["network_guesses_rejected"] = d["network_rejected"]
    return ctx, omega, Gamma, res, pre


# Reynolds numbers of the recorded runs, in hundredths of the workload's own
# (the held-out evaluation run is the workload itself, 100); the middle one is
# the validation run
TRAIN_RE = (60, 80, 120, 150, 200, 250, 300)


def _train_network(iim, w, torch, np, runs, steps, iters):
    """The learned guess's data and training: `runs` runs shaped like the
    workload (same grid, its bodies moved by a seeded sub-cell offset) at
    Reynolds numbers re / 100 times the workload's, re from TRAIN_RE (the
    viscosity scaled), impulsively started and advanced `steps` steps with
    the dense solver while every stage solve is recorded; one run (the middle
    re) is held out for validation, the others train one network (on the
    GPU, the library's own kernels) in chunks, keeping the parameters with the
    lowest validation loss.  The workload's own run (re 100, bodies in place)
    is never seen."""
    import dataclasses
    res = list(TRAIN_RE[:max(2, min(runs, len(TRAIN_RE)))])
    val_re = res[len(res) // 2]
    rng = np.random.default_rng(11)
    g0 = w.grid
    ctxs, offsets = {}, {}
    t0 = time.perf_counter()
    for re in res:
        dx, dy = (rng.uniform(-0.5, 0.5, 2) * g0.h).tolist()
        bodies = [dataclasses.replace(b, points=b.points + np.array([dx, dy]),
                                      center=(b.center[0] + dx, b.center[1] + dy)) for b in w.bodies]
        grid = dataclasses.replace(g0, nu=g0.nu * 100.0 / re)
        c = iim.Context(grid, bodies, solver=iim.SOLVER_DIRECT)
        c.record_solves(3 * steps)
        om = torch.zeros((grid.ny, grid.nx), dtype=torch.float64, device="cuda:0")
        c.rk3_steps(om, np.zeros(c.n_circ), w.dt, steps)
        ctxs[re], offsets[re] = c, (dx, dy)
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    train = [ctxs[r] for r in res if r != val_re]
    net = iim.Network(bf16=True, seed=0)
    chunk = max(1, min(iters, 250))
    best, curve, train_loss = (float("inf"), None, 0), [], []
    t0 = time.perf_counter()
    done = 0
    while done < iters:
        k = min(chunk, iters - done)
        losses = iim.warm_start_train_multi(train, net, iters=k, batch=64, lr=1e-3, seed=1 + done)
        done += k
        vl, nval = ctxs[val_re].warm_start_loss(net)
        curve.append((done, float(np.mean(losses[-min(50, k):])), vl))
        train_loss.append(losses)
        if vl < best[0]:
            best = (vl, net.get(), done)
    net.set(best[1])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    losses = np.concatenate(train_loss)
    recorded = {re: ctxs[re].warm_start_stats()["recorded"] for re in res}
    info = {"protocol": "runs shaped like the workload (its bodies moved by seeded sub-cell offsets) at re/100 "
                        "times its Reynolds number, re in %s, %d steps each from rest with every stage solve "
                        "recorded; %d runs train, the re %d run validates (the parameters with the lowest "
                        "validation loss are kept); evaluated on the workload's own run (re 100), never seen in "
                        "training" % (list(res), steps, len(train), val_re),
            "recorded_solves": recorded, "train_re": [r for r in res if r != val_re], "validation_re": val_re,
            "centre_offsets": {r: offsets[r] for r in res}, "record_s": t_rec, "train_s": t_train,
            "adam_steps": iters, "batch": 64, "validation_samples": nval,
            "loss_first100": float(losses[:100].mean()), "loss_last100": float(losses[-100:].mean()),
            "curve_step_trainloss_valloss": curve, "kept_step": best[2], "kept_validation_loss": best[0],
            "network": "4 circular conv1d layers, kernel 5, width 128, GELU; BF16 matrix-core products "
                       "(16x16x32 MFMA, LDS-staged operands), FP32 accumulation"}
    for c in ctxs.values():
        c.close()
    return net, info


def _segments_dev(torch, np, lengths):
    seg0, segl, pos, start = [], [], [], 0
    for L in lengths:
        seg0 += [start] * L
        segl += [L] * L
        pos += list(range(L))
        start += L
    return torch.as_tensor(np.array([seg0, segl, pos], dtype=np.int32), device="cuda:0")


def _net_roofline(iim, torch, np, B=64, P=384, reps=50):
    """The network's matrix-core throughput: forward passes and training
    steps (forward, backward, Adam) at the training batch shape (B sequences
    of P control points), and one forward pass at batch 1 (the inference
    inside a solve), timed with HIP events on the network's stream; FLOPs are
    the GEMMs' 2 M N K."""
    net = iim.Network(bf16=True, seed=0)
    cin, width, layers = net.shape
    chans = [cin] + [width] * (layers - 1) + [1]
    gen = torch.Generator(device="cuda:0").manual_seed(5)
    x = torch.randn((B, P, cin), generator=gen, device="cuda:0", dtype=torch.float32)
    t = torch.randn((B, P), generator=gen, device="cuda:0", dtype=torch.float32)
    y = torch.zeros((B, P), device="cuda:0", dtype=torch.float32)
    seq = _segments_dev(torch, np, [P])
    taps = 5
    fwd = sum(2.0 * B * P * taps * a * b for a, b in zip(chans[:-1], chans[1:]))
    bwd_w = fwd
    bwd_d = sum(2.0 * B * P * taps * a * b for a, b in zip(chans[1:-1], chans[2:]))
    out = {}
    for _ in range(5):
        net.forward(x, seq, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        net.forward(x, seq, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out["forward"] = {"batch": B, "P": P, "ms": ms, "gflop": fwd / 1e9, "tflops": fwd / (ms * 1e-3) / 1e12}
    net.train_step(x, seq, t, 1e-4)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        net.train_step(x, seq, t, 1e-4)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    tot = fwd + bwd_w + bwd_d
    out["train_step"] = {"batch": B, "P": P, "ms": ms, "gflop": tot / 1e9, "tflops": tot / (ms * 1e-3) / 1e12,
                         "note": "includes the loss copy to the host that every training step returns"}
    x1, y1 = x[:1].contiguous(), y[:1].contiguous()
    for _ in range(5):
        net.forward(x1, seq, y1)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        net.forward(x1, seq, y1)
    e1.record()
    torch.cuda.synchronize()
    out["inference_batch1_us"] = 1e3 * e0.elapsed_time(e1) / reps
    best = max(out["forward"]["tflops"], out["train_step"]["tflops"])
    out["roofline"] = {"bound": "mfma", "achieved": best, "peak": 2500.0, "unit": "TFLOP/s", "frac": best / 2500.0,
                       "dtype": "bf16 operands, fp32 accumulation"}
    net.close()
    return out


# library kernel names of the instrumented kernel ids
HIP_NAMES = {"fft_rows_fwd": "k_rows_fwd_reg", "fft_cols_conv": "k_cols_reg", "fft_rows_inv": "k_rows_inv_reg",
             "transport": "k_transport_all", "arnoldi": "k_arnoldi"}
HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(HERE, "paper_2109_13628_amd", "csrc", "kernels.hip")
# headline workloads: name -> (title of the profile summaries, generator)
WORKLOADS = {"cylinder_1024x512": "the 1024x512 free-space cylinder workload",
             "multi_body_2048": "the 2048x2048 four-body outflow workload"}


def _traffic_file(workload):
    return os.path.join(HERE, "profiles", "hbm_traffic_%s.txt" % workload)


def _src_hash():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _read_csv(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _summarize_trace(trace_dir, out, command, workload):
    """Top kernels of a --kernel-trace --stats run, and for the instrumented
    kernels the average duration per launch shape (the full-size launches of
    the RK3 steps are the largest grid)."""
    import glob
    stats = _read_csv(glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)[0])
    trace = _read_csv(glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)[0])
    lines = ["# rocprofv3 kernel trace: RK3 steps of " + WORKLOADS[workload], "",
             "command: " + command, ""]
    if "--no-autotune" in command:
        # a profiler's own overhead shifts the tuner's timings, so a profiled
        # run states its tile shapes instead of tuning them
        lines += ["FFT tile shapes: the defaults, which the autotuner keeps for this workload when bench.py "
                  "runs unprofiled (fft_tiles row_per 0, col_per 0 in its JSON line)", ""]
    lines += ["kernel | calls | avg us | total ms | share %", "---|---|---|---|---"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:16]:
        name = r["Name"].split("(")[0].replace("void ", "")
        lines.append("%s | %s | %.2f | %.3f | %.2f" % (name, r["Calls"], float(r["AverageNs"]) / 1e3,
                                                      float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    # launches inside the RK steps: from the first transport launch on (the
    # set-up before it builds the dense Schur matrix with pruned convolutions)
    t0 = min(int(r["Start_Timestamp"]) for r in trace if "k_transport_all" in r["Kernel_Name"])
    lines += ["", "launches inside the RK steps, per launch shape (grid size): calls, avg us", ""]
    for short, hip in HIP_NAMES.items():
        by = {}
        for r in trace:
            if (hip + "<" in r["Kernel_Name"] or hip + "(" in r["Kernel_Name"]) and int(r["Start_Timestamp"]) >= t0:
                by.setdefault(int(r["Grid_Size_X"]), []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        for grid in sorted(by, reverse=True):
            v = by[grid]
            lines.append("%s (%s) grid %d: %d calls, avg %.2f us" % (short, hip, grid, len(v), sum(v) / len(v) / 1e3))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _summarize_pmc(fetch_dir, write_dir, out, command, workload):
    """Mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the full-size
    launches of every instrumented kernel, and the scale that turns each
    counter into bytes: the counter reading of one plain 256 MiB device copy
    (the last copy dispatch of the run) against 256 MiB."""
    import glob
    res = {}
    for tag, d in (("fetch", fetch_dir), ("write", write_dir)):
        rows = _read_csv(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0])
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
        probe = max(copies, key=lambda r: int(r["Dispatch_Id"]))
        res[tag + "_scale"] = (256 * 1024) / float(probe["Counter_Value"])
        # dispatches inside the RK steps (from the first transport launch on)
        d0 = min(int(r["Dispatch_Id"]) for r in rows if "k_transport_all" in r["Kernel_Name"])
        for short, hip in HIP_NAMES.items():
            ks = [r for r in rows if (hip + "<" in r["Kernel_Name"] or hip + "(" in r["Kernel_Name"])
                  and int(r["Dispatch_Id"]) >= d0]
            if not ks:
                continue
            gmax = max(int(r["Grid_Size"]) for r in ks)
            v = [float(r["Counter_Value"]) for r in ks if int(r["Grid_Size"]) == gmax]
            res["%s_%s_kib" % (short, tag)] = sum(v) / len(v)
            res["%s_grid" % short] = gmax
    # the two runs differ in the counter and in the output folder
    fname, wname = os.path.basename(fetch_dir.rstrip("/")), os.path.basename(write_dir.rstrip("/"))
    lines = ["# HBM traffic per dispatch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE), full-size launches",
             "# inside the RK steps of " + WORKLOADS[workload] + "; bytes = KiB * 1024 * scale, where scale is",
             "# 256 MiB over the counter's reading for one plain 256 MiB device copy in the same run.", "",
             "command_fetch: " + command.replace("WRITE_SIZE", "FETCH_SIZE").replace(wname, fname),
             "command_write: " + command.replace("FETCH_SIZE", "WRITE_SIZE").replace(fname, wname),
             "kernel_source_sha256_16: " + _src_hash()]
    for k in sorted(res):
        lines.append("%s: %s" % (k, res[k]))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _summarize_mfma(pmc_dir, out, command):
    """Matrix-core counters of the network's GEMM kernels: per kernel
    instantiation and launch size, the mean over its dispatches of the BF16
    MFMA FLOPs (SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512) and of rocprofv3's
    MfmaUtil (MFMA busy cycles over the active cycles of all SIMDs, %)."""
    import glob
    rows = _read_csv(glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True)[0])
    per = {}
    for r in rows:
        name = r["Kernel_Name"]
        if "k_mm" not in name:
            continue
        short = name.replace("(anonymous namespace)::", "").replace("void ", "")
        short = short.split("(")[0].replace("iim::", "")
        d = per.setdefault((short, int(r["Grid_Size"])), {})
        d.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    lines = ["# Matrix-core counters of the network's GEMMs (rocprofv3 --pmc), the --net-only leg of bench.py:",
             "# forward passes and training steps at batch 64 x 384 control points, and batch-1 forward passes",
             "# (grid = threads of the launch; the small grids are the batch-1 inference layers).", "",
             "command: " + command, "",
             "kernel | grid | dispatches | BF16 GFLOP per dispatch | MfmaUtil %",
             "---|---|---|---|---"]
    for (short, grid), disp in sorted(per.items(), key=lambda kv: (kv[0][0], -kv[0][1])):
        vals = list(disp.values())
        fl = sum(v.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) * 512 for v in vals) / len(vals)
        ut = sum(v.get("MfmaUtil", 0.0) for v in vals) / len(vals)
        lines.append("%s | %d | %d | %.4f | %.2f" % (short[:90], grid, len(vals), fl / 1e9, ut))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _traffic(kernel, workload):
    """HBM bytes per full-size launch of `kernel` from the committed counter
    summary of the workload, or None when it is missing or the kernel source
    has changed since the counters were taken."""
    path = _traffic_file(workload)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != _src_hash():
        return None
    try:
        fb = float(kv[kernel + "_fetch_kib"]) * 1024 * float(kv["fetch_scale"])
        wb = float(kv[kernel + "_write_kib"]) * 1024 * float(kv["write_scale"])
    except KeyError:
        return None
    return {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb, "source": os.path.relpath(path, HERE)}


def main():
    args = _parse()
    if args.summarize_trace:
        _summarize_trace(args.summarize_trace[0], args.summarize_trace[1], args.command, args.workload)
        return
    if args.summarize_pmc:
        _summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.summarize_pmc[2], args.command,
                       args.workload)
        return
    if args.summarize_mfma:
        _summarize_mfma(args.summarize_mfma[0], args.summarize_mfma[1], args.command)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as wl
    import paper_2109_13628_amd as iim

    if args.net_only:
        print(json.dumps({"network": _net_roofline(iim, torch, np)}), flush=True)
        return
    if args.batch_only:
        try:
            res = _batch(iim, wl, torch, np, args.batch_sims, args.batch_steps)
        except Exception as e:   # reported to the parent as the leg's result
            res = {"error": repr(e)}
        print(json.dumps(res), flush=True)
        sys.exit(3 if "error" in res else 0)
    failed = []

    w = wl.cylinder() if args.workload == "cylinder_1024x512" else wl.multi_body(2048)
    g = w.grid
    prec = iim.PREC_FP64 if args.precision == "fp64" else iim.PREC_MIXED
    solver = iim.SOLVER_KRYLOV if args.solver == "krylov" else iim.SOLVER_DIRECT
    all_kernels = (1 << len(iim.KERNEL_NAMES)) - 1
    tag = "fp64" if prec == iim.PREC_FP64 else "mixed"

    # FFT tile shapes for this FFT size from the library's autotuner (timed on
    # a scratch context, outside every measurement)
    tiles = None
    if not args.no_autotune:
        _say("autotune of the FFT tile shapes")
        tctx = iim.Context(g, w.bodies, precision=prec, solver=iim.SOLVER_KRYLOV)
        tiles = tctx.autotune(reps=10)
        tctx.close()
    # headline path: warm-up (kernels timed with events only to find the dominant
    # one), then exactly `steps` timed steps without instrumentation
    _say("headline path: %d warm-up and %d timed steps on %s" % (args.warmup, args.steps, w.name))
    ctx, omega, Gamma, head, pre = _run_path(iim, w, torch, np, prec, solver, iim.GUESS_PREVIOUS,
                                             args.warmup, args.steps, profile_kernels=all_kernels, tiles=tiles)
    dominant = max(pre, key=lambda k: pre[k]["total_ms"]) if pre else "fft_cols_conv"
    total = sum(x["total_ms"] for x in pre.values()) or 1.0
    shares = {n: round(v["total_ms"] / total, 4) for n, v in pre.items()}

    # roofline of the dominant kernel: HIP events around each of its launches on
    # the context stream, over the same number of steps continuing the run;
    # then its largest launch repeated back to back between one event pair
    # (per-launch events also time the dispatch latency that back-to-back
    # launches hide, which a kernel profiler does not count)
    _say("roofline timing of %s" % dominant)
    ctx.profile(1 << iim.KERNEL_NAMES.index(dominant))
    Gamma, _ = ctx.rk3_steps(omega, Gamma, w.dt, args.steps)
    torch.cuda.synchronize()
    prof = ctx.profile_read().get(dominant, {})
    rep = None
    if dominant in ("fft_rows_fwd", "fft_cols_conv", "fft_rows_inv"):
        rep = ctx.profile_replay(dominant, 200)
        torch.cuda.synchronize()
    ctx.profile(0)
    achieved = rep["GBps"] if rep else prof.get("GBps")
    tr = _traffic(dominant, args.workload)
    roof = {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
            "frac": (achieved / 8000.0) if achieved else None,
            "traffic": tr["bytes_per_launch"] if tr else None, "traffic_detail": tr,
            "avg_us": rep["avg_us"] if rep else prof.get("avg_us"),
            "algorithmic_bytes_per_launch": rep["bytes_per_launch"] if rep else prof.get("bytes_per_launch"),
            "timing": ("HIP event pair around 200 back-to-back repeats of the kernel's full-size launch"
                       if rep else "HIP events around every launch"),
            "events_per_launch": {"avg_us": prof.get("avg_us"), "launches": prof.get("launches"),
                                  "GBps": prof.get("GBps"),
                                  "timing": "HIP events around every launch of this kernel over %d eager steps "
                                            "continuing the timed run" % args.steps}}

    paths = {tag + "_" + args.solver: head}
    warm = None
    net = None
    if not args.no_extra_workloads:
        try:
            paths.update(_extra_workloads(iim, wl, torch, np))
        except Exception as e:   # recorded; the other legs still run
            failed.append("workloads")
            paths["workloads_error"] = repr(e)
    if args.krylov_steps:
        try:
            net, warm = _krylov_paths(iim, w, torch, np, args, tiles, paths)
        except Exception as e:   # recorded; the other legs still run
            failed.append("krylov_paths")
            paths["krylov_error"] = repr(e)
        if not args.no_extra_workloads:
            try:
                paths.update(_krylov_large(iim, wl, torch, np, args.krylov_tol))
            except Exception as e:   # recorded; the other legs still run
                failed.append("krylov_large")
                paths["krylov_large_error"] = repr(e)

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
                   "fft": [ctx.info["fft_mx"], ctx.info["fft_my"]], "Re": (w.extra or {}).get("Re", 100), "dt": w.dt,
                   "precision": args.precision, "solver": args.solver, "krylov_tol_headline": 1e-13,
                   "fft_tiles": tiles,
                   "t_start": args.warmup * w.dt},
        "paths": paths,
        "warm_start": warm,
        "roofline": roof,
        "kernel_time_share_warmup": shares,
    }
    if "fp64_krylov_previous" in paths and "mixed_krylov_network" in paths:
        # the metric's named comparison on the paper's iterative solve:
        # plain FP64 GMRES against mixed precision with the learned guess
        a, b = paths["fp64_krylov_previous"], paths["mixed_krylov_network"]
        out["comparison"] = {"fp64_krylov_previous_cell_updates_per_s": a["value"],
                             "mixed_krylov_network_cell_updates_per_s": b["value"],
                             "speedup": b["value"] / a["value"],
                             "direct_fp64_cell_updates_per_s": head["value"]}
    if not args.no_cpu_baseline:
        ref_state = None
        try:
            _say("CPU baseline: the oracle over %d steps (and %d on one core)" % (args.cpu_steps,
                                                                               args.cpu_single_steps))
            cpu, ref_state = _cpu_baseline(w, args.cpu_steps, args.cpu_single_steps)
            out["cpu_baseline"] = cpu
        except Exception as e:
            failed.append("cpu_baseline")
            out["cpu_baseline"] = {"error": repr(e)}
        if ref_state is not None:
            # the state after the same steps from rest on the FP64 direct path
            # and on the mixed-precision network path (GMRES to the same
            # tolerance as 'paths') against the FP64 oracle
            try:
                _say("accuracy of the library's state against the oracle's")
                out["accuracy_vs_oracle"] = _accuracy(iim, w, torch, np, ref_state, net, args.krylov_tol)
            except Exception as e:
                failed.append("accuracy")
                out["accuracy_vs_oracle"] = {"error": repr(e)}
    if args.batch_sims:
        # in a child process: a failure there cannot take this line with it
        _say("batch of %d simulations (child process)" % args.batch_sims)
        out["batch"] = _batch_child(args)
        if "error" in out["batch"]:
            failed.append("batch")
    if failed:
        out["legs_failed"] = failed
    if args.copy_probe:
        # one copy kernel that reads and writes exactly 256 MiB: the reference
        # for converting FETCH_SIZE / WRITE_SIZE counters into bytes
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = src.numel() * 4
    # flushed at once: the line is on its way before the contexts are torn down
    print(json.dumps(out), flush=True)
    _say("result written")
    if failed:
        _say("legs failed: %s" % ", ".join(failed))
        sys.exit(3)


def _krylov_paths(iim, w, torch, np, args, tiles, paths):
    """The paper's iterative solve (GMRES with the FFT product, to a relative
    residual of args.krylov_tol) in FP64 and in mixed precision with the
    zero, previous-stage, extrapolated and learned guesses, every path timed
    over the same steps of the workload's run: the state after
    args.eval_start steps from rest (dense solver), then 3 warm-up and
    args.krylov_steps timed steps (the network's inference inside the timed
    steps).  Fills `paths`; returns the trained network and its record."""
    g = w.grid
    spin = iim.Context(g, w.bodies, solver=iim.SOLVER_DIRECT)
    om0 = torch.zeros((g.ny, g.nx), dtype=torch.float64, device="cuda:0")
    G0, _ = spin.rk3_steps(om0, np.zeros(spin.n_circ), w.dt, args.eval_start)
    torch.cuda.synchronize()
    spin.close()
    start = (om0, G0)
    net, warm = None, {}
    if args.train_runs:
        _say("warm-start network: %d recorded runs of %d steps, %d training iterations"
             % (args.train_runs, args.train_steps, args.train_iters))
        net, warm = _train_network(iim, w, torch, np, args.train_runs, args.train_steps, args.train_iters)
        _say("network matrix-core timing")
        warm["network_roofline"] = _net_roofline(iim, torch, np)
    kw = dict(warmup=3, steps=args.krylov_steps, tol=args.krylov_tol, per_step=True, tiles=tiles, start=start)
    guesses = [("zero", iim.GUESS_ZERO), ("previous", iim.GUESS_PREVIOUS), ("extrapolate", iim.GUESS_EXTRAPOLATE)]
    if net is not None:
        guesses.append(("network", iim.GUESS_NETWORK))
    for p_name, p_prec in (("fp64", iim.PREC_FP64), ("mixed", iim.PREC_MIXED)):
        for g_name, g_mode in guesses:
            _say("GMRES path %s, guess %s" % (p_name, g_name))
            c_, _, _, r_, _ = _run_path(iim, w, torch, np, p_prec, iim.SOLVER_KRYLOV, g_mode,
                                        net=net if g_mode == iim.GUESS_NETWORK else None, **kw)
            r_["t_start"] = (args.eval_start + 3) * w.dt
            paths["%s_krylov_%s" % (p_name, g_name)] = r_
            c_.close()
    base = paths["fp64_krylov_previous"]["ms_per_step"]
    warm["speedup_vs_fp64_krylov_previous"] = {k: base / v["ms_per_step"] for k, v in paths.items()
                                              if "krylov" in k and "ms_per_step" in v}
    warm["iterations_per_solve"] = {k: v["krylov"]["iterations_per_solve"] for k, v in paths.items()
                                    if "krylov" in k and "krylov" in v}
    return net, warm


def _batch_child(args):
    """The batched-serving leg in a child process (its own HIP runtime and
    device memory); its JSON object, or the failure."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--batch-only", "--batch-sims", str(args.batch_sims),
           "--batch-steps", str(args.batch_steps)]
    # the child's progress lines go straight to this process's stderr
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=args.batch_timeout)
    except subprocess.TimeoutExpired:
        return {"error": "timed out after %.0f s" % args.batch_timeout}
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    res = json.loads(lines[-1]) if lines else {}
    if r.returncode != 0 and "error" not in res:
        res["error"] = "exit status %d" % r.returncode
    return res


def _krylov_large(iim, wl, torch, np, tol, steps=3):
    """FP64 against mixed-precision GMRES (extrapolated guess, to tol) on the
    four-body 2048 x 2048 outflow configuration, where each product moves
    more bytes than at the headline size: 2 warm-up and `steps` timed steps
    from the state after 20 dense-solver steps."""
    w = wl.multi_body(2048)
    g = w.grid
    spin = iim.Context(g, w.bodies, solver=iim.SOLVER_DIRECT)
    om0 = torch.zeros((g.ny, g.nx), dtype=torch.float64, device="cuda:0")
    G0, _ = spin.rk3_steps(om0, np.zeros(spin.n_circ), w.dt, 20)
    torch.cuda.synchronize()
    spin.close()
    res = {}
    for name, prec in (("fp64", iim.PREC_FP64), ("mixed", iim.PREC_MIXED)):
        _say("multi_body_2048 GMRES %s" % name)
        c_, _, _, r_, _ = _run_path(iim, w, torch, np, prec, iim.SOLVER_KRYLOV, iim.GUESS_EXTRAPOLATE, warmup=2,
                                    steps=steps, tol=tol, per_step=True, start=(om0, G0))
        r_["fft"] = [c_.info["fft_mx"], c_.info["fft_my"]]
        r_["schur_unknowns"] = c_.info["n_affected"] + c_.info["n_circ"]
        res["multi_body_2048_outflow_krylov_%s_extrapolate" % name] = r_
        c_.close()
    return res


def _extra_workloads(iim, wl, torch, np):
    """The other single-GPU configurations, FP64 dense solver, graph replay:
    Taylor-Couette in the DST box (128 x 128, 20 steps), four nonconvex
    bodies with an outflow plane (2048 x 2048) and the cylinder of the
    headline in a periodic box (1024 x 512, mean velocity (1, 0))."""
    res = {}
    for name, w, warm, steps in (("taylor_couette_128_box", wl.taylor_couette(128), 5, 20),
                                 ("multi_body_2048_outflow", wl.multi_body(2048), 3, 10),
                                 ("periodic_cylinder_1024x512", wl.periodic_cylinder(
                                     nx=1024, ny=512, h=1.0 / 64, points=256, dt=0.0025, center=(4.0, 0.0)), 5, 20)):
        _say("workload %s: %d warm-up and %d timed steps" % (w.name, warm, steps))
        t0 = time.perf_counter()
        ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        om = torch.zeros((w.grid.ny, w.grid.nx), dtype=torch.float64, device="cuda:0")
        G = np.zeros(ctx.n_circ)
        G, _ = ctx.rk3_steps(om, G, w.dt, warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G, _ = ctx.rk3_steps(om, G, w.dt, steps)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        inf = ctx.info
        res[name] = {"value": w.grid.nx * w.grid.ny * steps / secs, "ms_per_step": 1e3 * secs / steps,
                     "steps": steps, "unit": "cell-updates/s", "nx": w.grid.nx, "ny": w.grid.ny,
                     "bodies": len(w.bodies), "schur_unknowns": inf["n_affected"] + inf["n_circ"],
                     "fft": [inf["fft_mx"], inf["fft_my"]], "dt": w.dt, "setup_s": setup,
                     "finite": bool(torch.isfinite(om).all())}
        ctx.close()
    return res


def _batch(iim, wl, torch, np, n_sims, steps):
    """Batched serving: n_sims independent simulations advanced by one HIP
    graph per batch step; aggregate throughput and batch-step latency."""
    ws = wl.batch_serving(n_sims, seed=5)
    _say("batch: creating %d simulations (dense Schur inverses, tile autotune, branch timing)" % n_sims)
    t0 = time.perf_counter()
    b = iim.Batch(ws)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    info = b.info()
    _say("batch: created in %.1f s, %d branches; warm-up steps" % (setup, info["branches"]))
    oms = [torch.zeros((w.grid.ny, w.grid.nx), dtype=torch.float64, device="cuda:0") for w in ws]
    Gs = [np.zeros(len(w.bodies)) for w in ws]
    dts = [w.dt for w in ws]
    b.step(oms, Gs, dts, 3)                  # graph capture + warm-up
    _say("batch: %d timed steps" % steps)
    st = b.step(oms, Gs, dts, steps)
    torch.cuda.synchronize()
    finite = all(bool(torch.isfinite(o).all()) for o in oms)
    b.close()
    return {"metric": "aggregate RK3 step cell-updates/s", "value": st["cells_per_step"] * steps / (st["ms_total"] * 1e-3),
            "unit": "cell-updates/s", "sims": n_sims, "steps": steps, "cells_per_step": st["cells_per_step"],
            "step_ms_p50": st["ms_p50"], "step_ms_p99": st["ms_p99"], "step_ms_max": st["ms_max"],
            "setup_s": setup, "branches": info["branches"], "branch_ms_tried": info["branch_ms"],
            "fft_tiles": info["tuning"], "finite": finite, "dtype": "f64",
            "branch_notes": info.get("notes"),
            "workload": "%d free-space simulations from rest, N x N nodes with N uniform in [256, 1024] on a 4 x 4 "
                        "domain, 1-6 seeded circles/ellipses each, u_inf = 1, Re uniform in [50, 500]" % n_sims,
            "timing": "HIP events around every batch-step graph launch"}


def _accuracy(iim, w, torch, np, ref, net, tol):
    om_ref, G_ref, n_steps, R, geo = ref
    g = w.grid
    res = {}
    for name, prec, guess in (("fp64_direct", iim.PREC_FP64, iim.GUESS_PREVIOUS),
                              ("mixed_krylov_network" if net is not None else "mixed_krylov_extrapolate",
                               iim.PREC_MIXED, iim.GUESS_NETWORK if net is not None else iim.GUESS_EXTRAPOLATE)):
        solver = iim.SOLVER_DIRECT if name == "fp64_direct" else iim.SOLVER_KRYLOV
        ctx = iim.Context(g, w.bodies, precision=prec, tol=tol, guess=guess, solver=solver)
        if guess == iim.GUESS_NETWORK:
            ctx.set_warm_start(guess, net)
        om = torch.zeros((g.ny, g.nx), dtype=torch.float64, device="cuda:0")
        G, _ = ctx.rk3_steps(om, np.zeros(ctx.n_circ), w.dt, n_steps)
        U = torch.zeros((g.ny + 2, g.nx + 2), dtype=torch.float64, device="cuda:0")
        V = torch.zeros_like(U)
        ctx.reconstruct(om, G, None, U, V)
        torch.cuda.synchronize()
        a = R.reconstruct(om_ref, G_ref)
        fl = np.pad(geo.fluid, 1)
        uv = np.stack([U.cpu().numpy()[fl], V.cpu().numpy()[fl]])
        uv_ref = np.stack([a.U[fl], a.V[fl]])
        om_gpu = om.cpu().numpy()[geo.fluid]
        res[name] = {"steps": n_steps, "krylov_tol": tol if solver == iim.SOLVER_KRYLOV else None,
                     "velocity_rel_error": float(np.linalg.norm(uv - uv_ref) / np.linalg.norm(uv_ref)),
                     "vorticity_rel_error": float(np.linalg.norm(om_gpu - om_ref[geo.fluid]) /
                                                  np.linalg.norm(om_ref[geo.fluid]))}
        ctx.close()
    return res


def _cpu_baseline(w, steps, single_steps):
    """The FP64 oracle, timed on this host's cores over a bounded sample of the
    same workload (RK3 steps from rest; set-up excluded), and on one core over
    a few more steps.  Also returns its state after the multi-core steps for
    the accuracy check.  The host share of one GPU is 16 cores, so at most 16
    threads are used."""
    import numpy as np
    import scipy.fft as sfft
    from oracle import geometry as OG, ns as ONS
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:          # BLAS threads then stay as configured
        threadpool_limits = None
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
    cpu = {"value": w.grid.nx * w.grid.ny * steps / secs, "unit": "cell-updates/s", "cores": cores,
           "kind": "oracle",
           "sample": "%d RK3 steps of the same 1024x512 cylinder workload after one set-up step from rest "
                     "(FP64 NumPy/SciPy, dense Schur LU, scipy.fft workers=%d)" % (steps, cores),
           "cpu_model": _cpu_model()}
    if single_steps:
        om1, G1 = om.copy(), G.copy()
        limit = threadpool_limits(limits=1) if threadpool_limits else None
        try:
            with sfft.set_workers(1):
                t0 = time.perf_counter()
                for _ in range(single_steps):
                    om1, G1 = st.step(om1, G1, w.dt)
                secs1 = time.perf_counter() - t0
        finally:
            if limit is not None:
                limit.unregister() if hasattr(limit, "unregister") else limit.__exit__(None, None, None)
        cpu["single_core"] = {"value": w.grid.nx * w.grid.ny * single_steps / secs1, "cores": 1,
                              "steps": single_steps, "blas_threads_limited": threadpool_limits is not None}
    return cpu, (om, G, steps + 1, st.rec, geo)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
