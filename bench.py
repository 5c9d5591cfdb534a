#!/usr/bin/env python3
"""Throughput of the explicit finite-volume Gatenby-Gawlinski step on one MI355X.

Workload: the 4096 x 4096 layered-tissue grid (64 seeded Voronoi regions with
piecewise-constant anisotropic tensors and two-cell low-diffusion membranes along
region borders, central tumour disk, delta1 = 12.5), stepped at 0.9 of the
explicit stability bound with the masses logged every 500 steps.  Inputs are
synthetic (seeded) and resident in HBM before the timed region starts.

One bench step = one forward-Euler step of the whole grid (one launch of the
step kernel); the timed region also contains the mass diagnostics every 500
steps.  The headline value is FP64; the compensated-FP32 and plain-FP32 variants
are measured beside it.  The oracle is timed on the host cores on a bounded
sample of the same workload.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

PEAK_HBM_GBS = 8000.0            # MI355X HBM3E peak
# Algorithmic HBM bytes per cell-update of one step: read u, v, w, a, b, c and
# write u, v, w once (the compensated state reads and writes a second word of u,
# v and w).
BYTES_PER_CELL = {"f64": 72, "f32c": 60, "f32": 36}
KERNEL_NAME = {"f64": "step_kernel<double, false, 1>", "f32c": "step_kernel<float, true, 2>",
               "f32": "step_kernel<float, false, 2>"}
METRIC = "Gcell-updates/s + % HBM peak, 4096² aniso FV step FP32/FP64; adjoint/fwd ratio"
# Algorithmic floating-point operations per cell-update (each face flux counted
# once, shared by its two cells): x/y faces of W 2 x 10, tangential differences
# 4, divergence of W 5, faces of V 2 x 6, divergence of V 5, reactions 14,
# Euler updates 6.  The library evaluates them without FMA contraction, so each
# is one vector operation.
FLOPS_PER_CELL = 66
# MI355X vector FP64 (and non-packed FP32) rate without FMA: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz = 39.3e12 operations per second (78.6 TFLOP/s counts an FMA
# as two operations).
PEAK_VALU_TFLOPS = 39.3
MASS_EVERY = 500


def measured_traffic(variant, kernel="single"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when a step kernel source changed since the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "profiles", "step_kernel_traffic.json")) as f:
            data = json.load(f)
        h = hashlib.sha256()
        for src in data["kernel_sources"]:
            with open(os.path.join(here, src), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    if h.hexdigest() != data.get("kernel_sources_sha256"):
        return None
    t = data["bytes_per_launch"].get(f"{variant}/{kernel}")
    return None if t is None else t["read"] + t["write"]


def roofline_of(variant, r):
    """Roofline of the kernel that dominates a timed run.  A single-step launch
    moves BYTES_PER_CELL bytes per cell and is HBM-bound; a fused launch reads
    and writes the same bytes for K steps and is bound by vector arithmetic, so
    it is placed against the non-FMA vector rate (FLOPS_PER_CELL per
    cell-update), with its HBM figures beside it."""
    if r["fused_steps"] == 1 and not r["tuning"].get("lane_shift"):
        return {"bound": "hbm", "achieved": r["achieved_GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": r["achieved_GBs"] / PEAK_HBM_GBS, "traffic": measured_traffic(variant),
                "kernel": KERNEL_NAME[variant], "kernel_avg_us": r["kernel_avg_us"],
                "bytes_per_cell_update": BYTES_PER_CELL[variant]}
    K = r["fused_steps"]
    if r["tuning"].get("lane_shift"):
        kname = f"fused_dpp_kernel<{'double' if variant == 'f64' else 'float'}, {str(variant == 'f32c').lower()}, " \
                f"{1 if variant == 'f64' else 2}, {K}>"
    else:
        kname = f"fused_kernel<{'double' if variant == 'f64' else 'float'}, {str(variant == 'f32c').lower()}, " \
                f"{1 if variant == 'f64' else 2}, {64 if (r['tuning']['threads'] == 64 or K == 4) else 128}, {K}>"
    return {"bound": "alu", "achieved": r["achieved_TFLOPs"], "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": r["achieved_TFLOPs"] / PEAK_VALU_TFLOPS, "traffic": measured_traffic(variant, f"fused{K}"),
            "kernel": kname,
            "kernel_avg_us": r["kernel_avg_us"], "steps_per_launch": K,
            "flops_per_cell_update": FLOPS_PER_CELL,
            "hbm_algorithmic_GBs": r["achieved_GBs"], "hbm_effective_GBs": r["effective_GBs"],
            "hbm_frac_effective": r["effective_GBs"] / PEAK_HBM_GBS}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_variant(pk, torch, w, dtype, steps, warmup, tune, force=None):
    """Time `steps` steps (after `warmup`) of the workload with the default
    single-step shape, or with the shape the autotuner picks (tune=True: the
    search runs before the timed region, on the same data, and restores it)."""
    stream = torch.cuda.current_stream()
    ctx = pk.Context(w.nx, w.ny, w.lx, w.ly, dtype=dtype, stream=stream.cuda_stream)
    ctx.set_params(w.params)
    ctx.set_tensor_eig(*w.eig)
    ctx.set_state(w.u0, w.v0, w.w0)
    dt = ctx.stable_dt(w.safety)
    if force is not None:
        ctx.set_tuning(*force)
        tuning = ctx.get_tuning()
    else:
        tuning = ctx.autotune(dt, trial_steps=12) if tune else ctx.get_tuning()
    K = max(1, tuning["fused_steps"])
    ctx.step(dt, warmup)
    torch.cuda.synchronize()
    segs = []
    masses = []
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    done = 0
    while done < steps:
        n = min(steps - done, MASS_EVERY - (done % MASS_EVERY))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.step(dt, n)
        e1.record(stream)
        segs.append((e0, e1, n))
        done += n
        if done % MASS_EVERY == 0:
            masses.append(ctx.diagnostics()["mass"].tolist())
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    step_ms = sum(a.elapsed_time(b) for a, b, _ in segs)
    launches = sum(n // K + n % K for _, _, n in segs)
    kernel_us = 1e3 * step_ms / launches          # average launch (K steps when fused)
    cells = w.nx * w.ny
    value = cells * steps / (total_ms * 1e-3) / 1e9
    d = ctx.diagnostics()
    ctx.close()
    per_launch_bytes = BYTES_PER_CELL[dtype] * cells
    return {
        "value": value, "ms_per_step": total_ms / steps, "kernel_avg_us": kernel_us,
        "wall_s": wall, "dt": dt, "tuning": tuning, "fused_steps": K,
        "achieved_GBs": per_launch_bytes / (kernel_us * 1e-6) / 1e9,
        "effective_GBs": K * per_launch_bytes / (kernel_us * 1e-6) / 1e9,
        "achieved_TFLOPs": FLOPS_PER_CELL * K * cells / (kernel_us * 1e-6) / 1e12,
        "mass_log": masses, "cfl": d["cfl"],
    }


def time_adjoint(pk, torch, steps=5000):
    """Gradient workload: 512^2 smooth anisotropic tensor, `steps` steps, loss of
    the final v and w; forward with square-root checkpoints, then the native
    reverse sweep (recompute + adjoint).  Returns times and their ratio."""
    from paper_2006_01748_amd import autograd as ag
    from paper_2006_01748_amd import workloads as wl
    w = wl.cfg4(steps=steps)
    stream = torch.cuda.current_stream()
    ctx = pk.Context(w.nx, w.ny, dtype="f64", stream=stream.cuda_stream)
    ctx.set_params(w.params)
    ctx.set_tensor_eig(*w.eig)
    dt = ctx.stable_dt(w.safety)
    every = ag.default_every(w.steps)
    sb = ctx.state_bytes()
    ckpt = torch.empty(-(-w.steps // every) * sb, dtype=torch.uint8, device="cuda")
    work = torch.empty((every - 1) * sb, dtype=torch.uint8, device="cuda")
    lam = [torch.zeros((w.ny, w.nx), dtype=torch.float64, device="cuda") for _ in range(3)]
    g = [torch.empty((w.ny, w.nx), dtype=torch.float64, device="cuda") for _ in range(3)]
    res = {}
    for rep in range(2):                    # first pass warms up
        ctx.set_state(w.u0, w.v0, w.w0)
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        ctx.step_checkpointed(dt, w.steps, every, ckpt)
        e1.record(stream)
        for x in lam:
            x.fill_(1e-6)
        ctx.adjoint_run(dt, w.steps, every, ckpt, work, lam, g)
        e2.record(stream)
        torch.cuda.synchronize()
        res = {"forward_ms": e0.elapsed_time(e1), "backward_ms": e1.elapsed_time(e2)}
    # per-launch kernel times: plain steps vs adjoint steps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.set_state(w.u0, w.v0, w.w0)
    torch.cuda.synchronize()
    e0.record(stream)
    ctx.step(dt, 1000)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_us = 1e3 * e0.elapsed_time(e1) / 1000
    ctx.close()
    ratio = res["backward_ms"] / res["forward_ms"]
    return {"workload": f"{w.nx}x{w.ny} smooth anisotropic tensor, {w.steps} steps, checkpoint every "
                        f"{every} steps (forward stores {-(-w.steps // every)} states, backward recomputes "
                        f"each segment and runs the adjoint through it)",
            "dtype": "f64", "forward_ms": res["forward_ms"], "backward_ms": res["backward_ms"],
            "backward_over_forward": ratio, "step_us": fwd_us,
            "adjoint_step_us_est": 1e3 * res["backward_ms"] / w.steps - fwd_us}


def time_ensemble(pk, torch, count=256, steps=500, loop_steps=50, force=None):
    """Ensemble workload: `count` instances (sides 64..512, own parameters, tensor
    and dt), compensated FP32.  Batched graph-replayed run versus a loop of
    single-instance launches of the same instances on the same GPU."""
    from paper_2006_01748_amd import workloads as wl
    ws = wl.cfg3(count, steps)
    # graph capture needs a stream other than the null stream: time on our own
    stream = torch.cuda.Stream()
    cells = sum(w.cells for w in ws)
    b = pk.Batch([(w.nx, w.ny) for w in ws], dtype="f32c", stream=stream.cuda_stream)
    dts = []
    for i, w in enumerate(ws):
        c = b[i]
        c.set_params(w.params)
        c.set_tensor_eig(*w.eig)
        c.set_state(w.u0, w.v0, w.w0)
        dts.append(c.stable_dt(w.safety))
        b.set_dt(i, dts[-1])
    tuned = b.autotune(trial_steps=10) if force is None else {"threads": force[0], "rows_per_strip": force[1]}
    b.set_tuning(threads=tuned["threads"], rows_per_strip=tuned["rows_per_strip"], graph_steps=50)
    b.run(50)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1)
    b.close()
    ctxs = []
    for i, w in enumerate(ws):
        c = pk.Context(w.nx, w.ny, dtype="f32c", stream=stream.cuda_stream)
        c.set_params(w.params)
        c.set_tensor_eig(*w.eig)
        c.set_state(w.u0, w.v0, w.w0)
        ctxs.append(c)
    for c, dt in zip(ctxs, dts):
        c.step(dt, 5)
    torch.cuda.synchronize()
    e0.record(stream)
    for c, dt in zip(ctxs, dts):
        c.step(dt, loop_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1)
    for c in ctxs:
        c.close()
    batch_rate = cells * steps / (batch_ms * 1e-3) / 1e9
    loop_rate = cells * loop_steps / (loop_ms * 1e-3) / 1e9
    return {"workload": f"{count} instances, sides 64..512 (total {cells} cells), own parameters, tensor and dt, "
                        f"compensated FP32", "dtype": "f32c", "tuning": tuned,
            "batched_Gcell_s": batch_rate, "batched_ms_per_step": batch_ms / steps,
            "loop_of_single_launches_Gcell_s": loop_rate, "loop_ms_per_step": loop_ms / loop_steps,
            "speedup": batch_rate / loop_rate,
            "batched_GBs": 60 * cells * steps / (batch_ms * 1e-3) / 1e9}


def copy_ceiling(torch, nbytes=1 << 30, reps=20):
    """Plain device-to-device copy bandwidth (read + write bytes per second)."""
    x = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(w, steps):
    import oracle
    a, b, c = oracle.tensor_from_eig(*w.eig)
    dt = oracle.stable_dt(a, b, c, w.params[2], w.safety)
    t0 = time.perf_counter()
    oracle.run(w.u0, w.v0, w.w0, a, b, c, w.params, dt, steps)
    sec = time.perf_counter() - t0
    return {"value": w.nx * w.ny * steps / sec / 1e9, "unit": "Gcell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} FP64 steps of the same {w.nx}x{w.ny} layered-tissue grid, one thread "
                      f"({sec:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=4096, help="grid side (4096 for the standard workload)")
    ap.add_argument("--variants", default="f64,f32c,f32")
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-ceiling", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="time the default single-step shape only")
    ap.add_argument("--force-tuning", default="",
                    help="VARIANT=ROWS,THREADS,FUSED[;...]: use these launch shapes instead of the autotuner "
                         "(reproducible profiling)")
    ap.add_argument("--ensemble-tuning", default="",
                    help="THREADS,ROWS: batched launch shape instead of the batch autotuner")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): this build has no multi-GPU "
              "path; the step would shard by row slabs with halo exchange.", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs as a single process on one GPU", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2006_01748_amd as pk
    from paper_2006_01748_amd import workloads as wl

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    log(f"generating {args.n}x{args.n} layered-tissue workload")
    w = wl.cfg2(n=args.n)
    variants = [v for v in args.variants.split(",") if v]
    res, single = {}, {}
    for v in variants:
        log(f"timing {v}, single-step kernel: {args.warmup} warm-up + {args.steps} timed steps")
        single[v] = time_variant(pk, torch, w, v, args.steps, args.warmup, tune=False)
        log(f"  {v} single-step: {single[v]['value']:.2f} Gcell/s, kernel {single[v]['kernel_avg_us']:.1f} us, "
            f"{single[v]['achieved_GBs']:.0f} GB/s ({100 * single[v]['achieved_GBs'] / PEAK_HBM_GBS:.1f}% of peak)")
        if not args.no_tune:
            log(f"timing {v}, autotuned shape")
            forced = dict(item.split("=") for item in args.force_tuning.split(";") if item)
            force = tuple(int(x) for x in forced[v].split(",")) if v in forced else None
            res[v] = time_variant(pk, torch, w, v, args.steps, args.warmup, tune=True, force=force)
            log(f"  {v} tuned {res[v]['tuning']}: {res[v]['value']:.2f} Gcell/s, launch {res[v]['kernel_avg_us']:.1f} us "
                f"({res[v]['fused_steps']} steps), effective {res[v]['effective_GBs']:.0f} GB/s")
        else:
            res[v] = single[v]
    adj = None
    if not args.no_adjoint:
        log("timing the gradient workload (forward with checkpoints, reverse sweep)")
        adj = time_adjoint(pk, torch)
        log(f"  backward/forward = {adj['backward_over_forward']:.2f}")
    ens = None
    if not args.no_ensemble:
        log("timing the ensemble (batched graph vs loop of single launches)")
        ens = time_ensemble(pk, torch, force=tuple(int(x) for x in args.ensemble_tuning.split(","))
                            if args.ensemble_tuning else None)
        log(f"  batched {ens['batched_Gcell_s']:.1f} Gcell/s vs loop {ens['loop_of_single_launches_Gcell_s']:.1f} "
            f"Gcell/s (x{ens['speedup']:.2f})")
    ceiling = None if args.no_copy_ceiling else copy_ceiling(torch)
    base = None
    if not args.no_cpu_baseline:
        log(f"timing the oracle on {args.cpu_steps} steps")
        base = cpu_baseline(w, args.cpu_steps)

    head = variants[0]
    r = res[head]
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {
            "workload": f"layered tissue {w.nx}x{w.ny}: 64 Voronoi regions with anisotropic tensors "
                        f"and membranes, central disk, delta1={w.params[0]}, dt=0.9 of the "
                        f"stability bound, masses every {MASS_EVERY} steps",
            "grid": [w.nx, w.ny], "params": list(w.params), "dt": r["dt"],
        },
        "roofline": roofline_of(head, r),
        "single_step_kernel": {
            "kernel": KERNEL_NAME[head], "value": single[head]["value"],
            "kernel_avg_us": single[head]["kernel_avg_us"], "bound": "hbm",
            "achieved": single[head]["achieved_GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": single[head]["achieved_GBs"] / PEAK_HBM_GBS, "traffic": measured_traffic(head),
            "bytes_per_cell_update": BYTES_PER_CELL[head]},
        "cpu_baseline": base,
        "variants": {v: {"tuned": res[v]["tuning"], "value": res[v]["value"],
                         "launch_avg_us": res[v]["kernel_avg_us"], "roofline": roofline_of(v, res[v]),
                         "single_step": {"value": single[v]["value"], "kernel_avg_us": single[v]["kernel_avg_us"],
                                         "achieved_GBs": single[v]["achieved_GBs"],
                                         "frac": single[v]["achieved_GBs"] / PEAK_HBM_GBS,
                                         "traffic": measured_traffic(v)}}
                     for v in variants},
        "adjoint": adj,
        "ensemble": ens,
        "copy_ceiling_GBs": ceiling,
        "mass_log": r["mass_log"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
