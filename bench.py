#!/usr/bin/env python3
"""Throughput of the explicit finite-volume Gatenby-Gawlinski step on one MI355X.

Workload: the 4096 x 4096 layered-tissue grid (64 seeded Voronoi regions with
piecewise-constant anisotropic tensors and two-cell low-diffusion membranes along
region borders, central tumour disk, delta1 = 12.5), stepped at 0.9 of the
explicit stability bound with the masses logged every 500 steps.  Inputs are
synthetic (seeded) and resident in HBM before the timed region starts.

One bench step = one forward-Euler step of the whole grid.  The headline runs
the library's fastest launch shape for the variant (several steps per launch,
the shapes below, which the library's autotuner picks on MI355X; --autotune
runs the search instead); the single-step kernel is timed beside it.  The
timed region also contains the mass diagnostics every 500 steps.  The headline
value is FP64; the compensated-FP32 and plain-FP32 variants are measured beside
it.  The oracle is timed on the host cores on a bounded sample of the same
workload.

Prints one JSON line.  With --summarize-profiles DIR it instead writes the
rocprofv3 summaries under profiles/ from the CSV output of the commands in
PROFILE_COMMANDS (run with DIR as $P).
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
# Launch shapes of the headline runs: (rows per strip, threads, steps per
# launch, lane-shift kernels: 1, or 2 for wide lanes).  Rows 0 is the library's
# height, the tallest strips whose waves fill the resident slots once.
HEADLINE_SHAPE = {"f64": (0, 64, 4, 2), "f32c": (0, 64, 4, 1), "f32": (0, 64, 4, 2)}
# The single-step kernel (one step per launch, the library's width and height).
SINGLE_SHAPE = (0, 0, 1, 0)
METRIC = "Gcell-updates/s + % HBM peak, 4096² aniso FV step FP32/FP64; adjoint/fwd ratio"
# Algorithmic floating-point operations per cell-update (each face flux counted
# once, shared by its two cells): x/y faces of W 2 x 10, tangential differences
# 4, divergence of W 5, faces of V 2 x 6, divergence of V 5, reactions 14,
# Euler updates 6.  FP64 and the compensated FP32 state evaluate them without
# fused multiply-adds, each one vector operation; plain FP32 fuses ten
# multiply-add pairs into single operations (its valu_frac still counts flops).
FLOPS_PER_CELL = 66
# MI355X vector FP64 (and non-packed FP32) rate without FMA: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz = 39.3e12 operations per second (78.6 TFLOP/s counts an FMA
# as two operations).
PEAK_VALU_TFLOPS = 39.3
MASS_EVERY = 500


def kernel_name(variant, tuning):
    """Name of the kernel a launch shape runs, as rocprofv3 prints it (without
    namespace and arguments), and its key in the traffic summary."""
    T = "double" if variant == "f64" else "float"
    comp = "true" if variant == "f32c" else "false"
    cpl = 1 if variant == "f64" else 2
    K = max(1, tuning.get("fused_steps", 1))
    if tuning.get("lane_shift") == 2:          # wide lanes: 16 bytes of columns per lane
        return f"fused_dpp_kernel<{T}, {comp}, {2 * cpl}, {K}>", f"wide{K}"
    if tuning.get("lane_shift"):
        return f"fused_dpp_kernel<{T}, {comp}, {cpl}, {K}>", f"lanes{K}"
    nt = tuning.get("threads") or 256
    return f"step_kernel<{T}, {comp}, {cpl}, {nt}>", "single"


# Sources of the three-dimensional kernels; every other csrc file belongs to the
# two-dimensional ones.
SOURCES_3D = ("ggfv3.hip", "ggfv_dpp.hpp", "ggfv_internal.hpp")


def traffic_sources(here, family="2d"):
    """Kernel sources whose change invalidates a counter summary of `family`
    (with the build script, whose flags shape the compiled kernels)."""
    out = [os.path.join("paper_2006_01748_amd", "build.py")]
    for d, _, fs in os.walk(os.path.join(here, "paper_2006_01748_amd", "csrc")):
        for f in fs:
            if not f.endswith((".hip", ".hpp")):
                continue
            keep = f in SOURCES_3D if family == "3d" else f != "ggfv3.hip"
            if keep:
                out.append(os.path.relpath(os.path.join(d, f), here))
    return sorted(set(out))


def sources_digest(here, srcs):
    import hashlib
    h = hashlib.sha256()
    for src in srcs:
        with open(os.path.join(here, src), "rb") as f:
            h.update(src.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(variant, tuning, rows):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when no summary covers this kernel and strip height, or a kernel source
    changed since the counters were taken."""
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "profiles", "step_kernel_traffic.json")) as f:
            data = json.load(f)
        if sources_digest(here, data["kernel_sources"]) != data.get("kernel_sources_sha256"):
            return None
        if data["kernel_sources"] != traffic_sources(here):
            return None
    except (OSError, KeyError, ValueError):
        return None
    _, key = kernel_name(variant, tuning)
    t = data["bytes_per_launch"].get(f"{variant}/{key}")
    if t is None or t.get("rows") != rows:
        return None
    return t["read"] + t["write"]


def measured_traffic3(dtype, shape):
    """HBM bytes per launch of the 3D step kernel from the committed counter
    summary, or None (no summary for this kernel and launch shape, or a 3D
    kernel source changed since)."""
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "profiles", "step3_kernel_traffic.json")) as f:
            data = json.load(f)
        if data["kernel_sources"] != traffic_sources(here, "3d"):
            return None
        if sources_digest(here, data["kernel_sources"]) != data.get("kernel_sources_sha256"):
            return None
    except (OSError, KeyError, ValueError):
        return None
    t = data["bytes_per_launch"].get(dtype)
    if t is None or t.get("launch_shape") != shape:
        return None
    return t["read"] + t["write"]


def roofline_of(variant, r):
    """Roofline of the kernel that dominates a timed run, against HBM: the
    algorithmic bytes of one launch (BYTES_PER_CELL per cell; a fused launch
    moves them once for its K steps) over the average launch time.  A fused
    launch also carries its vector figures: FLOPS_PER_CELL per cell-update
    against the non-FMA vector rate, and the measured VALU issue utilisation
    (counter summary) where it is known."""
    kname, _ = kernel_name(variant, r["tuning"])
    traffic = measured_traffic(variant, r["tuning"], r["rows"])
    hbm = {"achieved": r["achieved_GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": r["achieved_GBs"] / PEAK_HBM_GBS}
    out = {"bound": "hbm", **hbm, "traffic": traffic, "kernel": kname, "kernel_avg_us": r["kernel_avg_us"],
           "bytes_per_cell_update": BYTES_PER_CELL[variant]}
    if r["fused_steps"] > 1 or r["tuning"].get("lane_shift"):
        out.update({"steps_per_launch": r["fused_steps"],
                    "hbm_algorithmic_bytes_per_launch": BYTES_PER_CELL[variant] * r["cells"],
                    "hbm_effective_GBs": r["effective_GBs"],
                    "hbm_frac_effective": r["effective_GBs"] / PEAK_HBM_GBS,
                    "flops_per_cell_update": FLOPS_PER_CELL,
                    "valu_TFLOPs": r["achieved_TFLOPs"], "valu_peak_TFLOPs": PEAK_VALU_TFLOPS,
                    "valu_frac": r["achieved_TFLOPs"] / PEAK_VALU_TFLOPS})
        issue = measured_valu(variant, r["tuning"], r["rows"])
        if issue is not None:
            out["valu_issue_frac"] = issue / (VALU_ISSUE_PER_S * r["kernel_avg_us"] * 1e-6)
    return with_measured(out, r["kernel_avg_us"])


def measured_valu(variant, tuning, rows):
    """VALU wave instructions per launch from the committed counter summary, or
    None (no summary for this kernel and strip height, or a kernel source
    changed since the counters were taken)."""
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "profiles", "step_kernel_valu.json")) as f:
            data = json.load(f)
        if data["kernel_sources"] != traffic_sources(here):
            return None
        if sources_digest(here, data["kernel_sources"]) != data.get("kernel_sources_sha256"):
            return None
    except (OSError, KeyError, ValueError):
        return None
    _, key = kernel_name(variant, tuning)
    t = data["valu_per_launch"].get(f"{variant}/{key}")
    if t is None or t.get("rows") != rows:
        return None
    return t["valu"]


def with_measured(roof, kernel_us):
    """Add the measured HBM rate (the counters' bytes per launch over the live
    launch time) to a roofline object whose `traffic` is known."""
    if roof.get("traffic") is not None:
        roof["hbm_measured_GBs"] = roof["traffic"] / (kernel_us * 1e-6) / 1e9
        roof["hbm_measured_frac"] = roof["hbm_measured_GBs"] / PEAK_HBM_GBS
    return roof


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_variant(pk, torch, w, dtype, steps, warmup, tune, force=None):
    """Time `steps` steps (after `warmup`) of the workload in the launch shape
    `force`, on the single-step kernel (tune=False, no shape given), or with the
    shape the autotuner picks (tune=True: the search runs before the timed
    region, on the same data, and restores it)."""
    stream = torch.cuda.current_stream()
    ctx = pk.Context(w.nx, w.ny, w.lx, w.ly, dtype=dtype, stream=stream.cuda_stream)
    ctx.set_params(w.params)
    ctx.set_tensor_eig(*w.eig)
    ctx.set_state(w.u0, w.v0, w.w0)
    dt = ctx.stable_dt(w.safety)
    if force is None and not tune:
        force = SINGLE_SHAPE
    if force is not None:
        ctx.set_tuning(*force)
        tuning = ctx.get_tuning()
    else:
        tuning = ctx.autotune(dt, trial_steps=12)
    rows = tuning["rows_per_strip"]          # 0: the library's default strip height
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
        "wall_s": wall, "dt": dt, "tuning": tuning, "fused_steps": K, "rows": rows, "cells": cells,
        "achieved_GBs": per_launch_bytes / (kernel_us * 1e-6) / 1e9,
        "effective_GBs": K * per_launch_bytes / (kernel_us * 1e-6) / 1e9,
        "achieved_TFLOPs": FLOPS_PER_CELL * K * cells / (kernel_us * 1e-6) / 1e12,
        "mass_log": masses, "cfl": d["cfl"],
    }


def time_host_inclusive(pk, torch, w, dtype, steps, tuning, dt):
    """The same job with the host buffers in the timed region: the tensor (as
    eigenvalues and angle) and the state go up from pageable numpy arrays, the
    steps and the mass diagnostics run in the given launch shape, and the state
    comes back to numpy.  Wall clock, after one untimed round trip."""
    stream = torch.cuda.current_stream()
    ctx = pk.Context(w.nx, w.ny, w.lx, w.ly, dtype=dtype, stream=stream.cuda_stream)
    ctx.set_params(w.params)
    ctx.set_tuning(tuning["rows_per_strip"], tuning["threads"], tuning["fused_steps"], tuning["lane_shift"])
    out = [np.empty((w.ny, w.nx)) for _ in range(3)]
    walls = []
    for rep in range(2):                       # the first pass warms the path up
        n_steps = 10 if rep == 0 else steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.set_tensor_eig(*w.eig)
        ctx.set_state(w.u0, w.v0, w.w0)
        done = 0
        while done < n_steps:
            n = min(n_steps - done, MASS_EVERY - (done % MASS_EVERY))
            ctx.step(dt, n)
            done += n
            if done % MASS_EVERY == 0:
                ctx.diagnostics()
        ctx.get_state(out)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    ctx.close()
    cells = w.nx * w.ny
    up = 6 * cells * 8                          # FP64 host arrays: three eigen fields, three state fields
    down = 3 * cells * 8
    return {"value": cells * steps / walls[-1] / 1e9, "wall_ms": 1e3 * walls[-1], "steps": steps,
            "host_bytes_up": up, "host_bytes_down": down, "tuning": tuning}


def time_adjoint(pk, torch, steps=5000):
    """Gradient workload: 512^2 smooth anisotropic tensor, `steps` steps, loss of
    the final v and w; forward with square-root checkpoints, then the native
    reverse sweep (recompute + adjoint).  The forward runs twice, in the
    library's default shape (four steps per launch) and on the single-step
    kernel; the backward is the same either way.  Returns times and ratios."""
    from paper_2006_01748_amd import autograd as ag
    from paper_2006_01748_amd import workloads as wl
    w = wl.cfg4(steps=steps)
    stream = torch.cuda.current_stream()
    ctx = pk.Context(w.nx, w.ny, dtype="f64", stream=stream.cuda_stream)
    ctx.set_params(w.params)
    ctx.set_tensor_eig(*w.eig)
    dt = ctx.stable_dt(w.safety)
    default_shape = ctx.get_tuning()
    every = ag.default_every(w.steps)
    sb = ctx.state_bytes()
    ckpt = torch.empty(-(-w.steps // every) * sb, dtype=torch.uint8, device="cuda")
    work = torch.empty((every - 1) * sb, dtype=torch.uint8, device="cuda")
    lam = [torch.zeros((w.ny, w.nx), dtype=torch.float64, device="cuda") for _ in range(3)]
    g = [torch.empty((w.ny, w.nx), dtype=torch.float64, device="cuda") for _ in range(3)]
    res = {}
    for label, shape in (("fused", None), ("single_step", SINGLE_SHAPE)):
        if shape is None:
            ctx.set_tuning(*(default_shape[k] for k in ("rows_per_strip", "threads", "fused_steps", "lane_shift")))
        else:
            ctx.set_tuning(*shape)
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
            res[label] = {"forward_ms": e0.elapsed_time(e1), "backward_ms": e1.elapsed_time(e2)}
    # per-launch time of the single-step kernel (the backward's recomputation)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.set_state(w.u0, w.v0, w.w0)
    torch.cuda.synchronize()
    e0.record(stream)
    ctx.step(dt, 1000)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_us = 1e3 * e0.elapsed_time(e1) / 1000
    ctx.close()
    big = time_adjoint_kernel(pk, torch)
    bwd = res["fused"]["backward_ms"]
    return {"workload": f"{w.nx}x{w.ny} smooth anisotropic tensor, {w.steps} steps, checkpoint every "
                        f"{every} steps (forward stores {-(-w.steps // every)} states, backward recomputes "
                        f"each segment and runs the adjoint through it)",
            "dtype": "f64", "forward_shape": default_shape,
            "forward_ms": res["fused"]["forward_ms"], "backward_ms": bwd,
            "backward_over_forward": bwd / res["fused"]["forward_ms"],
            "forward_single_step_ms": res["single_step"]["forward_ms"],
            "backward_over_forward_single_step": res["single_step"]["backward_ms"] / res["single_step"]["forward_ms"],
            "step_us": fwd_us, "adjoint_step_us_est": 1e3 * bwd / w.steps - fwd_us,
            "adjoint_kernel_4096": big, "roofline": big["roofline"]}


# Algorithmic HBM bytes of one adjoint step per cell (FP64): read x^k (3),
# lam^{k+1} (3), a, b, c and the tensor gradient (3 + 3); write lam^k (3) and the
# tensor gradient (3).
ADJOINT_BYTES_PER_CELL = 18 * 8


def time_adjoint_kernel(pk, torch, n=4096, short=4, long=12):
    """The adjoint step at an HBM-resident size: the 4096^2 layered tissue, a
    reverse sweep with a checkpoint at every step (so it recomputes nothing and
    runs only adjoint steps), timed for `short` and `long` steps with HIP events
    on the context's stream; the difference over the extra steps is the time of
    one adjoint step, free of the sweep's fixed costs."""
    from paper_2006_01748_amd import workloads as wl
    w = wl.cfg2(n=n)
    stream = torch.cuda.current_stream()
    ctx = pk.Context(w.nx, w.ny, w.lx, w.ly, dtype="f64", stream=stream.cuda_stream)
    ctx.set_params(w.params)
    ctx.set_tensor_eig(*w.eig)
    dt = ctx.stable_dt(w.safety)
    sb = ctx.state_bytes()
    ckpt = torch.empty(long * sb, dtype=torch.uint8, device="cuda")
    work = torch.empty(sb, dtype=torch.uint8, device="cuda")
    lam = [torch.zeros((w.ny, w.nx), dtype=torch.float64, device="cuda") for _ in range(3)]
    g = [torch.empty((w.ny, w.nx), dtype=torch.float64, device="cuda") for _ in range(3)]
    ctx.set_state(w.u0, w.v0, w.w0)
    ctx.step_checkpointed(dt, long, 1, ckpt)
    ms = {}
    for k in (short, long, short, long):            # the first pair warms up
        for x in lam:
            x.fill_(1e-6)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.adjoint_run(dt, k, 1, ckpt, work, lam, g)
        e1.record(stream)
        torch.cuda.synchronize()
        ms[k] = e0.elapsed_time(e1)
    ctx.close()
    del ckpt, work
    us = 1e3 * (ms[long] - ms[short]) / (long - short)
    cells = w.nx * w.ny
    gbs = ADJOINT_BYTES_PER_CELL * cells / (us * 1e-6) / 1e9
    return {"workload": f"{w.nx}x{w.ny} layered tissue, FP64, reverse sweeps of {short} and {long} steps with a "
                        "checkpoint at every step", "adjoint_step_us": us,
            "roofline": {"bound": "hbm", "kernel": "adjoint_kernel<double>", "achieved": gbs, "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "traffic": measured_adjoint_traffic(),
                         "bytes_per_cell_update": ADJOINT_BYTES_PER_CELL, "kernel_avg_us": us}}


def measured_adjoint_traffic():
    """HBM bytes per adjoint step at 4096^2 from the committed counter summary,
    or None (none taken, or the adjoint source changed since)."""
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "profiles", "adjoint_kernel_traffic.json")) as f:
            data = json.load(f)
        if sources_digest(here, data["kernel_sources"]) != data.get("kernel_sources_sha256"):
            return None
        t = data["bytes_per_launch"]["adjoint_kernel<double>"]
    except (OSError, KeyError, ValueError):
        return None
    return t["read"] + t["write"]


def time_adaptive(pk, torch, w, steps=200):
    """Adaptive stepping on the headline grid (FP64): every step's size derived on
    the device from the state it starts from; one call of `steps` steps,
    timed with HIP events on the context's stream (it synchronizes once at the
    end)."""
    stream = torch.cuda.current_stream()
    ctx = pk.Context(w.nx, w.ny, w.lx, w.ly, dtype="f64", stream=stream.cuda_stream)
    ctx.set_params(w.params)
    ctx.set_tensor_eig(*w.eig)
    ctx.set_state(w.u0, w.v0, w.w0)
    log = torch.zeros(steps, dtype=torch.float64, device="cuda")
    ctx.step_adaptive(0.9, 10)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.step_adaptive(0.9, steps, log)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    dts = log.cpu().numpy()
    ctx.close()
    cells = w.nx * w.ny
    return {"workload": f"{w.nx}x{w.ny} layered tissue, FP64, safety 0.9, {steps} steps in one call",
            "value": cells * steps / (ms * 1e-3) / 1e9, "unit": "Gcell-updates/s",
            "ms_per_step": ms / steps, "dt_first": float(dts[0]), "dt_last": float(dts[-1])}


def time_front_sweep(pk, torch, t_end=2.0):
    """Invasion sweep (Section 2's propagating fronts and interstitial gap):
    delta1 in {0.5, 0.8, 1.5, 3, 6, 12.5} x ratio of the acid diffusivity along
    the propagation direction to the one across it in {1, 0.2}, 512 x 256 fronts
    on [0,1] x [0,0.5], FP64, one batch on the lane-shift kernel (4 steps per
    launch) with a common dt, run to t_end; then the fronts, the gap, the least
    u in the tumour bulk behind the front (v >= 0.9) and the LeVeque-Yee tumour
    speed of every instance."""
    from paper_2006_01748_amd import workloads as wl
    ws = wl.front_sweep()
    stream = torch.cuda.Stream()
    b = pk.Batch([(w.nx, w.ny) for w in ws], lx=ws[0].lx, ly=ws[0].ly, dtype="f64", stream=stream.cuda_stream)
    dts = []
    for i, w in enumerate(ws):
        c = b[i]
        c.set_params(w.params)
        c.set_tensor_eig(*w.eig)
        c.set_state(w.u0, w.v0, w.w0)
        dts.append(c.stable_dt(w.safety))
    dt = min(dts)
    for i in range(len(ws)):
        b.set_dt(i, dt)
    b.set_tuning(threads=64, rows_per_strip=16, graph_steps=48, fused_steps=4)
    m0 = [b[i].diagnostics()["mass"][1] for i in range(len(ws))]
    f0 = [b[i].front_diagnostics(0.25, 0.5)["tumour"][0] for i in range(len(ws))]
    n = int(t_end / dt) // 4 * 4
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.run(n)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cells = sum(w.cells for w in ws)
    out = []
    for i, w in enumerate(ws):
        d = b[i].diagnostics()
        f = b[i].front_diagnostics(0.25, 0.5)
        U, V, _ = b[i].get_state()
        out.append({"delta1": w.params[0], "kappa": round(float(w.eig[0][0, 0] / w.eig[1][0, 0]), 6),
                    "u_behind_min": float(U[V >= 0.9].min()) if (V >= 0.9).any() else None,
                    "tumour_front": float(f["tumour"][0]), "tumour_front_advance": float(f["tumour"][0] - f0[i]),
                    "gap_mean": float(f["gap"][0]) if f["rows_gap"] else None,
                    "gap_max": float(f["gap"][2]) if f["rows_gap"] else None,
                    "tumour_speed_leveque_yee": pk.front_speed(m0[i], d["mass"][1], 0.0, d["t"], w.ly, 1.0, 0.0)})
    b.close()
    return {"workload": f"{len(ws)} fronts 512x256 (delta1 sweep x 2 acid anisotropies), FP64, lane-shift "
                        f"batch, {n} steps to t = {n * dt:.3g}",
            "value": cells * n / (ms * 1e-3) / 1e9, "unit": "Gcell-updates/s", "ms": ms, "instances": out}


def time_3d(pk, torch, n=256, steps=100, warmup=10, dtypes=("f64", "f32"), trial_steps=20):
    """Three-dimensional step on the 256^3 slab tissue (19-point acid stencil,
    7-point tumour-cell stencil): for each dtype a short sweep of pencil shapes
    (rows per wave x planes per strip), then `steps` steps in the fastest, timed
    with HIP events on the context's stream.  Algorithmic bytes per cell-update:
    3 state values read, 6 tensor values read, 3 written."""
    from paper_2006_01748_amd import workloads as wl
    w = wl.tissue3(n=n)
    stream = torch.cuda.current_stream()
    out = {"workload": f"slab tissue {w.nx}x{w.ny}x{w.nz}, 8 z-slabs of random SPD tensors, tumour ball, "
                       f"dt=0.9 of the step bound, {steps} steps", "variants": {}}

    def timed(ctx, dt, k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.step(dt, k)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    for dt_name in dtypes:
        ctx = pk.Context3(w.nx, w.ny, w.nz, w.lx, w.ly, w.lz, dtype=dt_name, stream=stream.cuda_stream)
        ctx.set_params(w.params)
        ctx.set_tensor(*w.tensor)
        ctx.set_state(w.u0, w.v0, w.w0)
        dt = ctx.stable_dt(w.safety)
        sweep = {}
        for rows in (1, 2, 4):
            for zs in (16, 32, 64):
                for wx, wy in ((1, 1), (1, 2), (1, 4), (5, 1), (4, 2), (2, 2)):
                    ctx.set_tuning(zs, rows, wx, wy)
                    ctx.step(dt, 2)
                    torch.cuda.synchronize()
                    sweep[f"rows={rows},zs={zs},wx={wx},wy={wy}"] = timed(ctx, dt, trial_steps) * 1e3 / trial_steps
        best = min(sweep, key=sweep.get)
        rows, zs, wx, wy = (int(v.split("=")[1]) for v in best.split(","))
        ctx.set_tuning(zs, rows, wx, wy)
        shape = ctx.get_tuning()
        ctx.set_state(w.u0, w.v0, w.w0)
        ctx.step(dt, warmup)
        torch.cuda.synchronize()
        ms = timed(ctx, dt, steps)
        mass = ctx.mass()
        ctx.close()
        per = 12 * (8 if dt_name == "f64" else 4)
        us = ms * 1e3 / steps
        gbs = w.cells * per / (us * 1e-6) / 1e9
        out["variants"][dt_name] = {
            "value": w.cells * steps / (ms * 1e-3) / 1e9, "unit": "Gcell-updates/s", "kernel_avg_us": us,
            "launch_shape": shape, "kernel": f"step3_pencil_kernel<{'double' if dt_name == 'f64' else 'float'}, {rows}>",
            "roofline": with_measured({"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                       "frac": gbs / PEAK_HBM_GBS, "traffic": measured_traffic3(dt_name, shape)},
                                      us),
            "bytes_per_cell_update": per, "dt": dt, "mass": list(mass),
            "shape_sweep_us": {k: round(v, 1) for k, v in sweep.items()}}
    return out


def time_ensemble(pk, torch, count=256, steps=500, loop_steps=48, force=None):
    """Ensemble workload: `count` instances (sides 64..512, own parameters, tensor
    and dt), compensated FP32.  A batched graph-replayed run versus loops of
    single-instance launches of the same instances on the same GPU: one in the
    batch's own launch shape (same kernel family, steps per launch and strip
    height: the gain from batching alone) and one in each context's default
    shape."""
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
    if force is None:
        tuned = b.autotune(trial_steps=12)
        tuned["source"] = "batch autotuner"
    else:
        tuned = {"threads": force[0], "rows_per_strip": force[1], "fused_steps": force[2] if len(force) > 2 else 1,
                 "source": "fixed (--ensemble-tuning)"}
    K = tuned["fused_steps"]
    b.set_tuning(threads=tuned["threads"], rows_per_strip=tuned["rows_per_strip"], graph_steps=48, fused_steps=K)
    b.run(48)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1)
    b.close()
    launches = steps // K + steps % K

    def loop(shape):
        ctxs = []
        for w in ws:
            c = pk.Context(w.nx, w.ny, dtype="f32c", stream=stream.cuda_stream)
            c.set_params(w.params)
            c.set_tensor_eig(*w.eig)
            c.set_state(w.u0, w.v0, w.w0)
            if shape is not None:
                c.set_tuning(*shape)
            ctxs.append(c)
        for c, dt in zip(ctxs, dts):
            c.step(dt, 2 * K)
        torch.cuda.synchronize()
        e0.record(stream)
        for c, dt in zip(ctxs, dts):
            c.step(dt, loop_steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        for c in ctxs:
            c.close()
        return cells * loop_steps / (ms * 1e-3) / 1e9, ms / loop_steps

    same = (tuned["rows_per_strip"], 0, K, 1) if K > 1 else (tuned["rows_per_strip"], tuned["threads"], 1, 0)
    loop_rate, loop_ms = loop(same)
    default_rate, default_ms = loop(None)
    batch_rate = cells * steps / (batch_ms * 1e-3) / 1e9
    launch_us = 1e3 * batch_ms / launches
    alg = BYTES_PER_CELL["f32c"] * cells
    kname = (f"fused_dpp_batch_kernel<float, true, 2, {K}>" if K > 1
             else f"step_batch_kernel<float, true, 2, {tuned['threads']}>")
    return {"workload": f"{count} instances, sides 64..512 (total {cells} cells), own parameters, tensor and dt, "
                        f"compensated FP32", "dtype": "f32c", "tuning": tuned,
            "batched_Gcell_s": batch_rate, "batched_ms_per_step": batch_ms / steps,
            "loop_same_shape_Gcell_s": loop_rate, "loop_same_shape_ms_per_step": loop_ms,
            "loop_same_shape": dict(zip(("rows_per_strip", "threads", "fused_steps", "lane_shift"), same)),
            "loop_default_shape_Gcell_s": default_rate, "loop_default_shape_ms_per_step": default_ms,
            "speedup": batch_rate / loop_rate, "speedup_vs_default_shape_loop": batch_rate / default_rate,
            "roofline": {"bound": "hbm", "kernel": kname, "achieved": alg / (launch_us * 1e-6) / 1e9,
                         "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": alg / (launch_us * 1e-6) / 1e9 / PEAK_HBM_GBS,
                         "traffic": measured_ensemble_traffic(kname, tuned["rows_per_strip"]),
                         "launch_avg_us": launch_us, "steps_per_launch": K,
                         "note": "algorithmic bytes of one launch (60 B per cell of all instances) over the "
                                 "graph-replayed run's time per launch, gaps between launches included"}}


def measured_ensemble_traffic(kname, rows):
    """HBM bytes per launch of the batched kernel on the 256-instance ensemble
    from the committed counter summary, or None (none for this kernel, or a
    kernel source changed since)."""
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "profiles", "ensemble_kernel_traffic.json")) as f:
            data = json.load(f)
        if data["kernel_sources"] != traffic_sources(here):
            return None
        if sources_digest(here, data["kernel_sources"]) != data.get("kernel_sources_sha256"):
            return None
        t = data["bytes_per_launch"][kname]
        if t.get("rows") != rows:
            return None
    except (OSError, KeyError, ValueError, TypeError):
        return None
    return t["read"] + t["write"]


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


def host_identity():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(w, steps, single_steps):
    """The FP64 oracle on the host cores: all threads it is allowed (OpenMP over
    rows, the same bits as one thread) on `steps` steps, and one thread on
    `single_steps` steps, of the same grid."""
    import oracle
    a, b, c = oracle.tensor_from_eig(*w.eig)
    dt = oracle.stable_dt(a, b, c, w.params[2], w.safety)
    threads = oracle.set_threads()

    def timed(n):
        t0 = time.perf_counter()
        oracle.run(w.u0, w.v0, w.w0, a, b, c, w.params, dt, n)
        return time.perf_counter() - t0

    sec = timed(steps)
    oracle.set_threads(1)
    sec1 = timed(single_steps)
    oracle.set_threads(threads)
    cells = w.nx * w.ny
    return {"value": cells * steps / sec / 1e9, "unit": "Gcell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} FP64 steps of the same {w.nx}x{w.ny} layered-tissue grid on {threads} host "
                      f"threads ({sec:.1f} s)",
            "single_thread": {"value": cells * single_steps / sec1 / 1e9, "unit": "Gcell-updates/s", "cores": 1,
                              "sample": f"{single_steps} FP64 steps, one thread ({sec1:.1f} s)"},
            "host": host_identity()}


# The rocprofv3 runs behind the committed summaries under profiles/.  Run from
# /tmp with TMPDIR=/tmp; $R is the repository root, $P an output folder.
PROFILE_COMMANDS = {
    "trace": "timeout -k 10 500 rocprofv3 --kernel-trace --stats --output-format csv -d $P/trace -o trace "
             "-- python3 $R/bench.py --steps 200 --warmup 12 --no-cpu-baseline --no-fronts --no-adjoint --no-ensemble "
             "--no-3d > $P/trace_bench.json",
    "fronts": "timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d $P/fronts -o fronts "
              "-- python3 $R/bench.py --variants f64 --no-tune --steps 4 --warmup 4 --no-cpu-baseline --no-adjoint "
              "--no-ensemble --no-adaptive --no-copy-ceiling --no-3d --fronts-t 0.02 > $P/fronts_bench.json",
    "fetch": "timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $P/fetch -o fetch "
             "-- python3 $R/bench.py --steps 8 --warmup 4 --no-cpu-baseline --no-adjoint --no-ensemble "
             "--no-adaptive --no-fronts --no-3d --no-host-inclusive",
    "write": "timeout -s KILL 300 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $P/write -o write "
             "-- python3 $R/bench.py --steps 8 --warmup 4 --no-cpu-baseline --no-adjoint --no-ensemble "
             "--no-adaptive --no-fronts --no-3d --no-host-inclusive",
    # the three-dimensional kernel alone (with the copy used for calibration)
    "trace3": "timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d $P/trace3 -o trace3 "
              "-- python3 $R/bench.py --only-3d > $P/trace3_bench.json",
    "fetch3": "timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $P/fetch3 -o fetch3 "
              "-- python3 $R/bench.py --only-3d",
    "write3": "timeout -s KILL 300 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $P/write3 -o write3 "
              "-- python3 $R/bench.py --only-3d",
    # the ensemble alone: batched kernel trace (with the gaps between graph-replayed
    # launches) and its HBM traffic
    "etrace": "timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d $P/etrace -o etrace "
              "-- python3 $R/bench.py --only-ensemble --ensemble-tuning 64,32,4 > $P/etrace_bench.json",
    "efetch": "timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $P/efetch -o efetch "
              "-- python3 $R/bench.py --only-ensemble --ensemble-tuning 64,32,4",
    "ewrite": "timeout -s KILL 300 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $P/ewrite -o ewrite "
              "-- python3 $R/bench.py --only-ensemble --ensemble-tuning 64,32,4",
    # the adjoint alone (512^2 gradient workload, 4096^2 adjoint steps)
    "atrace": "timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d $P/atrace -o atrace "
              "-- python3 $R/bench.py --only-adjoint > $P/atrace_bench.json",
    "afetch": "timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $P/afetch -o afetch "
              "-- python3 $R/bench.py --only-adjoint",
    "awrite": "timeout -s KILL 300 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $P/awrite -o awrite "
              "-- python3 $R/bench.py --only-adjoint",
    # instruction counts of the 2D kernels (six SQ counters, one pass)
    "valu": "timeout -s KILL 300 rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD "
            "SQ_INSTS_VMEM_WR SQ_WAVES --output-format csv -d $P/valu -o valu "
            "-- python3 $R/bench.py --steps 8 --warmup 4 --no-cpu-baseline --no-adjoint --no-ensemble "
            "--no-adaptive --no-fronts --no-3d --no-host-inclusive --no-copy-ceiling",
}

# MI355X: 256 CUs, each issuing at most one wave64 vector instruction per cycle
# over its four SIMDs (16 lanes, 4 cycles per FP64 or non-packed FP32
# instruction), at 2.4 GHz.  The plain FP32 headline kernel reads 0.98-1.02 on
# different boxes: the four-cycle model does not hold exactly for every counted
# instruction, and such a value reads as the issue limit.
VALU_ISSUE_PER_S = 256 * 2.4e9


def summarize_valu(pdir, n=4096):
    """profiles/valu_step_kernels_4096_layered_tissue.md from the valu/ counter
    pass: instructions per cell-update of the single-step and headline kernels
    and the vector issue utilisation (instructions over 256 CUs x the
    dispatch's duration x 2.4 GHz)."""
    import csv
    import collections
    here = os.path.dirname(os.path.abspath(__file__))
    vals = collections.defaultdict(lambda: collections.defaultdict(float))
    meta = {}
    with open(os.path.join(pdir, "valu", "valu_counter_collection.csv")) as f:
        for row in csv.DictReader(f):
            d = int(row["Dispatch_Id"])
            vals[d][row["Counter_Name"]] += float(row["Counter_Value"])
            meta[d] = (_short(row["Kernel_Name"]), int(row["Grid_Size"]), int(row["Workgroup_Size"]),
                       (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3)
    agg = collections.defaultdict(list)
    for d, c in vals.items():
        agg[meta[d][:3]].append((c, meta[d][3]))
    counters = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR")
    rows, out, per_launch = [], {}, {}
    for v in ("f64", "f32c", "f32"):
        for label, tuning in (("single step", {"fused_steps": 1, "threads": 0}),
                              ("headline", dict(zip(("rows_per_strip", "threads", "fused_steps", "lane_shift"),
                                                    HEADLINE_SHAPE[v])))):
            kname, _ = kernel_name(v, tuning)
            keys = [k for k in agg if k[0] == kname]
            if not keys:
                continue
            k = max(keys, key=lambda x: x[1])         # the 4096^2 dispatches
            runs = agg[k]
            mean = {c: sum(r[0][c] for r in runs) / len(runs) for c in counters}
            us = sum(r[1] for r in runs) / len(runs)
            updates = n * n * max(1, tuning["fused_steps"])
            per = {c: mean[c] * 64 / updates for c in counters}
            util = mean["SQ_INSTS_VALU"] / (VALU_ISSUE_PER_S * us * 1e-6)
            out[f"{v}/{label}"] = {"kernel": kname, "dispatches": len(runs), "duration_us": us,
                                   "valu_per_cell_update": per["SQ_INSTS_VALU"], "valu_issue_util": util}
            _, key = kernel_name(v, tuning)
            per_launch[f"{v}/{key}"] = {"kernel": kname, "rows": tuning.get("rows_per_strip", 0),
                                        "valu": mean["SQ_INSTS_VALU"]}
            rows.append(f"| {v} | {label} | {kname} | {len(runs)} | {us:.1f} | {mean['SQ_INSTS_VALU']:.4g} | "
                        f"{per['SQ_INSTS_VALU']:.1f} | {per['SQ_INSTS_SALU']:.1f} | {per['SQ_INSTS_LDS']:.2f} | "
                        f"{per['SQ_INSTS_VMEM_RD']:.2f} | {per['SQ_INSTS_VMEM_WR']:.2f} | {100 * util:.0f}% |")
    with open(os.path.join(here, "profiles", "valu_step_kernels_4096_layered_tissue.md"), "w") as f:
        f.write("# Instruction counts of the 2D step kernels, 4096^2 layered tissue (rocprofv3 counters)\n\n"
                f"Command (from /tmp with TMPDIR=/tmp):\n\n```\n{PROFILE_COMMANDS['valu']}\n```\n\n"
                "Summary written by `python bench.py --summarize-profiles $P`.  Counts are wave instructions "
                "per dispatch, averaged over the dispatches of the 4096^2 runs; per cell-update they are "
                "lane instructions (x64) over 4096^2 x steps per launch.  Issue utilisation: VALU wave "
                "instructions over the most the chip can issue in the dispatch's duration (256 CUs x one "
                "wave instruction per cycle x 2.4 GHz x duration; every FP64 and non-packed FP32 "
                "instruction takes four cycles of a 16-lane SIMD).  Durations are those of the counter "
                "run.\n\n"
                "| variant | kernel role | kernel | dispatches | duration (us) | VALU instructions | "
                "VALU / cell-update | SALU / cell-update | LDS / cell-update | VMEM reads / cell-update | "
                "VMEM writes / cell-update | VALU issue utilisation |\n"
                "|---|---|---|---|---|---|---|---|---|---|---|---|\n" + "\n".join(rows) + "\n")
    srcs = traffic_sources(here)
    with open(os.path.join(here, "profiles", "step_kernel_valu.json"), "w") as f:
        json.dump({"note": "VALU wave instructions per dispatch (SQ_INSTS_VALU) of the 4096^2 step kernels; valid "
                           "for the kernel sources with this digest and the strip heights given (0: library "
                           "default).", "kernel_sources": srcs, "kernel_sources_sha256": sources_digest(here, srcs),
                   "valu_per_launch": per_launch}, f, indent=1)
    return out



def _short(name):
    name = name.replace("ggfv::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    name = name.replace("void ", "")
    depth, out = 0, []
    for ch in name:                      # drop the argument list
        if ch == "(" and depth == 0 and out:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def _counter_means(pdir, kind):
    """Mean counter value per (kernel, grid size, workgroup size) over the
    dispatches of one --pmc run (launch shapes with equal thread counts differ
    in workgroup size)."""
    import csv
    import collections
    vals, meta = collections.defaultdict(float), {}
    with open(os.path.join(pdir, kind, f"{kind}_counter_collection.csv")) as f:
        for row in csv.DictReader(f):
            d = int(row["Dispatch_Id"])
            vals[d] += float(row["Counter_Value"])
            meta[d] = (_short(row["Kernel_Name"]), int(row["Grid_Size"]), int(row["Workgroup_Size"]))
    agg = collections.defaultdict(list)
    for d, v in vals.items():
        agg[meta[d]].append(v)
    out = {k: sum(v) / len(v) for k, v in agg.items()}
    out["__per_dispatch__"] = [(meta[d], v) for d, v in sorted(vals.items())]
    return out


def _copy_calibration(fetch, write, copy_bytes=1 << 30):
    """Scale factors of FETCH_SIZE and WRITE_SIZE from the 1 GiB device copies of
    the copy-ceiling probe.  Copies of other sizes (checkpoints, state saves) run
    the same copy kernel with the same launch shape, so the calibration uses the
    largest copy dispatches of each run, identified per dispatch."""
    if isinstance(fetch, dict) and "__per_dispatch__" in fetch:
        fd, wd = fetch["__per_dispatch__"], write["__per_dispatch__"]
        fc = [v for (name, _, _), v in fd if name == "__amd_rocclr_copyBuffer"]
        wc = [v for (name, _, _), v in wd if name == "__amd_rocclr_copyBuffer"]
        fbig = [v for v in fc if v >= 0.9 * max(fc)]
        wbig = [v for v in wc if v >= 0.9 * max(wc)]
        f_mean, w_mean = sum(fbig) / len(fbig), sum(wbig) / len(wbig)
        return ("__amd_rocclr_copyBuffer", f_mean, w_mean), copy_bytes / (f_mean * 1024), copy_bytes / (w_mean * 1024)
    cal = [k for k in fetch if k[0] == "__amd_rocclr_copyBuffer"]
    ck = max(cal, key=lambda k: k[1])
    return ck, copy_bytes / (fetch[ck] * 1024), copy_bytes / (write[ck] * 1024)


def summarize_3d(pdir, tdir, fdir, wdir, bench_json):
    """profiles/step3_kernels_256cube_slab_tissue.md and profiles/step3_kernel_traffic.json."""
    import csv
    import collections
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(pdir, bench_json)) as f:
        three = json.loads(f.read().strip().splitlines()[-1])["three_d"]
    fetch, write = _counter_means(pdir, fdir), _counter_means(pdir, wdir)
    ck, f_scale, w_scale = _copy_calibration(fetch, write)
    durs = collections.defaultdict(list)
    with open(os.path.join(pdir, tdir, f"{tdir}_kernel_trace.csv")) as f:
        for row in csv.DictReader(f):
            name = _short(row["Kernel_Name"])
            if name.startswith("step3_pencil_kernel"):
                durs[(name, int(row["Grid_Size_X"]), int(row["Workgroup_Size_X"]))].append(
                    (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3)
    n3 = [int(x) for x in three["workload"].split()[2].rstrip(",").split("x")]
    cells3 = n3[0] * n3[1] * n3[2]
    rows3, traffic3 = [], {}
    for dt_name, vr in three["variants"].items():
        shape = vr["launch_shape"]
        threads = shape["workgroups"] * 64 * shape["waves_x"] * shape["waves_y"]
        key = (vr["kernel"], threads, 64 * shape["waves_x"] * shape["waves_y"])
        d = durs.get(key, [])
        alg = vr["bytes_per_cell_update"] * cells3
        alg_w = alg // 4                           # 3 of the 12 values are written
        rd = fetch.get(key, float("nan")) * 1024 * f_scale
        wr = write.get(key, float("nan")) * 1024 * w_scale
        if key in fetch and key in write:
            traffic3[dt_name] = {"kernel": vr["kernel"], "launch_shape": shape, "read": rd, "write": wr,
                                 "fetch_kib": fetch[key], "write_kib": write[key]}
        avg = sum(d) / len(d) if d else float("nan")
        rows3.append(f"| {dt_name} | {vr['kernel']} | {shape['rows_per_wave']} | {shape['z_per_strip']} | "
                     f"{shape['waves_x']}x{shape['waves_y']} | {shape['workgroups']} | {len(d)} | {avg:.1f} | "
                     f"{vr['kernel_avg_us']:.1f} | {alg / avg / 1e3:.0f} | {fetch.get(key, float('nan')):.0f} | "
                     f"{write.get(key, float('nan')):.0f} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | "
                     f"{(alg - alg_w) / 1e6:.1f} / {alg_w / 1e6:.1f} | {(rd + wr) / alg:.3f} |")
    srcs3 = traffic_sources(here, "3d")
    with open(os.path.join(here, "profiles", "step3_kernel_traffic.json"), "w") as f:
        json.dump({"note": f"HBM bytes per launch of the 3D step kernel on the {three['workload'].split(',')[0]} "
                           "grid, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (separate runs), scaled by "
                           f"the 1 GiB copyBuffer calibration (FETCH x{f_scale:.3f}, WRITE x{w_scale:.3f}); "
                           "valid for the kernel sources with this digest and the launch shape given.",
                   "kernel_sources": srcs3, "kernel_sources_sha256": sources_digest(here, srcs3),
                   "bytes_per_launch": traffic3}, f, indent=1)
    sweep = []
    for dt_name, vr in three["variants"].items():
        best = sorted(vr["shape_sweep_us"].items(), key=lambda x: x[1])
        sweep.append(f"| {dt_name} | " + "; ".join(f"{k}: {v}" for k, v in best[:6]) + " | " +
                     "; ".join(f"{k}: {v}" for k, v in best[-2:]) + " |")
    cmds = "\n".join(PROFILE_COMMANDS[k] for k in (tdir, fdir, wdir))
    with open(os.path.join(here, "profiles", "step3_kernels_256cube_slab_tissue.md"), "w") as f:
        f.write("# Three-dimensional step kernel, 256^3 slab tissue (rocprofv3)\n\n"
                "Commands (from /tmp with TMPDIR=/tmp; $R = repository root, $P = output folder):\n\n"
                f"```\n{cmds}\n```\n\nSummary written by `python bench.py --summarize-profiles $P`.\n\n"
                "The trace and counter rows are the dispatches of the launch shape bench.py picked in the "
                "traced run (a short sweep of rows per wave x planes per strip x waves per workgroup "
                "precedes the timed steps).  Algorithmic bytes per cell-update: u, v, w and the six tensor "
                "entries read once, u, v, w written once (96 B in FP64, 48 B in FP32).  Counter calibration: "
                f"the 1 GiB `__amd_rocclr_copyBuffer` reads FETCH_SIZE = {ck[1]:.0f} KiB and WRITE_SIZE = "
                f"{ck[2]:.0f} KiB, so FETCH_SIZE is scaled by {f_scale:.3f} and WRITE_SIZE by {w_scale:.3f}.\n\n"
                "| dtype | kernel | rows per wave | planes per strip | waves per workgroup | workgroups | "
                "dispatches (trace) | average (us, trace) | average (us, live HIP events) | algorithmic GB/s "
                "(trace) | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | scaled read (MB) | scaled write (MB) | "
                "algorithmic read / write (MB) | traffic / algorithmic |\n"
                "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|\n" + "\n".join(rows3) +
                "\n\n## Launch-shape sweep in the traced run (us per step): six fastest; two slowest\n\n"
                "| dtype | fastest | slowest |\n|---|---|---|\n" + "\n".join(sweep) + "\n")
    return traffic3


def _trace_rows(pdir, kind):
    """(short name, grid size, workgroup size, start ns, end ns) of every dispatch
    in a --kernel-trace run."""
    import csv
    out = []
    with open(os.path.join(pdir, kind, f"{kind}_kernel_trace.csv")) as f:
        for row in csv.DictReader(f):
            out.append((_short(row["Kernel_Name"]), int(row["Grid_Size_X"]), int(row["Workgroup_Size_X"]),
                        int(row["Start_Timestamp"]), int(row["End_Timestamp"])))
    return out


def _stats_table(rows, pred):
    import collections
    agg = collections.defaultdict(list)
    for name, grid, wg, t0, t1 in rows:
        if pred(name):
            agg[(name, grid)].append((t1 - t0) / 1e3)
    lines = []
    for (name, grid), d in sorted(agg.items(), key=lambda x: -sum(x[1])):
        lines.append(f"| {name} | {grid} | {len(d)} | {sum(d) / len(d):.1f} | {min(d):.1f} | {max(d):.1f} |")
    return ("| kernel | grid (threads) | calls | average (us) | min (us) | max (us) |\n|---|---|---|---|---|---|\n"
            + "\n".join(lines)), agg


def summarize_ensemble(pdir):
    """profiles/ensemble_kernels_256.md and profiles/ensemble_kernel_traffic.json
    from the etrace/, efetch/ and ewrite/ runs: the batched lane-shift kernel's
    launch time, the gap between its graph-replayed launches, and its traffic."""
    import statistics
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(pdir, "etrace_bench.json")) as f:
        ens = json.loads(f.read().strip().splitlines()[-1])["ensemble"]
    rows = _trace_rows(pdir, "etrace")
    table, agg = _stats_table(rows, lambda k: k.startswith(("fused_dpp_batch_kernel", "step_batch_kernel",
                                                             "fused_dpp_kernel", "step_kernel")))
    kname = ens["roofline"]["kernel"]
    batch = sorted((t0, t1) for name, grid, wg, t0, t1 in rows if name == kname)
    # gaps between consecutive batched launches (end to next start; the
    # timestamps of back-to-back launches may overlap by a few ns, read as 0);
    # those under 100 us belong to one run of graph replays
    gaps = [max(0.0, (b0 - a1) / 1e3) for (a0, a1), (b0, b1) in zip(batch, batch[1:])]
    run = sorted(g for g in gaps if g < 100.0)
    dur = [(t1 - t0) / 1e3 for t0, t1 in batch]
    gap_p90 = run[int(0.9 * (len(run) - 1))] if run else float("nan")
    gap_max = run[-1] if run else float("nan")
    gap_mean = sum(run) / len(run) if run else float("nan")
    fetch, write = _counter_means(pdir, "efetch"), _counter_means(pdir, "ewrite")
    ck, f_scale, w_scale = _copy_calibration(fetch, write)
    keys = [k for k in fetch if k[0] == kname]
    traffic = None
    if keys:
        k = max(keys, key=lambda x: x[1])
        traffic = {"kernel": kname, "rows": ens["tuning"]["rows_per_strip"], "read": fetch[k] * 1024 * f_scale,
                   "write": write.get(k, 0.0) * 1024 * w_scale, "fetch_kib": fetch[k], "write_kib": write.get(k, 0.0)}
    cells = int(ens["workload"].split("total ")[1].split(" cells")[0])
    alg = BYTES_PER_CELL["f32c"] * cells
    srcs = traffic_sources(here)
    gap_med = statistics.median(run) if run else float("nan")
    dur_med = statistics.median(dur) if dur else float("nan")
    with open(os.path.join(here, "profiles", "ensemble_kernel_traffic.json"), "w") as f:
        json.dump({"note": "HBM bytes per launch of the batched lane-shift kernel on the 256-instance ensemble "
                           "(sides 64..512, compensated FP32), from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE "
                           f"(separate runs) scaled by the 1 GiB copyBuffer (FETCH x{f_scale:.3f}, WRITE "
                           f"x{w_scale:.3f}); launch gaps from the kernel trace.",
                   "kernel_sources": srcs, "kernel_sources_sha256": sources_digest(here, srcs),
                   "bytes_per_launch": {kname: traffic} if traffic else {},
                   "launch_gap_us_median": gap_med, "launch_gap_us_mean": gap_mean, "launch_gap_us_max": gap_max,
                   "launch_us_median": dur_med}, f, indent=1)
    cmds = "\n".join(PROFILE_COMMANDS[k] for k in ("etrace", "efetch", "ewrite"))
    tr = (f"{(traffic['read'] + traffic['write']) / 1e6:.1f} MB per launch (read {traffic['read'] / 1e6:.1f}, "
          f"write {traffic['write'] / 1e6:.1f}; FETCH_SIZE {traffic['fetch_kib']:.0f} KiB, WRITE_SIZE "
          f"{traffic['write_kib']:.0f} KiB), {(traffic['read'] + traffic['write']) / alg:.3f} of the algorithmic "
          f"{alg / 1e6:.1f} MB" if traffic else "not collected")
    with open(os.path.join(here, "profiles", "ensemble_kernels_256.md"), "w") as f:
        f.write("# Ensemble kernels: 256 instances (sides 64..512), compensated FP32 (rocprofv3)\n\n"
                "Commands (from /tmp with TMPDIR=/tmp; $R = repository root, $P = output folder):\n\n"
                f"```\n{cmds}\n```\n\nSummary written by `python bench.py --summarize-profiles $P`.\n\n"
                f"## Kernel trace\n\n{table}\n\n"
                f"`{kname}` steps every instance 4 steps per launch (graph-replayed, 48 steps per graph; launch "
                f"shape {ens['tuning']}); "
                "`fused_dpp_kernel<float, true, 2, 4>` is the loop of single-instance launches in the same shape "
                "and `fused_dpp_kernel` / `step_kernel` rows of other shapes belong to the default-shape loop.\n\n"
                f"## Launches of the batched kernel\n\n"
                f"- median launch: {dur_med:.1f} us; gaps between consecutive launches (end to next start, "
                f"gaps under 100 us, {len(run)} gaps): median {gap_med:.2f} us, mean {gap_mean:.2f} us, 90th "
                f"percentile {gap_p90:.2f} us, largest {gap_max:.2f} us; the mean gap is "
                f"{100 * gap_mean / (dur_med + gap_mean):.2f}% of the time per launch.\n"
                f"- HBM traffic: {tr}.\n"
                f"- bench.py in the same run: batched {ens['batched_Gcell_s']:.1f} Gcell/s, loop in the same shape "
                f"{ens['loop_same_shape_Gcell_s']:.1f}, loop in the default shape "
                f"{ens['loop_default_shape_Gcell_s']:.1f} Gcell/s.\n")
    return {"launch_gap_us_median": gap_med, "launch_gap_us_mean": gap_mean, "launch_gap_us_max": gap_max,
            "launch_us_median": dur_med, "traffic": traffic}


def summarize_adjoint(pdir):
    """profiles/adjoint_kernels.md and profiles/adjoint_kernel_traffic.json from
    the atrace/, afetch/ and awrite/ runs: the adjoint kernel on the 512^2
    gradient workload and at 4096^2, and its HBM traffic at 4096^2."""
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(pdir, "atrace_bench.json")) as f:
        adj = json.loads(f.read().strip().splitlines()[-1])["adjoint"]
    rows = _trace_rows(pdir, "atrace")
    table, agg = _stats_table(rows, lambda k: k.startswith(("adjoint_kernel", "slots_reduce", "step_kernel<double",
                                                             "fused_dpp_kernel<double", "eig_backward")))
    fetch, write = _counter_means(pdir, "afetch"), _counter_means(pdir, "awrite")
    ck, f_scale, w_scale = _copy_calibration(fetch, write)
    keys = [k for k in fetch if k[0].startswith("adjoint_kernel<double")]
    k = max(keys, key=lambda x: fetch[x])             # the 4096^2 dispatches read the most
    rd, wr = fetch[k] * 1024 * f_scale, write.get(k, 0.0) * 1024 * w_scale
    n = 4096
    alg = ADJOINT_BYTES_PER_CELL * n * n
    big = [d for (name, grid), d in agg.items() if name == k[0] and grid == k[1]]
    avg = sum(big[0]) / len(big[0]) if big else float("nan")
    srcs = [os.path.join("paper_2006_01748_amd", "build.py")] + sorted(
        os.path.join("paper_2006_01748_amd", "csrc", x) for x in ("ggfv_adjoint.hip", "ggfv_dpp.hpp",
                                                                  "ggfv_step_common.hpp", "ggfv_internal.hpp"))
    traffic = {"kernel": k[0], "read": rd, "write": wr, "fetch_kib": fetch[k], "write_kib": write.get(k, 0.0)}
    with open(os.path.join(here, "profiles", "adjoint_kernel_traffic.json"), "w") as f:
        json.dump({"note": "HBM bytes per adjoint step on the 4096^2 layered-tissue grid (FP64), from rocprofv3 "
                           "--pmc FETCH_SIZE and WRITE_SIZE (separate runs) scaled by the 1 GiB copyBuffer "
                           f"(FETCH x{f_scale:.3f}, WRITE x{w_scale:.3f}).",
                   "kernel_sources": srcs, "kernel_sources_sha256": sources_digest(here, srcs),
                   "bytes_per_launch": {"adjoint_kernel<double>": traffic}}, f, indent=1)
    cmds = "\n".join(PROFILE_COMMANDS[x] for x in ("atrace", "afetch", "awrite"))
    with open(os.path.join(here, "profiles", "adjoint_kernels.md"), "w") as f:
        f.write("# Adjoint kernels: 512^2 gradient workload and 4096^2 adjoint steps, FP64 (rocprofv3)\n\n"
                "Commands (from /tmp with TMPDIR=/tmp; $R = repository root, $P = output folder):\n\n"
                f"```\n{cmds}\n```\n\nSummary written by `python bench.py --summarize-profiles $P`.\n\n"
                f"## Kernel trace\n\n{table}\n\n"
                "The smaller `adjoint_kernel` grid is the 512^2 gradient workload (5000 adjoint steps), the larger "
                "one the 4096^2 reverse sweeps of 4 and 12 steps.  `step_kernel<double, false, 1, 64>` recomputes "
                "each 512^2 segment; the forward runs in the default shape.\n\n"
                "## 4096^2 adjoint step\n\n"
                f"- trace average {avg:.1f} us; live HIP events in the same run "
                f"{adj['adjoint_kernel_4096']['adjoint_step_us']:.1f} us per step.\n"
                f"- algorithmic bytes {alg / 1e6:.1f} MB (144 B per cell: read x, lam', a, b, c and g; write lam and "
                f"g), {alg / (avg * 1e-6) / 1e9:.0f} GB/s over the trace average.\n"
                f"- counters: FETCH_SIZE {fetch[k]:.0f} KiB, WRITE_SIZE {write.get(k, 0.0):.0f} KiB per dispatch; "
                f"scaled read {rd / 1e6:.1f} MB, write {wr / 1e6:.1f} MB: {(rd + wr) / alg:.3f} of the algorithmic "
                f"bytes (calibration: FETCH x{f_scale:.3f}, WRITE x{w_scale:.3f} from the 1 GiB copyBuffer).\n"
                f"- bench.py in the same run: backward / forward = {adj['backward_over_forward']:.2f} (forward in "
                f"the default shape), {adj['backward_over_forward_single_step']:.2f} (single-step forward).\n")
    return {"adjoint_4096_us": avg, "traffic": traffic}


def summarize_fronts(pdir):
    """profiles/front_sweep_kernels_512x256.md from the fronts/ trace."""
    import csv
    here = os.path.dirname(os.path.abspath(__file__))
    head = "| kernel | calls | average (us) | min (us) | max (us) |\n|---|---|---|---|---|\n"
    fdir = os.path.join(pdir, "fronts")
    if os.path.isdir(fdir):
        fstats = {}
        with open(os.path.join(fdir, "fronts_kernel_stats.csv")) as f:
            for row in csv.DictReader(f):
                fstats[_short(row["Name"])] = (int(row["Calls"]), float(row["AverageNs"]) / 1e3,
                                              float(row["MinNs"]) / 1e3, float(row["MaxNs"]) / 1e3)
        with open(os.path.join(pdir, "fronts_bench.json")) as f:
            fb = json.loads(f.read().strip().splitlines()[-1])["front_sweep"]
        rows = [f"| {k} | {n} | {avg:.1f} | {lo:.1f} | {hi:.1f} |"
                for k, (n, avg, lo, hi) in sorted(fstats.items(), key=lambda x: -x[1][0] * x[1][1])
                if k.startswith(("fused_dpp_batch_kernel", "step_batch_kernel", "front_"))]
        with open(os.path.join(here, "profiles", "front_sweep_kernels_512x256.md"), "w") as f:
            f.write("# Invasion sweep: 12 fronts of 512x256 (delta1 sweep x 2 acid anisotropies), FP64 (rocprofv3)\n\n"
                    f"Command (from /tmp with TMPDIR=/tmp):\n\n```\n{PROFILE_COMMANDS['fronts']}\n```\n\n"
                    "## Kernel trace (--stats)\n\n" + head + "\n".join(rows) +
                    "\n\n`fused_dpp_batch_kernel<double, false, 1, 4>` steps all twelve fronts 4 steps per launch; "
                    "`front_row_kernel` / `front_final_kernel` are the front and gap diagnostics (one wave per row, "
                    f"then a fixed-order reduction).  bench.py in the same run: {fb['value']:.1f} Gcell/s over "
                    f"{fb['workload']}.\n")


def summarize_profiles(pdir):
    """Write profiles/*.md and profiles/step_kernel_traffic.json from the CSV
    output of PROFILE_COMMANDS (trace/, fetch/, write/ and trace_bench.json
    under pdir; trace3/, fetch3/, write3/ and trace3_bench.json for the 3D
    kernel and valu/ for the instruction counts, each of which may be present
    alone)."""
    if os.path.isdir(os.path.join(pdir, "valu")):
        print(json.dumps({"valu": summarize_valu(pdir)}, indent=1))
    if os.path.isdir(os.path.join(pdir, "etrace")):
        print(json.dumps({"ensemble": summarize_ensemble(pdir)}, indent=1))
    if os.path.isdir(os.path.join(pdir, "atrace")):
        print(json.dumps({"adjoint": summarize_adjoint(pdir)}, indent=1))
    if os.path.isdir(os.path.join(pdir, "fronts")):
        summarize_fronts(pdir)
    if not os.path.isdir(os.path.join(pdir, "trace")):
        if os.path.isdir(os.path.join(pdir, "trace3")):
            print(json.dumps({"three_d": summarize_3d(pdir, "trace3", "fetch3", "write3", "trace3_bench.json")},
                             indent=1))
        return
    import csv
    import collections
    here = os.path.dirname(os.path.abspath(__file__))
    stats = {}
    with open(os.path.join(pdir, "trace", "trace_kernel_stats.csv")) as f:
        for row in csv.DictReader(f):
            stats[_short(row["Name"])] = (int(row["Calls"]), float(row["AverageNs"]) / 1e3,
                                         float(row["MinNs"]) / 1e3, float(row["MaxNs"]) / 1e3)
    with open(os.path.join(pdir, "trace_bench.json")) as f:
        bench = json.loads(f.read().strip().splitlines()[-1])

    fetch, write = _counter_means(pdir, "fetch"), _counter_means(pdir, "write")
    ck, f_scale, w_scale = _copy_calibration(fetch, write)
    cells = bench["config"]["grid"][0] * bench["config"]["grid"][1]

    # kernels of the 4096^2 runs: single-step and headline shapes of each variant
    rows_md, traffic = [], {}
    for v, vr in bench["variants"].items():
        for label, tuning, rows in (("single", {"fused_steps": 1, "threads": 0}, 0),
                                    ("headline", vr["tuned"], vr["tuned"]["rows_per_strip"])):
            kname, key = kernel_name(v, tuning)
            ks = [k for k in fetch if k[0] == kname]
            if not ks:
                continue
            k = max(ks, key=lambda x: x[1])
            rd, wr = fetch[k] * 1024 * f_scale, write.get(k, 0.0) * 1024 * w_scale
            alg = BYTES_PER_CELL[v] * cells
            alg_w = (24 if v == "f64" else 12 if v == "f32" else 24) * cells
            traffic[f"{v}/{key}"] = {"kernel": kname, "rows": rows, "read": rd, "write": wr,
                                     "fetch_kib": fetch[k], "write_kib": write.get(k, 0.0)}
            st = stats.get(kname)
            rows_md.append(f"| {v} | {kname} | {rows or 'default'} | {st[0] if st else '-'} | "
                           f"{st[1] if st else float('nan'):.1f} | {fetch[k]:.0f} | {write.get(k, 0.0):.0f} | "
                           f"{rd / 1e6:.1f} | {wr / 1e6:.1f} | {(alg - alg_w) / 1e6:.1f} / {alg_w / 1e6:.1f} | "
                           f"{(rd + wr) / alg:.3f} |")
    srcs = traffic_sources(here)
    with open(os.path.join(here, "profiles", "step_kernel_traffic.json"), "w") as f:
        json.dump({"note": "HBM bytes per launch on the 4096x4096 layered-tissue grid, from rocprofv3 --pmc "
                           "FETCH_SIZE and WRITE_SIZE (separate runs), scaled by what a 1 GiB copyBuffer "
                           f"dispatch reads (FETCH x{f_scale:.3f}, WRITE x{w_scale:.3f}); valid for the kernel "
                           "sources with this digest and the strip heights given (0: library default).",
                   "kernel_sources": srcs, "kernel_sources_sha256": sources_digest(here, srcs),
                   "bytes_per_launch": traffic}, f, indent=1)

    def stat_rows(pred):
        out = []
        for k, (n, avg, lo, hi) in sorted(stats.items(), key=lambda x: -x[1][0] * x[1][1]):
            if pred(k):
                out.append(f"| {k} | {n} | {avg:.1f} | {lo:.1f} | {hi:.1f} |")
        return "\n".join(out)

    head = "| kernel | calls | average (us) | min (us) | max (us) |\n|---|---|---|---|---|\n"
    cmds = "\n".join(PROFILE_COMMANDS[k] for k in ("trace", "fetch", "write"))
    live = {v: vr["launch_avg_us"] for v, vr in bench["variants"].items()}
    with open(os.path.join(here, "profiles", "step_kernels_4096_layered_tissue.md"), "w") as f:
        f.write("# Step kernels, 4096x4096 layered-tissue workload (rocprofv3)\n\n"
                "Commands (from /tmp with TMPDIR=/tmp; $R = repository root, $P = output folder):\n\n"
                f"```\n{cmds}\n```\n\nSummary written by `python bench.py --summarize-profiles $P`.\n\n"
                "## Kernel trace (--stats), 4096^2 step kernels and diagnostics\n\n" + head +
                stat_rows(lambda k: k.startswith(("step_kernel<", "fused_dpp_kernel<", "fused_kernel<",
                                                  "step_adaptive_kernel<", "adapt_", "diag_kernel", "diag_final"))
                          and not k.endswith(", 64>")) +
                "\n\nAverage launch time measured live by bench.py with HIP events in the same traced run "
                "(headline shapes): " + ", ".join(f"{v} {us:.1f} us" for v, us in live.items()) + ".\n\n"
                "## HBM traffic per dispatch (--pmc, one counter per run)\n\n"
                f"Calibration: the 1 GiB `__amd_rocclr_copyBuffer` of the copy-ceiling probe reads "
                f"FETCH_SIZE = {ck[1]:.0f} KiB and WRITE_SIZE = {ck[2]:.0f} KiB per dispatch, so "
                f"FETCH_SIZE is scaled by {f_scale:.3f} and WRITE_SIZE by {w_scale:.3f}.  Algorithmic bytes: "
                "each launch reads u, v, w, a, b, c and writes u, v, w once (the compensated state reads "
                "and writes the low words too), whatever the number of steps it fuses.\n\n"
                "| variant | kernel | rows | calls (trace) | average (us) | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | "
                "scaled read (MB) | scaled write (MB) | algorithmic read / write (MB) | traffic / algorithmic |\n"
                "|---|---|---|---|---|---|---|---|---|---|---|\n" + "\n".join(rows_md) + "\n")
    if os.path.isdir(os.path.join(pdir, "trace3")):
        traffic["three_d"] = summarize_3d(pdir, "trace3", "fetch3", "write3", "trace3_bench.json")
    elif bench.get("three_d"):
        traffic["three_d"] = summarize_3d(pdir, "trace", "fetch", "write", "trace_bench.json")
    print(json.dumps({"calibration": {"fetch": f_scale, "write": w_scale}, "traffic": traffic}, indent=1))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=52)
    ap.add_argument("--n", type=int, default=4096, help="grid side (4096 for the standard workload)")
    ap.add_argument("--variants", default="f64,f32c,f32")
    ap.add_argument("--cpu-steps", type=int, default=200, help="oracle steps on all host threads")
    ap.add_argument("--cpu-steps-single", type=int, default=40, help="oracle steps on one host thread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-ceiling", action="store_true")
    ap.add_argument("--no-host-inclusive", action="store_true",
                    help="skip the run with host buffers (upload and download) inside the timed region")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-adaptive", action="store_true")
    ap.add_argument("--no-fronts", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--only-3d", action="store_true",
                    help="time the three-dimensional step and the copy ceiling only (for its profiles)")
    ap.add_argument("--only-adjoint", action="store_true",
                    help="time the gradient workload, the 4096^2 adjoint step and the copy ceiling only")
    ap.add_argument("--only-ensemble", action="store_true",
                    help="time the ensemble (in the benchmark's batched launch shape) and the copy ceiling only")
    ap.add_argument("--fronts-t", type=float, default=2.0, help="simulated time of the invasion sweep")
    ap.add_argument("--no-tune", action="store_true", help="time the default single-step shape only")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner for the headline shape instead of the fixed shapes")
    ap.add_argument("--force-tuning", default="",
                    help="VARIANT=ROWS,THREADS,FUSED,LANE_SHIFT[;...]: headline launch shapes")
    ap.add_argument("--ensemble-tuning", default="64,32,4",
                    help="THREADS,ROWS[,FUSED]: batched launch shape (default: the shape the batch autotuner "
                         "picks on this workload, which the committed ensemble profile covers)")
    ap.add_argument("--ensemble-autotune", action="store_true",
                    help="run the batch autotuner for the ensemble's launch shape instead")
    ap.add_argument("--summarize-profiles", metavar="DIR", default="",
                    help="write the profiles/ summaries from the output of PROFILE_COMMANDS in DIR; no GPU work")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
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
    if args.only_3d:
        three = time_3d(pk, torch)
        print(json.dumps({"three_d": three, "copy_ceiling_GBs": copy_ceiling(torch)}), flush=True)
        return
    if args.only_ensemble:
        ens = time_ensemble(pk, torch, force=None if args.ensemble_autotune or not args.ensemble_tuning
                            else tuple(int(x) for x in args.ensemble_tuning.split(",")))
        print(json.dumps({"ensemble": ens, "copy_ceiling_GBs": copy_ceiling(torch)}), flush=True)
        return
    if args.only_adjoint:
        adj = time_adjoint(pk, torch)
        print(json.dumps({"adjoint": adj, "copy_ceiling_GBs": copy_ceiling(torch)}), flush=True)
        return
    log(f"generating {args.n}x{args.n} layered-tissue workload")
    w = wl.cfg2(n=args.n)
    variants = [v for v in args.variants.split(",") if v]
    forced = dict(item.split("=") for item in args.force_tuning.split(";") if item)
    res, single = {}, {}
    for v in variants:
        log(f"timing {v}, single-step kernel: {args.warmup} warm-up + {args.steps} timed steps")
        single[v] = time_variant(pk, torch, w, v, args.steps, args.warmup, tune=False)
        log(f"  {v} single-step: {single[v]['value']:.2f} Gcell/s, kernel {single[v]['kernel_avg_us']:.1f} us, "
            f"{single[v]['achieved_GBs']:.0f} GB/s ({100 * single[v]['achieved_GBs'] / PEAK_HBM_GBS:.1f}% of peak)")
        if not args.no_tune:
            if v in forced:
                force = tuple(int(x) for x in forced[v].split(","))
            elif args.autotune:
                force = None
            else:
                force = HEADLINE_SHAPE[v]
            log(f"timing {v}, {'autotuned' if force is None else 'headline'} shape")
            res[v] = time_variant(pk, torch, w, v, args.steps, args.warmup, tune=True, force=force)
            log(f"  {v} shape {res[v]['tuning']}: {res[v]['value']:.2f} Gcell/s, launch {res[v]['kernel_avg_us']:.1f} us "
                f"({res[v]['fused_steps']} steps), effective {res[v]['effective_GBs']:.0f} GB/s")
        else:
            res[v] = single[v]
    host = None
    if not args.no_host_inclusive and not args.no_tune:
        hv = variants[0]
        log(f"timing {hv} with host buffers in the timed region (upload, {args.steps} steps, download)")
        host = time_host_inclusive(pk, torch, w, hv, args.steps, res[hv]["tuning"], res[hv]["dt"])
        host["vs_resident"] = host["value"] / res[hv]["value"]
        log(f"  {host['value']:.2f} Gcell/s ({host['wall_ms']:.1f} ms wall, {host['vs_resident']:.3f} of the "
            "HBM-resident rate)")
    adj = None
    if not args.no_adjoint:
        log("timing the gradient workload (forward with checkpoints, reverse sweep)")
        adj = time_adjoint(pk, torch)
        log(f"  backward/forward = {adj['backward_over_forward']:.2f} (fused forward), "
            f"{adj['backward_over_forward_single_step']:.2f} (single-step forward); adjoint step at 4096^2 "
            f"{adj['adjoint_kernel_4096']['adjoint_step_us']:.1f} us, "
            f"{adj['roofline']['achieved']:.0f} GB/s algorithmic")
    adaptive = None
    if not args.no_adaptive and "f64" in variants:
        log("timing adaptive stepping (device-side step size, FP64)")
        adaptive = time_adaptive(pk, torch, w)
        adaptive["vs_fixed_single_step"] = adaptive["value"] / single["f64"]["value"]
        log(f"  adaptive {adaptive['value']:.2f} Gcell/s ({adaptive['vs_fixed_single_step']:.3f} of the fixed-dt "
            "single-step rate)")
    fronts = None
    if not args.no_fronts:
        log("timing the invasion sweep (fronts and interstitial gap)")
        fronts = time_front_sweep(pk, torch, t_end=args.fronts_t)
        log(f"  {fronts['value']:.1f} Gcell/s; gaps " +
            ", ".join(f"d={x['delta1']}/k={x['kappa']:.1f}: {x['gap_mean'] if x['gap_mean'] is None else round(x['gap_mean'], 4)}"
                      for x in fronts["instances"]))
    three = None
    if not args.no_3d:
        log("timing the three-dimensional step (256^3 slab tissue)")
        three = time_3d(pk, torch)
        log("  " + ", ".join(f"{k}: {v['value']:.1f} Gcell/s, {v['kernel_avg_us']:.0f} us, "
                             f"{100 * v['roofline']['frac']:.1f}% of HBM" for k, v in three["variants"].items()))
    ens = None
    if not args.no_ensemble:
        log("timing the ensemble (batched graph vs loop of single launches)")
        ens = time_ensemble(pk, torch, force=None if args.ensemble_autotune or not args.ensemble_tuning
                            else tuple(int(x) for x in args.ensemble_tuning.split(",")))
        log(f"  batched {ens['batched_Gcell_s']:.1f} Gcell/s vs loop {ens['loop_same_shape_Gcell_s']:.1f} "
            f"Gcell/s in the same shape (x{ens['speedup']:.2f}), {ens['loop_default_shape_Gcell_s']:.1f} in the "
            f"default shape")
    ceiling = None if args.no_copy_ceiling else copy_ceiling(torch)
    base = None
    if not args.no_cpu_baseline:
        log(f"timing the oracle: {args.cpu_steps} steps on all host threads, {args.cpu_steps_single} on one")
        base = cpu_baseline(w, args.cpu_steps, args.cpu_steps_single)
        log(f"  {base['value']:.3f} Gcell/s on {base['cores']} threads, "
            f"{base['single_thread']['value']:.4f} on one ({base['host']['cpu_model']})")

    head = variants[0]
    r = res[head]
    s1 = single[head]
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
            "grid": [w.nx, w.ny], "params": list(w.params), "dt": r["dt"], "launch_shape": r["tuning"],
        },
        "roofline": roofline_of(head, r),
        "single_step_kernel": with_measured({
            "kernel": kernel_name(head, s1["tuning"])[0], "value": s1["value"],
            "kernel_avg_us": s1["kernel_avg_us"], "bound": "hbm",
            "achieved": s1["achieved_GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": s1["achieved_GBs"] / PEAK_HBM_GBS,
            "traffic": measured_traffic(head, s1["tuning"], s1["rows"]),
            "bytes_per_cell_update": BYTES_PER_CELL[head]}, s1["kernel_avg_us"]),
        "cpu_baseline": base,
        "variants": {v: {"tuned": res[v]["tuning"], "value": res[v]["value"],
                         "launch_avg_us": res[v]["kernel_avg_us"], "roofline": roofline_of(v, res[v]),
                         "single_step": {"value": single[v]["value"], "kernel_avg_us": single[v]["kernel_avg_us"],
                                         "achieved_GBs": single[v]["achieved_GBs"],
                                         "frac": single[v]["achieved_GBs"] / PEAK_HBM_GBS,
                                         "traffic": measured_traffic(v, single[v]["tuning"], single[v]["rows"])}}
                     for v in variants},
        "host_inclusive": host,
        "adjoint": adj,
        "adaptive": adaptive,
        "front_sweep": fronts,
        "three_d": three,
        "ensemble": ens,
        "copy_ceiling_GBs": ceiling,
        "mass_log": r["mass_log"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
