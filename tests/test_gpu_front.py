"""GPU front diagnostics and the invasion sweep (Section 2's propagating tumour
fronts and interstitial gap) against the oracle.

Bar: row counts, minima and maxima of the front positions bit for bit (each row
is the same FP64 expression on the same values); means within 1e-14 relative
(the GPU sums rows in a fixed tree order, the oracle serially).  The sweep's
states are checked against the paper's qualitative claims and its diagnostics
against the oracle applied to the GPU's own state.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2006_01748_amd as pk
from paper_2006_01748_amd import workloads as wl

pytestmark = pytest.mark.gpu


def same_front(got, ref):
    assert got["rows_front"] == ref["rows_front"] and got["rows_gap"] == ref["rows_gap"]
    for key in ("tumour", "tissue", "gap"):
        g, r = got[key], ref[key]
        assert g[1] == r[1] and g[2] == r[2], (key, g, r)
        assert math.isclose(g[0], r[0], rel_tol=1e-14, abs_tol=1e-300), (key, g, r)


def ramps(nx, ny, lx, seed):
    x = (np.arange(nx) + 0.5) * (lx / nx)
    g = np.random.Generator(np.random.PCG64(seed))
    av = g.uniform(0.2, 0.6, ny)
    au = av + g.uniform(0.05, 0.5, ny)
    v = np.clip(0.5 + (av[:, None] - x[None, :]) / g.uniform(0.02, 0.2, ny)[:, None], 0.0, 1.0)
    u = np.clip(0.25 + (x[None, :] - au[:, None]) / g.uniform(0.02, 0.2, ny)[:, None], 0.0, 1.0)
    v[::7] = 0.0                     # rows without a tumour front
    u[3::11] = 0.1                   # rows without a tissue front
    return u, v


@pytest.mark.parametrize("dtype", ["f64", "f32c", "f32"])
@pytest.mark.parametrize("shape", [(300, 77), (1, 9), (70, 1), (1000, 5)])
def test_front_diagnostics_match_oracle(dtype, shape):
    nx, ny = shape
    lx = 1.7
    u, v = ramps(nx, ny, lx, nx + ny)
    ctx = pk.Context(nx, ny, lx, 0.5, dtype=dtype)
    ctx.set_state(u, v, np.zeros_like(u))
    got = ctx.front_diagnostics(0.25, 0.5)
    U, V, _ = ctx.get_state()
    same_front(got, oracle.front_diag(U, V, 0.25, 0.5, lx))
    ctx.close()


def test_invasion_run_bitwise_and_fronts():
    """A narrow channel (the oracle's invasion pin): d = 12.5, 40000 steps on the
    GPU equal the oracle bit for bit, and so do the fronts."""
    nx, ny, lx, ly = 100, 2, 1.0, 0.02
    x = (np.arange(nx) + 0.5) / nx
    v0 = np.tile((x < 0.2).astype(float), (ny, 1))
    u0, w0, ones = np.ones((ny, nx)), np.zeros((ny, nx)), np.ones((ny, nx))
    prm = (12.5, 1.0, 0.01, 70.0, 70.0)
    ctx = pk.Context(nx, ny, lx, ly, dtype="f64")
    ctx.set_params(prm)
    ctx.set_tensor(ones, 0 * ones, ones)
    ctx.set_state(u0, v0, w0)
    dt = ctx.stable_dt(0.9)
    ctx.step(dt, 40000)
    U, V, W, _ = oracle.run(u0, v0, w0, ones, 0 * ones, ones, prm, dt, 40000, lx, ly)
    assert all(np.array_equal(p, q) for p, q in zip(ctx.get_state(), (U, V, W)))
    got = ctx.front_diagnostics(0.25, 0.5)
    same_front(got, oracle.front_diag(U, V, 0.25, 0.5, lx))
    assert got["gap"][1] > 0.05
    ctx.close()


def test_invasion_sweep_batch():
    """delta1 sweep across 1 (lower vertical acid diffusivity as a second set),
    256 x 128 fronts, batched lane-shift kernel, t = 0.5: the gap opens for large
    delta1 only and the tumour front travels faster with delta1; the front diagnostics of
    every instance equal the oracle's on the GPU state; the LeVeque-Yee speed of
    the tumour grows with delta1 as well."""
    ws = wl.front_sweep(deltas=(0.5, 0.8, 1.5, 3.0, 12.5), kappas=(1.0, 0.2), nx=256, ny=128)
    b = pk.Batch([(w.nx, w.ny) for w in ws], lx=ws[0].lx, ly=ws[0].ly, dtype="f32c")
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
    f0 = [b[i].front_diagnostics(0.25, 0.5) for i in range(len(ws))]
    m0 = [b[i].diagnostics()["mass"][1] for i in range(len(ws))]
    n = int(0.5 / dt)
    b.run(n)
    t = [b[i].diagnostics()["t"] for i in range(len(ws))]
    res = {}
    keys = [(k, d) for k in (1.0, 0.2) for d in (0.5, 0.8, 1.5, 3.0, 12.5)]   # front_sweep's order
    for i, w in enumerate(ws):
        f = b[i].front_diagnostics(0.25, 0.5)
        U, V, _ = b[i].get_state()
        same_front(f, oracle.front_diag(U, V, 0.25, 0.5, w.lx))
        m1 = b[i].diagnostics()["mass"][1]
        speed = pk.front_speed(m0[i], m1, 0.0, t[i], w.ly, 1.0, 0.0)
        disp = (f["tumour"][0] - f0[i]["tumour"][0]) / t[i]
        assert w.params[0] == keys[i][1]
        res[keys[i]] = (f, speed, disp)
    for kappa in (1.0, 0.2):
        gaps = [res[(kappa, d)][0]["gap"][0] if res[(kappa, d)][0]["rows_gap"] else 0.0
                for d in (0.5, 0.8, 1.5, 3.0, 12.5)]
        fronts = [res[(kappa, d)][0]["tumour"][0] for d in (0.5, 0.8, 1.5, 3.0, 12.5)]
        print(f"kappa {kappa}: fronts {np.round(fronts, 4)}, gaps {np.round(gaps, 4)}, speeds "
              f"{[round(res[(kappa, d)][1], 4) for d in (0.5, 0.8, 1.5, 3.0, 12.5)]}")
        # the gap belongs to the homogeneous (large delta1) invasion only
        assert gaps[0] < 0.02 and gaps[-1] > 0.05 and gaps[-1] > gaps[0], gaps
        assert all(f1 < f2 for f1, f2 in zip(fronts, fronts[1:])), fronts
        # the space-averaged (LeVeque-Yee) speed of the tumour orders the invasions
        # the same way (the fronts are still settling from their initial step at
        # this horizon, so it is not compared with the threshold's displacement)
        speeds = [res[(kappa, d)][1] for d in (0.5, 0.8, 1.5, 3.0, 12.5)]
        assert speeds[0] > 0 and all(s1 < s2 for s1, s2 in zip(speeds, speeds[1:])), speeds
    b.close()
