"""GPU parity of the adaptive time step (ggfv_step_adaptive) against the oracle's
adaptive run: the step size of every step is derived on the device from the
state that step starts from (Section 2, a new step size after each iteration).

Bar: FP64 states, step sizes and simulated time bit for bit (both sides evaluate
the same FP64 expressions in the same order); compensated FP32 within 1e-5 and
plain FP32 within 5e-4 relative against the FP64 oracle on the FP32-rounded
inputs.  The step size is a function of the state (proportional to
1/max|1-u|), so its relative error is bounded by the state's error times the
condition number max|u| / max|1-u| of that function.
"""
import numpy as np
import pytest

import oracle
import paper_2006_01748_amd as pk
from paper_2006_01748_amd import workloads as wl

pytestmark = pytest.mark.gpu

SEED = wl.BASE_SEED + 700
# Delta2 large enough that the tumour-cell term (with its mobility 1-u) sets the
# step size, so the step size changes from step to step as u evolves
PRM_MOB = (12.5, 1.0, 6.0, 70.0, 60.0)


def rng(k):
    return np.random.Generator(np.random.PCG64(SEED + k))


def inputs(nx, ny, k):
    g = rng(k)
    a, b, c = wl.random_abc(g, nx, ny)
    _, v, w = wl.random_state(g, nx, ny)
    u = 0.2 + 0.7 * g.random((ny, nx))
    return (u, v, w), (a, b, c)


def ctx_of(nx, ny, dtype, prm, state, abc, rows=0):
    ctx = pk.Context(nx, ny, dtype=dtype)
    ctx.set_params(prm)
    ctx.set_tensor(*abc)
    ctx.set_state(*state)
    if rows:
        ctx.set_tuning(rows)
    return ctx


@pytest.mark.parametrize("shape", [(160, 96), (300, 77), (1, 50), (50, 1), (513, 130), (3, 700)])
def test_adaptive_f64_bitwise(shape):
    torch = pytest.importorskip("torch")
    nx, ny = shape
    n = 25
    state, abc = inputs(nx, ny, nx + 7 * ny)
    ctx = ctx_of(nx, ny, "f64", PRM_MOB, state, abc)
    log = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.step_adaptive(0.9, n, log)
    got = ctx.get_state()
    U, V, W, ref_log, t = oracle.run_adaptive(*state, *abc, PRM_MOB, 0.9, n)
    assert np.array_equal(log.cpu().numpy(), ref_log), (log.cpu().numpy()[:4], ref_log[:4])
    assert all(np.array_equal(x, y) for x, y in zip(got, (U, V, W)))
    d = ctx.diagnostics()
    assert d["t"] == t and d["steps"] == n
    if nx * ny > 100:
        assert len(set(ref_log.tolist())) > 1, "the step size should change as u evolves"
    ctx.close()


def test_adaptive_continues_and_mixes_with_fixed_steps():
    """Two adaptive calls and a fixed-step call in between equal the oracle doing
    the same; strip heights do not change the bits."""
    torch = pytest.importorskip("torch")
    nx, ny = 129, 70
    state, abc = inputs(nx, ny, 3)
    for rows in (0, 3, 64):
        ctx = ctx_of(nx, ny, "f64", PRM_MOB, state, abc, rows=rows)
        ctx.step_adaptive(0.8, 7)
        ctx.step(2e-6, 3)
        log = torch.zeros(5, dtype=torch.float64, device="cuda")
        ctx.step_adaptive(0.8, 5, log)
        U, V, W, l1, t1 = oracle.run_adaptive(*state, *abc, PRM_MOB, 0.8, 7)
        U, V, W, _ = oracle.run(U, V, W, *abc, PRM_MOB, 2e-6, 3)
        U, V, W, l2, t2 = oracle.run_adaptive(U, V, W, *abc, PRM_MOB, 0.8, 5, t0=t1 + 3 * 2e-6)
        assert np.array_equal(log.cpu().numpy(), l2)
        assert all(np.array_equal(x, y) for x, y in zip(ctx.get_state(), (U, V, W))), rows
        assert ctx.diagnostics()["t"] == t2
        ctx.close()


def test_adaptive_full_size_layered_tissue():
    """4096^2 layered tissue, 6 adaptive steps, whole state and step sizes against
    the oracle (bitwise)."""
    torch = pytest.importorskip("torch")
    w = wl.cfg2(steps=6)
    a, b, c = oracle.tensor_from_eig(*w.eig)
    # the tensor goes in as (a, b, c): both sides then see identical inputs (the
    # eigen-description map evaluates sin/cos on each side separately)
    ctx = ctx_of(w.nx, w.ny, "f64", w.params, (w.u0, w.v0, w.w0), (a, b, c))
    log = torch.zeros(w.steps, dtype=torch.float64, device="cuda")
    ctx.step_adaptive(0.9, w.steps, log)
    U, V, W, ref_log, t = oracle.run_adaptive(w.u0, w.v0, w.w0, a, b, c, w.params, 0.9, w.steps)
    assert np.array_equal(log.cpu().numpy(), ref_log)
    assert all(np.array_equal(x, y) for x, y in zip(ctx.get_state(), (U, V, W)))
    assert ctx.diagnostics()["t"] == t
    ctx.close()


@pytest.mark.parametrize("dtype,tol", [("f32c", 1e-5), ("f32", 5e-4)])
def test_adaptive_fp32_against_oracle(dtype, tol):
    torch = pytest.importorskip("torch")
    nx, ny = 200, 150
    n = 400
    state, abc = inputs(nx, ny, 11)
    f32 = lambda x: np.float64(np.float32(x))
    state, abc = tuple(f32(x) for x in state), tuple(f32(x) for x in abc)
    prm = tuple(float(np.float32(p)) for p in PRM_MOB)
    ctx = ctx_of(nx, ny, dtype, prm, state, abc)
    log = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.step_adaptive(0.9, n, log)
    U, V, W, ref_log, t = oracle.run_adaptive(*state, *abc, prm, 0.9, n)
    got = ctx.get_state()
    err = max(float(np.max(np.abs(x - y)) / np.max(np.abs(y))) for x, y in zip(got, (U, V, W)))
    assert err <= tol, err
    cond = float(np.max(np.abs(U)) / np.max(np.abs(1.0 - U)))
    dt_err = float(np.max(np.abs(log.cpu().numpy() / ref_log - 1.0)))
    assert dt_err <= tol * cond, (dt_err, cond)
    ctx.close()


def test_adaptive_errors():
    torch = pytest.importorskip("torch")
    ctx = pk.Context(20, 10, dtype="f64")
    with pytest.raises(pk.GGFVError) as e:
        ctx.step_adaptive(0.9, 3)
    assert e.value.status == pk.GGFV_ESTATE
    state, abc = inputs(20, 10, 5)
    ctx.set_params(PRM_MOB)
    ctx.set_tensor(*abc)
    ctx.set_state(*state)
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(pk.GGFVError) as e:
            ctx.step_adaptive(bad, 3)
        assert e.value.status == pk.GGFV_EINVAL
    with pytest.raises(pk.GGFVError):
        ctx.step_adaptive(0.9, -1)
    with pytest.raises(ValueError):
        ctx.step_adaptive(0.9, 4, torch.zeros(3, dtype=torch.float64, device="cuda"))
    ctx.step_adaptive(0.9, 0)
    assert ctx.diagnostics()["steps"] == 0
    ctx.close()
