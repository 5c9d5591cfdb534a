"""GPU tests of the batched ensemble: every instance of a batched run equals the
same instance stepped alone (bit for bit), sampled instances match the FP64
oracle, graph replays equal eager launches, and the tuners restore the state."""
import numpy as np
import pytest

import oracle
import paper_2006_01748_amd as pk
from paper_2006_01748_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _instances(count, steps, sides=None):
    return [wl.cfg3_instance(i, steps, None if sides is None else sides[i % len(sides)]) for i in range(count)]


def _setup_single(w, dtype, dt):
    ctx = pk.Context(w.nx, w.ny, dtype=dtype)
    ctx.set_params(w.params)
    ctx.set_tensor_eig(*w.eig)
    ctx.set_state(w.u0, w.v0, w.w0)
    return ctx


def _setup_batch(ws, dtype):
    b = pk.Batch([(w.nx, w.ny) for w in ws], dtype=dtype)
    dts = []
    for i, w in enumerate(ws):
        c = b[i]
        c.set_params(w.params)
        c.set_tensor_eig(*w.eig)
        c.set_state(w.u0, w.v0, w.w0)
        dt = c.stable_dt(w.safety)
        b.set_dt(i, dt)
        dts.append(dt)
    return b, dts


@pytest.mark.parametrize("dtype", ["f64", "f32c", "f32"])
@pytest.mark.parametrize("threads", [64, 256])
def test_batch_equals_single_instances_bitwise(dtype, threads):
    ws = _instances(10, 37, sides=[64, 96, 130, 200, 512, 33])
    # a rectangular and a one-column instance as well
    ws.append(wl.Workload("rect", 47, 33, 1.0, 1.0, ws[0].params, *wl.disks_state(47, 33, [(0.5, 0.5)], 0.2),
                          eig=wl.random_eig(np.random.Generator(np.random.PCG64(5)), 47, 33), safety=0.9))
    ws.append(wl.Workload("col", 1, 40, 1.0, 1.0, ws[1].params, *wl.disks_state(1, 40, [(0.5, 0.5)], 0.2),
                          eig=wl.random_eig(np.random.Generator(np.random.PCG64(6)), 1, 40), safety=0.9))
    b, dts = _setup_batch(ws, dtype)
    b.set_tuning(threads=threads, rows_per_strip=0, graph_steps=10)
    b.run(37)                      # 3 graph replays + 7 single launches
    for i, w in enumerate(ws):
        got = b[i].get_state()
        ctx = _setup_single(w, dtype, dts[i])
        ctx.step(dts[i], 37)
        ref = ctx.get_state()
        assert all(np.array_equal(x, y) for x, y in zip(got, ref)), (i, w.nx, w.ny)
        assert b[i].diagnostics()["steps"] == 37
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32c", "f32"])
@pytest.mark.parametrize("K", [2, 3, 4])
def test_fused_batch_equals_single_instances_bitwise(dtype, K):
    """The ensemble form of the lane-shift kernel (K steps per launch, graph
    replays, single-step remainder) gives every instance the bits of that
    instance stepped alone."""
    ws = _instances(9, 37, sides=[64, 96, 130, 200, 33])
    ws.append(wl.Workload("rect", 47, 33, 1.0, 1.0, ws[0].params, *wl.disks_state(47, 33, [(0.5, 0.5)], 0.2),
                          eig=wl.random_eig(np.random.Generator(np.random.PCG64(7)), 47, 33), safety=0.9))
    ws.append(wl.Workload("col", 1, 40, 1.0, 1.0, ws[1].params, *wl.disks_state(1, 40, [(0.5, 0.5)], 0.2),
                          eig=wl.random_eig(np.random.Generator(np.random.PCG64(8)), 1, 40), safety=0.9))
    ws.append(wl.Workload("row", 150, 1, 1.0, 1.0, ws[2].params, *wl.disks_state(150, 1, [(0.5, 0.5)], 0.2),
                          eig=wl.random_eig(np.random.Generator(np.random.PCG64(9)), 150, 1), safety=0.9))
    refs = []
    b, dts = _setup_batch(ws, dtype)
    for i, w in enumerate(ws):
        ctx = _setup_single(w, dtype, dts[i])
        ctx.step(dts[i], 37)
        refs.append(ctx.get_state())
        ctx.close()
    for rows, graph in ((0, 10), (5, 0), (1, 24)):
        for i, w in enumerate(ws):
            b[i].set_state(w.u0, w.v0, w.w0)
        b.set_tuning(threads=64, rows_per_strip=rows, graph_steps=graph, fused_steps=K)
        assert b.get_tuning()["fused_steps"] == K
        b.run(37)
        for i, w in enumerate(ws):
            got = b[i].get_state()
            assert all(np.array_equal(x, y) for x, y in zip(got, refs[i])), (i, w.nx, w.ny, rows, graph)
    b.close()


def test_fused_batch_graph_replays_and_split_runs():
    """Runs split at arbitrary step counts (odd launch counts, remainders) and
    repeated graph replays with host reads in between equal one eager run."""
    ws = _instances(5, 40, sides=[64, 160, 256])
    b1, _ = _setup_batch(ws, "f32c")
    b1.set_tuning(threads=64, graph_steps=0, fused_steps=1)
    b2, _ = _setup_batch(ws, "f32c")
    b2.set_tuning(threads=64, rows_per_strip=8, graph_steps=16, fused_steps=4)
    for n in (17, 16, 33, 5, 40):
        b1.run(n)
        b2.run(n)
        for i in range(len(ws)):
            x, y = b1[i].get_state(), b2[i].get_state()
            assert all(np.array_equal(p, q) for p, q in zip(x, y)), (n, i)
            assert b2[i].diagnostics()["steps"] == b1[i].diagnostics()["steps"]
    b1.close()
    b2.close()


def _oracle_sample(ws):
    """Sixteen instances of the ensemble for the oracle: the first instance of
    every side 64, 96, ..., 512 and the second 512^2 one."""
    first = {}
    for i, w in enumerate(ws):
        first.setdefault(w.nx, []).append(i)
    pick = [first[s][0] for s in sorted(first)]
    pick.append(first[max(first)][1])
    return pick


@pytest.fixture(scope="module")
def ensemble_oracle():
    """The 256-instance ensemble (sides 64..512, 5000 steps) with FP32-rounded
    inputs and steps from the oracle's own tensor map and step bound, and the
    FP64 oracle's final states of 16 instances covering every side."""
    ws = wl.cfg3(256, 5000)
    f32 = lambda x: np.float64(np.float32(x))
    inputs = []
    for w in ws:
        abc = tuple(f32(x) for x in oracle.tensor_from_eig(*(f32(x) for x in w.eig)))
        prm = tuple(float(np.float32(p)) for p in w.params)
        st = tuple(f32(x) for x in (w.u0, w.v0, w.w0))
        dt = float(np.float32(oracle.stable_dt(*abc, prm[2], w.safety)))
        inputs.append((abc, prm, st, dt))
    pick = _oracle_sample(ws)
    assert len(pick) == 16 and len({ws[i].nx for i in pick}) == 15
    refs = {}
    for i in pick:
        abc, prm, st, dt = inputs[i]
        refs[i] = oracle.run(*st, *abc, prm, dt, ws[i].steps)[:3]
    return ws, inputs, refs


@pytest.mark.timeout(900)
@pytest.mark.parametrize("fused", [1, 4])
def test_full_ensemble_against_oracle_sampled(ensemble_oracle, fused):
    """256 instances (sides 64..512), compensated FP32, 5000 steps in one batched
    run (one or four steps per launch, graph replays); 16 instances, one of
    every side and two of 512^2, against the FP64 oracle on the same FP32
    inputs (1e-5 relative max-norm per field)."""
    ws, inputs, refs = ensemble_oracle
    f32 = lambda x: np.asarray(x, np.float32)
    b = pk.Batch([(w.nx, w.ny) for w in ws], dtype="f32c")
    for i, (abc, prm, st, dt) in enumerate(inputs):
        b.set(i, prm, dt, tuple(f32(x) for x in abc), tuple(f32(x) for x in st))
    b.set_tuning(threads=64, rows_per_strip=16, graph_steps=48, fused_steps=fused)
    b.run(5000)
    worst = 0.0
    for i, ref in refs.items():
        got = b[i].get_state()
        err = max(float(np.max(np.abs(x - y)) / np.max(np.abs(y))) for x, y in zip(got, ref))
        worst = max(worst, err)
        assert err <= 1e-5, (i, ws[i].nx, err)
    print(f"ensemble: worst per-instance max-norm error vs FP64 oracle over {len(refs)} instances "
          f"(sides {sorted({ws[i].nx for i in refs})}): {worst:.3e}")
    for i in range(len(ws)):
        d = b[i].diagnostics()
        assert d["nonfinite"] == 0 and d["steps"] == 5000
    b.close()


def test_graph_replays_equal_eager_launches():
    ws = _instances(6, 40, sides=[64, 160, 256])
    b1, _ = _setup_batch(ws, "f64")
    b1.set_tuning(threads=64, graph_steps=0)
    b2, _ = _setup_batch(ws, "f64")
    b2.set_tuning(threads=64, graph_steps=4)
    for rep in range(5):                        # several replays, host reads in between
        b1.run(8)
        b2.run(8)
        for i in range(len(ws)):
            x, y = b1[i].get_state(), b2[i].get_state()
            assert all(np.array_equal(p, q) for p, q in zip(x, y)), (rep, i)
    b1.close()
    b2.close()


def test_batch_autotune_keeps_results():
    ws = _instances(5, 30, sides=[64, 128, 300])
    b, dts = _setup_batch(ws, "f32c")
    before = [b[i].get_state() for i in range(len(ws))]
    best = b.autotune(trial_steps=4)
    assert best["threads"] in (64, 256) and best["rows_per_strip"] in (4, 8, 16, 32, 64)
    assert best["fused_steps"] in (1, 2, 3, 4) and b.get_tuning()["fused_steps"] == best["fused_steps"]
    for i in range(len(ws)):
        assert all(np.array_equal(p, q) for p, q in zip(before[i], b[i].get_state()))
        assert b[i].diagnostics()["steps"] == 0
    b.run(30)
    ref, _ = _setup_batch(ws, "f32c")
    ref.run(30)
    for i in range(len(ws)):
        assert all(np.array_equal(p, q) for p, q in zip(b[i].get_state(), ref[i].get_state()))
    b.close()
    ref.close()


def test_single_context_autotune_and_narrow_width():
    w = wl.cfg1(n=300, steps=20)
    ctx = pk.Context(w.nx, w.ny, dtype="f64")
    ctx.set_params(w.params)
    ctx.set_tensor_eig(*w.eig)
    ctx.set_state(w.u0, w.v0, w.w0)
    dt = ctx.stable_dt(0.9)
    before = ctx.get_state()
    best = ctx.autotune(dt, trial_steps=3)
    assert best["threads"] in (64, 128, 256)
    assert all(np.array_equal(p, q) for p, q in zip(before, ctx.get_state()))
    ctx.step(dt, 20)
    tuned = ctx.get_state()
    for threads, rows in ((64, 8), (256, 13), (64, 300), (128, 5)):
        ctx.set_tuning(rows, threads)
        ctx.set_state(w.u0, w.v0, w.w0)
        ctx.step(dt, 20)
        assert all(np.array_equal(p, q) for p, q in zip(tuned, ctx.get_state())), (threads, rows)


def test_batch_errors():
    ws = _instances(2, 5, sides=[64])
    b = pk.Batch([(w.nx, w.ny) for w in ws], dtype="f64")
    with pytest.raises(pk.GGFVError) as e:
        b.run(1)
    assert e.value.status == pk.GGFV_ESTATE
    with pytest.raises(pk.GGFVError):
        b.set_tuning(threads=100)
    with pytest.raises(pk.GGFVError):
        b.set_tuning(threads=64, fused_steps=5)
    with pytest.raises(pk.GGFVError):
        b.set_dt(5, 1e-6)
    with pytest.raises(pk.GGFVError):
        b.set_dt(0, -1.0)
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32c"])
def test_batch_set_and_get_state_calls(dtype):
    """ggfv_batch_set (parameters, tensor, state and dt of an instance in one
    call) and ggfv_batch_get_state give the bits of the per-instance calls."""
    g = np.random.Generator(np.random.PCG64(wl.BASE_SEED + 77))
    sizes = [(70, 33), (1, 20), (129, 64)]
    prms = [(12.5, 1.0, 0.01, 70.0, 70.0), (3.0, 1.0, 0.05, 40.0, 30.0), (0.5, 1.0, 0.002, 90.0, 90.0)]
    cases = []
    for (nx, ny), prm in zip(sizes, prms):
        abc = wl.random_abc(g, nx, ny)
        st = wl.random_state(g, nx, ny)
        dt = oracle.stable_dt(*abc, prm[2], 0.8)
        cases.append((prm, dt, abc, st))
    b = pk.Batch(sizes, dtype=dtype)
    for i, (prm, dt, abc, st) in enumerate(cases):
        b.set(i, prm, dt, abc, st)
    b.run(9)
    for i, (prm, dt, abc, st) in enumerate(cases):
        nx, ny = sizes[i]
        ctx = pk.Context(nx, ny, dtype=dtype)
        ctx.set_params(prm)
        ctx.set_tensor(*abc)
        ctx.set_state(*st)
        ctx.step(dt, 9)
        ref = ctx.get_state()
        ctx.close()
        got = b.get_state(i)
        assert all(np.array_equal(x, y) for x, y in zip(got, ref)), i
        assert all(np.array_equal(x, y) for x, y in zip(b[i].get_state(), ref)), i
    with pytest.raises(pk.GGFVError) as e:
        b.set(3, prms[0], 1e-6, cases[0][2], cases[0][3])
    assert e.value.status == pk.GGFV_EINVAL
    with pytest.raises(pk.GGFVError) as e:
        b.set(0, prms[0], 0.0, cases[0][2], cases[0][3])
    assert e.value.status == pk.GGFV_EINVAL
    with pytest.raises(pk.GGFVError):
        b.get_state(-1)
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32c"])
def test_batch_device_tensor_io_orders_with_torch(dtype):
    """Instance state written by torch kernels on torch's stream just before
    set_state, and read by a torch kernel just after get_state, with no
    synchronization in between: the batch's own stream is ordered with
    torch's, so the device-pointer path gives the bits of the host path."""
    torch = pytest.importorskip("torch")
    ws = _instances(4, 24, sides=[64, 200, 96, 512])
    host, _ = _setup_batch(ws, dtype)
    host.set_tuning(threads=64, graph_steps=8, fused_steps=4)
    host.run(24)
    ref = [host[i].get_state() for i in range(len(ws))]
    host.close()
    b, _ = _setup_batch(ws, dtype)
    b.set_tuning(threads=64, graph_steps=8, fused_steps=4)
    big = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
    for i, w in enumerate(ws):
        # state produced on the device behind a long torch kernel
        st = [torch.from_numpy(x).cuda() for x in (w.u0, w.v0, w.w0)]
        for _ in range(4):
            big.mul_(1.0)
        dev = [x * (big[0] * 1.0) for x in st]
        b[i].set_state(*dev)
    b.run(24)
    for i, w in enumerate(ws):
        out = [torch.full((w.ny, w.nx), float("nan"), dtype=torch.float64, device="cuda") for _ in range(3)]
        b[i].get_state(out=out)
        copies = [x.clone() for x in out]          # a torch kernel right behind the library's
        for x, r in zip(copies, ref[i]):
            assert np.array_equal(x.cpu().numpy(), r), (i, w.nx)
    b.close()
