"""GPU parity of the HIP step against the FP64 oracle (through the C ABI).

Bar: FP64 within 1e-12 relative max-norm per field (bitwise agreement is expected
since both sides follow the same arithmetic order without FMA, and is checked
where both sides see identical inputs); FP32 with compensated state within 1e-5
relative after 1e4 steps against the FP64 oracle run on the FP32-rounded inputs.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2006_01748_amd as pk
from paper_2006_01748_amd import workloads as wl

pytestmark = pytest.mark.gpu

SEED = wl.BASE_SEED + 300
PRM = wl.PARAMS_REF


def rng(k):
    return np.random.Generator(np.random.PCG64(SEED + k))


def rel_err(got, ref):
    return max(float(np.max(np.abs(np.asarray(g, np.float64) - r)) / max(np.max(np.abs(r)), 1e-300))
               for g, r in zip(got, ref))


# launch shape of the single-step kernel (one step per launch, default width)
SINGLE = (0, 0, 1, 0)


def gpu_ctx(nx, ny, dtype, params, state, abc=None, eig=None, lx=1.0, ly=1.0, rows=0):
    """A context in the library's default launch shape, or (rows > 0) on the
    single-step kernel with that strip height."""
    ctx = pk.Context(nx, ny, lx, ly, dtype=dtype)
    ctx.set_params(params)
    if abc is not None:
        ctx.set_tensor(*abc)
    else:
        ctx.set_tensor_eig(*eig)
    ctx.set_state(*state)
    if rows:
        ctx.set_tuning(rows)
    return ctx


def test_default_launch_shape_follows_the_grid_size():
    """A new context's launch shape: four steps per launch on the lane-shift
    kernels (wide lanes except for the compensated state) on large grids, two
    on mid-sized ones, the single-step kernel on small ones; several steps per
    launch need the lane-shift kernels."""
    for n, K in ((4096, 4), (1024, 2), (256, 1)):
        for dtype, lanes in (("f64", 2), ("f32c", 1)):
            ctx = pk.Context(n, n, dtype=dtype)
            want = {"rows_per_strip": 0, "threads": 0, "fused_steps": K, "lane_shift": lanes if K > 1 else 0}
            assert ctx.get_tuning() == want, (n, dtype, ctx.get_tuning())
            ctx.close()
    ctx = pk.Context(64, 48, dtype="f64")
    with pytest.raises(pk.GGFVError) as e:
        ctx.set_tuning(0, 64, 2, lane_shift=0)
    assert e.value.status == pk.GGFV_EINVAL
    ctx.close()


@pytest.mark.parametrize("nx,ny,rows", [(300, 77, 0), (1, 50, 7), (50, 1, 0), (257, 3, 2), (64, 64, 5),
                                        (513, 130, 0), (2, 2, 1), (1000, 9, 4), (3, 700, 0)])
def test_f64_ragged_shapes_bitwise(nx, ny, rows):
    g = rng(nx * 7 + ny)
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    prm = (12.5, 1.0, 0.05, 70.0, 55.0)
    lx, ly = 1.0, 0.8
    dt = oracle.stable_dt(a, b, c, prm[2], 0.9, lx, ly)
    ref = oracle.run(u, v, w, a, b, c, prm, dt, 25, lx, ly)[:3]
    # the single-step kernel at this strip height, then the default shape
    for single in (True, False):
        ctx = gpu_ctx(nx, ny, "f64", prm, (u, v, w), abc=(a, b, c), lx=lx, ly=ly)
        if single:
            ctx.set_tuning(rows)
        assert ctx.stable_dt(0.9) == dt
        ctx.step(dt, 25)
        got = ctx.get_state()
        ctx.close()
        assert rel_err(got, ref) <= 1e-12
        assert all(np.array_equal(x, y) for x, y in zip(got, ref)), single


def test_f64_smooth_anisotropic_eig_tensor():
    """cfg1 recipe at 256^2; each side maps (lambda1, lambda2, theta) itself."""
    w = wl.cfg1(n=256, steps=1000)
    a, b, c = oracle.tensor_from_eig(*w.eig)
    dt = oracle.stable_dt(a, b, c, w.params[2], 0.9)
    ctx = gpu_ctx(w.nx, w.ny, "f64", w.params, (w.u0, w.v0, w.w0), eig=w.eig)
    ga, gb, gc = ctx.get_tensor()
    scale = np.max(w.eig[0])
    for x, y in ((ga, a), (gb, b), (gc, c)):
        assert np.max(np.abs(x - y)) <= 4e-16 * scale
    gdt = ctx.stable_dt(0.9)
    assert math.isclose(gdt, dt, rel_tol=1e-15)
    ctx.step(gdt, w.steps)
    got = ctx.get_state()
    ref = oracle.run(w.u0, w.v0, w.w0, a, b, c, w.params, dt, w.steps)[:3]
    assert rel_err(got, ref) <= 1e-12


def _patch_reference(w, a, b, c, dt, steps, j0, j1, i0, i1):
    """Oracle on a sub-window grown by `steps` cells on every side that is not a
    domain edge; the inner window is then exact (the scheme has a one-cell
    stencil per step)."""
    J0, J1 = max(0, j0 - steps), min(w.ny, j1 + steps)
    I0, I1 = max(0, i0 - steps), min(w.nx, i1 + steps)
    sl = (slice(J0, J1), slice(I0, I1))
    dx = w.lx / w.nx
    dy = w.ly / w.ny
    lx, ly = (I1 - I0) * dx, (J1 - J0) * dy
    # idx and idy must be the full grid's: same cell size, so nx'/lx' = nx/lx
    u, v, ww, _ = oracle.run(w.u0[sl], w.v0[sl], w.w0[sl], a[sl], b[sl], c[sl], w.params, dt, steps, lx, ly)
    inner = (slice(j0 - J0, j1 - J0), slice(i0 - I0, i1 - I0))
    return u[inner], v[inner], ww[inner]


@pytest.mark.parametrize("dtype", ["f64"])
def test_full_size_layered_tissue_patches(dtype):
    """4096^2 layered tissue (Voronoi regions + membranes), launch shape as timed
    by the benchmark, 60 steps; outputs sampled on corner, edge and interior
    windows, each recomputed exactly by the oracle on a grown sub-window."""
    w = wl.cfg2(steps=60)
    a, b, c = oracle.tensor_from_eig(*w.eig)
    ctx = gpu_ctx(w.nx, w.ny, dtype, w.params, (w.u0, w.v0, w.w0), eig=w.eig)
    dt = oracle.stable_dt(a, b, c, w.params[2], 0.9)
    assert math.isclose(ctx.stable_dt(0.9), dt, rel_tol=1e-15)
    ctx.step(dt, w.steps)
    got = ctx.get_state()
    n = w.nx
    windows = [(0, 40, 0, 40), (n - 40, n, n - 40, n), (0, 40, 2000, 2060), (2030, 2070, 2030, 2070),
               (1000, 1040, n - 40, n)]
    for (j0, j1, i0, i1) in windows:
        ref = _patch_reference(w, a, b, c, dt, w.steps, j0, j1, i0, i1)
        sub = [x[j0:j1, i0:i1] for x in got]
        for s, r in zip(sub, ref):
            assert np.max(np.abs(s - r)) <= 1e-12 * max(np.max(np.abs(r)), 1.0)


def test_smooth_anisotropic_1024_2000_steps_headline_shape():
    """The smooth anisotropic workload at its full 1024^2, 2000 FP64 steps in the
    headline launch shape (four steps per launch, wide lanes, the library's
    strip height), against a full oracle run: equal bit for bit."""
    w = wl.cfg1(n=1024, steps=2000)
    a, b, c = oracle.tensor_from_eig(*w.eig)
    dt = oracle.stable_dt(a, b, c, w.params[2], 0.9)
    ctx = gpu_ctx(w.nx, w.ny, "f64", w.params, (w.u0, w.v0, w.w0), abc=(a, b, c))
    ctx.set_tuning(0, 64, 4, lane_shift=2)
    ctx.step(dt, w.steps)
    got = ctx.get_state()
    ctx.close()
    ref = oracle.run(w.u0, w.v0, w.w0, a, b, c, w.params, dt, w.steps)[:3]
    for name, x, r in zip("uvw", got, ref):
        assert np.array_equal(x, r), (name, float(np.max(np.abs(x - r))))


@pytest.mark.parametrize("delta1", [1.0, 12.5, 20.0])
def test_full_size_500_steps_headline_shape_each_delta1(delta1):
    """4096^2 layered tissue, 500 FP64 steps in the benchmark's launch shape
    (four steps per launch, wide lanes, the library's strip height), for each
    kill rate of the workload recipe; an 8x8 window on the tumour disk's edge
    (and, for the largest rate, a corner) recomputed exactly by the oracle on a
    sub-grid grown by 500 cells: equal bit for bit."""
    w = wl.cfg2(delta1=delta1, steps=500)
    a, b, c = oracle.tensor_from_eig(*w.eig)
    ctx = gpu_ctx(w.nx, w.ny, "f64", w.params, (w.u0, w.v0, w.w0), abc=(a, b, c))
    ctx.set_tuning(0, 64, 4, lane_shift=2)
    dt = oracle.stable_dt(a, b, c, w.params[2], 0.9)
    ctx.step(dt, w.steps)
    got = ctx.get_state()
    ctx.close()
    windows = [(2044, 2052, 2250, 2258)] + ([(0, 8, 0, 8)] if delta1 == 20.0 else [])
    for (j0, j1, i0, i1) in windows:
        ref = _patch_reference(w, a, b, c, dt, w.steps, j0, j1, i0, i1)
        for name, x, r in zip("uvw", (x[j0:j1, i0:i1] for x in got), ref):
            assert np.array_equal(x, r), (name, j0, i0, float(np.max(np.abs(x - r))))


@pytest.mark.parametrize("dtype,shape", [("f64", (0, 64, 4, 2)), ("f32", (0, 64, 4, 2)), ("f32c", (0, 64, 4, 1))])
def test_full_size_10000_steps_transpose_and_reflection(dtype, shape):
    """The scheme is equivariant, bit for bit, under the transpose (x <-> y with
    a <-> c) and the reflection x -> 1 - x (with b -> -b); the oracle pins both,
    and the device matches the oracle bit for bit, so the device must keep them
    exactly at any size and length (the FP32 kernels evaluate the same
    expressions, so they keep them too).  4096^2 layered tissue with a
    perturbed, asymmetric state, the workload's 10000 steps in the benchmark's
    launch shape of each precision: the transposed and the mirrored problems
    (which fall on different strips, lanes and strip seams) give the transposed
    and mirrored result."""
    w = wl.cfg2(steps=10000)
    a, b, c = oracle.tensor_from_eig(*w.eig)
    g = rng(77)
    u0 = np.clip(w.u0 + 0.05 * g.random(w.u0.shape), 0.0, 1.0)
    w0 = 0.1 * g.random(w.u0.shape)
    state = (u0, w.v0, w0)
    C = np.ascontiguousarray

    def run(st, abc, dt=None):
        ctx = gpu_ctx(w.nx, w.ny, dtype, w.params, [C(x) for x in st], abc=[C(x) for x in abc])
        ctx.set_tuning(*shape)
        dt = ctx.stable_dt(0.9) if dt is None else dt
        ctx.step(dt, w.steps)
        out = ctx.get_state()
        ctx.close()
        return out, dt

    base, dt = run(state, (a, b, c))
    print(f"base run done, dt={dt!r}", flush=True)
    tr, _ = run([x.T for x in state], (c.T, b.T, a.T), dt)
    for name, x, y in zip("uvw", tr, base):
        assert np.array_equal(x, y.T), f"{name}: transposed run differs"
    mi, _ = run([x[:, ::-1] for x in state], (a[:, ::-1], -b[:, ::-1], c[:, ::-1]), dt)
    for name, x, y in zip("uvw", mi, base):
        assert np.array_equal(x, y[:, ::-1]), f"{name}: mirrored run differs"


@pytest.mark.parametrize("dtype,shape,tol", [("f64", (0, 64, 4, 2), 1e-10), ("f32", (0, 64, 4, 2), 1e-4),
                                             ("f32c", (0, 64, 4, 1), 1e-7)])
def test_full_size_10000_steps_conservation_and_equilibria(dtype, shape, tol):
    """Properties that hold at any size, at the benchmark's size and length in
    each precision's headline shape.  With the reactions off, zero boundary
    flux conserves the tumour-cell and acid masses: every face flux leaves one
    cell and enters the other, so only the rounding of each cell's update moves
    the sum (bars: 10^4 steps x 10 x the unit roundoff, FP64 1e-10, FP32 1e-4,
    compensated FP32 1e-7).  The homogeneous equilibria (1, 0, 0) and
    (0, 1, rho3/delta3) stay exactly in place."""
    w = wl.cfg2(steps=10000)
    g = rng(78)
    state = (np.clip(w.u0 + 0.05 * g.random(w.u0.shape), 0.0, 1.0), w.v0, 0.1 * g.random(w.u0.shape))
    off = (0.0, 0.0, w.params[2], 0.0, 0.0)               # no reactions, Delta2 kept
    ctx = gpu_ctx(w.nx, w.ny, dtype, off, state, eig=w.eig)
    ctx.set_tuning(*shape)
    dt = ctx.stable_dt(0.9)
    m0 = ctx.diagnostics()["mass"]
    ctx.step(dt, w.steps)
    m1 = ctx.diagnostics()["mass"]
    drift = np.abs(m1[1:] - m0[1:]) / m0[1:]
    print(f"{dtype}: relative mass drift of v, w after {w.steps} steps: {drift}", flush=True)
    assert np.all(drift <= tol)
    ctx.set_params(w.params)
    rho3, delta3 = w.params[3], w.params[4]
    for eq in ((1.0, 0.0, 0.0), (0.0, 1.0, rho3 / delta3)):
        ctx.set_state(*[np.full((w.ny, w.nx), x) for x in eq])
        ctx.step(dt, w.steps)
        for name, x, e in zip("uvw", ctx.get_state(), eq):
            assert np.all(x == np.float32(e) if dtype != "f64" else x == e), (dtype, eq, name)
    ctx.close()


@pytest.mark.parametrize("dtype,shape,tol", [("f32", (0, 64, 4, 2), 5e-4), ("f32c", (0, 64, 4, 1), 1e-5)])
def test_full_size_fp32_headline_shapes(dtype, shape, tol):
    """4096^2 layered tissue in the FP32 launch shapes the benchmark times (wide
    lanes for plain FP32, 8-byte lanes for the compensated state, the library's
    strip height), 40 steps: bit for bit the single-step kernel's result, and
    sampled windows within the FP32 bars of the FP64 oracle run on the device's
    own FP32 tensor, state and step."""
    import dataclasses
    w = wl.cfg2(steps=40)
    r32 = lambda x: np.float64(np.float32(x))
    # FP32-rounded inputs for both sides: tensor from the oracle's map of the
    # FP32 eigen-fields, state, parameters and step
    a, b, c = (r32(x) for x in oracle.tensor_from_eig(*(r32(x) for x in w.eig)))
    w32 = dataclasses.replace(w, u0=r32(w.u0), v0=r32(w.v0), w0=r32(w.w0),
                              params=tuple(float(np.float32(p)) for p in w.params))
    dt = float(np.float32(oracle.stable_dt(a, b, c, w32.params[2], 0.9)))
    f32 = lambda x: np.asarray(x, np.float32)
    st32 = tuple(f32(x) for x in (w32.u0, w32.v0, w32.w0))
    ctx = gpu_ctx(w.nx, w.ny, dtype, w32.params, st32, abc=tuple(f32(x) for x in (a, b, c)))
    ctx.set_tuning(*SINGLE)
    ctx.step(dt, w.steps)
    single = ctx.get_state()
    ctx.set_state(*st32)
    ctx.set_tuning(*shape)
    ctx.step(dt, w.steps)
    got = ctx.get_state()
    for name, x, y in zip("uvw", got, single):
        assert np.array_equal(x, y), f"{name}: headline shape differs from single steps"
    ctx.close()
    n = w.nx
    for (j0, j1, i0, i1) in [(0, 30, 0, 30), (n - 30, n, 2000, 2030), (2030, 2060, 2030, 2060)]:
        ref = _patch_reference(w32, a, b, c, dt, w.steps, j0, j1, i0, i1)
        for x, r in zip((x[j0:j1, i0:i1] for x in got), ref):
            assert np.max(np.abs(x - r)) <= tol * max(np.max(np.abs(r)), 1.0)


# ---------------------------------------------------------------------------
# FP32: compensated state meets 1e-5 after 1e4 steps; plain FP32 does not

def _f32_inputs(n=256):
    w = wl.cfg1(n=n, steps=10000)
    f = lambda x: np.asarray(x, np.float32)
    eig = tuple(f(x) for x in w.eig)
    st = tuple(f(x) for x in (w.u0, w.v0, w.w0))
    prm32 = tuple(float(np.float32(p)) for p in w.params)
    # oracle tensor from the same FP32 eigen-fields, rounded to FP32 like the device
    a, b, c = (np.float64(np.float32(x)) for x in oracle.tensor_from_eig(*[np.float64(x) for x in eig]))
    # step of the 1024^2 grid (4x finer): the increments per step then match cfg1's
    dt = float(np.float32(oracle.stable_dt(a, b, c, prm32[2], 0.9) / 16.0))
    return w, eig, st, prm32, (a, b, c), dt


@pytest.fixture(scope="module")
def f32_case():
    w, eig, st, prm32, abc, dt = _f32_inputs()
    ref = oracle.run(*[np.float64(x) for x in st], *abc, prm32, dt, w.steps)[:3]
    return w, eig, st, prm32, abc, dt, ref


def test_f32c_tolerance_after_1e4_steps(f32_case):
    w, eig, st, prm32, abc, dt, ref = f32_case
    ctx = gpu_ctx(w.nx, w.ny, "f32c", prm32, st, eig=eig)
    ga, gb, gc = ctx.get_tensor()
    for x, y in zip((ga, gb, gc), abc):
        assert np.max(np.abs(x - y)) <= 2.5e-7 * np.max(np.abs(y))
    ctx.step(dt, w.steps)
    got = ctx.get_state()
    err = rel_err(got, ref)
    print(f"f32c rel err after {w.steps} steps: {err:.3e}")
    assert err <= 1e-5


def test_f32_plain_stated_tolerance(f32_case):
    w, eig, st, prm32, abc, dt, ref = f32_case
    ctx = gpu_ctx(w.nx, w.ny, "f32", prm32, st, eig=eig)
    ctx.step(dt, w.steps)
    got = ctx.get_state()
    err = rel_err(got, ref)
    print(f"f32 plain rel err after {w.steps} steps: {err:.3e}")
    assert err <= 5e-4


# ---------------------------------------------------------------------------
# properties on the device

def test_diagnostics_parity_and_unstable_flag():
    nx, ny = 333, 211
    g = rng(1)
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    prm = (3.0, 1.0, 0.2, 2.0, 1.0)
    dt = oracle.stable_dt(a, b, c, prm[2], 0.5)
    ctx = gpu_ctx(nx, ny, "f64", prm, (u, v, w), abc=(a, b, c))
    ctx.step(dt, 3)
    ref = oracle.run(u, v, w, a, b, c, prm, dt, 3)[:3]
    d = ctx.diagnostics()
    od = oracle.diagnostics(*ref, a, b, c, prm[2], dt)
    assert np.allclose(d["mass"], od["mass"], rtol=1e-12, atol=0)
    assert np.array_equal(d["vmin"], od["vmin"]) and np.array_equal(d["vmax"], od["vmax"])
    assert math.isclose(d["cfl"], od["cfl"], rel_tol=1e-14) and d["cfl"] <= 0.5 + 1e-12
    assert d["nonfinite"] == 0
    # determinism of the reduction order
    d2 = ctx.diagnostics()
    assert np.array_equal(d["mass"], d2["mass"])
    # a state with non-finite values is flagged
    w2 = w.copy()
    w2[5, 7] = np.nan
    w2[100, 3] = np.inf
    ctx.set_state(u, v, w2)
    with pytest.raises(pk.GGFVError) as e:
        ctx.diagnostics()
    assert e.value.status == pk.GGFV_EUNSTABLE
    assert ctx.diagnostics(allow_unstable=True)["nonfinite"] == 2


def test_conservation_on_device():
    nx, ny = 400, 250
    g = rng(2)
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    prm = (3.0, 0.0, 0.05, 0.0, 0.0)
    ctx = gpu_ctx(nx, ny, "f64", prm, (u, v, w), abc=(a, b, c))
    dt = ctx.stable_dt(0.9)
    ctx.step(dt, 1)
    m0 = ctx.diagnostics()["mass"]
    ctx.step(dt, 3000)
    m1 = ctx.diagnostics()["mass"]
    assert abs(m1[1] - m0[1]) <= 1e-12 * m0[1]
    assert abs(m1[2] - m0[2]) <= 1e-12 * m0[2]


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32c"])
def test_equilibria_bitwise_on_device(dtype):
    nx, ny = 190, 130
    g = rng(3)
    a, b, c = wl.random_abc(g, nx, ny)
    ones, zeros = np.ones((ny, nx)), np.zeros((ny, nx))
    for st in ((ones, zeros, zeros), (zeros, ones, ones)):
        ctx = gpu_ctx(nx, ny, dtype, PRM, st, abc=(a, b, c))
        ctx.step(ctx.stable_dt(0.9), 1000)
        got = ctx.get_state()
        assert all(np.array_equal(x, y) for x, y in zip(got, st))


def test_determinism_resume_and_launch_shape_invariance():
    nx, ny = 700, 300
    g = rng(4)
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    ctx = gpu_ctx(nx, ny, "f64", PRM, (u, v, w), abc=(a, b, c))
    dt = ctx.stable_dt(0.9)
    ctx.step(dt, 100)
    full = ctx.get_state()
    ctx.set_state(u, v, w)
    ctx.step(dt, 100)
    again = ctx.get_state()
    assert all(np.array_equal(x, y) for x, y in zip(full, again))
    ctx.set_state(u, v, w)
    ctx.step(dt, 50)
    half = ctx.get_state()
    ctx.set_state(*half)
    ctx.step(dt, 50)
    assert all(np.array_equal(x, y) for x, y in zip(full, ctx.get_state()))
    for rows in (1, 3, 17, 300):
        ctx.set_tuning(rows)
        ctx.set_state(u, v, w)
        ctx.step(dt, 100)
        assert all(np.array_equal(x, y) for x, y in zip(full, ctx.get_state())), rows


def test_device_pointer_io_matches_host_io():
    torch = pytest.importorskip("torch")
    nx, ny = 129, 65
    g = rng(5)
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    dev = [torch.from_numpy(x).cuda() for x in (u, v, w)]
    tdev = [torch.from_numpy(x).cuda() for x in (a, b, c)]
    ctx = pk.Context(nx, ny, dtype="f64")
    ctx.set_params(PRM)
    ctx.set_tensor(*tdev)
    ctx.set_state(*dev)
    dt = oracle.stable_dt(a, b, c, PRM[2], 0.9)
    ctx.step(dt, 10)
    outs = [torch.empty((ny, nx), dtype=torch.float64, device="cuda") for _ in range(3)]
    ctx.get_state(out=outs)
    torch.cuda.synchronize()
    ref = oracle.run(u, v, w, a, b, c, PRM, dt, 10)[:3]
    assert all(np.array_equal(o.cpu().numpy(), r) for o, r in zip(outs, ref))


def test_f32c_io_roundtrip_and_conversions():
    nx, ny = 70, 33
    g = rng(6)
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    ctx = gpu_ctx(nx, ny, "f32c", PRM, (u, v, w), abc=(a, b, c))
    got = ctx.get_state()
    for x, y in zip(got, (u, v, w)):
        assert np.max(np.abs(x - y)) <= 2.0 ** -46 * np.max(np.abs(y))
    hi = ctx.get_state(dtype="f32")
    for x, y in zip(hi, (u, v, w)):
        assert np.array_equal(x, y.astype(np.float32))


def test_error_paths():
    nx, ny = 16, 12
    ones, zeros = np.ones((ny, nx)), np.zeros((ny, nx))
    ctx = pk.Context(nx, ny, dtype="f64")
    with pytest.raises(pk.GGFVError) as e:
        ctx.step(1e-4, 1)
    assert e.value.status == pk.GGFV_ESTATE
    ctx.set_params(PRM)
    with pytest.raises(pk.GGFVError) as e:
        ctx.set_tensor(ones, 2 * ones, ones)        # a c - b^2 < 0
    assert e.value.status == pk.GGFV_EINVAL
    with pytest.raises(pk.GGFVError) as e:
        ctx.set_tensor(-ones, zeros, ones)          # a < 0
    assert e.value.status == pk.GGFV_EINVAL
    ctx.set_tensor(ones, zeros, ones)
    ctx.set_state(ones, zeros, zeros)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(pk.GGFVError) as e:
            ctx.step(bad, 1)
        assert e.value.status == pk.GGFV_EINVAL
    with pytest.raises(pk.GGFVError):
        ctx.step(1e-4, -1)
    ctx.step(1e-4, 0)
    with pytest.raises(pk.GGFVError):
        ctx.set_params((1.0, 1.0, -0.1, 1.0, 1.0))
    with pytest.raises(ValueError):
        ctx.set_state(np.ones(5), np.ones(5), np.ones(5))
    # an unstable step is detected by the diagnostics
    ctx.set_state(*wl.random_state(rng(7), nx, ny))
    dt = ctx.stable_dt(0.9)
    ctx.step(dt * 5.0, 1)
    with pytest.raises(pk.GGFVError) as e:
        ctx.diagnostics()
    assert e.value.status == pk.GGFV_EUNSTABLE


# ---------------------------------------------------------------------------
# several steps fused per launch: identical bits to single steps

@pytest.mark.parametrize("dtype,lanes", [("f64", 1), ("f32c", 1), ("f32", 1), ("f64", 2), ("f32", 2)])
@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_lane_shift_steps_bitwise(dtype, lanes, K):
    """The one-wave kernels with register rows and lane shifts (8 or, with wide
    lanes, 16 bytes of columns per lane) give the bits of single steps, for
    every fused depth, strip height and ragged shape (widths spanning several
    waves, one column, one row)."""
    shapes = [(300, 77), (1, 50), (50, 1), (513, 130), (3, 700), (129, 129), (125, 9)]
    for (nx, ny) in shapes:
        g = rng(nx * 17 + ny + K)
        a, b, c = wl.random_abc(g, nx, ny)
        u, v, w = wl.random_state(g, nx, ny)
        ctx = gpu_ctx(nx, ny, dtype, PRM, (u, v, w), abc=(a, b, c))
        ctx.set_tuning(*SINGLE)
        dt = ctx.stable_dt(0.9)
        n = 3 * K + 2 if K > 1 else 5             # fused launches plus single-step remainder
        ctx.step(dt, n)
        ref = ctx.get_state()
        for rows in (0, 1, 3, 2 * K + 1, 37):
            ctx.set_tuning(rows, 0, K, lane_shift=lanes)
            ctx.set_state(u, v, w)
            ctx.step(dt, n)
            got = ctx.get_state()
            for name, x, y in zip("uvw", got, ref):
                if not np.array_equal(x, y):
                    bad = np.argwhere(x != y)
                    raise AssertionError(f"{name} differs at {len(bad)} cells, first {bad[:4].tolist()} "
                                         f"(shape {nx}x{ny}, rows {rows})")
            assert ctx.get_tuning()["lane_shift"] == lanes
        ctx.close()


def test_wide_lanes_rejected_for_compensated_state():
    ctx = gpu_ctx(64, 64, "f32c", PRM, wl.random_state(rng(5), 64, 64), abc=wl.random_abc(rng(6), 64, 64))
    with pytest.raises(pk.GGFVError):
        ctx.set_tuning(0, 0, 4, lane_shift=2)
    with pytest.raises(pk.GGFVError):
        ctx.set_tuning(0, 0, 4, lane_shift=3)
    ctx.close()


@pytest.mark.parametrize("lanes", [1, 2])
def test_lane_shift_full_size_against_oracle_patches(lanes):
    """4096^2 layered tissue, four steps per launch on the lane-shift kernels
    (default strip height, as the benchmark runs them), 40 steps; windows at
    corners and edges against the oracle."""
    w = wl.cfg2(steps=40)
    a, b, c = oracle.tensor_from_eig(*w.eig)
    ctx = gpu_ctx(w.nx, w.ny, "f64", w.params, (w.u0, w.v0, w.w0), eig=w.eig)
    ctx.set_tuning(0, 0, 4, lane_shift=lanes)
    dt = oracle.stable_dt(a, b, c, w.params[2], 0.9)
    ctx.step(dt, w.steps)
    got = ctx.get_state()
    n = w.nx
    for (j0, j1, i0, i1) in [(0, 30, 0, 30), (n - 30, n, n - 30, n), (2000, 2030, 55, 85)]:
        ref = _patch_reference(w, a, b, c, dt, w.steps, j0, j1, i0, i1)
        for s_, r in zip((x[j0:j1, i0:i1] for x in got), ref):
            assert np.max(np.abs(s_ - r)) <= 1e-12 * max(np.max(np.abs(r)), 1.0)
    ctx.close()


def test_fused_full_size_patches_and_checkpoints():
    """4096^2 layered tissue with three steps per launch (narrow lanes), 60 steps, sampled
    windows against the oracle; checkpointed stepping with fusion keeps the
    same states."""
    torch = pytest.importorskip("torch")
    w = wl.cfg2(steps=60)
    a, b, c = oracle.tensor_from_eig(*w.eig)
    ctx = gpu_ctx(w.nx, w.ny, "f64", w.params, (w.u0, w.v0, w.w0), eig=w.eig)
    ctx.set_tuning(0, 0, 3, lane_shift=1)
    dt = oracle.stable_dt(a, b, c, w.params[2], 0.9)
    ctx.step(dt, w.steps)
    got = ctx.get_state()
    n = w.nx
    for (j0, j1, i0, i1) in [(0, 30, 0, 30), (n - 30, n, 1000, 1030), (2000, 2030, n - 30, n)]:
        ref = _patch_reference(w, a, b, c, dt, w.steps, j0, j1, i0, i1)
        for s_, r in zip((x[j0:j1, i0:i1] for x in got), ref):
            assert np.max(np.abs(s_ - r)) <= 1e-12 * max(np.max(np.abs(r)), 1.0)
    # checkpointed run with fusion: same final state, and checkpoint 1 equals the
    # state after `every` single steps
    every = 7
    ckpt = torch.empty(-(-w.steps // every) * ctx.state_bytes(), dtype=torch.uint8, device="cuda")
    ctx.set_state(w.u0, w.v0, w.w0)
    ctx.step_checkpointed(dt, w.steps, every, ckpt)
    assert all(np.array_equal(x, y) for x, y in zip(ctx.get_state(), got))
    ctx.close()


def test_autotune_picks_a_valid_shape_and_keeps_state():
    w = wl.cfg1(n=512, steps=10)
    ctx = gpu_ctx(w.nx, w.ny, "f64", w.params, (w.u0, w.v0, w.w0), eig=w.eig)
    dt = ctx.stable_dt(0.9)
    before = ctx.get_state()
    best = ctx.autotune(dt, trial_steps=4)
    assert best["fused_steps"] in (1, 2, 3, 4) and best["threads"] in (64, 128, 256)
    assert ctx.get_tuning() == best
    assert all(np.array_equal(p, q) for p, q in zip(before, ctx.get_state()))
    assert ctx.diagnostics()["steps"] == 0
