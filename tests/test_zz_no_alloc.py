"""ggfv_diagnostics_noalloc (through the C ABI) against ggfv_diagnostics on
the same state, tensor and step: bit for bit, on two calls in a row, the
second on a smaller grid; argument errors before any device work."""
import ctypes

import numpy as np
import pytest

import paper_2006_01748_amd as pk
from paper_2006_01748_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(nx, ny, dtype, seed, steps=12, lx=1.0, ly=0.7):
    g = np.random.Generator(np.random.PCG64(wl.BASE_SEED + seed))
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    prm = (12.5, 1.0, 0.03, 70.0, 60.0)
    ctx = pk.Context(nx, ny, lx, ly, dtype=dtype)
    ctx.set_params(prm)
    ctx.set_tensor(a, b, c)
    ctx.set_state(u, v, w)
    dt = ctx.stable_dt(0.9)
    if dtype != "f64":
        dt = float(np.float32(dt))
    ctx.step(dt, steps)
    d = ctx.diagnostics()
    tdt = torch.float64 if dtype in ("f64", "f32c") else torch.float32
    st = [torch.empty((ny, nx), dtype=tdt, device="cuda") for _ in range(3)]
    ab = [torch.empty((ny, nx), dtype=tdt, device="cuda") for _ in range(3)]
    ctx.get_state(out=st)
    ctx.get_tensor(out=ab)
    torch.cuda.synchronize()
    ctx.close()
    return d, st, ab, prm[2], dt, lx, ly


def _noalloc(st, ab, D2, dt, lx, ly):
    out = torch.full((11,), float("nan"), dtype=torch.float64, device="cuda")
    pk.diagnostics_noalloc(*st, *ab, D2, dt, out, lx, ly)
    return out.cpu().numpy()          # synchronizes torch's stream


def _same(d, r):
    assert np.array_equal(r[0:3], d["mass"]), (r[0:3], d["mass"])
    assert np.array_equal(r[3:6], d["vmin"]) and np.array_equal(r[6:9], d["vmax"])
    assert r[9] == d["cfl"] and r[10] == d["nonfinite"] == 0


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32c"])
def test_noalloc_diagnostics_equal_context_diagnostics(dtype):
    big = _case(1000, 613, dtype, 1)
    small = _case(77, 5, dtype, 2)
    for d, st, ab, D2, dt, lx, ly in (big, small):    # two calls in a row, the second smaller
        _same(d, _noalloc(st, ab, D2, dt, lx, ly))
    # and the large one again after the small one (the shared partials are rewritten)
    d, st, ab, D2, dt, lx, ly = big
    _same(d, _noalloc(st, ab, D2, dt, lx, ly))


def test_noalloc_diagnostics_rejects_bad_arguments():
    lib = pk.lib()
    x = torch.zeros(64, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(x.data_ptr())
    args = lambda nx, ny, io, ptr, D2, dev: (nx, ny, 1.0, 1.0, io, ptr, p, p, p, p, p, D2, 1e-3, p, dev, None)
    for bad in (args(0, 8, pk.GGFV_F64, p, 0.01, 0), args(1 << 20, 1 << 15, pk.GGFV_F64, p, 0.01, 0),
                args(8, 8, pk.GGFV_F32C, p, 0.01, 0), args(8, 8, pk.GGFV_F64, None, 0.01, 0),
                args(8, 8, pk.GGFV_F64, p, -1.0, 0), args(8, 8, pk.GGFV_F64, p, 0.01, 999)):
        assert lib.ggfv_diagnostics_noalloc(*bad) == pk.GGFV_EINVAL
        assert lib.ggfv_last_error(None) != b""
