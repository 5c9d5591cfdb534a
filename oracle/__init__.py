"""FP64 CPU oracle for the explicit finite-volume Gatenby-Gawlinski step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it to check and time the HIP library.  The product path
never imports it.  It shares no code with the HIP path; the only common module
is the seeded input generator, which holds none of the scheme's arithmetic.

The arithmetic lives in ``ggfv_oracle.c`` (plain loops, FP64, no FMA).  This
wrapper builds it with gcc into ``libggfv_oracle.so`` next to the source and
exposes numpy-level functions.  Every function states the passage it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ggfv_oracle.c")
_SRC_ADJ = os.path.join(_HERE, "ggfv_oracle_adjoint.c")
_SRC_3D = os.path.join(_HERE, "ggfv_oracle3d.c")
LIB_PATH = os.path.join(_HERE, "libggfv_oracle.so")
CFLAGS = ["-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp"]

_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def sources():
    return [p for p in (_SRC, _SRC_ADJ, _SRC_3D) if os.path.exists(p)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (portable x86-64, no -march=native)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", *CFLAGS, *sources(), "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build(force=True)
    _lib = bind(ctypes.CDLL(LIB_PATH))
    return _lib


def use_library(path):
    """Bind another build of the oracle source (mutation tests); returns the
    previous binding so the caller can restore it with ``restore_library``."""
    global _lib
    prev = _lib
    _lib = bind(ctypes.CDLL(path))
    return prev


def restore_library(prev):
    global _lib
    _lib = prev


def bind(lib):
    i, d, l, p = ctypes.c_int, ctypes.c_double, ctypes.c_long, _D
    lib.orc_tensor_from_eig.argtypes = [l, p, p, p, p, p, p]
    lib.orc_lambda_max.argtypes = [d, d, d]
    lib.orc_lambda_max.restype = d
    lib.orc_count_not_spd.argtypes = [l, p, p, p]
    lib.orc_count_not_spd.restype = l
    lib.orc_stable_dt.argtypes = [i, i, d, d, p, p, p, d, d]
    lib.orc_stable_dt.restype = d
    lib.orc_div_w.argtypes = [i, i, d, d, p, p, p, p, p]
    lib.orc_div_v.argtypes = [i, i, d, d, p, p, p]
    lib.orc_step.argtypes = [i, i, d, d, p, d, p, p, p, p, p, p, p, p, p, p, p, p]
    lib.orc_diag.argtypes = [i, i, d, d, p, p, p, p, p, p, d, d, p]
    lib.orc_run.argtypes = [i, i, d, d, p, d, l, p, p, p, p, p, p, l, p]
    lib.orc_adaptive_dt.argtypes = [i, i, d, d, p, p, p, p, d, d]
    lib.orc_adaptive_dt.restype = d
    lib.orc_run_adaptive.argtypes = [i, i, d, d, p, d, l, p, p, p, p, p, p, p, p]
    lib.orc_front_diag.argtypes = [i, i, d, p, p, d, d, p]
    pp = ctypes.POINTER(_D)
    lib.orc3_div_w.argtypes = [i, i, i, d, d, d, p, pp, p]
    lib.orc3_div_v.argtypes = [i, i, i, d, d, d, p, p, p]
    lib.orc3_step.argtypes = [i, i, i, d, d, d, p, d, p, p, p, pp, p, p, p]
    lib.orc3_run.argtypes = [i, i, i, d, d, d, p, d, l, p, p, p, pp]
    lib.orc3_stable_dt.argtypes = [i, i, i, d, d, d, pp, d, d]
    lib.orc3_stable_dt.restype = d
    lib.orc3_mass.argtypes = [i, i, i, d, d, d, p, p, p, p]
    lib.orc_front_speed.argtypes = [d, d, d, d, d, d, d]
    lib.orc_front_speed.restype = d
    lib.orc_adjoint_step.argtypes = [i, i, d, d, p, d, p, p, p, p, p, p,
                                     p, p, p, p, p, p, p, p, p, p]
    lib.orc_eig_backward.argtypes = [l, p, p, p, p, p, p, p, p, p]
    lib.orc_adjoint_run.argtypes = [i, i, d, d, p, d, l, p, p, p, p, p, p, p, p, p, p, p, p, p]
    lib.orc_adjoint_run_ckpt.argtypes = [i, i, d, d, p, d, l, l, p, p, p, p, p, p, p, p, p, p, p, p, p]
    lib.orc_set_threads.argtypes = [i]
    lib.orc_set_threads.restype = i
    return lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(x):
    return None if x is None else x.ctypes.data_as(_D)


def tensor_from_eig(lam1, lam2, theta):
    """(lambda1, lambda2, theta) -> (a, b, c): A = R diag(l1, l2) R^T (eq. (2))."""
    lam1, lam2, theta = _f64(lam1), _f64(lam2), _f64(theta)
    a, b, c = (np.empty_like(lam1) for _ in range(3))
    _load().orc_tensor_from_eig(lam1.size, _ptr(lam1), _ptr(lam2), _ptr(theta),
                                _ptr(a), _ptr(b), _ptr(c))
    return a, b, c


def lambda_max(a, b, c) -> float:
    return _load().orc_lambda_max(float(a), float(b), float(c))


def count_not_spd(a, b, c) -> int:
    """Cells violating Sylvester's criterion for A = [[a,b],[b,c]] (eq. (2))."""
    a, b, c = _f64(a), _f64(b), _f64(c)
    return int(_load().orc_count_not_spd(a.size, _ptr(a), _ptr(b), _ptr(c)))


def stable_dt(a, b, c, Delta2, safety, lx=1.0, ly=1.0) -> float:
    """Explicit step bound (Section 2, CFL restriction of the explicit scheme)."""
    a, b, c = _f64(a), _f64(b), _f64(c)
    ny, nx = a.shape
    return _load().orc_stable_dt(nx, ny, lx, ly, _ptr(a), _ptr(b), _ptr(c),
                                 float(Delta2), float(safety))


def div_w(W, a, b, c, lx=1.0, ly=1.0):
    """D2(W; A): Table 2 in flux form with zero boundary flux."""
    W, a, b, c = _f64(W), _f64(a), _f64(b), _f64(c)
    ny, nx = W.shape
    out = np.empty_like(W)
    _load().orc_div_w(nx, ny, lx, ly, _ptr(W), _ptr(a), _ptr(b), _ptr(c), _ptr(out))
    return out


def div_v(U, V, lx=1.0, ly=1.0):
    """D1(V; U): Table 1 in flux form with zero boundary flux."""
    U, V = _f64(U), _f64(V)
    ny, nx = V.shape
    out = np.empty_like(V)
    _load().orc_div_v(nx, ny, lx, ly, _ptr(U), _ptr(V), _ptr(out))
    return out


def step(u, v, w, a, b, c, params, dt, lx=1.0, ly=1.0, sources=None):
    """One forward-Euler step of eq. (3); returns new (u, v, w)."""
    u, v, w, a, b, c = (_f64(x) for x in (u, v, w, a, b, c))
    ny, nx = u.shape
    prm = _f64(params)
    un, vn, wn = np.empty_like(u), np.empty_like(v), np.empty_like(w)
    su = sv = sw = None
    if sources is not None:
        su, sv, sw = (_f64(s) for s in sources)
    _load().orc_step(nx, ny, lx, ly, _ptr(prm), float(dt), _ptr(u), _ptr(v), _ptr(w),
                     _ptr(a), _ptr(b), _ptr(c), _ptr(un), _ptr(vn), _ptr(wn),
                     _ptr(su), _ptr(sv), _ptr(sw))
    return un, vn, wn


def run(u, v, w, a, b, c, params, dt, nsteps, lx=1.0, ly=1.0, mass_every=0):
    """nsteps steps of eq. (3).  Returns (u, v, w, mass_log) with mass_log of shape
    (nsteps // mass_every, 3) (empty when mass_every == 0)."""
    u, v, w = (np.array(x, dtype=np.float64, copy=True, order="C") for x in (u, v, w))
    a, b, c = _f64(a), _f64(b), _f64(c)
    ny, nx = u.shape
    prm = _f64(params)
    nlog = nsteps // mass_every if mass_every > 0 else 0
    log = np.zeros((max(nlog, 1), 3))
    _load().orc_run(nx, ny, lx, ly, _ptr(prm), float(dt), int(nsteps), _ptr(u), _ptr(v),
                    _ptr(w), _ptr(a), _ptr(b), _ptr(c), int(mass_every), _ptr(log))
    return u, v, w, log[:nlog]


def adaptive_dt(u, a, b, c, Delta2, safety, lx=1.0, ly=1.0) -> float:
    """Step size of the adaptive scheme on the state u (Section 2: a new step size
    after every iteration, for stability): the dt whose per-cell Gershgorin
    number equals `safety`."""
    u, a, b, c = (_f64(x) for x in (u, a, b, c))
    ny, nx = u.shape
    return _load().orc_adaptive_dt(nx, ny, lx, ly, _ptr(u), _ptr(a), _ptr(b), _ptr(c),
                                   float(Delta2), float(safety))


def run_adaptive(u, v, w, a, b, c, params, safety, nsteps, lx=1.0, ly=1.0, t0=0.0):
    """nsteps steps of eq. (3), each with the adaptive step size of the state it
    starts from.  Returns (u, v, w, dt_log, t) with t = t0 + sum of the steps."""
    u, v, w = (np.array(x, dtype=np.float64, copy=True, order="C") for x in (u, v, w))
    a, b, c = _f64(a), _f64(b), _f64(c)
    ny, nx = u.shape
    prm = _f64(params)
    log = np.zeros(max(int(nsteps), 1))
    t = ctypes.c_double(float(t0))
    _load().orc_run_adaptive(nx, ny, lx, ly, _ptr(prm), float(safety), int(nsteps), _ptr(u), _ptr(v),
                             _ptr(w), _ptr(a), _ptr(b), _ptr(c), _ptr(log),
                             ctypes.byref(t))
    return u, v, w, log[:int(nsteps)], t.value


def front_diag(u, v, theta_u=0.5, theta_v=0.5, lx=1.0) -> dict:
    """Tumour front, tissue front and interstitial gap along +x (per row, then
    mean / min / max over rows); see orc_front_diag."""
    u, v = _f64(u), _f64(v)
    ny, nx = u.shape
    out = np.zeros(11)
    _load().orc_front_diag(nx, ny, float(lx), _ptr(u), _ptr(v), float(theta_u), float(theta_v), _ptr(out))
    return {"tumour": out[0:3].copy(), "tissue": out[3:6].copy(), "gap": out[6:9].copy(),
            "rows_front": int(out[9]), "rows_gap": int(out[10])}


def front_speed(mass0, mass1, t0, t1, ly=1.0, behind=1.0, ahead=0.0) -> float:
    """LeVeque-Yee space-averaged front speed from two masses of one population."""
    return _load().orc_front_speed(float(mass0), float(mass1), float(t0), float(t1), float(ly),
                                   float(behind), float(ahead))


# ---------------------------------------------------------------------------
# three dimensions: fields of shape (nz, ny, nx), the tensor as the six fields
# (axx, ayy, azz, axy, axz, ayz)

def _tensor3(A):
    arrs = [_f64(x) for x in A]
    if len(arrs) != 6:
        raise ValueError("the 3D tensor has six fields (axx, ayy, azz, axy, axz, ayz)")
    ptrs = (ctypes.POINTER(ctypes.c_double) * 6)(*[_ptr(x) for x in arrs])
    return arrs, ptrs


def div_w3(W, A, lx=1.0, ly=1.0, lz=1.0):
    """div(A grad W) of the 3D scheme (19-point stencil in flux form)."""
    W = _f64(W)
    nz, ny, nx = W.shape
    keep, ptrs = _tensor3(A)
    out = np.empty_like(W)
    _load().orc3_div_w(nx, ny, nz, lx, ly, lz, _ptr(W), ptrs, _ptr(out))
    return out


def div_v3(U, V, lx=1.0, ly=1.0, lz=1.0):
    """div((1-U) grad V) of the 3D scheme (7-point stencil in flux form)."""
    U, V = _f64(U), _f64(V)
    nz, ny, nx = V.shape
    out = np.empty_like(V)
    _load().orc3_div_v(nx, ny, nz, lx, ly, lz, _ptr(U), _ptr(V), _ptr(out))
    return out


def step3(u, v, w, A, params, dt, lx=1.0, ly=1.0, lz=1.0):
    """One step of the 3D scheme; returns new (u, v, w)."""
    u, v, w = (_f64(x) for x in (u, v, w))
    nz, ny, nx = u.shape
    keep, ptrs = _tensor3(A)
    prm = _f64(params)
    un, vn, wn = np.empty_like(u), np.empty_like(v), np.empty_like(w)
    _load().orc3_step(nx, ny, nz, lx, ly, lz, _ptr(prm), float(dt), _ptr(u), _ptr(v), _ptr(w), ptrs,
                      _ptr(un), _ptr(vn), _ptr(wn))
    return un, vn, wn


def run3(u, v, w, A, params, dt, nsteps, lx=1.0, ly=1.0, lz=1.0):
    """nsteps steps of the 3D scheme; returns (u, v, w)."""
    u, v, w = (np.array(x, dtype=np.float64, copy=True, order="C") for x in (u, v, w))
    nz, ny, nx = u.shape
    keep, ptrs = _tensor3(A)
    prm = _f64(params)
    _load().orc3_run(nx, ny, nz, lx, ly, lz, _ptr(prm), float(dt), int(nsteps), _ptr(u), _ptr(v), _ptr(w),
                     ptrs)
    return u, v, w


def stable_dt3(A, Delta2, safety, lx=1.0, ly=1.0, lz=1.0) -> float:
    """Explicit step bound of the 3D scheme (Gershgorin bound of max lambda)."""
    keep, ptrs = _tensor3(A)
    nz, ny, nx = keep[0].shape
    return _load().orc3_stable_dt(nx, ny, nz, lx, ly, lz, ptrs, float(Delta2), float(safety))


def mass3(u, v, w, lx=1.0, ly=1.0, lz=1.0):
    u, v, w = (_f64(x) for x in (u, v, w))
    nz, ny, nx = u.shape
    out = np.zeros(3)
    _load().orc3_mass(nx, ny, nz, lx, ly, lz, _ptr(u), _ptr(v), _ptr(w), _ptr(out))
    return out


def diagnostics(u, v, w, a, b, c, Delta2, dt, lx=1.0, ly=1.0) -> dict:
    """Masses, min/max, CFL number and non-finite count of a state."""
    u, v, w, a, b, c = (_f64(x) for x in (u, v, w, a, b, c))
    ny, nx = u.shape
    out = np.zeros(11)
    _load().orc_diag(nx, ny, lx, ly, _ptr(u), _ptr(v), _ptr(w), _ptr(a), _ptr(b), _ptr(c),
                     float(Delta2), float(dt), _ptr(out))
    return {"mass": out[0:3].copy(), "vmin": out[3:6].copy(), "vmax": out[6:9].copy(),
            "cfl": float(out[9]), "nonfinite": int(out[10])}


def adjoint_step(u, v, w, a, b, c, params, dt, lam_next, lx=1.0, ly=1.0):
    """Transpose of one step of eq. (3) (dt fixed).  Returns (lam, g_abc, g_params):
    lam = (dF/dx)^T lam_next, g_abc = (dF/d(a,b,c))^T lam_next (three arrays),
    g_params = (dF/d(delta1, rho2, Delta2, rho3, delta3))^T lam_next."""
    u, v, w, a, b, c = (_f64(x) for x in (u, v, w, a, b, c))
    lu1, lv1, lw1 = (_f64(x) for x in lam_next)
    ny, nx = u.shape
    prm = _f64(params)
    lu, lv, lw = (np.empty_like(u) for _ in range(3))
    ga, gb, gc = (np.zeros_like(u) for _ in range(3))
    gp = np.zeros(5)
    _load().orc_adjoint_step(nx, ny, lx, ly, _ptr(prm), float(dt), _ptr(u), _ptr(v), _ptr(w),
                             _ptr(a), _ptr(b), _ptr(c), _ptr(lu1), _ptr(lv1), _ptr(lw1),
                             _ptr(lu), _ptr(lv), _ptr(lw), _ptr(ga), _ptr(gb), _ptr(gc), _ptr(gp))
    return (lu, lv, lw), (ga, gb, gc), gp


def eig_backward(lam1, lam2, theta, ga, gb, gc):
    """Chain rule of the tensor map (lambda1, lambda2, theta) -> (a, b, c)."""
    lam1, lam2, theta, ga, gb, gc = (_f64(x) for x in (lam1, lam2, theta, ga, gb, gc))
    g1, g2, gt = (np.empty_like(lam1) for _ in range(3))
    _load().orc_eig_backward(lam1.size, _ptr(lam1), _ptr(lam2), _ptr(theta), _ptr(ga), _ptr(gb),
                             _ptr(gc), _ptr(g1), _ptr(g2), _ptr(gt))
    return g1, g2, gt


def adjoint_run(u0, v0, w0, a, b, c, params, dt, nsteps, lam_final, lx=1.0, ly=1.0):
    """Reverse sweep over nsteps steps from x^0 (all states kept; small grids only).
    Returns (lam0, g_abc, g_params) for the loss whose gradient at x^N is lam_final."""
    u0, v0, w0, a, b, c = (_f64(x) for x in (u0, v0, w0, a, b, c))
    lu, lv, lw = (np.array(x, dtype=np.float64, copy=True, order="C") for x in lam_final)
    ny, nx = u0.shape
    prm = _f64(params)
    ga, gb, gc = (np.zeros_like(u0) for _ in range(3))
    gp = np.zeros(5)
    _load().orc_adjoint_run(nx, ny, lx, ly, _ptr(prm), float(dt), int(nsteps), _ptr(u0), _ptr(v0),
                            _ptr(w0), _ptr(a), _ptr(b), _ptr(c), _ptr(lu), _ptr(lv), _ptr(lw),
                            _ptr(ga), _ptr(gb), _ptr(gc), _ptr(gp))
    return (lu, lv, lw), (ga, gb, gc), gp


def adjoint_run_ckpt(u0, v0, w0, a, b, c, params, dt, nsteps, lam_final, every, lx=1.0, ly=1.0):
    """adjoint_run with the states stored every `every` steps and each segment
    recomputed before its adjoint steps (same results; about nsteps/every +
    every states in memory, so full-length sweeps on large grids fit)."""
    u0, v0, w0, a, b, c = (_f64(x) for x in (u0, v0, w0, a, b, c))
    lu, lv, lw = (np.array(x, dtype=np.float64, copy=True, order="C") for x in lam_final)
    ny, nx = u0.shape
    prm = _f64(params)
    ga, gb, gc = (np.zeros_like(u0) for _ in range(3))
    gp = np.zeros(5)
    _load().orc_adjoint_run_ckpt(nx, ny, lx, ly, _ptr(prm), float(dt), int(nsteps), int(every), _ptr(u0),
                                 _ptr(v0), _ptr(w0), _ptr(a), _ptr(b), _ptr(c), _ptr(lu), _ptr(lv), _ptr(lw),
                                 _ptr(ga), _ptr(gb), _ptr(gc), _ptr(gp))
    return (lu, lv, lw), (ga, gb, gc), gp


def set_threads(n: int = 0) -> int:
    """Threads the oracle's per-face and per-cell loops may use (n < 1: leave
    the current setting, by default OMP_NUM_THREADS or every core); returns
    the number in effect.  Results do not depend on it."""
    return int(_load().orc_set_threads(int(n)))
