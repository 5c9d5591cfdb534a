"""ctypes binding of ``libggfv.so`` (the C ABI of include/ggfv.h and include/ggfv3.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Arrays may be numpy arrays (host memory) or torch tensors; a torch
tensor on the GPU is passed as device memory and work is enqueued on torch's
current stream unless another stream is given.  If the library has not been
built the binding raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libggfv.so")

GGFV_OK, GGFV_EINVAL, GGFV_ENOMEM, GGFV_EHIP, GGFV_ESTATE, GGFV_EUNSTABLE = range(6)
GGFV_F32, GGFV_F64, GGFV_F32C = 1, 2, 3
GGFV_HOST, GGFV_DEVICE = 0, 1

DTYPES = {"f32": GGFV_F32, "f64": GGFV_F64, "f32c": GGFV_F32C}

# Every function of the ABI, in header order: (name, restype, argtypes).
_c = ctypes
_VP = _c.c_void_p
_SIGNATURES = [
    ("ggfv_create", _c.c_int, [_c.POINTER(_VP), _c.c_int, _c.c_int, _c.c_double, _c.c_double,
                               _c.c_int, _c.c_int, _VP]),
    ("ggfv_destroy", None, [_VP]),
    ("ggfv_set_stream", _c.c_int, [_VP, _VP]),
    ("ggfv_set_params", _c.c_int, [_VP, _VP]),
    ("ggfv_set_tensor", _c.c_int, [_VP, _VP, _VP, _VP, _c.c_int, _c.c_int]),
    ("ggfv_set_tensor_eig", _c.c_int, [_VP, _VP, _VP, _VP, _c.c_int, _c.c_int]),
    ("ggfv_get_tensor", _c.c_int, [_VP, _VP, _VP, _VP, _c.c_int, _c.c_int]),
    ("ggfv_set_state", _c.c_int, [_VP, _VP, _VP, _VP, _c.c_int, _c.c_int]),
    ("ggfv_get_state", _c.c_int, [_VP, _VP, _VP, _VP, _c.c_int, _c.c_int]),
    ("ggfv_stable_dt", _c.c_int, [_VP, _c.c_double, _c.POINTER(_c.c_double)]),
    ("ggfv_step", _c.c_int, [_VP, _c.c_double, _c.c_longlong]),
    ("ggfv_diagnostics", _c.c_int, [_VP, _VP]),
    ("ggfv_diagnostics_noalloc", _c.c_int, [_c.c_int, _c.c_int, _c.c_double, _c.c_double, _c.c_int] + [_VP] * 6
     + [_c.c_double, _c.c_double, _VP, _c.c_int, _VP]),
    ("ggfv_state_bytes", _c.c_longlong, [_VP]),
    ("ggfv_step_checkpointed", _c.c_int, [_VP, _c.c_double, _c.c_longlong, _c.c_longlong, _VP, _c.c_longlong]),
    ("ggfv_adjoint_step", _c.c_int, [_VP, _c.c_double] + [_VP] * 12 + [_c.POINTER(_c.c_double), _c.c_int, _c.c_int]),
    ("ggfv_adjoint_run", _c.c_int, [_VP, _c.c_double, _c.c_longlong, _c.c_longlong, _VP, _c.c_longlong, _VP,
                                    _c.c_longlong] + [_VP] * 6 + [_c.POINTER(_c.c_double), _c.c_int, _c.c_int]),
    ("ggfv_eig_backward", _c.c_int, [_VP] * 10 + [_c.c_int, _c.c_int]),
    ("ggfv_set_tuning", _c.c_int, [_VP, _VP]),
    ("ggfv_get_tuning", _c.c_int, [_VP, _VP]),
    ("ggfv_autotune", _c.c_int, [_VP, _c.c_double, _c.c_int, _VP]),
    ("ggfv_batch_create", _c.c_int, [_c.POINTER(_VP), _c.c_int, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int),
                                     _c.c_double, _c.c_double, _c.c_int, _c.c_int, _VP]),
    ("ggfv_batch_destroy", None, [_VP]),
    ("ggfv_batch_instance", _VP, [_VP, _c.c_int]),
    ("ggfv_batch_set_dt", _c.c_int, [_VP, _c.c_int, _c.c_double]),
    ("ggfv_batch_set", _c.c_int, [_VP, _c.c_int, _VP, _c.c_double] + [_VP] * 6 + [_c.c_int, _c.c_int]),
    ("ggfv_batch_get_state", _c.c_int, [_VP, _c.c_int, _VP, _VP, _VP, _c.c_int, _c.c_int]),
    ("ggfv_batch_run", _c.c_int, [_VP, _c.c_longlong]),
    ("ggfv_batch_set_tuning", _c.c_int, [_VP, _c.c_int, _c.c_int, _c.c_int]),
    ("ggfv_batch_autotune", _c.c_int, [_VP, _c.c_int, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int)]),
    ("ggfv_batch_set_fused_steps", _c.c_int, [_VP, _c.c_int]),
    ("ggfv_step_adaptive", _c.c_int, [_VP, _c.c_double, _c.c_longlong, _VP]),
    ("ggfv_front_diagnostics", _c.c_int, [_VP, _c.c_double, _c.c_double, _c.POINTER(_c.c_double)]),
    ("ggfv_front_speed", _c.c_double, [_c.c_double] * 7),
    ("ggfv_batch_get_tuning", _c.c_int, [_VP, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int), _c.POINTER(_c.c_int),
                                         _c.POINTER(_c.c_int)]),
    ("ggfv_batch_last_error", _c.c_char_p, [_VP]),
    ("ggfv_last_error", _c.c_char_p, [_VP]),
    ("ggfv_status_string", _c.c_char_p, [_c.c_int]),
    # include/ggfv3.h
    ("ggfv3_create", _c.c_int, [_c.POINTER(_VP), _c.c_int, _c.c_int, _c.c_int, _c.c_double, _c.c_double,
                                _c.c_double, _c.c_int, _c.c_int, _VP]),
    ("ggfv3_destroy", None, [_VP]),
    ("ggfv3_set_params", _c.c_int, [_VP, _VP]),
    ("ggfv3_set_tensor", _c.c_int, [_VP] + [_VP] * 6 + [_c.c_int, _c.c_int]),
    ("ggfv3_set_state", _c.c_int, [_VP, _VP, _VP, _VP, _c.c_int, _c.c_int]),
    ("ggfv3_get_state", _c.c_int, [_VP, _VP, _VP, _VP, _c.c_int, _c.c_int]),
    ("ggfv3_stable_dt", _c.c_int, [_VP, _c.c_double, _c.POINTER(_c.c_double)]),
    ("ggfv3_step", _c.c_int, [_VP, _c.c_double, _c.c_longlong]),
    ("ggfv3_mass", _c.c_int, [_VP, _c.POINTER(_c.c_double)]),
    ("ggfv3_time", _c.c_int, [_VP, _c.POINTER(_c.c_double), _c.POINTER(_c.c_longlong)]),
    ("ggfv3_set_tuning", _c.c_int, [_VP, _c.c_int, _c.c_int, _c.c_int, _c.c_int]),
    ("ggfv3_get_tuning", _c.c_int, [_VP] + [_c.POINTER(_c.c_int)] * 4 + [_c.POINTER(_c.c_longlong)]),
    ("ggfv3_last_error", _c.c_char_p, [_VP]),
]


class Params(ctypes.Structure):
    _fields_ = [("delta1", ctypes.c_double), ("rho2", ctypes.c_double),
                ("Delta2", ctypes.c_double), ("rho3", ctypes.c_double),
                ("delta3", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("steps", ctypes.c_longlong),
                ("mass", ctypes.c_double * 3), ("vmin", ctypes.c_double * 3),
                ("vmax", ctypes.c_double * 3), ("cfl", ctypes.c_double),
                ("nonfinite", ctypes.c_longlong)]


class Tuning(ctypes.Structure):
    _fields_ = [("rows_per_strip", ctypes.c_int), ("threads", ctypes.c_int), ("fused_steps", ctypes.c_int),
                ("lane_shift", ctypes.c_int)]


class GGFVError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status


_lib = None


def _status_name(s):
    names = ["GGFV_OK", "GGFV_EINVAL", "GGFV_ENOMEM", "GGFV_EHIP", "GGFV_ESTATE", "GGFV_EUNSTABLE"]
    return names[s] if 0 <= s < len(names) else f"status {s}"


def lib():
    """The loaded library; raises if it was never built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2006_01748_amd.build` "
                          "(there is no CPU fallback)")
    # One HIP runtime per process: when torch is present its bundled runtime
    # (same soname) must be loaded first so that the library binds to it and
    # torch's streams and device pointers are valid in the library's calls.
    _torch()
    L = ctypes.CDLL(LIB_PATH)
    for name, res, args in _SIGNATURES:
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def front_speed(mass0, mass1, t0, t1, ly=1.0, behind=1.0, ahead=0.0):
    """LeVeque-Yee space-averaged front speed from two masses (ggfv_front_speed)."""
    return float(lib().ggfv_front_speed(float(mass0), float(mass1), float(t0), float(t1), float(ly),
                                        float(behind), float(ahead)))


def diagnostics_noalloc(u, v, w, a, b, c, Delta2, dt, out, lx=1.0, ly=1.0, device=0, stream=None):
    """ggfv_diagnostics_noalloc: diagnostics of a state and tensor in torch device
    tensors (all (ny, nx), float64 or float32) into `out`, a float64 device
    tensor of 11 values, enqueued on torch's current stream (or `stream`);
    allocates nothing.  Returns `out`."""
    arrays = (u, v, w, a, b, c)
    if not all(_is_device_tensor(x) and x.is_contiguous() for x in arrays):
        raise TypeError("diagnostics_noalloc takes contiguous device tensors")
    io = _io_of(u)
    if any(_io_of(x) != io or tuple(x.shape) != tuple(u.shape) for x in arrays):
        raise TypeError("all arrays must share one shape and dtype")
    if not (_is_device_tensor(out) and out.is_contiguous() and out.numel() >= 11 and out.dtype == _torch().float64):
        raise TypeError("out must be a contiguous float64 device tensor of at least 11 values")
    ny, nx = (int(u.shape[0]), int(u.shape[1])) if u.dim() == 2 else (1, int(u.numel()))
    if stream is None:
        stream = _current_stream()
    rc = lib().ggfv_diagnostics_noalloc(nx, ny, float(lx), float(ly), io,
                                        *[ctypes.c_void_p(x.data_ptr()) for x in arrays], float(Delta2),
                                        float(dt), ctypes.c_void_p(out.data_ptr()), int(device), stream)
    if rc != GGFV_OK:
        raise GGFVError(rc, lib().ggfv_last_error(None).decode())
    return out


def exported_names():
    return [s[0] for s in _SIGNATURES]


def _torch():
    try:
        import torch
        return torch
    except ImportError:  # pragma: no cover
        return None


def _is_device_tensor(x):
    t = _torch()
    return t is not None and isinstance(x, t.Tensor) and x.is_cuda


def _io_of(x):
    if _is_device_tensor(x):
        t = _torch()
        if x.dtype == t.float64:
            return GGFV_F64
        if x.dtype == t.float32:
            return GGFV_F32
        raise TypeError(f"unsupported tensor dtype {x.dtype}")
    if x.dtype == np.float64:
        return GGFV_F64
    if x.dtype == np.float32:
        return GGFV_F32
    raise TypeError(f"unsupported array dtype {x.dtype}")


def _current_stream():
    t = _torch()
    if t is None or not t.cuda.is_available():
        return None
    return ctypes.c_void_p(t.cuda.current_stream().cuda_stream)


def _prep_arrays(arrays, count):
    """(pointers, where, io, keepalive) for input arrays of `count` values each."""
    if all(_is_device_tensor(x) for x in arrays):
        xs = [x.contiguous() for x in arrays]
        io = _io_of(xs[0])
        if any(_io_of(x) != io for x in xs):
            raise TypeError("all arrays must share a dtype")
        for x in xs:
            if x.numel() != count:
                raise ValueError(f"expected {count} values, got {x.numel()}")
        return [ctypes.c_void_p(x.data_ptr()) for x in xs], GGFV_DEVICE, io, xs
    xs = []
    for x in arrays:
        if _torch() is not None and isinstance(x, _torch().Tensor):
            x = x.cpu().numpy()
        x = np.asarray(x)
        if x.dtype not in (np.float32, np.float64):
            x = x.astype(np.float64)
        x = np.ascontiguousarray(x)
        if x.size != count:
            raise ValueError(f"expected {count} values, got {x.size}")
        xs.append(x)
    io = _io_of(xs[0])
    xs = [x.astype(xs[0].dtype, copy=False) for x in xs]
    return [x.ctypes.data_as(ctypes.c_void_p) for x in xs], GGFV_HOST, io, xs


def _call_out3(obj, fn, outs, count):
    """Call fn(handle, p0, p1, p2, where, io) into three outputs of `count` values."""
    if all(_is_device_tensor(x) for x in outs):
        for x in outs:
            if not x.is_contiguous() or x.numel() != count:
                raise ValueError(f"device outputs must be contiguous with {count} values")
        ptrs = [ctypes.c_void_p(x.data_ptr()) for x in outs]
        obj._check(fn(obj._h, *ptrs, GGFV_DEVICE, _io_of(outs[0])))
    else:
        for x in outs:
            if not (isinstance(x, np.ndarray) and x.flags.c_contiguous and x.size == count):
                raise ValueError(f"host outputs must be contiguous numpy arrays with {count} values")
        ptrs = [x.ctypes.data_as(ctypes.c_void_p) for x in outs]
        obj._check(fn(obj._h, *ptrs, GGFV_HOST, _io_of(outs[0])))
    return tuple(outs)


class Context:
    """One grid, its tensor, parameters and state on one GPU (see include/ggfv.h)."""

    def __init__(self, nx, ny, lx=1.0, ly=1.0, dtype="f64", device=0, stream=None, _handle=None):
        self._lib = lib()
        if _handle is not None:          # an instance owned by a Batch
            self.nx, self.ny, self.lx, self.ly = int(nx), int(ny), float(lx), float(ly)
            self.dtype = dtype
            self._h = _handle
            self._owned = False
            return
        self._owned = True
        self.nx, self.ny, self.lx, self.ly = int(nx), int(ny), float(lx), float(ly)
        self.dtype = dtype
        h = ctypes.c_void_p()
        if stream is None:
            stream = _current_stream()
        rc = self._lib.ggfv_create(ctypes.byref(h), self.nx, self.ny, self.lx, self.ly,
                                   DTYPES[dtype], int(device), stream)
        if rc != GGFV_OK:
            why = self._lib.ggfv_last_error(None).decode()
            raise GGFVError(rc, f"ggfv_create({nx}, {ny}, {lx}, {ly}, {dtype}, device={device}) failed: {why}")
        self._h = h

    # -- plumbing ----------------------------------------------------------
    def _check(self, rc):
        if rc != GGFV_OK:
            raise GGFVError(rc, self._lib.ggfv_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owned", True):
                self._lib.ggfv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def _prep_in(self, arrays):
        return _prep_arrays(arrays, self.nx * self.ny)

    def _out(self, out, dtype):
        if out is not None:
            return out
        dt = np.float64 if dtype == "f64" else np.float32
        return [np.empty((self.ny, self.nx), dtype=dt) for _ in range(3)]

    def _call_out(self, fn, out, dtype):
        return _call_out3(self, fn, self._out(out, dtype), self.nx * self.ny)

    # -- API ---------------------------------------------------------------
    def set_stream(self, stream):
        self._check(self._lib.ggfv_set_stream(self._h, stream))

    def set_params(self, params):
        p = Params(*[float(x) for x in params])
        self._check(self._lib.ggfv_set_params(self._h, ctypes.byref(p)))

    def set_tensor(self, a, b, c):
        ptrs, where, io, keep = self._prep_in((a, b, c))
        self._check(self._lib.ggfv_set_tensor(self._h, *ptrs, where, io))

    def set_tensor_eig(self, lam1, lam2, theta):
        ptrs, where, io, keep = self._prep_in((lam1, lam2, theta))
        self._check(self._lib.ggfv_set_tensor_eig(self._h, *ptrs, where, io))

    def get_tensor(self, out=None, dtype="f64"):
        return self._call_out(self._lib.ggfv_get_tensor, out, dtype)

    def set_state(self, u, v, w):
        ptrs, where, io, keep = self._prep_in((u, v, w))
        self._check(self._lib.ggfv_set_state(self._h, *ptrs, where, io))

    def get_state(self, out=None, dtype="f64"):
        return self._call_out(self._lib.ggfv_get_state, out, dtype)

    def stable_dt(self, safety):
        d = ctypes.c_double()
        self._check(self._lib.ggfv_stable_dt(self._h, float(safety), ctypes.byref(d)))
        return d.value

    def step(self, dt, nsteps=1):
        self._check(self._lib.ggfv_step(self._h, float(dt), int(nsteps)))

    def front_diagnostics(self, theta_u=0.5, theta_v=0.5):
        """Tumour front, tissue front and interstitial gap along +x (ggfv_front_diagnostics)."""
        out = (ctypes.c_double * 11)()
        self._check(self._lib.ggfv_front_diagnostics(self._h, float(theta_u), float(theta_v), out))
        o = list(out)
        return {"tumour": np.array(o[0:3]), "tissue": np.array(o[3:6]), "gap": np.array(o[6:9]),
                "rows_front": int(o[9]), "rows_gap": int(o[10])}

    def step_adaptive(self, safety, nsteps=1, dt_log=None):
        """nsteps steps, each with the step size the device derives from the state
        it starts from (ggfv_step_adaptive).  dt_log: None or a CUDA float64
        tensor of at least nsteps elements that receives the step sizes."""
        ptr = None
        if dt_log is not None:
            if not dt_log.is_cuda or str(dt_log.dtype) != "torch.float64" or not dt_log.is_contiguous():
                raise ValueError("dt_log must be a contiguous CUDA float64 tensor")
            if dt_log.numel() < int(nsteps):
                raise ValueError("dt_log holds fewer than nsteps elements")
            ptr = ctypes.c_void_p(dt_log.data_ptr())
        self._check(self._lib.ggfv_step_adaptive(self._h, float(safety), int(nsteps), ptr))

    # -- gradients -----------------------------------------------------------
    def state_bytes(self):
        return int(self._lib.ggfv_state_bytes(self._h))

    def step_checkpointed(self, dt, nsteps, every, ckpt):
        """Step and store the state before every `every`-th step into the device
        tensor `ckpt` (at least ceil(nsteps/every) * state_bytes() bytes)."""
        self._check(self._lib.ggfv_step_checkpointed(self._h, float(dt), int(nsteps), int(every),
                                                     ctypes.c_void_p(ckpt.data_ptr()),
                                                     ckpt.numel() * ckpt.element_size()))

    def _ptrs9(self, arrays):
        dev = [_is_device_tensor(x) for x in arrays]
        if all(dev):
            for x in arrays:
                if not x.is_contiguous() or x.numel() != self.nx * self.ny:
                    raise ValueError("device arrays must be contiguous with nx*ny values")
            io = _io_of(arrays[0])
            return [ctypes.c_void_p(x.data_ptr()) for x in arrays], GGFV_DEVICE, io
        if any(dev):
            raise TypeError("mixing host and device arrays")
        for x in arrays:
            if not (isinstance(x, np.ndarray) and x.flags.c_contiguous and x.size == self.nx * self.ny):
                raise ValueError("host arrays must be C-contiguous numpy arrays with nx*ny values")
        io = _io_of(arrays[0])
        if any(x.dtype != arrays[0].dtype for x in arrays):
            raise TypeError("all arrays must share a dtype")
        return [x.ctypes.data_as(ctypes.c_void_p) for x in arrays], GGFV_HOST, io

    def adjoint_step(self, dt, x, lam_next, g_abc):
        """One adjoint step at state x: returns (lam, g_params) with lam = (dF/dx)^T
        lam_next; the tensor gradient is added into g_abc in place."""
        if _is_device_tensor(x[0]):
            outs = [x[0].new_empty((self.ny, self.nx)) for _ in range(3)]
        else:
            outs = [np.empty((self.ny, self.nx), dtype=np.asarray(x[0]).dtype) for _ in range(3)]
        p1, where, io = self._ptrs9(list(x) + list(lam_next) + outs)
        p2, where2, io2 = self._ptrs9(list(g_abc) + list(x))
        if (where2, io2) != (where, io):
            raise TypeError("gradient arrays must match the other arrays' location and dtype")
        gp = (ctypes.c_double * 5)()
        self._check(self._lib.ggfv_adjoint_step(self._h, float(dt), *p1, *p2[:3], gp, where, io))
        return tuple(outs), np.array(gp[:])

    def adjoint_run(self, dt, nsteps, every, ckpt, work, lam, g_abc):
        """Reverse sweep: lam (3 arrays, in: dL/dx^N, out: dL/dx^0), g_abc (3 arrays,
        overwritten).  Returns the five parameter gradients."""
        ptrs = self._ptrs9(list(lam))[0] + self._ptrs9(list(g_abc))[0]
        _, where, io = self._ptrs9(list(lam))
        gp = (ctypes.c_double * 5)()
        self._check(self._lib.ggfv_adjoint_run(
            self._h, float(dt), int(nsteps), int(every), ctypes.c_void_p(ckpt.data_ptr()),
            ckpt.numel() * ckpt.element_size(), ctypes.c_void_p(work.data_ptr()),
            work.numel() * work.element_size(), *ptrs, gp, where, io))
        return np.array(gp[:])

    def eig_backward(self, lam1, lam2, theta, ga, gb, gc):
        arrays = [lam1, lam2, theta, ga, gb, gc]
        if all(_is_device_tensor(x) for x in arrays):
            outs = [lam1.new_empty(lam1.shape) for _ in range(3)]
        else:
            outs = [np.empty((self.ny, self.nx), dtype=np.asarray(lam1).dtype) for _ in range(3)]
        ptrs, where, io = self._ptrs9(arrays + outs)
        self._check(self._lib.ggfv_eig_backward(self._h, *ptrs, where, io))
        return tuple(outs)

    def set_tuning(self, rows_per_strip=0, threads=0, fused_steps=1, lane_shift=0):
        t = Tuning(int(rows_per_strip), int(threads), int(fused_steps), int(lane_shift))
        self._check(self._lib.ggfv_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self):
        t = Tuning()
        self._check(self._lib.ggfv_get_tuning(self._h, ctypes.byref(t)))
        return {"rows_per_strip": t.rows_per_strip, "threads": t.threads, "fused_steps": t.fused_steps,
                "lane_shift": t.lane_shift}

    def autotune(self, dt, trial_steps=20):
        t = Tuning()
        self._check(self._lib.ggfv_autotune(self._h, float(dt), int(trial_steps), ctypes.byref(t)))
        return {"rows_per_strip": t.rows_per_strip, "threads": t.threads, "fused_steps": t.fused_steps,
                "lane_shift": t.lane_shift}

    def diagnostics(self, allow_unstable=False):
        d = Diag()
        rc = self._lib.ggfv_diagnostics(self._h, ctypes.byref(d))
        if rc != GGFV_OK and not (allow_unstable and rc == GGFV_EUNSTABLE):
            self._check(rc)
        return {"t": d.t, "steps": d.steps, "mass": np.array(d.mass[:]), "vmin": np.array(d.vmin[:]),
                "vmax": np.array(d.vmax[:]), "cfl": d.cfl, "nonfinite": d.nonfinite,
                "status": rc}


class Batch:
    """An ensemble of independent instances stepped together (see include/ggfv.h)."""

    def __init__(self, sizes, lx=1.0, ly=1.0, dtype="f32c", device=0, stream=None):
        self._lib = lib()
        n = len(sizes)
        nx = (ctypes.c_int * n)(*[int(s[0]) for s in sizes])
        ny = (ctypes.c_int * n)(*[int(s[1]) for s in sizes])
        if stream is None:
            stream = _current_stream()
        h = ctypes.c_void_p()
        rc = self._lib.ggfv_batch_create(ctypes.byref(h), n, nx, ny, float(lx), float(ly), DTYPES[dtype],
                                         int(device), stream)
        if rc != GGFV_OK:
            raise GGFVError(rc, "ggfv_batch_create failed: " + self._lib.ggfv_batch_last_error(None).decode())
        self._h = h
        self.sizes = [(int(a), int(b)) for a, b in sizes]
        self.dtype = dtype
        self.instances = [Context(sx, sy, lx, ly, dtype, device,
                                  _handle=ctypes.c_void_p(self._lib.ggfv_batch_instance(h, i)))
                          for i, (sx, sy) in enumerate(self.sizes)]

    def _check(self, rc):
        if rc != GGFV_OK:
            raise GGFVError(rc, self._lib.ggfv_batch_last_error(self._h).decode())

    def __len__(self):
        return len(self.instances)

    def __getitem__(self, i):
        # re-fetch so the batch knows the instance may change
        self._lib.ggfv_batch_instance(self._h, int(i))
        return self.instances[i]

    def set_dt(self, i, dt):
        self._check(self._lib.ggfv_batch_set_dt(self._h, int(i), float(dt)))

    def set(self, i, params, dt, abc, state):
        """Parameters, tensor (a, b, c), state (u, v, w) and dt of instance i in one
        call (ggfv_batch_set)."""
        i = int(i)
        p = Params(*[float(x) for x in params])
        if not 0 <= i < len(self.sizes):     # let the library report the bad index
            self._check(self._lib.ggfv_batch_set(self._h, i, ctypes.byref(p), float(dt), *([None] * 6),
                                                 GGFV_HOST, GGFV_F64))
        nx, ny = self.sizes[i]
        ptrs, where, io, keep = _prep_arrays(tuple(abc) + tuple(state), nx * ny)
        self._check(self._lib.ggfv_batch_set(self._h, i, ctypes.byref(p), float(dt), *ptrs, where, io))

    def get_state(self, i, out=None, dtype="f64"):
        """State of instance i (ggfv_batch_get_state)."""
        idx = int(i)
        if not 0 <= idx < len(self.sizes):   # let the library report the bad index
            self._check(self._lib.ggfv_batch_get_state(self._h, idx, None, None, None, GGFV_HOST, GGFV_F64))
        nx, ny = self.sizes[idx]
        if out is None:
            dt = np.float64 if dtype == "f64" else np.float32
            out = [np.empty((ny, nx), dtype=dt) for _ in range(3)]
        return _call_out3(self, lambda h, *rest: self._lib.ggfv_batch_get_state(h, idx, *rest), out, nx * ny)

    def run(self, nsteps):
        self._check(self._lib.ggfv_batch_run(self._h, int(nsteps)))

    def set_tuning(self, threads=64, rows_per_strip=0, graph_steps=50, fused_steps=None):
        self._check(self._lib.ggfv_batch_set_tuning(self._h, int(threads), int(rows_per_strip), int(graph_steps)))
        if fused_steps is not None:
            self._check(self._lib.ggfv_batch_set_fused_steps(self._h, int(fused_steps)))

    def get_tuning(self):
        v = [ctypes.c_int() for _ in range(4)]
        self._check(self._lib.ggfv_batch_get_tuning(self._h, *(ctypes.byref(x) for x in v)))
        return {"threads": v[0].value, "rows_per_strip": v[1].value, "graph_steps": v[2].value,
                "fused_steps": v[3].value}

    def autotune(self, trial_steps=10):
        t, r = ctypes.c_int(), ctypes.c_int()
        self._check(self._lib.ggfv_batch_autotune(self._h, int(trial_steps), ctypes.byref(t), ctypes.byref(r)))
        return {"threads": t.value, "rows_per_strip": r.value, "fused_steps": self.get_tuning()["fused_steps"]}

    def close(self):
        if getattr(self, "_h", None):
            for c in self.instances:
                c._h = None
            self._lib.ggfv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Context3:
    """One three-dimensional grid, its tensor, parameters and state on one GPU
    (see include/ggfv3.h).  Arrays are (nz, ny, nx), x fastest."""

    def __init__(self, nx, ny, nz, lx=1.0, ly=1.0, lz=1.0, dtype="f64", device=0, stream=None):
        self._lib = lib()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.lx, self.ly, self.lz = float(lx), float(ly), float(lz)
        self.dtype = dtype
        if dtype not in ("f64", "f32"):
            raise ValueError("Context3 dtype must be 'f64' or 'f32'")
        h = ctypes.c_void_p()
        if stream is None:
            stream = _current_stream()
        rc = self._lib.ggfv3_create(ctypes.byref(h), self.nx, self.ny, self.nz, self.lx, self.ly, self.lz,
                                    DTYPES[dtype], int(device), stream)
        if rc != GGFV_OK:
            why = self._lib.ggfv3_last_error(None).decode()
            raise GGFVError(rc, f"ggfv3_create({nx}, {ny}, {nz}, {dtype}, device={device}) failed: {why}")
        self._h = h

    @property
    def count(self):
        return self.nx * self.ny * self.nz

    def _check(self, rc):
        if rc != GGFV_OK:
            raise GGFVError(rc, self._lib.ggfv3_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ggfv3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_params(self, params):
        p = Params(*[float(x) for x in params])
        self._check(self._lib.ggfv3_set_params(self._h, ctypes.byref(p)))

    def set_tensor(self, axx, ayy, azz, axy, axz, ayz):
        ptrs, where, io, keep = _prep_arrays((axx, ayy, azz, axy, axz, ayz), self.count)
        self._check(self._lib.ggfv3_set_tensor(self._h, *ptrs, where, io))

    def set_state(self, u, v, w):
        ptrs, where, io, keep = _prep_arrays((u, v, w), self.count)
        self._check(self._lib.ggfv3_set_state(self._h, *ptrs, where, io))

    def get_state(self, out=None, dtype="f64"):
        if out is None:
            dt = np.float64 if dtype == "f64" else np.float32
            out = [np.empty((self.nz, self.ny, self.nx), dtype=dt) for _ in range(3)]
        return _call_out3(self, self._lib.ggfv3_get_state, out, self.count)

    def stable_dt(self, safety):
        d = ctypes.c_double()
        self._check(self._lib.ggfv3_stable_dt(self._h, float(safety), ctypes.byref(d)))
        return d.value

    def step(self, dt, nsteps=1):
        self._check(self._lib.ggfv3_step(self._h, float(dt), int(nsteps)))

    def mass(self):
        m = (ctypes.c_double * 3)()
        self._check(self._lib.ggfv3_mass(self._h, m))
        return tuple(m)

    def time(self):
        t, n = ctypes.c_double(), ctypes.c_longlong()
        self._check(self._lib.ggfv3_time(self._h, ctypes.byref(t), ctypes.byref(n)))
        return t.value, n.value

    def set_tuning(self, z_per_strip=0, rows_per_wave=0, waves_x=0, waves_y=0):
        self._check(self._lib.ggfv3_set_tuning(self._h, int(z_per_strip), int(rows_per_wave), int(waves_x),
                                               int(waves_y)))

    def get_tuning(self):
        """Effective launch shape, with the number of workgroups a step launches."""
        v = [ctypes.c_int() for _ in range(4)]
        g = ctypes.c_longlong()
        self._check(self._lib.ggfv3_get_tuning(self._h, *(ctypes.byref(x) for x in v), ctypes.byref(g)))
        return {"z_per_strip": v[0].value, "rows_per_wave": v[1].value, "waves_x": v[2].value,
                "waves_y": v[3].value, "workgroups": g.value}
