"""Host-side checks of the C ABI: the built library loads, exports every function
that include/*.h declare, the binding covers exactly those, argument checks
that run before any device work reject bad input, and the product path has no
CPU fallback.  No GPU is used."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

import paper_2006_01748_amd as pk
from paper_2006_01748_amd import _binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def header_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(ggfv3?_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(_binding.LIB_PATH):
        from paper_2006_01748_amd import build
        build.build()
    return _binding.LIB_PATH


def test_every_declared_symbol_is_exported(built):
    lib = ctypes.CDLL(built)
    names = header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header_exactly():
    assert sorted(pk.exported_names()) == header_functions()


def test_library_does_not_contain_oracle(built):
    out = subprocess.run(["nm", "-D", built], capture_output=True, text=True).stdout
    assert "orc_" not in out
    assert "ggfv_step" in out


def test_status_strings(built):
    lib = pk.lib()
    assert lib.ggfv_status_string(0) == b"GGFV_OK"
    assert lib.ggfv_status_string(5) == b"GGFV_EUNSTABLE"
    assert lib.ggfv_status_string(99) == b"GGFV_UNKNOWN"


@pytest.mark.parametrize("nx,ny,lx,ly,dtype", [
    (0, 4, 1.0, 1.0, pk.GGFV_F64), (4, -1, 1.0, 1.0, pk.GGFV_F64), (4, 4, 0.0, 1.0, pk.GGFV_F64),
    (4, 4, 1.0, float("nan"), pk.GGFV_F64), (4, 4, 1.0, 1.0, 7), (1 << 20, 1 << 20, 1.0, 1.0, pk.GGFV_F64)])
def test_create_rejects_bad_arguments_before_device_work(built, nx, ny, lx, ly, dtype):
    lib = pk.lib()
    h = ctypes.c_void_p(123)
    rc = lib.ggfv_create(ctypes.byref(h), nx, ny, lx, ly, dtype, 0, None)
    assert rc == pk.GGFV_EINVAL
    assert h.value is None


def test_null_context_is_rejected(built):
    lib = pk.lib()
    assert lib.ggfv_step(None, 1e-3, 1) == pk.GGFV_EINVAL
    assert lib.ggfv_set_params(None, None) == pk.GGFV_EINVAL
    assert lib.ggfv_diagnostics(None, None) == pk.GGFV_EINVAL
    assert lib.ggfv_create(None, 4, 4, 1.0, 1.0, pk.GGFV_F64, 0, None) == pk.GGFV_EINVAL
    lib.ggfv_destroy(None)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_binding, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_binding, "_lib", None)
    with pytest.raises(ImportError):
        _binding.lib()


def test_create_failure_message_is_reported(built):
    lib = pk.lib()
    h = ctypes.c_void_p()
    assert lib.ggfv_create(ctypes.byref(h), 0, 5, 1.0, 1.0, pk.GGFV_F64, 0, None) == pk.GGFV_EINVAL
    assert b"grid" in lib.ggfv_last_error(None)


@pytest.mark.parametrize("nx,ny,nz,lz,dtype", [
    (0, 4, 4, 1.0, pk.GGFV_F64), (4, 4, -2, 1.0, pk.GGFV_F64), (4, 4, 4, 0.0, pk.GGFV_F64),
    (4, 4, 4, float("inf"), pk.GGFV_F64), (4, 4, 4, 1.0, pk.GGFV_F32C), (2048, 2048, 2048, 1.0, pk.GGFV_F64)])
def test_create3_rejects_bad_arguments_before_device_work(built, nx, ny, nz, lz, dtype):
    lib = pk.lib()
    h = ctypes.c_void_p(123)
    rc = lib.ggfv3_create(ctypes.byref(h), nx, ny, nz, 1.0, 1.0, lz, dtype, 0, None)
    assert rc == pk.GGFV_EINVAL
    assert h.value is None
    assert lib.ggfv3_last_error(None) != b""


def test_null_context3_is_rejected(built):
    lib = pk.lib()
    assert lib.ggfv3_step(None, 1e-3, 1) == pk.GGFV_EINVAL
    assert lib.ggfv3_set_params(None, None) == pk.GGFV_EINVAL
    assert lib.ggfv3_mass(None, None) == pk.GGFV_EINVAL
    assert lib.ggfv3_set_tuning(None, 4, 0, 0, 0) == pk.GGFV_EINVAL
    assert lib.ggfv3_create(None, 4, 4, 4, 1.0, 1.0, 1.0, pk.GGFV_F64, 0, None) == pk.GGFV_EINVAL
    lib.ggfv3_destroy(None)


def test_null_batch_calls_are_rejected(built):
    lib = pk.lib()
    assert lib.ggfv_batch_set(None, 0, None, 1e-3, *([None] * 6), pk.GGFV_HOST, pk.GGFV_F64) == pk.GGFV_EINVAL
    assert lib.ggfv_batch_get_state(None, 0, None, None, None, pk.GGFV_HOST, pk.GGFV_F64) == pk.GGFV_EINVAL


def test_build_flags_name_existing_sources():
    """Per-source compiler flags are keyed by file name: a renamed source would
    silently lose its instruction schedule.  The lane-shift instances are split
    by precision across exactly the two sources the flags distinguish."""
    from paper_2006_01748_amd import build as b
    names = {os.path.basename(p) for p in b.sources()}
    assert set(b.SOURCE_FLAGS) <= names
    assert {"ggfv_fused_dpp.hip", "ggfv_fused_dpp_f64.hip"} <= names
    assert "ggfv_fused_dpp_f64.hip" not in b.SOURCE_FLAGS
