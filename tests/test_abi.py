"""The C-ABI library loads and exports what include/hj.h declares; host-only
argument checks (no GPU work is started by any call here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hj.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hj_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2002_12115_amd import hj
    if not os.path.exists(hj.LIB_PATH):
        pytest.fail("libhj.so is not built; run __graft_entry__.build()")
    return hj.load()


def test_header_declares_the_boundary():
    names = declared()
    for n in ("hj_create", "hj_upload", "hj_sweep", "hj_residual", "hj_download", "hj_destroy",
              "hj_batch_create", "hj_batch_sweep", "hj_autotune", "hj_batch_autotune"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    assert lib.hj_status_string(0) == b"HJ_OK"
    assert lib.hj_status_string(-7) == b"HJ_ERR_HANDLE"
    assert lib.hj_status_string(123) == b"HJ_ERR_UNKNOWN"


def test_slab_bytes_layout(lib):
    b = ctypes.c_ulonglong()
    assert lib.hj_slab_bytes(0, 34, 34, 66, ctypes.byref(b)) == 0
    # 14 fields, rows padded to 128-byte lines: at least the dense size
    assert b.value >= 14 * 34 * 34 * 66 * 8
    b32 = ctypes.c_ulonglong()
    assert lib.hj_slab_bytes(1, 34, 34, 66, ctypes.byref(b32)) == 0
    assert b32.value < b.value
    assert lib.hj_slab_bytes(0, 2, 34, 66, ctypes.byref(b)) == -2
    assert lib.hj_slab_bytes(7, 34, 34, 66, ctypes.byref(b)) == -3
    assert lib.hj_slab_bytes(0, 34, 34, 66, None) == -1


def test_host_side_argument_errors(lib):
    h = ctypes.c_void_p()
    assert lib.hj_create(ctypes.byref(h), 5, 10, 10, 10, None) == -3
    assert lib.hj_create(ctypes.byref(h), 0, 10, 2, 10, None) == -2
    assert lib.hj_create(None, 0, 10, 10, 10, None) == -1
    assert b"dtype" in lib.hj_last_error() or b"NULL" in lib.hj_last_error()
    # operations on a handle the library never issued
    bogus = ctypes.c_void_p(0x1234)
    g = ctypes.c_double()
    assert lib.hj_sweep(bogus, 1, 0.8, None, None) == -7
    assert lib.hj_residual(None, ctypes.byref(g)) == -7
    assert lib.hj_destroy(bogus) == -7
    assert lib.hj_batch_sweep(bogus, 1, 0.8, None, None) == -7
    nx = (ctypes.c_int * 1)(10)
    assert lib.hj_batch_create(ctypes.byref(h), 9, 1, nx, nx, nx, None) == -3
    assert lib.hj_batch_create(ctypes.byref(h), 0, 0, nx, nx, nx, None) == -1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2002_12115_amd import hj
    monkeypatch.setattr(hj, "_lib", None)
    monkeypatch.setattr(hj, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        hj.load()
