"""hj_sweep_noalloc, called through the C ABI: the same iterations as
hj_sweep_async with nothing allocated (per-tile gosa partials in the
library's file-scope device array). Two calls in a row, the second on a
smaller grid, each compared with hj_sweep_async on the same inputs (FP64
field bitwise, gosa within 1e-10; FP32 field within 1e-5) and with the
oracle; device memory in use is unchanged across a call; a configuration
whose partials do not fit the array is refused before anything runs."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2002_12115_amd import hj, inputs
from _hjtest import F32_FIELD_RTOL, F64_GOSA_RTOL, field_err, gosa_err, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

H = ctypes.c_void_p


def _ok(lib, rc, where):
    assert rc == 0, "%s: %d %s" % (where, rc, lib.hj_last_error().decode())


def _solver(lib, dtype, shape, f):
    h = H()
    _ok(lib, lib.hj_create(ctypes.byref(h), dtype, *shape, None), "hj_create")
    for name in inputs.INPUTS:
        a = np.ascontiguousarray(f[name], dtype=np.float64)
        _ok(lib, lib.hj_upload_f64(h, inputs.FIELD_ID[name], a.ctypes.data), "hj_upload_f64")
    return h


def _download(lib, h, dtype, shape):
    out = np.empty(shape, dtype=np.float64 if dtype == hj.F64 else np.float32)
    _ok(lib, lib.hj_download(h, inputs.FIELD_ID["p"], out.ctypes.data), "hj_download")
    return out


def _run(lib, entry, dtype, shape, f, n, omega, check_memory=False):
    """Field and gosa history after n iterations through `entry`
    (hj_sweep_async or hj_sweep_noalloc), gosa to a device buffer."""
    h = _solver(lib, dtype, shape, f)
    try:
        dev = torch.zeros(n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0] if check_memory else None
        _ok(lib, getattr(lib, entry)(h, n, ctypes.c_double(omega), ctypes.c_void_p(dev.data_ptr())), entry)
        _ok(lib, lib.hj_sync(h), "hj_sync")
        free1 = torch.cuda.mem_get_info()[0] if check_memory else None
        p = _download(lib, h, dtype, shape)
        hist = dev.cpu().numpy().copy()
    finally:
        _ok(lib, lib.hj_destroy(h), "hj_destroy")
    return p, hist, (free0, free1)


@pytest.fixture(scope="module")
def lib():
    torch.cuda.set_device(0)
    return hj.load()


# two calls in a row, the second on a smaller grid (and fewer iterations)
CALLS = [((66, 70, 134), 9), ((18, 21, 35), 4)]


@pytest.mark.parametrize("dtype", [hj.F64, hj.F32])
def test_noalloc_matches_async_two_calls(lib, dtype):
    omega = 0.8
    for q, (shape, n) in enumerate(CALLS):
        f = inputs.fields(2002 + q, shape)
        say("hj_sweep_async", "f64" if dtype == hj.F64 else "f32", shape, n)
        p_a, g_a, _ = _run(lib, "hj_sweep_async", dtype, shape, f, n, omega)
        say("hj_sweep_noalloc", "f64" if dtype == hj.F64 else "f32", shape, n)
        p_b, g_b, (free0, free1) = _run(lib, "hj_sweep_noalloc", dtype, shape, f, n, omega, check_memory=True)
        pref, _, href = oracle.sweep(f, n, omega, nthreads=4)
        assert free1 == free0, "device memory in use changed by %d bytes" % (free0 - free1)
        if dtype == hj.F64:
            assert np.array_equal(p_b, p_a), (shape, field_err(p_b, p_a))
            assert np.array_equal(p_b, pref), (shape, field_err(p_b, pref))
            assert gosa_err(g_b, g_a) <= F64_GOSA_RTOL
            assert gosa_err(g_b, href) <= F64_GOSA_RTOL
        else:
            assert field_err(p_b, p_a.astype(np.float64)) <= F32_FIELD_RTOL
            assert field_err(p_b, pref) <= F32_FIELD_RTOL
            assert gosa_err(g_b, g_a) < 1e-4


def test_noalloc_refuses_partials_beyond_its_array(lib):
    """The direct kernel (bj 2) on 1028x1028x3 has 1026*513 = 526,338 tiles
    per iteration, more than the array's 524,288 doubles: HJ_ERR_ARG, checked
    before anything is uploaded or launched."""
    h = H()
    _ok(lib, lib.hj_create(ctypes.byref(h), hj.F32, 1028, 1028, 3, None), "hj_create")
    try:
        c = hj.Config.make(kernel=hj.KERNEL_DIRECT, bj=2, vec=1, ichunk=1, nontemporal=0, use_graph=0,
                           xcd_remap=0, persistent=0, tsteps=1, reread=0)
        _ok(lib, lib.hj_set_config(h, ctypes.byref(c)), "hj_set_config")
        dev = torch.zeros(2, dtype=torch.float64, device="cuda")
        rc = lib.hj_sweep_noalloc(h, 2, ctypes.c_double(0.8), ctypes.c_void_p(dev.data_ptr()))
        assert rc == -1 and b"scratch" in lib.hj_last_error()
        rc = lib.hj_sweep_noalloc(h, 2, ctypes.c_double(0.8), None)
        assert rc == -1 and b"NULL" in lib.hj_last_error()
    finally:
        _ok(lib, lib.hj_destroy(h), "hj_destroy")


def test_noalloc_captured_in_a_graph_and_replayed(lib):
    """The allocation-free call captured into a caller's HIP graph (torch's
    graph capture on the handle's stream) and replayed three times, with
    downloads between the replays: after replay r the FP64 field equals the
    oracle's after 4r iterations bitwise, and the gosa the replay wrote equals
    the oracle's history for those iterations. Four iterations are two
    two-iteration launches, so the field returns to its buffer each time."""
    shape, n, omega = (34, 36, 70), 4, 0.8
    f = inputs.fields(11, shape)
    stream = torch.cuda.Stream()
    h = H()
    _ok(lib, lib.hj_create(ctypes.byref(h), hj.F64, *shape, ctypes.c_void_p(stream.cuda_stream)), "hj_create")
    try:
        for name in inputs.INPUTS:
            a = np.ascontiguousarray(f[name], dtype=np.float64)
            _ok(lib, lib.hj_upload_f64(h, inputs.FIELD_ID[name], a.ctypes.data), "hj_upload_f64")
        c = hj.Config()
        _ok(lib, lib.hj_get_config(h, ctypes.byref(c)), "hj_get_config")
        assert c.tsteps == 2
        dev = torch.zeros(n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        say("capture hj_sweep_noalloc", shape, n)
        with torch.cuda.graph(g, stream=stream):
            _ok(lib, lib.hj_sweep_noalloc(h, n, ctypes.c_double(omega), ctypes.c_void_p(dev.data_ptr())),
                "hj_sweep_noalloc (captured)")
        _, _, href = oracle.sweep(f, 3 * n, omega, nthreads=4)
        for r in range(1, 4):
            say("replay", r)
            g.replay()
            torch.cuda.synchronize()
            p = _download(lib, h, hj.F64, shape)
            pref = oracle.sweep(f, r * n, omega, nthreads=4)[0]
            assert np.array_equal(p, pref), (r, field_err(p, pref))
            assert gosa_err(dev.cpu().numpy(), href[(r - 1) * n:r * n]) <= F64_GOSA_RTOL, r
    finally:
        _ok(lib, lib.hj_destroy(h), "hj_destroy")


FRESH_CAPTURE = r"""
import ctypes, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
sys.path.insert(0, sys.argv[1] + "/tests")
import oracle
from paper_2002_12115_amd import hj, inputs
lib = hj.load()
shape, n, omega = (34, 36, 70), 4, 0.8
f = inputs.fields(5, shape)
stream = torch.cuda.Stream()
h = ctypes.c_void_p()
assert lib.hj_create(ctypes.byref(h), hj.F64, *shape, ctypes.c_void_p(stream.cuda_stream)) == 0
for name in inputs.INPUTS:
    a = np.ascontiguousarray(f[name], dtype=np.float64)
    assert lib.hj_upload_f64(h, inputs.FIELD_ID[name], a.ctypes.data) == 0
c = hj.Config.make(kernel=1, bj=8, vec=2, ichunk=7, nontemporal=0, use_graph=1, xcd_remap=1, persistent=0,
                   tsteps=2, reread=0)
assert lib.hj_set_config(h, ctypes.byref(c)) == 0
dev = torch.zeros(n, dtype=torch.float64, device="cuda")
torch.cuda.synchronize()
g = torch.cuda.CUDAGraph()
with torch.cuda.graph(g, stream=stream):      # the first launch of this kernel in the process
    assert lib.hj_sweep_noalloc(h, n, ctypes.c_double(omega), ctypes.c_void_p(dev.data_ptr())) == 0
g.replay()
torch.cuda.synchronize()
out = np.empty(shape, dtype=np.float64)
assert lib.hj_download(h, inputs.FIELD_ID["p"], out.ctypes.data) == 0
assert lib.hj_destroy(h) == 0
pref = oracle.sweep(f, n, omega, nthreads=4)[0]
assert np.array_equal(out, pref)
print("fresh capture ok", flush=True)
"""


def test_noalloc_first_launch_inside_a_capture_in_a_fresh_process():
    """In a new process, the first launch of a two-iteration kernel with the
    XCD remap happens inside a caller's graph capture: the configuration call
    made the runtime queries beforehand, so the capture holds, and one replay
    gives the oracle's field bitwise."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    say("fresh-process capture of hj_sweep_noalloc")
    r = subprocess.run([sys.executable, "-c", FRESH_CAPTURE, root], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "fresh capture ok" in r.stdout
