"""ctypes binding of libhj (declared in include/hj.h).

Argument marshalling only: every step of a sweep runs in the library's HIP
kernels. PyTorch, when present, supplies device memory (``hj_attach`` on a
torch uint8 tensor) and the stream; without it the library allocates.
The library must be built (``paper_2002_12115_amd.build``): there is no
fallback path, and loading fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Iterable, List, Mapping, Optional, Sequence, Tuple

import numpy as np

from .inputs import FIELDS, FIELD_ID, INPUTS

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhj.so")

F64, F32 = 0, 1
KERNEL_DIRECT, KERNEL_MARCH, KERNEL_FLAT = 0, 1, 2
STATUS = {0: "HJ_OK", -1: "HJ_ERR_ARG", -2: "HJ_ERR_SHAPE", -3: "HJ_ERR_DTYPE", -4: "HJ_ERR_OOM",
          -5: "HJ_ERR_HIP", -6: "HJ_ERR_STATE", -7: "HJ_ERR_HANDLE", -8: "HJ_ERR_TUNE"}


class HJError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__("%s: %s (%s)" % (where, STATUS.get(status, status), detail))
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("bj", ctypes.c_int), ("vec", ctypes.c_int),
                ("ichunk", ctypes.c_int), ("nontemporal", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("xcd_remap", ctypes.c_int), ("persistent", ctypes.c_int), ("tsteps", ctypes.c_int),
                ("reread", ctypes.c_int)]

    def as_dict(self) -> Dict[str, int]:
        return {n: int(getattr(self, n)) for n, _ in self._fields_}

    @classmethod
    def make(cls, **kw) -> "Config":
        c = cls()
        for n, v in kw.items():
            setattr(c, n, int(v))
        return c

    def __repr__(self):
        return "Config(%s)" % ", ".join("%s=%d" % kv for kv in self.as_dict().items())


_lib = None


def load() -> ctypes.CDLL:
    """Load libhj.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhj.so is not built (%s); run paper_2002_12115_amd.build.build() "
                          "or __graft_entry__.build()" % LIB_PATH)
    # torch ships its own libamdhip64 with the same soname as the system one.
    # One process must hold one HIP runtime: load torch's first (when torch is
    # installed) so libhj binds to it and torch can still see the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    i32, dbl, vp, u64 = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_ulonglong
    ip, dp, cp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(Config)
    H = ctypes.c_void_p
    sig = {
        "hj_slab_bytes": [i32, i32, i32, i32, ctypes.POINTER(u64)],
        "hj_create": [ctypes.POINTER(H), i32, i32, i32, i32, vp],
        "hj_attach": [ctypes.POINTER(H), i32, i32, i32, i32, vp, u64, vp],
        "hj_upload": [H, i32, vp],
        "hj_upload_f64": [H, i32, vp],
        "hj_download": [H, i32, vp],
        "hj_snapshot": [H, vp],
        "hj_snapshot_wait": [H],
        "hj_sweep": [H, i32, dbl, dp, dp],
        "hj_sweep_async": [H, i32, dbl, vp],
        "hj_sweep_noalloc": [H, i32, dbl, vp],
        "hj_residual": [H, dp],
        "hj_get_config": [H, cp],
        "hj_set_config": [H, cp],
        "hj_autotune": [H, i32, i32, cp, dp],
        "hj_sync": [H],
        "hj_get_stream": [H, ctypes.POINTER(vp)],
        "hj_destroy": [H],
        "hj_batch_create": [ctypes.POINTER(H), i32, i32, ip, ip, ip, vp],
        "hj_batch_upload": [H, i32, i32, vp],
        "hj_batch_upload_f64": [H, i32, i32, vp],
        "hj_batch_download": [H, i32, i32, vp],
        "hj_batch_sweep": [H, i32, dbl, dp, dp],
        "hj_batch_residual": [H, dp],
        "hj_batch_get_config": [H, cp],
        "hj_batch_set_config": [H, cp],
        "hj_batch_autotune": [H, i32, i32, cp, dp],
        "hj_batch_destroy": [H],
        "hj_copy_probe": [vp, vp, u64, vp, dp],
        "hj_stream_probe": [H, i32, i32, i32, dp],
        "hj_autotune_ga": [H, i32, i32, u64, dbl, dbl, i32, i32, cp, dp, ip],
        "hj_batch_autotune_ga": [H, i32, i32, u64, dbl, dbl, i32, i32, cp, dp, ip],
        "hj_gene_config": [i32, i32, i32, i32, i32, ctypes.c_uint, cp],
        "hj_ga_run": [i32, i32, i32, u64, dbl, dbl, vp, ctypes.POINTER(ctypes.c_uint), dp, vp, ip],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = i32
    lib.hj_status_string.argtypes = [i32]
    lib.hj_status_string.restype = ctypes.c_char_p
    lib.hj_last_error.argtypes = []
    lib.hj_last_error.restype = ctypes.c_char_p
    lib.hj_last_sweep_ms.argtypes = []
    lib.hj_last_sweep_ms.restype = dbl
    _lib = lib
    return lib


def check(rc: int, where: str) -> None:
    if rc != 0:
        lib = load()
        raise HJError(rc, where, (lib.hj_last_error() or b"").decode(errors="replace"))


def last_sweep_ms() -> float:
    return float(load().hj_last_sweep_ms())


def _dtype_code(dtype) -> int:
    if dtype in (F64, "f64", "float64", np.float64):
        return F64
    if dtype in (F32, "f32", "float32", np.float32):
        return F32
    if isinstance(dtype, np.dtype):
        return _dtype_code(dtype.type)
    raise ValueError("dtype must be f64 or f32, got %r" % (dtype,))


def _np_dtype(code: int):
    return np.float64 if code == F64 else np.float32


def _torch_cuda():
    try:
        import torch
    except ImportError:
        return None
    return torch if torch.cuda.is_available() else None


def _field(name) -> int:
    return FIELD_ID[name] if isinstance(name, str) else int(name)


class Solver:
    """One resident Jacobi solve (``hj_solver``).

    use_torch: allocate the device slab as a torch tensor and run on torch's
    current stream (default when torch sees a GPU); otherwise the library
    allocates and creates its own stream.
    """

    def __init__(self, dtype, shape: Sequence[int], use_torch: Optional[bool] = None, stream=None):
        self.lib = load()
        self.dtype = _dtype_code(dtype)
        self.np_dtype = _np_dtype(self.dtype)
        self.shape = tuple(int(s) for s in shape)
        nx, ny, nz = self.shape
        self._h = ctypes.c_void_p()
        self._slab = None
        torch = _torch_cuda() if use_torch in (None, True) else None
        if use_torch and torch is None:
            raise RuntimeError("use_torch=True but torch sees no GPU")
        if stream is None and torch is not None:
            stream = torch.cuda.current_stream().cuda_stream
        st = ctypes.c_void_p(int(stream)) if stream else None
        if torch is not None:
            nbytes = ctypes.c_ulonglong()
            check(self.lib.hj_slab_bytes(self.dtype, nx, ny, nz, ctypes.byref(nbytes)), "hj_slab_bytes")
            self._slab = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device="cuda")
            base = self._slab.data_ptr()
            aligned = (base + 255) // 256 * 256
            check(self.lib.hj_attach(ctypes.byref(self._h), self.dtype, nx, ny, nz, ctypes.c_void_p(aligned),
                                     nbytes.value, st), "hj_attach")
        else:
            check(self.lib.hj_create(ctypes.byref(self._h), self.dtype, nx, ny, nz, st), "hj_create")
        self.gosa_history: Optional[np.ndarray] = None
        self._snap: Optional[np.ndarray] = None
        self.last_ms: float = 0.0

    # -- data movement --
    def upload(self, name, array: np.ndarray) -> None:
        a = np.ascontiguousarray(array)
        if a.shape != self.shape:
            raise ValueError("array shape %s != solver shape %s" % (a.shape, self.shape))
        f = _field(name)
        if a.dtype == np.float64:
            check(self.lib.hj_upload_f64(self._h, f, a.ctypes.data), "hj_upload_f64(%s)" % (name,))
        else:
            a = np.ascontiguousarray(a, dtype=self.np_dtype)
            check(self.lib.hj_upload(self._h, f, a.ctypes.data), "hj_upload(%s)" % (name,))

    def upload_all(self, arrays: Mapping[str, np.ndarray]) -> None:
        for n in INPUTS:
            self.upload(n, arrays[n])

    def download(self, name="p", out: Optional[np.ndarray] = None) -> np.ndarray:
        """The field as a new array, or written into `out` (C-contiguous, the
        solver's shape and dtype; a pinned buffer is copied to directly)."""
        if out is None:
            out = np.empty(self.shape, dtype=self.np_dtype)
        elif out.shape != self.shape or out.dtype != self.np_dtype or not out.flags.c_contiguous:
            raise ValueError("out must be a C-contiguous %s array of shape %s" % (self.np_dtype, self.shape))
        check(self.lib.hj_download(self._h, _field(name), out.ctypes.data), "hj_download(%s)" % (name,))
        return out

    def snapshot(self, out: np.ndarray) -> None:
        """Start sending the current field to `out` (C-contiguous, the
        solver's shape and dtype; pinned for the transfer to overlap later
        sweeps). `out` must stay untouched until snapshot_wait()."""
        if out.shape != self.shape or out.dtype != self.np_dtype or not out.flags.c_contiguous:
            raise ValueError("out must be a C-contiguous %s array of shape %s" % (self.np_dtype, self.shape))
        self._snap = out          # keep the array alive while the copy runs
        check(self.lib.hj_snapshot(self._h, out.ctypes.data), "hj_snapshot")

    def snapshot_wait(self) -> None:
        check(self.lib.hj_snapshot_wait(self._h), "hj_snapshot_wait")
        self._snap = None

    # -- compute --
    def sweep(self, n_iter: int, omega: float) -> float:
        hist = np.zeros(max(int(n_iter), 1), dtype=np.float64)
        last = ctypes.c_double(float("nan"))
        check(self.lib.hj_sweep(self._h, int(n_iter), float(omega), ctypes.byref(last),
                                hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "hj_sweep")
        self.gosa_history = hist[:n_iter]
        self.last_ms = last_sweep_ms()
        return float(last.value)

    def sweep_async(self, n_iter: int, omega: float, dev_gosa_hist: int = 0) -> None:
        check(self.lib.hj_sweep_async(self._h, int(n_iter), float(omega),
                                      ctypes.c_void_p(dev_gosa_hist) if dev_gosa_hist else None),
              "hj_sweep_async")

    def sweep_noalloc(self, n_iter: int, omega: float, dev_gosa_hist: int) -> None:
        """hj_sweep_noalloc: enqueue n_iter iterations without any allocation;
        dev_gosa_hist is the device address of n_iter doubles."""
        check(self.lib.hj_sweep_noalloc(self._h, int(n_iter), float(omega), ctypes.c_void_p(dev_gosa_hist)),
              "hj_sweep_noalloc")

    def residual(self) -> float:
        g = ctypes.c_double()
        check(self.lib.hj_residual(self._h, ctypes.byref(g)), "hj_residual")
        return float(g.value)

    def sync(self) -> None:
        check(self.lib.hj_sync(self._h), "hj_sync")

    def stream_probe(self, vec: int = 1, ichunk: int = 16, n_rep: int = 10) -> float:
        """ms per launch of the 13-read/1-write streaming probe on these arrays."""
        ms = ctypes.c_double()
        check(self.lib.hj_stream_probe(self._h, int(vec), int(ichunk), int(n_rep), ctypes.byref(ms)),
              "hj_stream_probe")
        return float(ms.value)

    @property
    def stream(self) -> int:
        s = ctypes.c_void_p()
        check(self.lib.hj_get_stream(self._h, ctypes.byref(s)), "hj_get_stream")
        return int(s.value or 0)

    # -- configuration --
    @property
    def config(self) -> Config:
        c = Config()
        check(self.lib.hj_get_config(self._h, ctypes.byref(c)), "hj_get_config")
        return c

    @config.setter
    def config(self, c: Config) -> None:
        check(self.lib.hj_set_config(self._h, ctypes.byref(c)), "hj_set_config")

    def set(self, **kw) -> Config:
        c = self.config
        for n, v in kw.items():
            setattr(c, n, int(v))
        self.config = c
        return c

    def autotune(self, n_sweeps: int = 3, repeats: int = 3) -> Tuple[Config, float]:
        c = Config()
        ms = ctypes.c_double()
        check(self.lib.hj_autotune(self._h, int(n_sweeps), int(repeats), ctypes.byref(c), ctypes.byref(ms)),
              "hj_autotune")
        return c, float(ms.value)

    def autotune_ga(self, population: int = 10, generations: int = 10, seed: int = 2002, pc: float = 0.9,
                    pm: float = 0.05, n_sweeps: int = 3, repeats: int = 3) -> Tuple[Config, float, int]:
        """The paper's genetic search over the configuration (returns config, ms, evaluations)."""
        c = Config()
        ms = ctypes.c_double()
        ev = ctypes.c_int()
        check(self.lib.hj_autotune_ga(self._h, int(population), int(generations), int(seed), float(pc), float(pm),
                                      int(n_sweeps), int(repeats), ctypes.byref(c), ctypes.byref(ms),
                                      ctypes.byref(ev)), "hj_autotune_ga")
        return c, float(ms.value), int(ev.value)

    def close(self) -> None:
        if self._h:
            check(self.lib.hj_destroy(self._h), "hj_destroy")   # waits for a pending snapshot
            self._h = ctypes.c_void_p()
        self._slab = None
        self._snap = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._h:
                self.lib.hj_destroy(self._h)
        except Exception:
            pass


class Batch:
    """Many independent solves advanced together (``hj_batch``)."""

    def __init__(self, dtype, shapes: Sequence[Sequence[int]], stream=None):
        self.lib = load()
        self.dtype = _dtype_code(dtype)
        self.np_dtype = _np_dtype(self.dtype)
        self.shapes = [tuple(int(s) for s in sh) for sh in shapes]
        n = len(self.shapes)
        nx = (ctypes.c_int * n)(*[s[0] for s in self.shapes])
        ny = (ctypes.c_int * n)(*[s[1] for s in self.shapes])
        nz = (ctypes.c_int * n)(*[s[2] for s in self.shapes])
        self._h = ctypes.c_void_p()
        st = ctypes.c_void_p(int(stream)) if stream else None
        check(self.lib.hj_batch_create(ctypes.byref(self._h), self.dtype, n, nx, ny, nz, st), "hj_batch_create")
        self.gosa_history: Optional[np.ndarray] = None
        self.last_ms = 0.0

    @property
    def n(self) -> int:
        return len(self.shapes)

    def upload(self, inst: int, name, array: np.ndarray) -> None:
        a = np.ascontiguousarray(array)
        if a.shape != self.shapes[inst]:
            raise ValueError("instance %d: array shape %s != %s" % (inst, a.shape, self.shapes[inst]))
        f = _field(name)
        if a.dtype == np.float64:
            check(self.lib.hj_batch_upload_f64(self._h, inst, f, a.ctypes.data), "hj_batch_upload_f64")
        else:
            a = np.ascontiguousarray(a, dtype=self.np_dtype)
            check(self.lib.hj_batch_upload(self._h, inst, f, a.ctypes.data), "hj_batch_upload")

    def upload_all(self, inst: int, arrays: Mapping[str, np.ndarray]) -> None:
        for n in INPUTS:
            self.upload(inst, n, arrays[n])

    def download(self, inst: int, name="p", out: Optional[np.ndarray] = None) -> np.ndarray:
        """Instance inst's field as a new array, or written into `out`
        (C-contiguous, the instance's shape and the batch's dtype)."""
        shape = tuple(self.shapes[inst])
        if out is None:
            out = np.empty(shape, dtype=self.np_dtype)
        elif out.shape != shape or out.dtype != self.np_dtype or not out.flags.c_contiguous:
            raise ValueError("out must be a C-contiguous %s array of shape %s" % (self.np_dtype, shape))
        check(self.lib.hj_batch_download(self._h, inst, _field(name), out.ctypes.data), "hj_batch_download")
        return out

    def sweep(self, n_iter: int, omega: float) -> np.ndarray:
        hist = np.zeros((max(int(n_iter), 1), self.n), dtype=np.float64)
        last = np.zeros(self.n, dtype=np.float64)
        check(self.lib.hj_batch_sweep(self._h, int(n_iter), float(omega),
                                      last.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "hj_batch_sweep")
        self.gosa_history = hist[:n_iter]
        self.last_ms = last_sweep_ms()
        return last

    def residual(self) -> np.ndarray:
        g = np.zeros(self.n, dtype=np.float64)
        check(self.lib.hj_batch_residual(self._h, g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
              "hj_batch_residual")
        return g

    @property
    def config(self) -> Config:
        c = Config()
        check(self.lib.hj_batch_get_config(self._h, ctypes.byref(c)), "hj_batch_get_config")
        return c

    @config.setter
    def config(self, c: Config) -> None:
        check(self.lib.hj_batch_set_config(self._h, ctypes.byref(c)), "hj_batch_set_config")

    def set(self, **kw) -> Config:
        c = self.config
        for n, v in kw.items():
            setattr(c, n, int(v))
        self.config = c
        return c

    def autotune(self, n_sweeps: int = 3, repeats: int = 3) -> Tuple[Config, float]:
        c = Config()
        ms = ctypes.c_double()
        check(self.lib.hj_batch_autotune(self._h, int(n_sweeps), int(repeats), ctypes.byref(c),
                                         ctypes.byref(ms)), "hj_batch_autotune")
        return c, float(ms.value)

    def autotune_ga(self, population: int = 10, generations: int = 10, seed: int = 2002, pc: float = 0.9,
                    pm: float = 0.05, n_sweeps: int = 3, repeats: int = 3) -> Tuple[Config, float, int]:
        c = Config()
        ms = ctypes.c_double()
        ev = ctypes.c_int()
        check(self.lib.hj_batch_autotune_ga(self._h, int(population), int(generations), int(seed), float(pc),
                                            float(pm), int(n_sweeps), int(repeats), ctypes.byref(c),
                                            ctypes.byref(ms), ctypes.byref(ev)), "hj_batch_autotune_ga")
        return c, float(ms.value), int(ev.value)

    def close(self) -> None:
        if self._h:
            check(self.lib.hj_batch_destroy(self._h), "hj_batch_destroy")
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._h:
                self.lib.hj_batch_destroy(self._h)
        except Exception:
            pass


def copy_probe(nbytes: int) -> float:
    """Time the library's copy kernel over nbytes (device to device); returns ms."""
    torch = _torch_cuda()
    if torch is None:
        raise RuntimeError("copy_probe needs torch with a GPU for its buffers")
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ms = ctypes.c_double()
    st = torch.cuda.current_stream().cuda_stream
    check(load().hj_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                               ctypes.c_void_p(st) if st else None, ctypes.byref(ms)), "hj_copy_probe")
    return float(ms.value)
