"""CPU oracle for the Jacobi pressure sweep -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU
baseline leg may import this package. The product library never does; it
shares no code with it.

``oracle.c`` is the plain FP64 triple loop (the operator, the evaluation
order and the gosa definition are stated in its header). This module is the
ctypes binding: it copies the caller's arrays, runs the loop, and returns new
arrays, so callers' inputs are never modified.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Mapping, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORDER = ("p", "a0", "a1", "a2", "a3", "b0", "b1", "b2", "c0", "c1", "c2", "bnd", "wrk1", "wrk2")
COMPILE = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile liboracle.so (gcc -O2 -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(COMPILE + [_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i32, dbl, vp, i64 = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_longlong
        arr14 = ctypes.c_void_p * 14
        lib.oracle_sweep.restype = i32
        lib.oracle_sweep.argtypes = [i32, i32, i32, arr14, i32, dbl, vp, i32]
        lib.oracle_residual.restype = dbl
        lib.oracle_residual.argtypes = [i32, i32, i32, arr14, i32]
        lib.oracle_cells.restype = i32
        lib.oracle_cells.argtypes = [i32, i32, i32, arr14, dbl, i64, vp, vp, vp]
        lib.oracle_max_threads.restype = i32
        lib.oracle_max_threads.argtypes = []
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _prepare(arrays: Mapping[str, np.ndarray]) -> Tuple[Dict[str, np.ndarray], Tuple[int, int, int]]:
    shape = np.asarray(arrays["p"]).shape
    if len(shape) != 3:
        raise ValueError("arrays must be 3-D [nx][ny][nz]")
    work = {}
    for name in ORDER:
        if name == "wrk2" and "wrk2" not in arrays:
            src = arrays["p"]
        else:
            src = arrays[name]
        a = np.array(src, dtype=np.float64, order="C", copy=True)
        if a.shape != shape:
            raise ValueError("array %s has shape %s, expected %s" % (name, a.shape, shape))
        work[name] = a
    return work, shape


def _ptrs(work: Mapping[str, np.ndarray]):
    return (ctypes.c_void_p * 14)(*[work[n].ctypes.data for n in ORDER])


def _in_place(arrays: Mapping[str, np.ndarray]) -> Tuple[Dict[str, np.ndarray], Tuple[int, int, int]]:
    """The caller's own arrays (FP64, C-contiguous, one shape), with a wrk2
    made from p when none is given: no copy of the 13 inputs."""
    shape = np.asarray(arrays["p"]).shape
    work = {}
    for name in ORDER:
        if name == "wrk2" and "wrk2" not in arrays:
            work[name] = np.array(arrays["p"], dtype=np.float64, order="C", copy=True)
            continue
        a = arrays[name]
        if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags.c_contiguous or a.shape != shape:
            raise ValueError("copy=False needs C-contiguous float64 arrays of one shape (%s)" % name)
        work[name] = a
    if len(shape) != 3:
        raise ValueError("arrays must be 3-D [nx][ny][nz]")
    return work, shape


def sweep(arrays: Mapping[str, np.ndarray], n_iter: int, omega: float,
          nthreads: int = 1, copy: bool = True) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """n_iter Jacobi iterations from the given arrays.

    Returns (p, wrk2, gosa_hist): the field after the last iteration, the
    last iteration's wrk2 (shell copied from the initial p when wrk2 is not
    given), and the per-iteration gosa, each from the pre-update field.
    With copy=True (the default) the arrays are copied and left unchanged;
    with copy=False they must be C-contiguous float64 arrays, and p (and
    wrk2, when given) are updated in place -- for grids too large to hold twice.
    """
    work, (nx, ny, nz) = _prepare(arrays) if copy else _in_place(arrays)
    hist = np.zeros(max(n_iter, 0), dtype=np.float64)
    rc = _load().oracle_sweep(nx, ny, nz, _ptrs(work), int(n_iter), float(omega),
                              hist.ctypes.data if n_iter > 0 else None, int(nthreads))
    if rc != 0:
        raise ValueError("oracle_sweep failed with %d (shape %s)" % (rc, (nx, ny, nz)))
    return work["p"], work["wrk2"], hist


def residual(arrays: Mapping[str, np.ndarray], nthreads: int = 1) -> float:
    """gosa of the given p with no update."""
    work, (nx, ny, nz) = _prepare(arrays)
    g = float(_load().oracle_residual(nx, ny, nz, _ptrs(work), int(nthreads)))
    if g < 0:
        raise ValueError("oracle_residual rejected its arguments")
    return g


def cells(arrays: Mapping[str, np.ndarray], omega: float,
          idx: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """(ss, wrk2) of one iteration at the given dense interior indices.

    Reads the arrays in place (no copy), so it is usable on grids too large
    to duplicate.
    """
    shape = np.asarray(arrays["p"]).shape
    nx, ny, nz = shape
    keep = []
    ptrs = []
    for name in ORDER:
        a = arrays.get(name, arrays["p"]) if name == "wrk2" else arrays[name]
        if a.dtype != np.float64 or not a.flags.c_contiguous or a.shape != shape:
            a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        ptrs.append(a.ctypes.data)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    ss = np.zeros(idx.size, np.float64)
    w2 = np.zeros(idx.size, np.float64)
    rc = _load().oracle_cells(nx, ny, nz, (ctypes.c_void_p * 14)(*ptrs), float(omega),
                              int(idx.size), idx.ctypes.data, ss.ctypes.data, w2.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_cells failed with %d" % rc)
    return ss, w2
