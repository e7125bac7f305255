"""Seeded synthetic inputs for the Jacobi pressure sweep (host side only).

The numbers come from ``hjgen.c`` (counter-based SplitMix64 + Box-Muller);
this module is the ctypes binding plus the named workloads. It holds none of
the sweep's arithmetic, so the CPU oracle and the HIP path can both consume
its arrays without sharing any of the method's code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field as _field
from typing import Dict, List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hjgen.c")
_LIB = os.path.join(_HERE, "libhjgen.so")

# Field order shared by every component: index = field id of the C generator
# and of the library's field enum.
FIELDS: Tuple[str, ...] = ("p", "a0", "a1", "a2", "a3", "b0", "b1", "b2",
                           "c0", "c1", "c2", "bnd", "wrk1", "wrk2")
INPUTS: Tuple[str, ...] = FIELDS[:13]          # what a caller uploads
FIELD_ID: Dict[str, int] = {n: i for i, n in enumerate(FIELDS)}

DEFAULT_SIGMA = 0.01   # wrk1 ~ N(0, sigma): 0.01 is read as the standard deviation


def build(force: bool = False) -> str:
    """Compile libhjgen.so with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u64, i32, dbl = ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        vp = ctypes.c_void_p
        lib.hjgen_mix.restype = u64
        lib.hjgen_mix.argtypes = [u64]
        lib.hjgen_bits.restype = u64
        lib.hjgen_bits.argtypes = [u64, i32, u64]
        lib.hjgen_uniform.restype = dbl
        lib.hjgen_uniform.argtypes = [u64, i32, u64]
        lib.hjgen_normal.restype = dbl
        lib.hjgen_normal.argtypes = [u64, i32, u64, dbl]
        lib.hjgen_fill_f64.restype = i32
        lib.hjgen_fill_f64.argtypes = [u64, i32, i32, i32, i32, dbl, i32, vp]
        lib.hjgen_fill_f32.restype = i32
        lib.hjgen_fill_f32.argtypes = [u64, i32, i32, i32, i32, dbl, i32, vp]
        lib.hjgen_values_f64.restype = i32
        lib.hjgen_values_f64.argtypes = [u64, i32, i32, i32, i32, dbl, i32, ctypes.c_longlong, vp, vp]
        lib.hjgen_batch.restype = i32
        lib.hjgen_batch.argtypes = [u64, i32, i32, i32, i32, i32, vp, vp, vp, vp]
        _lib = lib
    return _lib


def mix(z: int) -> int:
    return int(_load().hjgen_mix(z & 0xFFFFFFFFFFFFFFFF))


def bits(seed: int, fid: int, n: int) -> int:
    return int(_load().hjgen_bits(seed & 0xFFFFFFFFFFFFFFFF, fid, n))


def uniform(seed: int, fid: int, n: int) -> float:
    return float(_load().hjgen_uniform(seed & 0xFFFFFFFFFFFFFFFF, fid, n))


def normal(seed: int, fid: int, n: int, sigma: float = 1.0) -> float:
    return float(_load().hjgen_normal(seed & 0xFFFFFFFFFFFFFFFF, fid, n, sigma))


def field(seed: int, name, shape: Sequence[int], dtype=np.float64,
          sigma: float = DEFAULT_SIGMA, bnd_mode: int = 0, out: np.ndarray | None = None) -> np.ndarray:
    """One dense C-order [nx][ny][nz] array of field `name` (name or id 0..12)."""
    fid = FIELD_ID[name] if isinstance(name, str) else int(name)
    if not 0 <= fid <= 12:
        raise ValueError("field %r is not a drawn or derived input" % (name,))
    nx, ny, nz = (int(s) for s in shape)
    dtype = np.dtype(dtype)
    if out is None:
        out = np.empty((nx, ny, nz), dtype=dtype)
    if out.shape != (nx, ny, nz) or out.dtype != dtype or not out.flags.c_contiguous:
        raise ValueError("out must be a C-contiguous %s array of shape %s" % (dtype, (nx, ny, nz)))
    lib = _load()
    if dtype == np.float64:
        rc = lib.hjgen_fill_f64(seed & 0xFFFFFFFFFFFFFFFF, fid, nx, ny, nz, sigma, bnd_mode,
                                out.ctypes.data)
    elif dtype == np.float32:
        rc = lib.hjgen_fill_f32(seed & 0xFFFFFFFFFFFFFFFF, fid, nx, ny, nz, sigma, bnd_mode,
                                out.ctypes.data)
    else:
        raise ValueError("dtype must be float64 or float32")
    if rc != 0:
        raise ValueError("hjgen rejected field=%d shape=%s" % (fid, (nx, ny, nz)))
    return out


def values(seed: int, name, shape: Sequence[int], idx, sigma: float = DEFAULT_SIGMA,
           bnd_mode: int = 0) -> np.ndarray:
    """FP64 values of one field at the given dense linear indices of a grid."""
    fid = FIELD_ID[name] if isinstance(name, str) else int(name)
    nx, ny, nz = (int(s) for s in shape)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.shape, dtype=np.float64)
    rc = _load().hjgen_values_f64(seed & 0xFFFFFFFFFFFFFFFF, fid, nx, ny, nz, sigma, bnd_mode,
                                  int(idx.size), idx.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise ValueError("hjgen_values rejected field=%r or an index" % (name,))
    return out


def neighbourhood(seed: int, shape: Sequence[int], centres, sigma: float = DEFAULT_SIGMA,
                  bnd_mode: int = 0, dtype=np.float64, radius: int = 1) -> Dict[str, np.ndarray]:
    """The 13 inputs on the (2r+1)^3 block around each centre (i,j,k).

    Returns arrays of shape [m, 2r+1, 2r+1, 2r+1]; block q holds cells
    (i-r..i+r, j-r..j+r, k-r..k+r) of centre q, with the values the full
    grid has there (rounded to `dtype`, then widened back to FP64). Every
    block must lie inside the grid.
    """
    nx, ny, nz = (int(s) for s in shape)
    c = np.asarray(centres, dtype=np.int64).reshape(-1, 3)
    d = np.arange(-radius, radius + 1)
    ii = c[:, 0, None, None, None] + d[None, :, None, None]
    jj = c[:, 1, None, None, None] + d[None, None, :, None]
    kk = c[:, 2, None, None, None] + d[None, None, None, :]
    lin = (ii * ny + jj) * nz + kk
    out = {}
    for n in INPUTS:
        v = values(seed, n, shape, lin.ravel(), sigma, bnd_mode).reshape(lin.shape)
        out[n] = v.astype(dtype).astype(np.float64)
    return out


def fields(seed: int, shape: Sequence[int], dtype=np.float64, sigma: float = DEFAULT_SIGMA,
           bnd_mode: int = 0) -> Dict[str, np.ndarray]:
    """The 13 input arrays (p, a0..a3, b0..b2, c0..c2, bnd, wrk1)."""
    return {n: field(seed, n, shape, dtype, sigma, bnd_mode) for n in INPUTS}


def batch_shapes(seed: int, n: int, lo_xy: int = 17, hi_xy: int = 129, lo_z: int = 33,
                 hi_z: int = 257) -> Tuple[List[Tuple[int, int, int]], List[int]]:
    """Sizes (boundary included) and per-instance seeds of a batch of solves."""
    nx = np.zeros(n, np.int32)
    ny = np.zeros(n, np.int32)
    nz = np.zeros(n, np.int32)
    sd = np.zeros(n, np.uint64)
    rc = _load().hjgen_batch(seed & 0xFFFFFFFFFFFFFFFF, n, lo_xy, hi_xy, lo_z, hi_z,
                             nx.ctypes.data, ny.ctypes.data, nz.ctypes.data, sd.ctypes.data)
    if rc != 0:
        raise ValueError("bad batch size range")
    return [(int(a), int(b), int(c)) for a, b, c in zip(nx, ny, nz)], [int(s) for s in sd]


@dataclass(frozen=True)
class Workload:
    """A named solve: grid (boundary included, k contiguous), dtype, iterations."""
    name: str
    shape: Tuple[int, int, int]
    dtype: str                 # "f64" or "f32"
    iters: int
    omega: float = 0.8
    seed: int = 2002
    batch: int = 0             # >0: number of independent instances (sizes drawn from seed)
    note: str = ""

    @property
    def interior(self) -> int:
        if self.batch:
            shapes, _ = batch_shapes(self.seed, self.batch)
            return sum((a - 2) * (b - 2) * (c - 2) for a, b, c in shapes)
        nx, ny, nz = self.shape
        return (nx - 2) * (ny - 2) * (nz - 2)


# The five workloads of the Himeno-style pressure solve. The paper evaluates
# the Himeno benchmark (section 5.1.1) without stating its grid, precision or
# iteration count; these seeded synthetic grids stand in for it.
WORKLOADS: Dict[str, Workload] = {
    "small_f64": Workload("small_f64", (34, 34, 66), "f64", 50,
                          note="34x34x66 FP64, 50 iterations (parity case)"),
    "medium_f64": Workload("medium_f64", (130, 130, 258), "f64", 200,
                           note="130x130x258 FP64, 200 iterations, all arrays resident"),
    "large_f32": Workload("large_f32", (258, 258, 514), "f32", 500,
                          note="258x258x514 FP32 storage, FP64 gosa, 500 iterations"),
    "batch64": Workload("batch64", (0, 0, 0), "f32", 100, batch=64,
                        note="64 uneven solves nx,ny~U{17..129}, nz~U{33..257}, 100 iterations"),
    "huge_f32": Workload("huge_f32", (514, 514, 1026), "f32", 1000,
                         note="514x514x1026 FP32 storage, FP64 gosa, 1000 iterations"),
}
