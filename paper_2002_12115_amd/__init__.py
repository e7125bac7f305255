"""MI355X-native Jacobi pressure sweep (19-point, variable coefficients, fused gosa).

The compute path is ``libhj.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/hj.h``); ``paper_2002_12115_amd.hj`` is its thin ctypes
binding. Importing this package loads nothing: ``inputs`` is host-only and
the binding loads the library on first use and fails loudly without it.
"""
import importlib

__all__ = ["hj", "inputs"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
