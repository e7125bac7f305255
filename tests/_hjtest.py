"""Helpers shared by the GPU tests: run the HIP path and the oracle on the
same seeded inputs and measure their difference."""
import sys

import numpy as np

import oracle
from paper_2002_12115_amd import hj, inputs

F64_FIELD_RTOL = 1e-12     # FP64 field (expected bitwise: identical evaluation order)
F64_GOSA_RTOL = 1e-10      # FP64 gosa (reduction order differs)
F32_FIELD_RTOL = 1e-5      # FP32 field against the FP64 oracle


def say(*a):
    """Name the case before each GPU step (flushed, so a fault still shows it)."""
    print("[case]", *a, file=sys.stderr, flush=True)


def field_err(x, ref):
    """Normwise relative error max|x - ref| / max|ref|."""
    x = np.asarray(x, dtype=np.float64)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def gosa_err(g, ref):
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(g - ref) / np.maximum(np.abs(ref), 1e-300)))


def gpu_run(shape, dtype, n_iter, omega=0.8, seed=2002, cfg=None, bnd_mode=0, use_torch=None,
            arrays=None):
    """(p, gosa_hist, solver config) from the HIP path, or None when the
    configuration cannot run this grid (a flat kernel too wide for it)."""
    f = arrays if arrays is not None else inputs.fields(seed, shape, bnd_mode=bnd_mode)
    with hj.Solver(dtype, shape, use_torch=use_torch) as s:
        if cfg is not None:
            try:
                s.config = cfg
            except hj.HJError as e:
                if cfg.kernel == hj.KERNEL_FLAT and e.status == -1:
                    return None
                raise
        s.upload_all(f)
        s.sweep(n_iter, omega)
        p = s.download("p")
        return p, s.gosa_history.copy(), s.config


def oracle_run(shape, n_iter, omega=0.8, seed=2002, bnd_mode=0, nthreads=8, arrays=None):
    f = arrays if arrays is not None else inputs.fields(seed, shape, bnd_mode=bnd_mode)
    p, _, hist = oracle.sweep(f, n_iter, omega, nthreads=nthreads)
    return p, hist


def cfg(**kw):
    base = dict(kernel=hj.KERNEL_MARCH, bj=4, vec=1, ichunk=8, nontemporal=1, use_graph=1,
                xcd_remap=1, persistent=0, tsteps=1, reread=0)
    base.update(kw)
    return hj.Config.make(**base)


def f64_configs():
    out = []
    for bj in (2, 4, 8):
        for nt in (0, 1):
            out.append(cfg(kernel=hj.KERNEL_DIRECT, bj=bj, nontemporal=nt, xcd_remap=nt))
    for bj in (1, 2, 4, 8):
        for v in (1, 2):
            for ich, nt, rm in ((1, 1, 0), (3, 0, 1), (16, 1, 1), (1000, 0, 0)):
                out.append(cfg(bj=bj, vec=v, ichunk=ich, nontemporal=nt, xcd_remap=rm))
    out.extend(fused_configs())
    out.extend(flat_configs())
    return out


def flat_configs():
    """Runs of consecutive interior (j,k) cells."""
    out = []
    for nw in (2, 4, 8):
        for ich, nt, rm in ((1, 1, 0), (3, 0, 1), (1000, 1, 1)):
            out.append(cfg(kernel=hj.KERNEL_FLAT, bj=nw, vec=1, ichunk=ich, nontemporal=nt, xcd_remap=rm))
    return out


def fused_configs():
    """Two iterations per pass (tsteps 2)."""
    out = []
    for bj in (2, 4, 6, 8, 14):
        for ich, nt, rm, rr in ((1, 1, 0, 0), (2, 0, 1, 1), (5, 1, 0, 1), (1000, 0, 1, 0)):
            out.append(cfg(bj=bj, vec=1, ichunk=ich, nontemporal=nt, xcd_remap=rm, tsteps=2, reread=rr))
    for bj in (2, 4, 6, 8, 12):          # 64-cell rows with a halo wave
        for ich, nt, rm, rr in ((1, 0, 1, 0), (3, 1, 0, 1), (1000, 0, 1, 1)):
            out.append(cfg(bj=bj, vec=2, ichunk=ich, nontemporal=nt, xcd_remap=rm, tsteps=2, reread=rr))
    for bj in (6, 14, 22, 30):           # two 30-cell rows per wave
        for ich, nt, rm, rr in ((1, 1, 1, 0), (4, 0, 0, 1), (1000, 0, 1, 0)):
            out.append(cfg(bj=bj, vec=4, ichunk=ich, nontemporal=nt, xcd_remap=rm, tsteps=2, reread=rr))
    return out


def f32_configs():
    out = [cfg(kernel=hj.KERNEL_DIRECT, bj=4, nontemporal=1, vec=1)]
    for bj in (1, 2, 4, 8):
        for v in (1, 2, 4):
            for ich, nt, rm in ((2, 1, 1), (7, 0, 0)):
                out.append(cfg(bj=bj, vec=v, ichunk=ich, nontemporal=nt, xcd_remap=rm))
    out.extend(fused_configs())
    out.extend(flat_configs())
    return out


def cfg_id(c):
    d = c.as_dict()
    k = ("direct" if d["kernel"] == 0 else "flat" if d["kernel"] == 2 else
         ({1: "fused%d", 2: "wide%d", 4: "narrow%d"}[d["vec"]]) % d["reread"] if d["tsteps"] == 2 else "march")
    return "%s-bj%d-v%d-ic%d-nt%d-rm%d" % (k, d["bj"], d["vec"], d["ichunk"], d["nontemporal"], d["xcd_remap"])
