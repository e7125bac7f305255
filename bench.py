#!/usr/bin/env python3
"""Benchmark of the resident 19-point Jacobi sweep on one MI355X.

A step is one full solve of the workload on resident arrays: n_iter Jacobi
iterations with the fused FP64 gosa of every iteration brought back to the
host (hj_sweep). Inputs are uploaded before the timed region. The printed
JSON line reports GLUPS (interior lattice updates per second) over the
timed steps; the dominant kernel's HBM rate against the 8 TB/s peak, both
algorithmic (the bytes a pass must move: each of the 14 arrays once) and
measured (rocprofv3 counter bytes, when taken on the current kernel code);
the field and gosa error of every result against the FP64 CPU oracle; and
the oracle itself timed on the host cores as a reported baseline. The oracle
runs only in that last leg (cpu_baseline_leg): the GPU legs keep the results
to check, and the leg times the oracle and compares them with it.

  python bench.py [--steps K] [--warmup W] [--workload medium_f64] [--retune]
                  [--no-cpu-baseline] [--no-extra] [--profile]
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GLUPS + HBM GB/s (% of peak), FP32-batched vs FP64 plain at 1e-5 rel error"
PEAK_HBM_GBPS = 8000.0          # MI355X HBM3E, vendor figure
KERNEL_SOURCES = ["paper_2002_12115_amd/csrc/sweep_kernels.hpp", "paper_2002_12115_amd/csrc/sweep_types.hpp",
                  "paper_2002_12115_amd/csrc/hj_kernels.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
TUNE_CACHE = os.path.join(ROOT, "paper_2002_12115_amd", "tune_cache.txt")


_T0 = time.perf_counter()


def log(*a):
    print("[bench +%.1fs]" % (time.perf_counter() - _T0), *a, file=sys.stderr, flush=True)


_CPP_TOKENS = re.compile(r'"(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\'|//[^\n]*|/\*.*?\*/', re.S)


def code_only(src: str) -> str:
    """C++ source without its comments, whitespace runs collapsed: edits to
    comments or layout do not change it."""
    kept = _CPP_TOKENS.sub(lambda m: m.group(0) if m.group(0)[0] in "\"'" else " ", src)
    return " ".join(kept.split())


def kernel_hash() -> str:
    """Identity of the kernel code the stored counter figures were taken on."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()[:16]


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def cache_has(kind: str, dtype: str, key: str) -> bool:
    """Whether the tuning cache (HJ_TUNE_CACHE) holds this problem."""
    path = os.environ.get("HJ_TUNE_CACHE")
    if not path or not os.path.exists(path):
        return False
    arch = device_arch()
    with open(path) as f:
        for line in f:
            t = line.split()
            if len(t) >= 4 and t[:4] == [kind, arch, dtype, key]:
                return True
    return False


def batch_key(shapes) -> str:
    h = 1469598103934665603
    for sh in shapes:
        for d in sh:
            h ^= d & 0xFFFFFFFF
            h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return "n%d-%016x" % (len(shapes), h)


def interior(shape):
    nx, ny, nz = shape
    return (nx - 2) * (ny - 2) * (nz - 2)


def esize(dtype: str) -> int:
    return 8 if dtype == "f64" else 4


def kernel_name(cfg: dict) -> str:
    """The kernel a configuration launches for its passes."""
    if cfg.get("tsteps") == 2:
        return "wide_kernel" if cfg.get("vec") == 2 else "fused_kernel"
    return {0: "direct_kernel", 1: "march_kernel", 2: "flat_kernel"}[cfg["kernel"]]


def load_traffic(workload: str, cfg: dict):
    """HBM bytes per launch measured by rocprofv3 counters, if they were taken
    on the current kernel sources and the same launch configuration."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(workload)
    if not e or e.get("kernel_hash") != kernel_hash() or e.get("config") != cfg:
        return None
    return e.get("bytes_per_launch")


def roofline(esz: int, n_int: int, tsteps: int, avg_launch_ms: float, traffic):
    """HBM figures of one launch of a kernel that advances every interior cell
    of n_int by tsteps iterations in one pass over memory.

    achieved: algorithmic bytes per launch / average launch time. The
    algorithmic bytes are what the pass must move at least: the 12
    coefficient arrays and p read once and wrk2 written once per interior
    cell, 14 * esz * n_int, i.e. 14 * esz / tsteps per lattice update (112 B
    FP64, 56 B FP32 with one iteration per pass; half with two). It is a lower
    bound on the real traffic, so frac never exceeds what HBM moved.
    measured: rocprofv3 FETCH_SIZE + WRITE_SIZE bytes per launch (calibrated
    against a copy of known size) / the same time, when the counters were
    taken on the current kernel code and configuration (else null). These
    count every byte that leaves the L2s; the memory-side cache may answer
    part of the reads, so they bound the HBM bytes from above.
    per_update_equiv: the bytes a one-iteration kernel would move for the
    same updates, per second (a speed figure, not a fraction of HBM)."""
    s = avg_launch_ms * 1e-3
    alg = 14 * esz * n_int
    out = {"bound": "hbm", "achieved": alg / s / 1e9, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
           "frac": alg / s / 1e9 / PEAK_HBM_GBPS, "traffic": traffic,
           "achieved_basis": "algorithmic: 14 arrays x %d B x %d interior cells per launch (%d iteration%s)"
                             % (esz, n_int, tsteps, "s" if tsteps > 1 else ""),
           "iterations_per_launch": tsteps, "lattice_updates_per_launch": n_int * tsteps,
           "algorithmic_bytes_per_launch": alg, "avg_launch_ms": avg_launch_ms,
           "measured_gbps": None, "measured_frac": None, "traffic_over_algorithmic": None,
           "per_update_equiv_gbps": alg * tsteps / s / 1e9}
    if traffic:
        out["traffic_basis"] = ("L2 egress: FETCH_SIZE + WRITE_SIZE per launch, calibrated; an upper bound on "
                                "HBM bytes (the memory-side cache may serve part of the reads)")
        out["measured_gbps"] = traffic / s / 1e9
        out["measured_frac"] = traffic / s / 1e9 / PEAK_HBM_GBPS
        out["traffic_over_algorithmic"] = traffic / alg
    return out


def cpu_baseline(w, arrays, budget_s: float):
    """Oracle on the host cores: whole grid, as many iterations as fit the
    budget; when the whole solve fits, repeated solves until the budget is
    spent (a steadier figure)."""
    import oracle
    nthreads = oracle.max_threads()      # OpenMP's default: OMP_NUM_THREADS or all cores
    t0 = time.perf_counter()
    oracle.sweep(arrays, 1, w.omega, nthreads=nthreads)
    t1 = time.perf_counter() - t0
    iters = max(1, min(w.iters, int(budget_s / max(t1, 1e-6))))
    solves, dt = 0, 0.0
    while solves == 0 or dt + dt / solves <= budget_s:
        t0 = time.perf_counter()
        oracle.sweep(arrays, iters, w.omega, nthreads=nthreads)
        dt += time.perf_counter() - t0
        solves += 1
    return {"value": interior(w.shape) * iters * solves / dt / 1e9, "unit": "GLUPS", "cores": nthreads,
            "kind": "oracle",
            "sample": "%s grid %s, %d x %d of %d iterations, FP64, %d OpenMP threads, %.1f s"
                      % (w.name, "x".join(map(str, w.shape)), solves, iters, w.iters, nthreads, dt),
            "host": host_cpu()}


def host_cpu() -> dict:
    """The host the oracle ran on: CPU model, logical CPUs, CPUs this process may use."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def accuracy(w, arrays, p_gpu, hist_gpu, iters: int):
    import oracle
    pref, _, href = oracle.sweep(arrays, iters, w.omega, nthreads=oracle.max_threads())
    ferr = float(np.abs(p_gpu.astype(np.float64) - pref).max() / np.abs(pref).max())
    gerr = float(np.max(np.abs(hist_gpu - href) / href))
    out = {"field_rel_err": ferr, "gosa_rel_err": gerr, "iters_checked": iters,
           "field_bitwise": bool(np.array_equal(p_gpu.astype(np.float64), pref))}
    if p_gpu.dtype == np.float32:
        # FP32 residuals reach the FP32 rounding floor as the solve converges,
        # far below the FP64 oracle's gosa: reported, not gated
        out["gosa_gated"] = False
    return out


def whole_grid_accuracy(w, inputs, p_gpu, hist_gpu, iters: int):
    """Field and gosa error of a grid too large to hold twice: the FP64
    inputs are regenerated and the oracle updates them in place."""
    import oracle
    f = inputs.fields(w.seed, w.shape)
    pref, _, href = oracle.sweep(f, iters, w.omega, nthreads=oracle.max_threads(), copy=False)
    ferr = float(np.abs(p_gpu.astype(np.float64) - pref).max() / np.abs(pref).max())
    gerr = float(np.max(np.abs(hist_gpu - href) / href))
    del f, pref
    return {"field_rel_err": ferr, "gosa_rel_err": gerr, "iters_checked": iters, "cells_checked": "all"}


def run_single(w, args, hj, inputs, steps: int, warmup: int, check_iters: int, keep_arrays: bool):
    """Time `steps` full solves of workload w on resident arrays."""
    n_int = interior(w.shape)
    log("workload", w.name, w.shape, w.dtype, "iters", w.iters)
    t0 = time.perf_counter()
    s = hj.Solver(w.dtype, w.shape)
    arrays = None
    if keep_arrays:
        arrays = inputs.fields(w.seed, w.shape)   # FP64 master copies (the oracle's inputs)
        gen_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        s.upload_all(arrays)
        upload_s = time.perf_counter() - t0
    else:
        # one field at a time in the solver's dtype (RNE of the FP64 draws)
        dt = np.float64 if w.dtype == "f64" else np.float32
        gen_s = upload_s = 0.0
        for name in inputs.INPUTS:
            t1 = time.perf_counter()
            a = inputs.field(w.seed, name, w.shape, dtype=dt)
            t2 = time.perf_counter()
            s.upload(name, a)
            gen_s += t2 - t1
            upload_s += time.perf_counter() - t2
            del a
    log("inputs generated in %.1f s, uploaded in %.2f s" % (gen_s, upload_s))
    tuned_ms = None
    key = "%dx%dx%d" % tuple(w.shape)
    if args.config and w.name == args.workload:
        c = s.config.as_dict()
        for kv in args.config.split(","):
            k, v = kv.split("=")
            if k not in c:
                raise SystemExit("--config: unknown field %r" % k)
            c[k] = int(v)
        s.config = hj.Config.make(**c)
        log("configuration from --config:", s.config)
    elif args.retune or not cache_has("solve", w.dtype, key):
        c, tuned_ms = s.autotune(n_sweeps=args.tune_sweeps, repeats=3)
        log("autotuned:", c, "%.3f ms per %d sweeps" % (tuned_ms, args.tune_sweeps))
    else:
        log("configuration from the tuning cache:", s.config)
    cfg = s.config.as_dict()

    # the first solve's result from the initial field, kept for the
    # cpu_baseline leg to compare with the oracle
    check = None
    if check_iters:
        # the first check_iters iterations from the initial field, compared
        # whole with the oracle in the cpu_baseline leg
        n_chk = min(check_iters, w.iters)
        s.sweep(n_chk, w.omega)
        check = {"w": w, "n": n_chk, "p": s.download("p"), "hist": s.gosa_history.copy(), "arrays": arrays}
        if arrays is not None:
            s.upload("p", arrays["p"])
        else:
            s.upload("p", inputs.field(w.seed, "p", w.shape,
                                       dtype=np.float64 if w.dtype == "f64" else np.float32))

    import torch
    for _ in range(warmup):
        s.sweep(w.iters, w.omega)
    torch.cuda.synchronize()
    kernel_ms = 0.0
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        s.sweep(w.iters, w.omega)
        step_ms.append(s.last_ms)       # HIP events on the solver's stream around each solve
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = sum(step_ms)
    updates = n_int * w.iters * steps
    glups = updates / wall / 1e9
    # A launch of t iterations advances every interior cell t times; a
    # remainder of a solve runs single-iteration launches, whose time is
    # folded in pro rata (one iteration = 1/t of a launch).
    tsteps = max(1, int(cfg.get("tsteps", 1)))
    launches = w.iters * steps / tsteps
    avg_launch_ms = kernel_ms / launches
    traffic = load_traffic(w.name, cfg)
    roof = roofline(esize(w.dtype), n_int, tsteps, avg_launch_ms, traffic)
    roof["kernel"] = kernel_name(cfg)
    ceilings = None
    if args.ceilings:
        # the library's probes on this GPU: a plain copy, and 13 reads + 1 write
        # per cell over these very arrays (the sweep's traffic without its stencil)
        nb = 2 << 30
        hj.copy_probe(nb)
        copy_ms = min(hj.copy_probe(nb) for _ in range(3))
        sv = 2 if w.dtype == "f64" else 4
        st_ms = min(s.stream_probe(sv, ich, 10) for ich in (2, 4, 8))
        ceilings = {"copy_gbps": 2 * nb / copy_ms / 1e6,
                    "stream13r1w_gbps": 14 * esize(w.dtype) * n_int / st_ms / 1e6}
        ceilings["achieved_over_stream13r1w"] = roof["achieved"] / ceilings["stream13r1w_gbps"]
        if roof["measured_gbps"]:
            ceilings["measured_over_stream13r1w"] = roof["measured_gbps"] / ceilings["stream13r1w_gbps"]
    roof["measured_ceilings"] = ceilings
    res = {
        "glups": glups, "ms_per_step": wall * 1e3 / steps, "wall_s": wall, "roofline": roof,
        "upload_s": upload_s, "pcie_inclusive_glups": updates / (wall + upload_s) / 1e9,
        "config": cfg, "tuned_ms": tuned_ms, "accuracy": None, "check": check,
        "last_gosa": float(s.gosa_history[-1]), "steps": steps,
        "step_ms_device": {"median": float(np.median(step_ms)), "min": float(min(step_ms)),
                           "max": float(max(step_ms))},
    }
    s.close()
    return res, arrays


def solve_ms(s, w, reps: int = 5) -> float:
    """Median device time of `reps` whole solves (w.iters iterations) in the
    handle's installed configuration."""
    s.sweep(w.iters, w.omega)
    t = []
    for _ in range(reps):
        s.sweep(w.iters, w.omega)
        t.append(s.last_ms)
    return float(np.median(t))


def tuner_comparison(w, hj, inputs, arrays, sweeps: int = 40, seeds=(2002, 1, 7)):
    """Exhaustive search against the paper's genetic search (population and
    generations 10, at most the gene length; Pc 0.9, Pm 0.05) on the same
    arrays. Every measurement times `sweeps` sweeps (2-3 ms on medium_f64, so
    that timing noise does not decide fitness), median of 3. Each search's
    winner is then timed on whole solves, and the genetic winner is reported
    as a fraction of the exhaustive winner's speed, for each seed."""
    out = {"sweeps_per_measurement": sweeps, "repeats": 3}
    saved = os.environ.get("HJ_TUNE_CACHE", "")
    os.environ["HJ_TUNE_CACHE"] = ""              # never write the committed cache
    try:
        runs = [("exhaustive", None)] + [("genetic_seed%d" % sd, sd) for sd in seeds]
        for kind, seed in runs:
            s = hj.Solver(w.dtype, w.shape)
            s.upload_all(arrays)
            t0 = time.perf_counter()
            if seed is None:
                c, ms = s.autotune(n_sweeps=sweeps, repeats=3)
                ev = None
            else:
                c, ms, ev = s.autotune_ga(10, 10, seed, 0.9, 0.05, n_sweeps=sweeps, repeats=3)
            dt = time.perf_counter() - t0
            solve = solve_ms(s, w)
            out[kind] = {"config": c.as_dict(), "evaluations": ev, "tune_s": dt,
                         "search_ms_per_sweep": ms / sweeps, "solve_ms": solve,
                         "glups": interior(w.shape) * w.iters / solve / 1e6}
            s.close()
            log("tuner", kind, c, "%.3f ms per solve" % solve)
    finally:
        os.environ["HJ_TUNE_CACHE"] = saved
    ex = out["exhaustive"]["solve_ms"]
    out["genetic_speed_over_exhaustive"] = {str(sd): ex / out["genetic_seed%d" % sd]["solve_ms"] for sd in seeds}
    return out


def transfer_ablation(w, hj, arrays):
    """The same solve under the transfer placements of paper_2002_12115_amd.transfer."""
    from paper_2002_12115_amd import transfer
    out = {}
    ref = None
    for policy, n, pinned in (("resident", w.iters, False), ("p_every_k", w.iters, False),
                              ("p_every_iter", 20, False), ("all_every_iter", 10, False),
                              ("p_every_k", w.iters, True), ("p_every_iter", 20, True),
                              ("all_every_iter", 10, True), ("observe_every_k", w.iters, True),
                              ("observe_every_k_async", w.iters, True)):
        s = hj.Solver(w.dtype, w.shape)
        r = transfer.run(s, arrays, policy, n, w.omega, k=10, pinned=pinned)
        s.close()
        if policy == "resident":
            ref = r
        same = None
        if n == ref["iters"]:
            same = bool(np.array_equal(r["field"], ref["field"]))
        out[policy + ("_pinned" if pinned else "")] = {"glups": interior(w.shape) * n / r["wall_s"] / 1e9, "iters": n, "k": r["k"],
                       "ms_per_iter": r["wall_s"] * 1e3 / n,
                       "pcie_gbps": (r["h2d_bytes"] + r["d2h_bytes"]) / r["wall_s"] / 1e9,
                       "field_equals_resident": same}
    return out


def one_iteration_config(hj, dtype: str, shape) -> dict:
    """The plain one-iteration configuration of a single solve (one launch per
    iteration): march kernel, 16-byte lanes (bj 4 for FP64, 8 for FP32),
    non-temporal streams, the i-chunk that gives the grid about 4096 workgroups."""
    bj, vec = (4, 2) if dtype == "f64" else (8, 4)
    kt = -(-(shape[2] - 2) // (64 * vec))
    jt = -(-(shape[1] - 2) // bj)
    nchunks = max(1, -(-4096 // (kt * jt)))
    ichunk = max(1, -(-(shape[0] - 2) // nchunks))
    return dict(kernel=hj.KERNEL_MARCH, bj=bj, vec=vec, ichunk=ichunk, nontemporal=1, use_graph=0, xcd_remap=0,
                persistent=0, tsteps=1, reread=0)


BATCH_MODES = ("batched", "per_instance", "per_instance_default")


def run_batch(args, hj, inputs, dtype: str, iters: int, mode: str, tune: bool):
    """The 64 uneven solves of batch64, `iters` iterations each.

    batched: one launch per pass over every instance's tiles, the loop
    replayed as one graph (the library's batch path), in its tuned
    configuration; timed with HIP events around each batch solve.
    per_instance: one launch per instance per iteration, instance after
    instance on one stream (the one-iteration kernel, no graph).
    per_instance_default: each instance its own solve in the library's
    default configuration (two iterations per launch, graph per solve),
    still one launch per instance per pass. Both per-instance modes are
    timed on the host clock around all instances' solves."""
    w = inputs.WORKLOADS["batch64"]
    shapes, seeds = inputs.batch_shapes(w.seed, w.batch)
    n_int = sum(interior(sh) for sh in shapes)
    import torch
    if mode != "batched":
        solvers = []
        stream = None
        for sh, sd in zip(shapes, seeds):
            s = hj.Solver(dtype, sh, stream=stream)   # all instances on one stream
            stream = stream or s.stream
            if mode == "per_instance":
                s.config = hj.Config.make(**one_iteration_config(hj, dtype, sh))
            s.upload_all(inputs.fields(sd, sh))
            solvers.append(s)
        for s in solvers:
            s.sweep_async(2, w.omega)
        for s in solvers:
            s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            for s in solvers:
                s.sweep_async(iters, w.omega)
            for s in solvers:
                s.sync()
        wall = time.perf_counter() - t0
        if mode == "per_instance":
            cfg = dict(one_iteration_config(hj, dtype, shapes[0]), ichunk="about 4096 workgroups per instance")
        else:
            cfg = dict(solvers[0].config.as_dict(), ichunk="one wave of resident workgroups per instance")
        tsteps = 1 if mode == "per_instance" else max(1, int(solvers[0].config.tsteps))
        for s in reversed(solvers):          # the first one owns the shared stream
            s.close()
        dev_ms = wall * 1e3 / args.batch_steps
    else:
        b = hj.Batch(dtype, shapes)
        for t, (sh, sd) in enumerate(zip(shapes, seeds)):
            b.upload_all(t, inputs.fields(sd, sh))
        if tune or not cache_has("batch", dtype, batch_key(shapes)):
            c, ms = b.autotune(n_sweeps=6, repeats=3)
            log("batch autotuned", dtype, c, ms)
        else:
            log("batch configuration from the tuning cache:", dtype, b.config)
        b.sweep(2, w.omega)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dms = []
        for _ in range(args.batch_steps):
            b.sweep(iters, w.omega)
            dms.append(b.last_ms)
        wall = time.perf_counter() - t0
        cfg = b.config.as_dict()
        tsteps = max(1, int(cfg.get("tsteps", 1)))
        b.close()
        dev_ms = float(np.median(dms))
    name = "batch64_%s%s" % (dtype, "" if mode == "batched" else "_" + mode)
    # one "launch" here is one pass over every instance (a single launch when
    # batched; one launch per instance otherwise)
    roof = roofline(esize(dtype), n_int, tsteps, dev_ms / (iters / tsteps), load_traffic(name, cfg))
    return {"glups": n_int * iters * args.batch_steps / wall / 1e9, "dtype": dtype, "iters": iters,
            "mode": mode, "instances": len(shapes), "interior_cells": n_int,
            "launches_per_pass": len(shapes) if mode != "batched" else 1, "config": cfg,
            "ms_per_solve": dev_ms, "roofline": roof}


def batch_results(hj, inputs, n_iter: int):
    """Both dtypes' batched fields and gosa histories after n_iter
    iterations from the same inputs, for the cpu_baseline leg to compare
    with the oracle."""
    w = inputs.WORKLOADS["batch64"]
    shapes, seeds = inputs.batch_shapes(w.seed, w.batch)
    arrs = [inputs.fields(sd, sh) for sh, sd in zip(shapes, seeds)]
    out = {"w": w, "n": n_iter, "arrays": arrs}
    for dtype in ("f64", "f32"):
        b = hj.Batch(dtype, shapes)
        for t, a in enumerate(arrs):
            b.upload_all(t, a)
        b.sweep(n_iter, w.omega)
        out[dtype] = {"p": [b.download(t) for t in range(len(shapes))], "hist": b.gosa_history.copy(),
                      "config": b.config.as_dict()}
        b.close()
    return out


def batch_accuracy(r):
    """Per-instance error of both batched dtypes against the FP64 oracle
    (one oracle solve per instance): FP64 field bitwise and gosa, FP32 field
    and gosa, the worst instance of each."""
    import oracle
    acc = {"iters_checked": r["n"], "instances": len(r["arrays"]), "f64_field_bitwise": True,
           "f64_field_rel_err_max": 0.0, "f64_gosa_rel_err_max": 0.0,
           "f32_field_rel_err_max": 0.0, "f32_gosa_rel_err_max": 0.0}
    for t, a in enumerate(r["arrays"]):
        pref, _, href = oracle.sweep(a, r["n"], r["w"].omega, nthreads=oracle.max_threads())
        for dt in ("f64", "f32"):
            p = r[dt]["p"][t].astype(np.float64)
            fe = float(np.abs(p - pref).max() / np.abs(pref).max())
            ge = float(np.max(np.abs(r[dt]["hist"][:, t] - href) / href))
            acc[dt + "_field_rel_err_max"] = max(acc[dt + "_field_rel_err_max"], fe)
            acc[dt + "_gosa_rel_err_max"] = max(acc[dt + "_gosa_rel_err_max"], ge)
        acc["f64_field_bitwise"] = acc["f64_field_bitwise"] and bool(np.array_equal(r["f64"]["p"][t], pref))
    return acc


def cpu_baseline_leg(w, arrays, budget_s: float, checks: dict, inputs):
    """The only part of this script that runs the oracle: the error of every
    checked GPU result against it, then its timing on the host cores.
    checks: name -> the result a GPU leg kept (see run_single, batch_results)."""
    acc = {}
    for name, c in checks.items():
        if c is None:
            continue
        if "hist" in c:
            acc[name] = (accuracy(c["w"], c["arrays"], c["p"], c["hist"], c["n"]) if c["arrays"] is not None
                         else whole_grid_accuracy(c["w"], inputs, c["p"], c["hist"], c["n"]))
        else:
            acc[name] = batch_accuracy(c)
        log("accuracy", name, acc[name])
    return cpu_baseline(w, arrays, budget_s), acc


def counter_means(run_dir: str, counter: str) -> dict:
    """Per-kernel mean of one rocprofv3 --pmc counter (KiB per dispatch) over
    every *counter_collection.csv under run_dir: {kernel: (mean, dispatches)}."""
    import csv
    import glob
    sums, counts = {}, {}
    for path in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                k = row["Kernel_Name"]
                sums[k] = sums.get(k, 0.0) + float(row["Counter_Value"])
                counts[k] = counts.get(k, 0) + 1
    return {k: (sums[k] / counts[k], counts[k]) for k in sums}


def ingest_counters(key: str, kernel: str, fetch_dir: str, write_dir: str, bench_json: str, copy_bytes: int,
                    per_pass: int = 1) -> dict:
    """Record the HBM bytes of `kernel` in profiles/traffic.json under `key`:
    FETCH_SIZE and WRITE_SIZE from two rocprofv3 --pmc runs of the same bench
    command, each scaled by what the counter read for the library's copy
    kernel over copy_bytes in that run (the calibration), times per_pass
    dispatches per pass (the per-instance batch modes launch one kernel per
    instance). The entry is keyed by the current kernel code and by the
    configuration the profiled run used (its JSON line in bench_json), so
    bench.py reports it only while both still hold."""
    fetch, write = counter_means(fetch_dir, "FETCH_SIZE"), counter_means(write_dir, "WRITE_SIZE")
    cal = {}
    for name, tab, full in (("fetch", fetch, copy_bytes / 1024.0), ("write", write, copy_bytes / 1024.0)):
        copies = [k for k in tab if "copy_kernel" in k]
        if len(copies) != 1:
            raise SystemExit("%s run: expected one copy_kernel calibration entry, found %r" % (name, copies))
        cal[name] = (full / tab[copies[0]][0], tab[copies[0]][0])
    names = [k for k in fetch if kernel in k and k in write]
    if len(names) != 1:
        raise SystemExit("kernel %r matches %r in both runs" % (kernel, names))
    kname = names[0]
    fk, nf = fetch[kname]
    wk, nw = write[kname]
    fb, wb = fk * 1024 * cal["fetch"][0] * per_pass, wk * 1024 * cal["write"][0] * per_pass
    with open(bench_json) as f:
        line = json.loads([ln for ln in f if ln.strip().startswith("{")][-1])
    if "config" in line and "kernel_config" in line["config"]:
        cfg = line["config"]["kernel_config"]
    else:
        cfg = [v for v in line.values() if isinstance(v, dict) and "config" in v][0]["config"]
    entry = {"kernel_hash": kernel_hash(), "config": cfg, "kernel": kname, "bytes_per_launch": int(round(fb + wb)),
             "fetch_bytes": int(round(fb)), "write_bytes": int(round(wb)), "fetch_kib_raw": fk, "write_kib_raw": wk,
             "dispatches": [nf, nw], "dispatches_per_pass": per_pass,
             "copy_calibration": {"bytes": copy_bytes, "fetch_kib_raw": cal["fetch"][1],
                                  "write_kib_raw": cal["write"][1], "fetch_scale": cal["fetch"][0],
                                  "write_scale": cal["write"][0]}}
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        t = {}
    t[key] = entry
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)
        f.write("\n")
    return entry


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--ingest-counters":
        ig = argparse.ArgumentParser(prog="bench.py --ingest-counters")
        ig.add_argument("key")
        ig.add_argument("kernel", help="a substring naming the kernel, e.g. 'wide_kernel<double'")
        ig.add_argument("fetch_dir")
        ig.add_argument("write_dir")
        ig.add_argument("bench_json", help="the JSON line the profiled bench command printed")
        ig.add_argument("--copy-bytes", type=int, default=1 << 30)
        ig.add_argument("--per-pass", type=int, default=1)
        a = ig.parse_args(sys.argv[2:])
        e = ingest_counters(a.key, a.kernel, a.fetch_dir, a.write_dir, a.bench_json, a.copy_bytes, a.per_pass)
        print(json.dumps({a.key: e}, indent=1))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="medium_f64")
    ap.add_argument("--retune", action="store_true",
                    help="autotune even when the tuning cache has this problem")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run the library's copy kernel over this many bytes (counter calibration)")
    ap.add_argument("--tune-sweeps", type=int, default=6,
                    help="sweeps per tuning measurement (even, so two-iteration passes have no remainder)")
    ap.add_argument("--check-iters", type=int, default=-1,
                    help="iterations compared with the oracle (default: all for small grids)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-ceilings", dest="ceilings", action="store_false",
                    help="skip the copy and 13-read/1-write bandwidth probes")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--batch-dtype", default="f32", choices=["f32", "f64"],
                    help="dtype of the batch64 workload when it runs alone (--profile --workload batch64)")
    ap.add_argument("--batch-mode", default="batched", choices=list(BATCH_MODES),
                    help="how the batch64 workload runs when it runs alone (--profile --workload batch64)")
    ap.add_argument("--config", default="",
                    help="run the main workload in this configuration instead of the tuned one, "
                         "as field=value pairs, e.g. tsteps=1,vec=2,bj=4,ichunk=2,nontemporal=1")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: no oracle, no extras")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sweep would shard as i-slabs with one halo plane exchanged per iteration)",
              file=sys.stderr)
        sys.exit(2)

    os.environ.setdefault("HJ_TUNE_CACHE", TUNE_CACHE)
    import torch
    from paper_2002_12115_amd import hj, inputs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    hj.load()
    w = inputs.WORKLOADS[args.workload]
    if w.batch:
        if not args.profile:
            raise SystemExit("the main line is a single solve; batch64 is reported under extra "
                             "(or run it alone with --profile)")
        r = run_batch(args, hj, inputs, args.batch_dtype, w.iters, args.batch_mode, args.retune)
        if args.copy_probe:          # the counters' calibration leg, as for single solves
            ms = hj.copy_probe(args.copy_probe)
            log("copy probe: %d bytes in %.3f ms" % (args.copy_probe, ms))
        print(json.dumps({"workload": w.name, "batch64_%s_%s" % (args.batch_dtype, args.batch_mode): r}), flush=True)
        return
    if args.profile:
        args.no_cpu_baseline = True
        args.no_extra = True
        args.check_iters = 0
        args.ceilings = False
    if args.check_iters < 0:
        args.check_iters = w.iters if interior(w.shape) * w.iters <= 2e9 else 20

    res, arrays = run_single(w, args, hj, inputs, args.steps, args.warmup, args.check_iters, True)
    if args.copy_probe:
        ms = hj.copy_probe(args.copy_probe)
        log("copy probe: %d bytes in %.3f ms = %.0f GB/s" % (args.copy_probe, ms, 2 * args.copy_probe / ms / 1e6))
    out = {
        "metric": METRIC,
        "value": res["glups"],
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.dtype,
        "data": "synthetic: seeded SplitMix64 fields (p~U[0,1), a,c~U[0.9,1.1), b~U[-0.05,0.05), "
                "wrk1~N(0,0.01), derived a3 and bnd) standing in for the Himeno benchmark",
        "config": {"workload": w.name, "grid": list(w.shape), "iters_per_step": w.iters,
                   "omega": w.omega, "seed": w.seed, "kernel_config": res["config"]},
        "roofline": res["roofline"],
        "step_ms_device": res["step_ms_device"],
        "accuracy": res["accuracy"],
        "upload_s": res["upload_s"],
        "pcie_inclusive_glups": res["pcie_inclusive_glups"],
    }
    checks = {"main": res.pop("check")}
    if not args.no_extra:
        extra = {}
        log("tuner comparison...")
        extra["tuner_exhaustive_vs_genetic"] = tuner_comparison(w, hj, inputs, arrays)
        log("transfer placement...")
        extra["transfer_placement"] = transfer_ablation(w, hj, arrays)
        for dtype, mode in (("f32", "batched"), ("f64", "batched"), ("f64", "per_instance"),
                            ("f64", "per_instance_default")):
            log("batch64", dtype, mode, "...")
            extra["batch64_%s_%s" % (dtype, mode)] = run_batch(args, hj, inputs, dtype, 100, mode, args.retune)
        plain = max(extra["batch64_f64_per_instance"]["glups"], extra["batch64_f64_per_instance_default"]["glups"])
        extra["batch64_f32_vs_f64_per_instance"] = extra["batch64_f32_batched"]["glups"] / plain
        log("batch64 results for the oracle...")
        checks["batch64"] = batch_results(hj, inputs, inputs.WORKLOADS["batch64"].iters)
        saved = args.ceilings
        args.ceilings = False
        # large_f32: the whole 500-iteration solve; huge_f32: 11 iterations
        # (five two-iteration passes and a one-iteration remainder), whole grid
        for name, steps, chk, keep in (("large_f32", 3, 500, True), ("huge_f32", 2, 11, False)):
            log(name, "...")
            r, _ = run_single(inputs.WORKLOADS[name], args, hj, inputs, steps, 1, chk, keep)
            checks[name] = r.pop("check")
            extra[name] = {k: r[k] for k in ("glups", "ms_per_step", "roofline", "config", "steps", "upload_s")}
        args.ceilings = saved
        out["extra"] = extra
    if not args.no_cpu_baseline:
        log("cpu baseline leg (oracle): timing and the error of every checked result...")
        out["cpu_baseline"], acc = cpu_baseline_leg(w, arrays, args.cpu_budget, checks, inputs)
        out["accuracy"] = acc.get("main")
        if "extra" in out:
            for name in ("large_f32", "huge_f32"):
                if name in out["extra"]:
                    out["extra"][name]["accuracy"] = acc.get(name)
            if "batch64" in acc:
                out["extra"]["batch64_accuracy"] = acc["batch64"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
