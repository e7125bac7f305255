"""Runtime behaviour around the sweep: device memory released after tuning,
the tuner's failure paths (forced from the host with HJ_TUNE_INJECT, so every
kernel still runs normally), and the graph cache's eviction under
asynchronous sweeps. Results are checked against the oracle or against the
same solve run another way."""
import csv

import numpy as np
import pytest

import oracle
from paper_2002_12115_amd import hj, inputs
from _hjtest import F32_FIELD_RTOL, field_err, oracle_run, say

pytestmark = pytest.mark.gpu

SHAPE = (40, 36, 140)
LEAK_SLACK = 32 << 20          # bytes of device memory a repeated call may move


def free_device_bytes():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_autotune_returns_its_device_memory():
    """A solve's tuning session frees its saved field and parity reference:
    free device memory after three more autotunes is what it was after the
    first (each leaked session would hold two 35 MB fields)."""
    shape = (130, 130, 258)
    f = inputs.fields(2002, shape)
    with hj.Solver("f64", shape, use_torch=False) as s:
        s.upload_all(f)
        say("leak: first autotune")
        s.autotune(n_sweeps=2, repeats=1)
        s.sweep(4, 0.8)
        base = free_device_bytes()
        for r in range(3):
            say("leak: autotune", r)
            s.autotune(n_sweeps=2, repeats=1)
        s.sweep(4, 0.8)
        after = free_device_bytes()
        assert abs(after - base) <= LEAK_SLACK, (base, after)
        p = s.download("p")
    assert np.array_equal(p, oracle.sweep(f, 8, 0.8, nthreads=oracle.max_threads())[0])


def test_batch_autotune_returns_its_device_memory():
    """A batch's tuning session frees its copy of the slab (here 4 instances,
    about 300 MB)."""
    shapes = [(66, 66, 130), (60, 50, 120), (66, 40, 100), (30, 66, 130)]
    arrays = [inputs.fields(11 + t, sh) for t, sh in enumerate(shapes)]
    with hj.Batch("f64", shapes) as b:
        for t, a in enumerate(arrays):
            b.upload_all(t, a)
        say("batch leak: first autotune")
        b.autotune(n_sweeps=2, repeats=1)
        b.sweep(4, 0.8)
        base = free_device_bytes()
        for r in range(2):
            say("batch leak: autotune", r)
            b.autotune(n_sweeps=2, repeats=1)
        b.sweep(4, 0.8)
        after = free_device_bytes()
        assert abs(after - base) <= LEAK_SLACK, (base, after)
        outs = [b.download(t) for t in range(len(shapes))]
    for a, p in zip(arrays, outs):
        assert np.array_equal(p, oracle.sweep(a, 8, 0.8)[0])


def read_log(path):
    rows = []
    with open(path) as f:
        for r in csv.reader(f):
            rows.append(dict(kernel=int(r[5]), bj=int(r[6]), vec=int(r[7]), ichunk=int(r[8]),
                             nontemporal=int(r[9]), xcd_remap=int(r[10]), persistent=int(r[11]), ms=float(r[12]),
                             verdict=r[13], tsteps=int(r[14]), reread=int(r[15])))
    return rows


@pytest.mark.parametrize("search", ["exhaustive", "genetic"])
def test_injected_launch_failures_are_never_chosen(search, tmp_path, monkeypatch):
    """Every two-iteration candidate is made to fail its launch: the search
    scores them as failed (the genetic search as 1000 s), logs them as such,
    installs a one-iteration configuration, and the solve still matches the
    oracle."""
    log = tmp_path / "tune.csv"
    monkeypatch.setenv("HJ_TUNE_LOG", str(log))
    monkeypatch.setenv("HJ_TUNE_INJECT", "launch:tsteps=2")
    f = inputs.fields(2002, SHAPE)
    with hj.Solver("f64", SHAPE) as s:
        s.upload_all(f)
        say("inject launch", search)
        if search == "exhaustive":
            best, ms = s.autotune(n_sweeps=2, repeats=1)
        else:
            best, ms, ev = s.autotune_ga(population=10, generations=10, seed=2002, n_sweeps=2, repeats=1)
            assert ev >= 1
        assert best.tsteps == 1 and s.config.tsteps == 1
        s.sweep(5, 0.8)
        p = s.download("p")
    rows = read_log(log)
    two = [r for r in rows if r["tsteps"] == 2]
    assert two, "the search measured no two-iteration candidate"
    assert all(r["verdict"] == "launch-failed" and r["ms"] == float("inf") for r in two)
    assert any(r["verdict"] == "ok" for r in rows)
    assert np.array_equal(p, oracle_run(SHAPE, 5)[0])


def test_injected_parity_failures_are_never_chosen(tmp_path, monkeypatch):
    """Candidates of the march kernel run but are scored as differing from the
    reference: the winner is a direct or flat configuration."""
    log = tmp_path / "tune.csv"
    monkeypatch.setenv("HJ_TUNE_LOG", str(log))
    monkeypatch.setenv("HJ_TUNE_INJECT", "parity:kernel=1")
    f = inputs.fields(2002, SHAPE)
    with hj.Solver("f32", SHAPE) as s:
        s.upload_all(f)
        say("inject parity")
        best, _ = s.autotune(n_sweeps=2, repeats=1)
        assert best.kernel in (hj.KERNEL_DIRECT, hj.KERNEL_FLAT)
        s.sweep(4, 0.8)
        p = s.download("p")
    rows = read_log(log)
    assert all(r["verdict"] == "parity-failed" for r in rows if r["kernel"] == 1)
    assert field_err(p, oracle_run(SHAPE, 4)[0]) <= F32_FIELD_RTOL


@pytest.mark.parametrize("search", ["exhaustive", "genetic"])
def test_every_candidate_failing_leaves_the_solve_unchanged(search, monkeypatch):
    """When no candidate passes, tuning returns HJ_ERR_TUNE (for the genetic
    search: every gene scored 1000 s), and the field and configuration are
    those from before the call."""
    monkeypatch.setenv("HJ_TUNE_INJECT", "launch:kernel=0;launch:kernel=1;launch:kernel=2")
    f = inputs.fields(5, SHAPE)
    with hj.Solver("f64", SHAPE) as s:
        s.upload_all(f)
        s.sweep(3, 0.8)
        before, cfg0 = s.download("p"), s.config.as_dict()
        say("inject all", search)
        with pytest.raises(hj.HJError) as e:
            if search == "exhaustive":
                s.autotune(n_sweeps=2, repeats=1)
            else:
                s.autotune_ga(population=6, generations=4, seed=1, n_sweeps=2, repeats=1)
        assert e.value.status == -8
        assert np.array_equal(s.download("p"), before)
        assert s.config.as_dict() == cfg0
        s.sweep(2, 0.8)
        p = s.download("p")
    assert np.array_equal(p, oracle_run(SHAPE, 5, seed=5)[0])


def test_batch_injected_failures_are_never_chosen(monkeypatch):
    monkeypatch.setenv("HJ_TUNE_INJECT", "launch:tsteps=2;parity:kernel=2")
    shapes = [(20, 30, 70), (35, 17, 40), (18, 18, 130)]
    arrays = [inputs.fields(20 + t, sh) for t, sh in enumerate(shapes)]
    with hj.Batch("f64", shapes) as b:
        for t, a in enumerate(arrays):
            b.upload_all(t, a)
        say("batch inject")
        best, _ = b.autotune(n_sweeps=2, repeats=1)
        assert best.tsteps == 1 and best.kernel == hj.KERNEL_MARCH
        best, _, _ = b.autotune_ga(population=8, generations=6, seed=3, n_sweeps=2, repeats=1)
        assert best.tsteps == 1 and best.kernel == hj.KERNEL_MARCH
        b.sweep(5, 0.8)
        outs = [b.download(t) for t in range(len(shapes))]
    for a, p in zip(arrays, outs):
        assert np.array_equal(p, oracle.sweep(a, 5, 0.8)[0])


def test_async_sweeps_cycle_more_graphs_than_the_cache_holds():
    """Ten distinct iteration counts enqueued back to back with
    hj_sweep_async (the cache keeps eight graphs, so executables are evicted
    while earlier ones may still be queued): the field equals one synchronous
    solve of the total count, bit for bit."""
    shape = (34, 34, 66)
    f = inputs.fields(9, shape)
    counts = list(range(1, 11))
    with hj.Solver("f64", shape) as s:
        s.upload_all(f)
        say("graph cache cycle", counts)
        for n in counts:
            s.sweep_async(n, 0.8)
        s.sync()
        p_async = s.download("p")
    with hj.Solver("f64", shape) as s:
        s.upload_all(f)
        s.sweep(sum(counts), 0.8)
        p_sync = s.download("p")
    assert np.array_equal(p_async, p_sync)
    assert np.array_equal(p_sync, oracle.sweep(f, sum(counts), 0.8, nthreads=4)[0])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_exhaustive_search_measures_every_gene(dtype, tmp_path, monkeypatch):
    """Both searches cover one space: every configuration an 11-bit gene names
    for this grid (hj_gene_config) is among those the exhaustive search
    measures (its tuning log)."""
    import ctypes
    log = tmp_path / "tune.csv"
    monkeypatch.setenv("HJ_TUNE_LOG", str(log))
    lib = hj.load()
    lib.hj_gene_config.argtypes = [ctypes.c_int] * 5 + [ctypes.c_uint, ctypes.POINTER(hj.Config)]
    code = hj.F64 if dtype == "f64" else hj.F32
    keys = ("kernel", "bj", "vec", "ichunk", "nontemporal", "xcd_remap", "persistent", "tsteps", "reread")
    genes = set()
    for g in range(2 ** 11):
        c = hj.Config()
        assert lib.hj_gene_config(code, *SHAPE, 0, g, ctypes.byref(c)) == 0
        genes.add(tuple(c.as_dict()[k] for k in keys))
    f = inputs.fields(2002, SHAPE)
    with hj.Solver(dtype, SHAPE) as s:
        s.upload_all(f)
        say("exhaustive log", dtype)
        s.autotune(n_sweeps=2, repeats=1)
    measured = {tuple(r[k] for k in keys) for r in read_log(log)}
    missing = genes - measured
    assert not missing, sorted(missing)[:5]
