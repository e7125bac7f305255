"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

FP64 fields must be bitwise equal (same evaluation order, no contraction),
FP64 gosa within 1e-10 relative, FP32 fields within 1e-5 relative of the
FP64 oracle. Shapes cover several tiles in every direction, ragged tails in
k, j and i, single-cell interiors and random bnd masks.
"""
import numpy as np
import pytest

import oracle
from paper_2002_12115_amd import hj, inputs
from _hjtest import (F32_FIELD_RTOL, F64_GOSA_RTOL, cfg, cfg_id, f32_configs, f64_configs,
                     field_err, gosa_err, gpu_run, oracle_run, say)

pytestmark = pytest.mark.gpu

SHAPES = [(3, 3, 3), (3, 4, 5), (5, 3, 4), (34, 34, 66), (19, 23, 37), (7, 9, 130),
          (6, 5, 259), (40, 17, 67), (4, 70, 3)]

_oracle_cache = {}


def oracle_cached(shape, n_iter, seed=2002, bnd_mode=0):
    key = (shape, n_iter, seed, bnd_mode)
    if key not in _oracle_cache:
        _oracle_cache[key] = oracle_run(shape, n_iter, seed=seed, bnd_mode=bnd_mode)
    return _oracle_cache[key]


@pytest.mark.parametrize("c", f64_configs(), ids=cfg_id)
def test_f64_bitwise_all_shapes(c):
    for shape in SHAPES:
        for bnd_mode in (0, 1):
            n = 7
            say("f64", cfg_id(c), shape, "bnd_mode", bnd_mode)
            r = gpu_run(shape, "f64", n, cfg=c, bnd_mode=bnd_mode)
            if r is None:
                continue                       # this flat width does not fit the grid
            p, hist, _ = r
            pref, href = oracle_cached(shape, n, bnd_mode=bnd_mode)
            assert np.array_equal(p, pref), (shape, bnd_mode, field_err(p, pref))
            assert gosa_err(hist, href) <= F64_GOSA_RTOL, (shape, hist, href)


@pytest.mark.parametrize("c", f32_configs(), ids=cfg_id)
def test_f32_within_tolerance_all_shapes(c):
    for shape in SHAPES:
        n = 7
        say("f32", cfg_id(c), shape)
        r = gpu_run(shape, "f32", n, cfg=c)
        if r is None:
            continue
        p, hist, _ = r
        pref, href = oracle_cached(shape, n)
        assert field_err(p, pref) <= F32_FIELD_RTOL, (shape, field_err(p, pref))
        assert np.all(np.isfinite(hist)) and gosa_err(hist, href) < 1e-3


def test_f32_configs_agree_bitwise():
    shape = (19, 23, 137)
    f = inputs.fields(1, shape)
    ref = None
    for c in f32_configs():
        say("f32 agree", cfg_id(c))
        r = gpu_run(shape, "f32", 5, cfg=c, arrays=f)
        if r is None:
            continue
        p, hist, _ = r
        if ref is None:
            ref = (p, hist)
        else:
            assert np.array_equal(p, ref[0]), cfg_id(c)
            assert gosa_err(hist, ref[1]) < 1e-12


def test_small_f64_workload_50_iterations():
    w = inputs.WORKLOADS["small_f64"]
    say("small_f64 default config")
    p, hist, _ = gpu_run(w.shape, "f64", w.iters, omega=w.omega, seed=w.seed)
    pref, href = oracle_run(w.shape, w.iters, omega=w.omega, seed=w.seed)
    assert np.array_equal(p, pref)
    assert gosa_err(hist, href) <= F64_GOSA_RTOL
    assert np.all(np.diff(hist) < 0)   # monotone decrease on this operator


@pytest.mark.parametrize("seed", [2002, 1, 7])
def test_seeds_and_torch_vs_library_memory(seed):
    shape = (21, 18, 70)
    pref, href = oracle_run(shape, 9, seed=seed)
    for use_torch in (True, False):
        say("seed", seed, "use_torch", use_torch)
        p, hist, _ = gpu_run(shape, "f64", 9, seed=seed, use_torch=use_torch)
        assert np.array_equal(p, pref)
        assert gosa_err(hist, href) <= F64_GOSA_RTOL


def test_residual_matches_oracle_and_history():
    shape = (17, 20, 45)
    f = inputs.fields(7, shape)
    for dtype in ("f64", "f32"):
        say("residual", dtype)
        with hj.Solver(dtype, shape) as s:
            s.upload_all(f)
            g0 = s.residual()
            ref0 = oracle.residual(f)
            tol = 1e-12 if dtype == "f64" else 1e-4
            assert abs(g0 - ref0) <= tol * ref0
            s.sweep(4, 0.8)
            assert s.gosa_history[0] == pytest.approx(g0, rel=1e-12)
            g4 = s.residual()
            p4, _, _ = oracle.sweep(f, 4, 0.8)
            ref4 = oracle.residual(dict(f, p=p4))
            assert abs(g4 - ref4) <= tol * ref4
            # one more sweep: its history entry is this residual
            s.sweep(1, 0.8)
            assert s.gosa_history[0] == pytest.approx(g4, rel=1e-12)


GRAPH_CONFIGS = [None,
                 dict(kernel=1, bj=4, vec=2, ichunk=4, nontemporal=1, xcd_remap=0, tsteps=1, reread=0),
                 dict(kernel=1, bj=8, vec=2, ichunk=7, nontemporal=0, xcd_remap=1, tsteps=2, reread=0),
                 dict(kernel=1, bj=14, vec=4, ichunk=9, nontemporal=0, xcd_remap=1, tsteps=2, reread=1)]


@pytest.mark.parametrize("extra", GRAPH_CONFIGS, ids=["default", "one", "wide", "narrow"])
def test_graph_replays_match_eager(extra):
    """Replays of captured loops (two cached graphs alternate when a call has
    an odd number of passes) equal eager launches, with host work between."""
    shape = (30, 33, 100)
    f = inputs.fields(2002, shape)
    for dtype in ("f64", "f32"):
        res = {}
        for graph in (0, 1):
            say("graph", graph, dtype, extra)
            with hj.Solver(dtype, shape) as s:
                if extra:
                    s.set(**extra)
                s.set(use_graph=graph)
                s.upload_all(f)
                hs, ps = [], []
                for rep in range(4):         # replays with eager host work between them
                    s.sweep(6, 0.8)
                    hs.append(s.gosa_history.copy())
                    ps.append(s.download("p"))
                    _ = s.residual()
                res[graph] = (hs, ps)
        for a, b in zip(res[0][0], res[1][0]):
            assert np.array_equal(a, b)
        for a, b in zip(res[0][1], res[1][1]):
            assert np.array_equal(a, b)


def test_sweep_in_pieces_equals_one_call():
    shape = (12, 13, 70)
    f = inputs.fields(1, shape)
    with hj.Solver("f64", shape) as s:
        s.upload_all(f)
        h = []
        for n in (1, 2, 3, 5):
            say("pieces", n)
            s.sweep(n, 0.8)
            h.extend(s.gosa_history)
        p_pieces = s.download("p")
        assert np.array_equal(s.download("wrk2"), p_pieces)
    pref, href = oracle_run(shape, 11, seed=1)
    assert np.array_equal(p_pieces, pref)
    assert gosa_err(h, href) <= F64_GOSA_RTOL


def test_default_is_the_two_iteration_kernel():
    """A new solve with no tuning-cache entry starts on the two-iteration
    kernel (64-cell rows, 8 rows per tile) and, with odd and even counts,
    gives the oracle's field."""
    shape = (66, 40, 130)
    f = inputs.fields(5, shape)
    with hj.Solver("f64", shape) as s:
        c = s.config
        assert (c.kernel, c.bj, c.vec, c.tsteps, c.reread, c.xcd_remap) == (1, 8, 2, 2, 0, 1)
        assert 1 <= c.ichunk <= shape[0] - 2
        s.upload_all(f)
        say("default config", c)
        s.sweep(5, 0.8)
        h = list(s.gosa_history)
        s.sweep(4, 0.8)
        h.extend(s.gosa_history)
        p = s.download("p")
    pref, href = oracle_run(shape, 9, seed=5)
    assert np.array_equal(p, pref)
    assert gosa_err(h, href) <= F64_GOSA_RTOL


def test_run_to_run_deterministic():
    shape = (50, 40, 300)
    f = inputs.fields(7, shape)
    outs = []
    for _ in range(3):
        say("determinism")
        p, hist, _ = gpu_run(shape, "f64", 5, arrays=f)
        outs.append((p, hist))
    for p, hist in outs[1:]:
        assert np.array_equal(p, outs[0][0])
        assert np.array_equal(hist, outs[0][1])   # fixed-order reduction: same bits


@pytest.mark.parametrize("dtype,c", [
    ("f64", dict(bj=4, vec=2, ichunk=1)), ("f64", dict(bj=8, vec=1, ichunk=2)),
    ("f32", dict(bj=8, vec=2, ichunk=1)), ("f32", dict(bj=14, vec=4, ichunk=3))],
    ids=["f64-wide", "f64-fused", "f32-wide", "f32-narrow"])
def test_remap_windows_with_a_partial_last_window(dtype, c):
    """Single-grid two-iteration launches deal tiles to XCDs in windows of
    the workgroups resident at once; a grid of several windows and a
    partial last one (thousands of tiles, not a multiple of the window)
    still computes every tile exactly once."""
    shape = (41, 131, 133)          # 39 planes in chunks of 1-3; ragged j and k tiles
    n = 4
    conf = cfg(nontemporal=0, xcd_remap=1, tsteps=2, reread=0, **c)
    say("remap windows", dtype, shape, cfg_id(conf))
    p, hist, _ = gpu_run(shape, dtype, n, cfg=conf)
    pref, href = oracle_cached(shape, n)
    if dtype == "f64":
        assert np.array_equal(p, pref)
        assert gosa_err(hist, href) <= F64_GOSA_RTOL
    else:
        assert field_err(p, pref) <= F32_FIELD_RTOL


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_coefficient_upload_between_sweeps(dtype):
    """Coefficients uploaded between sweeps reach every cell the two-iteration
    tiles read, the columns on the k tile edges included (the upload refreshes
    the compact copy of those that the 64-cell-row kernel reads)."""
    shape = (12, 19, 140)   # three 64-cell k tiles, the last one ragged
    f, g = inputs.fields(2002, shape), inputs.fields(7, shape, bnd_mode=1)
    with hj.Solver(dtype, shape) as s:
        s.config = cfg(bj=8, vec=2, ichunk=5, nontemporal=0, xcd_remap=1, tsteps=2)
        say("coefficient upload", dtype, shape, cfg_id(s.config))
        s.upload_all(f)
        s.sweep(2, 0.8)
        for n in inputs.INPUTS[1:]:
            s.upload(n, g[n])
        s.sweep(4, 0.8)
        p, hist = s.download("p"), s.gosa_history.copy()
    p1, w1, _ = oracle.sweep(f, 2, 0.8)
    pref, _, href = oracle.sweep(dict(g, p=p1, wrk2=w1), 4, 0.8)
    if dtype == "f64":
        assert np.array_equal(p, pref)
        assert gosa_err(hist, href) <= F64_GOSA_RTOL
    else:
        assert field_err(p, pref) <= F32_FIELD_RTOL


def test_download_coefficients_round_trip():
    shape = (6, 7, 9)
    f = inputs.fields(2002, shape)
    with hj.Solver("f32", shape) as s:
        s.upload_all(f)
        for n in inputs.INPUTS:
            assert np.array_equal(s.download(n), f[n].astype(np.float32)), n


def test_error_paths():
    shape = (5, 6, 7)
    f = inputs.fields(1, shape)
    with hj.Solver("f64", shape) as s:
        with pytest.raises(hj.HJError) as e:
            s.sweep(1, 0.8)
        assert e.value.status == -6            # not every input uploaded
        with pytest.raises(hj.HJError) as e:
            s.upload("wrk2", f["p"])
        assert e.value.status == -1
        with pytest.raises(hj.HJError) as e:
            s.config = cfg(bj=3)
        assert e.value.status == -1
        with pytest.raises(hj.HJError) as e:
            s.config = cfg(vec=4)              # vec 4 is FP32 only
        assert e.value.status == -1
        s.upload_all(f)
        with pytest.raises(hj.HJError):
            s.sweep(-1, 0.8)
        p0 = s.download("p")
        s.sweep(0, 0.8)                        # no-op
        assert np.array_equal(s.download("p"), p0)
        h = s._h
    lib = hj.load()
    assert lib.hj_sweep(h, 1, 0.8, None, None) == -7     # destroyed handle


def test_device_memory_is_not_a_host_array():
    """A device pointer passed where the ABI takes a host array is refused
    with HJ_ERR_ARG, not copied through the host."""
    import torch
    shape = (5, 6, 7)
    dev = torch.zeros(int(np.prod(shape)), dtype=torch.float64, device="cuda")
    lib = hj.load()
    with hj.Solver("f64", shape) as s:
        assert lib.hj_upload(s._h, 1, dev.data_ptr()) == -1
        assert lib.hj_upload_f64(s._h, 1, dev.data_ptr()) == -1
        assert lib.hj_download(s._h, 0, dev.data_ptr()) == -1
        assert lib.hj_snapshot(s._h, dev.data_ptr()) == -1
        assert b"device memory" in lib.hj_last_error()
    with hj.Batch("f64", [shape, (4, 4, 4)]) as b:
        assert lib.hj_batch_upload(b._h, 0, 1, dev.data_ptr()) == -1
        assert lib.hj_batch_download(b._h, 0, 0, dev.data_ptr()) == -1


def test_out_of_memory_is_reported_and_recoverable():
    """A grid larger than the device (about 3 TB of arrays) fails with
    HJ_ERR_OOM, and later handles work normally (the error is not kept)."""
    with pytest.raises(hj.HJError) as e:
        hj.Solver("f64", (3000, 3000, 3000), use_torch=False)
    assert e.value.status == -4
    with pytest.raises(hj.HJError) as e:
        hj.Batch("f64", [(20, 20, 20), (3000, 3000, 3000)])
    assert e.value.status == -4
    shape = (12, 13, 70)
    f = inputs.fields(4, shape)
    with hj.Solver("f64", shape, use_torch=False) as s:
        s.upload_all(f)
        s.sweep(3, 0.8)
        assert np.array_equal(s.download("p"), oracle.sweep(f, 3, 0.8)[0])


def test_autotune_restores_state_and_keeps_parity():
    shape = (40, 36, 140)
    f = inputs.fields(2002, shape)
    for dtype in ("f64", "f32"):
        with hj.Solver(dtype, shape) as s:
            s.upload_all(f)
            s.sweep(3, 0.8)
            before = s.download("p")
            say("autotune", dtype)
            best, ms = s.autotune(n_sweeps=2, repeats=1)
            assert ms > 0
            assert np.array_equal(s.download("p"), before)
            s.sweep(4, 0.8)
            p = s.download("p")
        pref, _ = oracle_run(shape, 7, seed=2002)
        if dtype == "f64":
            assert np.array_equal(p, pref), best
        else:
            assert field_err(p, pref) <= F32_FIELD_RTOL


def test_tuning_cache_round_trip(tmp_path, monkeypatch):
    """The autotune winner is recorded in HJ_TUNE_CACHE and a new handle for
    the same problem starts from it; malformed lines, other shapes and
    unsupported configurations in the file are ignored."""
    path = tmp_path / "cache.txt"
    shape = (40, 36, 140)
    path.write_text("not a cache line\n"
                    "solve gfx950 f64 9x9x9 1 4 2 2 1 0 0 0.1 1 0\n"
                    "solve gfx950 f64 40x36x140 1 3 7 2 1 0 0 0.1 1 0\n")   # bj 3, vec 7: unsupported
    monkeypatch.setenv("HJ_TUNE_CACHE", str(path))
    f = inputs.fields(3, shape)
    with hj.Solver("f64", shape) as s:
        assert s.config.bj != 3                 # the unsupported line was not applied
        s.upload_all(f)
        say("cache round trip")
        best, _ = s.autotune(n_sweeps=2, repeats=1)
    lines = [ln for ln in path.read_text().splitlines() if " 40x36x140 " in ln]
    assert len(lines) == 1                      # the winner replaced the old line for this shape
    assert "not a cache line" in path.read_text() and " 9x9x9 " in path.read_text()
    with hj.Solver("f64", shape) as s:
        assert s.config.as_dict() == dict(best.as_dict(), use_graph=1)
        s.upload_all(f)
        s.sweep(3, 0.8)
        assert np.array_equal(s.download("p"), oracle.sweep(f, 3, 0.8)[0])


def test_genetic_search_restores_state_and_keeps_parity():
    shape = (40, 36, 140)
    f = inputs.fields(7, shape)
    for dtype in ("f64", "f32"):
        with hj.Solver(dtype, shape) as s:
            s.upload_all(f)
            s.sweep(2, 0.8)
            before = s.download("p")
            say("genetic search", dtype)
            best, ms, evals = s.autotune_ga(population=10, generations=10, seed=2002, n_sweeps=2, repeats=1)
            assert ms > 0 and 1 <= evals <= 100
            assert np.array_equal(s.download("p"), before)
            assert s.config.as_dict() == dict(best.as_dict(), use_graph=1)
            s.sweep(3, 0.8)
            p = s.download("p")
        pref, _ = oracle_run(shape, 5, seed=7)
        if dtype == "f64":
            assert np.array_equal(p, pref), best
        else:
            assert field_err(p, pref) <= F32_FIELD_RTOL


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_transfer_placements_give_the_same_solve(dtype):
    """Every host-transfer placement gives the resident solve's field bit for
    bit. gosa agrees to rounding: a placement that sweeps one iteration per
    call runs those on the one-iteration kernel, whose per-tile partials are
    summed in another order than the two-iteration kernel's."""
    from paper_2002_12115_amd import transfer
    shape = (34, 34, 66)
    f = inputs.fields(2002, shape)
    res = {}
    for policy in transfer.POLICIES:
        say("transfer", policy, dtype)
        with hj.Solver(dtype, shape) as s:
            res[policy] = transfer.run(s, f, policy, 12, 0.8, k=5)
    ref = res["resident"]
    for policy, r in res.items():
        assert np.array_equal(r["field"], ref["field"]), policy
        assert gosa_err(r["gosa_history"], ref["gosa_history"]) <= 1e-13, policy
    assert res["p_every_iter"]["d2h_bytes"] == 12 * f["p"].size * (8 if dtype == "f64" else 4)
    if dtype == "f64":
        pref, _ = oracle_run(shape, 12)
        assert np.array_equal(ref["field"], pref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pinned_host_buffers_match_pageable(dtype):
    """Uploads from and downloads into pinned host memory (copied directly,
    without the library's staging buffers) give the same arrays, the same
    solve and the same transfer placements as pageable arrays."""
    from paper_2002_12115_amd import transfer
    shape = (21, 34, 70)
    f = inputs.fields(9, shape)
    say("pinned buffers", dtype)
    with hj.Solver(dtype, shape) as s:
        pin = {n: transfer.pinned_like(f[n], s.np_dtype) for n in inputs.INPUTS}
        s.upload_all(pin)
        for n in inputs.INPUTS:
            out = s.download(n, out=transfer.pinned_like(np.zeros(shape), s.np_dtype))
            assert np.array_equal(out, f[n].astype(s.np_dtype)), n
        s.sweep(5, 0.8)
        p_pin = s.download("p", out=transfer.pinned_like(np.zeros(shape), s.np_dtype))
        assert np.array_equal(p_pin, s.download("p"))
        with pytest.raises(ValueError):
            s.download("p", out=np.zeros((3, 3, 3), dtype=s.np_dtype))
    with hj.Solver(dtype, shape) as s:
        s.upload_all(f)
        s.sweep(5, 0.8)
        assert np.array_equal(s.download("p"), p_pin)
    runs = {}
    for pinned in (False, True):
        with hj.Solver(dtype, shape) as s:
            runs[pinned] = transfer.run(s, f, "p_every_iter", 6, 0.8, pinned=pinned)
    assert np.array_equal(runs[True]["field"], runs[False]["field"])
    assert np.array_equal(runs[True]["gosa_history"], runs[False]["gosa_history"])
    if dtype == "f64":
        assert np.array_equal(runs[True]["field"], oracle.sweep(f, 6, 0.8)[0])


def test_snapshots_equal_the_field_when_taken():
    """hj_snapshot sends the field as it stands when called, while later
    sweeps run; pageable targets work too, and destroying a handle with a
    snapshot in flight waits for it. The observe placements (synchronous and
    overlapped) give the resident field."""
    from paper_2002_12115_amd import transfer
    shape = (30, 33, 100)
    f = inputs.fields(11, shape)
    say("snapshots")
    snaps, done = [], 0
    with hj.Solver("f64", shape) as s:
        s.upload_all(f)
        for n in (1, 2, 3):
            s.sweep(n, 0.8)
            done += n
            snap = transfer.pinned_like(np.zeros(shape))
            s.snapshot(snap)
            s.sweep(2, 0.8)                      # runs while the snapshot is sent
            snaps.append((done, snap))
            done += 2
            s.snapshot_wait()
        final = s.download()
        pageable = np.zeros(shape)
        s.snapshot(pageable)
        s.snapshot_wait()
        assert np.array_equal(pageable, final)
        with pytest.raises(ValueError):
            s.snapshot(np.zeros((3, 3, 3)))
        s.snapshot(transfer.pinned_like(np.zeros(shape)))   # still in flight at destroy
    for n_done, snap in snaps:
        assert np.array_equal(snap, oracle.sweep(f, n_done, 0.8)[0]), n_done
    assert np.array_equal(final, oracle.sweep(f, done, 0.8)[0])
    res = {}
    for policy in ("resident", "observe_every_k", "observe_every_k_async"):
        with hj.Solver("f64", shape) as s:
            res[policy] = transfer.run(s, f, policy, 13, 0.8, k=4, pinned=True)
    for policy in ("observe_every_k", "observe_every_k_async"):
        assert np.array_equal(res[policy]["field"], res["resident"]["field"]), policy
        assert res[policy]["d2h_bytes"] == 4 * f["p"].size * 8


def test_f32_snapshot_equals_download():
    from paper_2002_12115_amd import transfer
    shape = (17, 40, 130)
    f = inputs.fields(12, shape)
    say("f32 snapshot")
    with hj.Solver("f32", shape) as s:
        s.upload_all(f)
        s.sweep(3, 0.8)
        snap = transfer.pinned_like(np.zeros(shape), np.float32)
        s.snapshot(snap)
        want = s.download()
        s.sweep(3, 0.8)
        s.snapshot_wait()
        assert np.array_equal(snap, want)
        assert field_err(snap, oracle.sweep(f, 3, 0.8)[0]) <= F32_FIELD_RTOL


def test_flat_fit_is_enforced():
    """A flat run too wide for the grid is refused, never launched."""
    # FP64 staged plane: 1280 values. nz = 300: runs of 128 cells touch 4 rows
    # (1200 values), runs of 512 touch 5 (1500).
    shape = (5, 9, 300)
    with hj.Solver("f64", shape) as s:
        with pytest.raises(hj.HJError) as e:
            s.config = cfg(kernel=hj.KERNEL_FLAT, bj=8, vec=1, ichunk=2)
        assert e.value.status == -1
        s.config = cfg(kernel=hj.KERNEL_FLAT, bj=2, vec=1, ichunk=2)     # 2 waves fit
        f = inputs.fields(3, shape)
        s.upload_all(f)
        s.sweep(3, 0.8)
        assert np.array_equal(s.download("p"), oracle.sweep(f, 3, 0.8)[0])
