"""GPU parity of the batched path: every instance of a batch (one launch per
iteration, or per two iterations) equals its own single solve and the oracle."""
import numpy as np
import pytest

import oracle
from paper_2002_12115_amd import hj, inputs
from _hjtest import F32_FIELD_RTOL, F64_GOSA_RTOL, field_err, gosa_err, say

pytestmark = pytest.mark.gpu


def small_batch(seed=2002, n=7):
    shapes, seeds = inputs.batch_shapes(seed, n, lo_xy=3, hi_xy=21, lo_z=3, hi_z=80)
    shapes[0] = (3, 3, 3)          # a single-cell interior among the others
    return shapes, seeds


def batch_configs(dtype):
    out = []
    for nw in (2, 4, 8):
        for ich, nt, per in ((1, 1, 0), (5, 0, 1)):
            out.append(hj.Config.make(kernel=2, bj=nw, vec=1, ichunk=ich, nontemporal=nt, use_graph=1, xcd_remap=0,
                                      persistent=per))
    vmax = 2 if dtype == "f64" else 4
    for bj in (1, 2, 4, 8):
        v = 1
        while v <= vmax:
            for ich, nt, per in ((1, 1, 0), (5, 0, 1), (64, 1, 1)):
                out.append(hj.Config.make(kernel=1, bj=bj, vec=v, ichunk=ich, nontemporal=nt,
                                          use_graph=1, xcd_remap=0, persistent=per))
            v *= 2
    for bj in (2, 4, 6, 8, 14):                 # two iterations per pass
        for ich, rr, rm in ((1, 0, 0), (5, 1, 1), (64, 0, 1)):
            out.append(hj.Config.make(kernel=1, bj=bj, vec=1, ichunk=ich, nontemporal=0, use_graph=1,
                                      xcd_remap=rm, persistent=0, tsteps=2, reread=rr))
    for bj in (2, 6, 12):                       # two iterations, 64-cell rows with a halo wave
        for ich, rr, rm in ((1, 1, 1), (7, 0, 0), (64, 1, 0)):
            out.append(hj.Config.make(kernel=1, bj=bj, vec=2, ichunk=ich, nontemporal=0, use_graph=1,
                                      xcd_remap=rm, persistent=0, tsteps=2, reread=rr))
    for bj in (6, 14, 22, 30):                  # two iterations, two 30-cell rows per wave
        for ich, rr, rm in ((1, 0, 1), (9, 1, 0)):
            out.append(hj.Config.make(kernel=1, bj=bj, vec=4, ichunk=ich, nontemporal=0, use_graph=1,
                                      xcd_remap=rm, persistent=0, tsteps=2, reread=rr))
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_matches_oracle_every_config(dtype):
    shapes, seeds = small_batch()
    arrays = [inputs.fields(sd, sh) for sh, sd in zip(shapes, seeds)]
    refs = [oracle.sweep(a, 6, 0.8, nthreads=4) for a in arrays]
    for c in batch_configs(dtype):
        say("batch", dtype, c)
        with hj.Batch(dtype, shapes) as b:
            b.config = c
            for t, a in enumerate(arrays):
                b.upload_all(t, a)
            b.sweep(6, 0.8)
            hist = b.gosa_history
            for t in range(len(shapes)):
                p = b.download(t, "p")
                pref, _, href = refs[t]
                if dtype == "f64":
                    assert np.array_equal(p, pref), (t, shapes[t])
                    assert gosa_err(hist[:, t], href) <= F64_GOSA_RTOL
                else:
                    assert field_err(p, pref) <= F32_FIELD_RTOL, (t, shapes[t])


def test_batch_equals_single_solves_bitwise():
    shapes, seeds = inputs.batch_shapes(7, 5, lo_xy=10, hi_xy=40, lo_z=20, hi_z=150)
    arrays = [inputs.fields(sd, sh) for sh, sd in zip(shapes, seeds)]
    for dtype in ("f64", "f32"):
        say("batch vs single", dtype)
        with hj.Batch(dtype, shapes) as b:
            for t, a in enumerate(arrays):
                b.upload_all(t, a)
            b.sweep(9, 0.8)
            hist = b.gosa_history.copy()
            res = b.residual()
            outs = [b.download(t) for t in range(len(shapes))]
        for t, a in enumerate(arrays):
            with hj.Solver(dtype, shapes[t]) as s:
                s.upload_all(a)
                s.sweep(9, 0.8)
                assert np.array_equal(s.download(), outs[t])
                assert gosa_err(hist[:, t], s.gosa_history) < 1e-12
                assert res[t] == pytest.approx(s.residual(), rel=1e-12)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dispatch_order_leaves_results_bitwise_unchanged(dtype):
    """A two-iteration batch dispatches its tiles longest-first without XCD
    renumbering and instance by instance with it; each tile's gosa partials
    go to its instance-major place, so fields and gosa histories are bitwise
    the same in both orders (and over chunk lengths that leave remainders)."""
    shapes, seeds = inputs.batch_shapes(11, 9, lo_xy=5, hi_xy=70, lo_z=10, hi_z=140)
    arrays = [inputs.fields(sd, sh) for sh, sd in zip(shapes, seeds)]
    outs = []
    for rm in (1, 0):
        c = hj.Config.make(kernel=1, bj=6, vec=4 if dtype == "f64" else 2, ichunk=9, nontemporal=0, use_graph=1,
                           xcd_remap=rm, persistent=0, tsteps=2, reread=0)
        say("dispatch order", dtype, "xcd_remap", rm)
        with hj.Batch(dtype, shapes) as b:
            b.config = c
            for t, a in enumerate(arrays):
                b.upload_all(t, a)
            b.sweep(8, 0.8)
            outs.append(([b.download(t) for t in range(len(shapes))], b.gosa_history.copy()))
    (p1, h1), (p0, h0) = outs
    for t in range(len(shapes)):
        assert np.array_equal(p1[t], p0[t]), t
    assert np.array_equal(h1, h0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_iteration_batch_odd_counts_and_residual(dtype):
    """Odd iteration counts end on a one-iteration pass; the residual and the
    gosa history continue across calls, as for single solves."""
    shapes, seeds = inputs.batch_shapes(11, 6, lo_xy=5, hi_xy=40, lo_z=5, hi_z=150)
    arrays = [inputs.fields(sd, sh) for sh, sd in zip(shapes, seeds)]
    c = hj.Config.make(kernel=1, bj=6, vec=2, ichunk=7, nontemporal=0, use_graph=1, xcd_remap=1, persistent=0,
                       tsteps=2, reread=0)
    say("two-iteration batch, odd counts", dtype)
    with hj.Batch(dtype, shapes) as b:
        b.config = c
        assert b.config.tsteps == 2 and b.config.xcd_remap == 1
        for t, a in enumerate(arrays):
            b.upload_all(t, a)
        b.sweep(3, 0.8)
        h1 = b.gosa_history.copy()
        b.sweep(4, 0.8)
        h2 = b.gosa_history.copy()
        res = b.residual()
        outs = [b.download(t) for t in range(len(shapes))]
    for t, a in enumerate(arrays):
        pref, _, href = oracle.sweep(a, 7, 0.8)
        if dtype == "f64":
            assert np.array_equal(outs[t], pref), (t, shapes[t])
            assert gosa_err(np.concatenate([h1[:, t], h2[:, t]]), href) <= F64_GOSA_RTOL
            assert res[t] == pytest.approx(oracle.residual(dict(a, p=pref)), rel=1e-10)
        else:
            assert field_err(outs[t], pref) <= F32_FIELD_RTOL, (t, shapes[t])


@pytest.mark.parametrize("tsteps", [1, 2])
def test_batch_graph_replays_match_eager(tsteps):
    shapes, seeds = inputs.batch_shapes(5, 5, lo_xy=5, hi_xy=30, lo_z=5, hi_z=100)
    arrays = [inputs.fields(sd, sh) for sh, sd in zip(shapes, seeds)]
    extra = dict(bj=6, vec=1, ichunk=5, xcd_remap=1, tsteps=2) if tsteps == 2 else dict(bj=4, vec=1, ichunk=4)
    res = {}
    for graph in (0, 1):
        say("batch graph", graph, tsteps)
        with hj.Batch("f64", shapes) as b:
            b.config = hj.Config.make(**dict(b.config.as_dict(), use_graph=graph, **extra))
            for t, a in enumerate(arrays):
                b.upload_all(t, a)
            hs, ps = [], []
            for rep in range(4):
                b.sweep(5, 0.8)
                hs.append(b.gosa_history.copy())
                ps.append([b.download(t) for t in range(len(shapes))])
                _ = b.residual()
            res[graph] = (hs, ps)
    for a, c in zip(res[0][0], res[1][0]):
        assert np.array_equal(a, c)
    for a, c in zip(res[0][1], res[1][1]):
        for x, y in zip(a, c):
            assert np.array_equal(x, y)


def test_batch_of_one_and_zero_iterations():
    shape = (20, 21, 70)
    f = inputs.fields(9, shape)
    say("batch of one")
    with hj.Batch("f64", [shape]) as b:
        b.config = hj.Config.make(kernel=1, bj=14, vec=4, ichunk=6, nontemporal=0, use_graph=1, xcd_remap=1,
                                  persistent=0, tsteps=2, reread=0)
        b.upload_all(0, f)
        b.sweep(0, 0.8)                          # no-op
        assert np.array_equal(b.download(0), f["p"])
        assert b.residual()[0] == pytest.approx(oracle.residual(f), rel=1e-10)
        b.sweep(5, 0.8)
        pref, _, href = oracle.sweep(f, 5, 0.8)
        assert np.array_equal(b.download(0), pref)
        assert gosa_err(b.gosa_history[:, 0], href) <= F64_GOSA_RTOL


def test_batch_autotune_keeps_parity():
    shapes, seeds = small_batch(1, 5)
    arrays = [inputs.fields(sd, sh) for sh, sd in zip(shapes, seeds)]
    with hj.Batch("f64", shapes) as b:
        for t, a in enumerate(arrays):
            b.upload_all(t, a)
        say("batch autotune")
        best, ms = b.autotune(n_sweeps=2, repeats=1)
        assert ms > 0 and best.kernel in (1, 2)
        b.sweep(4, 0.8)
        for t, a in enumerate(arrays):
            pref, _, _ = oracle.sweep(a, 4, 0.8)
            assert np.array_equal(b.download(t), pref)


def test_batch_errors():
    with pytest.raises(hj.HJError) as e:
        hj.Batch("f64", [(3, 3, 3), (2, 5, 5)])
    assert e.value.status == -2
    with hj.Batch("f32", [(4, 4, 4), (5, 5, 5)]) as b:
        with pytest.raises(hj.HJError) as e:
            b.sweep(1, 0.8)
        assert e.value.status == -6
        with pytest.raises(hj.HJError):
            b.config = hj.Config.make(kernel=0, bj=4, vec=1, ichunk=4, nontemporal=0, use_graph=1,
                                      xcd_remap=0, persistent=0)
        with pytest.raises(hj.HJError):          # two-iteration passes have no persistent grid
            b.config = hj.Config.make(kernel=1, bj=8, vec=1, ichunk=4, nontemporal=0, use_graph=1,
                                      xcd_remap=0, persistent=1, tsteps=2)
        b.config = hj.Config.make(kernel=1, bj=4, vec=1, ichunk=4, nontemporal=0, use_graph=1, xcd_remap=1,
                                  persistent=0, tsteps=1, reread=1)
        assert b.config.xcd_remap == 0 and b.config.reread == 0   # one-iteration batches clear them
    with hj.Batch("f64", [(4, 4, 4), (5, 6, 900)]) as b:
        with pytest.raises(hj.HJError) as e:      # a flat run too wide for one instance
            b.config = hj.Config.make(kernel=2, bj=8, vec=1, ichunk=4, nontemporal=0, use_graph=1,
                                      xcd_remap=0, persistent=0)
        assert e.value.status == -1
        with pytest.raises(ValueError):
            b.upload(1, "p", np.zeros((4, 4, 4)))


def test_batch_genetic_search_keeps_parity():
    shapes, seeds = small_batch(3, 5)
    arrays = [inputs.fields(sd, sh) for sh, sd in zip(shapes, seeds)]
    with hj.Batch("f64", shapes) as b:
        for t, a in enumerate(arrays):
            b.upload_all(t, a)
        say("batch genetic search")
        best, ms, evals = b.autotune_ga(population=8, generations=6, seed=1, n_sweeps=2, repeats=1)
        assert ms > 0 and best.kernel in (1, 2) and evals >= 1
        b.sweep(4, 0.8)
        for t, a in enumerate(arrays):
            pref, _, _ = oracle.sweep(a, 4, 0.8)
            assert np.array_equal(b.download(t), pref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_pinned_host_arrays_match_pageable(dtype):
    """Batch uploads from and downloads into pinned host memory (copied
    directly) give the same instances as pageable arrays."""
    from paper_2002_12115_amd import transfer
    shapes, seeds = inputs.batch_shapes(21, 4, lo_xy=4, hi_xy=30, lo_z=4, hi_z=90)
    arrays = [inputs.fields(sd, sh) for sh, sd in zip(shapes, seeds)]
    say("batch pinned", dtype)
    outs = {}
    for pinned in (False, True):
        with hj.Batch(dtype, shapes) as b:
            for t, a in enumerate(arrays):
                src = {n: transfer.pinned_like(a[n], b.np_dtype) for n in inputs.INPUTS} if pinned else a
                b.upload_all(t, src)
            b.sweep(4, 0.8)
            got = []
            for t, sh in enumerate(shapes):
                if pinned:
                    got.append(b.download(t, out=transfer.pinned_like(np.zeros(sh), b.np_dtype)).copy())
                else:
                    got.append(b.download(t))
            with pytest.raises(ValueError):
                b.download(0, out=np.zeros((2, 2, 2), dtype=b.np_dtype))
            outs[pinned] = got
    for x, y in zip(outs[False], outs[True]):
        assert np.array_equal(x, y)
    if dtype == "f64":
        for t, a in enumerate(arrays):
            assert np.array_equal(outs[True][t], oracle.sweep(a, 4, 0.8)[0])
