"""Different handles used from different host threads at once: each result
equals the oracle's (FP64 bitwise), whatever the interleaving."""
import threading

import numpy as np
import pytest

import oracle
from paper_2002_12115_amd import hj, inputs
from _hjtest import cfg, say

pytestmark = pytest.mark.gpu


def test_concurrent_handles_on_threads():
    jobs = [((30, 40, 70), 1, cfg(bj=8, vec=2, ichunk=7, nontemporal=0, xcd_remap=1, tsteps=2, reread=0)),
            ((50, 20, 90), 2, cfg(bj=4, vec=2, ichunk=3, nontemporal=1, xcd_remap=0)),
            ((19, 33, 140), 3, cfg(bj=6, vec=4, ichunk=5, nontemporal=0, xcd_remap=1, tsteps=2, reread=1))]
    batch_shapes, batch_seeds = inputs.batch_shapes(4, 4, lo_xy=5, hi_xy=30, lo_z=5, hi_z=90)
    n = 7
    results, errors = {}, []
    hj.load()                                    # load the library once, on this thread

    def solve(idx, shape, seed, c):
        try:
            f = inputs.fields(seed, shape)
            with hj.Solver("f64", shape) as s:
                s.config = c
                s.upload_all(f)
                for _ in range(3):               # several calls, so the threads interleave
                    s.sweep(n, 0.8)
                    s.upload("p", f["p"])
                s.sweep(n, 0.8)
                results[idx] = (f, s.download("p"))
        except Exception as e:                   # reported in the main thread
            errors.append((idx, repr(e)))

    def batch():
        try:
            arrays = [inputs.fields(sd, sh) for sh, sd in zip(batch_shapes, batch_seeds)]
            with hj.Batch("f64", batch_shapes) as b:
                for t, a in enumerate(arrays):
                    b.upload_all(t, a)
                b.sweep(n, 0.8)
                results["batch"] = (arrays, [b.download(t) for t in range(len(arrays))])
        except Exception as e:
            errors.append(("batch", repr(e)))

    say("threads", len(jobs) + 1)
    threads = [threading.Thread(target=solve, args=(q, sh, sd, c)) for q, (sh, sd, c) in enumerate(jobs)]
    threads.append(threading.Thread(target=batch))
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
        assert not t.is_alive()
    assert not errors, errors
    for q in range(len(jobs)):
        f, p = results[q]
        assert np.array_equal(p, oracle.sweep(f, n, 0.8)[0]), jobs[q]
    arrays, outs = results["batch"]
    for a, p in zip(arrays, outs):
        assert np.array_equal(p, oracle.sweep(a, n, 0.8)[0])
