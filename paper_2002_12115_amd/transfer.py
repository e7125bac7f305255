"""Where the CPU-GPU transfers of a solve are placed.

The paper's offload method moves variables between CPU and GPU at the
outermost loop it can (section 3.2). It sends variables that are not needed
back and forth once, before all GPU work, and returns them after it; data
already on the GPU is marked present (section 3.3). This module runs the same
Jacobi solve under different placements, so the cost the rule avoids can be
measured on MI355X. Every placement computes the same iterations with the
same kernels; only the transfers around them differ, so the final field is
bitwise the same.

Placements:
  resident          upload once, all iterations on the device, download once
  p_every_k         the field goes to the host and back every k iterations
  p_every_iter      ... every iteration
  all_every_iter    all 13 inputs are uploaded before every iteration and the
                    field is downloaded after it (per-loop offload with no
                    data region)
  observe_every_k   the host reads the field every k iterations (no upload)
  observe_every_k_async   the same reads, each sent by hj_snapshot while the
                    next k iterations run (overlapped; pinned host arrays)

With pinned=True the host side of every transfer is pinned memory (copies
of the inputs made before the timed region), which the library copies to
and from directly; otherwise ordinary (pageable) arrays, which it stages
through its own pinned buffers.
"""
from __future__ import annotations

import time
from typing import Dict, Mapping

import numpy as np

from .inputs import INPUTS

POLICIES = ("resident", "p_every_k", "p_every_iter", "all_every_iter", "observe_every_k",
            "observe_every_k_async")


def pinned_like(a: np.ndarray, dtype=None) -> np.ndarray:
    """A copy of `a` in pinned host memory (allocated through torch)."""
    import torch
    dt = np.dtype(dtype or a.dtype)
    t = torch.empty(a.shape, dtype=torch.float64 if dt == np.float64 else torch.float32, pin_memory=True)
    out = t.numpy()
    out[...] = a
    return out


def run(solver, arrays: Mapping[str, np.ndarray], policy: str, n_iter: int, omega: float,
        k: int = 10, pinned: bool = False) -> Dict[str, object]:
    """Upload `arrays`, run n_iter iterations under `policy`, return timings,
    bytes moved, the final field and the gosa history."""
    if policy not in POLICIES:
        raise ValueError("unknown policy %r" % (policy,))
    esz = np.dtype(solver.np_dtype).itemsize
    cells = int(np.prod(solver.shape))
    field_bytes = cells * esz
    if pinned:   # the inputs in the solver's dtype, pinned, before the timed region
        arrays = {n: pinned_like(arrays[n], solver.np_dtype) for n in INPUTS}
    solver.upload_all(arrays)
    if pinned:
        host = solver.download("p", out=pinned_like(arrays["p"]))   # the host's copy of the field
    else:
        host = np.array(solver.download("p"))
    h2d = d2h = 0
    hist = []
    # observe placements: two host arrays, so the host may read one while the
    # other is written (allocated here, outside the timed region)
    spare = None
    if policy.startswith("observe_every_k"):
        spare = pinned_like(host) if pinned else np.empty_like(host)
    t0 = time.perf_counter()
    if policy == "resident":
        solver.sweep(n_iter, omega)
        hist.extend(solver.gosa_history)
    elif policy.startswith("observe_every_k"):
        overlap = policy.endswith("_async")
        views = [host, spare]
        done = 0
        while done < n_iter:
            n = min(k, n_iter - done)
            solver.sweep(n, omega)
            hist.extend(solver.gosa_history)
            done += n
            dst = views[(done // k) % 2]
            if overlap:
                solver.snapshot_wait()          # the previous snapshot's array is complete
                solver.snapshot(dst)
            else:
                solver.download("p", out=dst)
            d2h += field_bytes
        if overlap:
            solver.snapshot_wait()
    else:
        step = k if policy == "p_every_k" else 1
        done = 0
        while done < n_iter:
            n = min(step, n_iter - done)
            if policy == "all_every_iter":
                for name in INPUTS:
                    solver.upload(name, host if name == "p" else arrays[name])
                h2d += len(INPUTS) * field_bytes
            solver.sweep(n, omega)
            hist.extend(solver.gosa_history)
            host = solver.download("p", out=host if pinned else None)
            d2h += field_bytes
            if policy != "all_every_iter":
                solver.upload("p", host)
                h2d += field_bytes
            done += n
    wall = time.perf_counter() - t0
    final = solver.download("p")
    return {"policy": policy, "pinned": pinned, "iters": n_iter, "k": k if policy == "p_every_k" else None,
            "wall_s": wall, "h2d_bytes": h2d, "d2h_bytes": d2h, "field": final,
            "gosa_history": np.asarray(hist)}
