"""Pins of the CPU oracle against facts that do not come from its own code.

* Taylor closed form: for a quadratic field p, every face pair and every
  mixed bracket of the stencil has an exact value in terms of the analytic
  derivatives of p (a p(x+e) + c p(x-e) = (a+c)p + (a-c) dp + (a+c)/2 d2p,
  and each 2x2 mixed bracket = 4 d_u d_v p). With per-cell random dyadic
  coefficients every operation is exact, so the oracle must match bitwise.
  A swapped face pair, a wrong axis, a wrong plane for a b coefficient, a
  wrong sign in a bracket, a dropped term or an in-place (Gauss-Seidel)
  update all change the result.
* Textbook case: a = c = 1, b = 0, a3 = 1/6, omega = 1 is the 7-point Jacobi
  average, checked with scipy.ndimage.correlate.
* Fixed point and contraction: a field built (from the closed form) to be
  the exact fixed point is recovered from a perturbed start at the rate
  bounded by ||M||_inf = (1-omega) + omega max a3 * rowsum.
* Invariants: mirror symmetry, omega-linearity, monotone ||ss||_inf and gosa,
  thread-count independence, gosa history == residual of the pre-update field.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2002_12115_amd import inputs

COEF = ("a0", "a1", "a2", "a3", "b0", "b1", "b2", "c0", "c1", "c2", "bnd", "wrk1")


def grid(shape):
    nx, ny, nz = shape
    return np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64),
                       np.arange(nz, dtype=np.float64), indexing="ij")


def dyadic_case(shape, rng, random_bnd=False):
    """Per-cell coefficients that are multiples of 1/64 (a3 of 1/1024)."""
    q = lambda lo, hi, d: rng.integers(lo, hi + 1, size=shape).astype(np.float64) / d
    f = {
        "a0": q(58, 70, 64), "a1": q(58, 70, 64), "a2": q(58, 70, 64),
        "c0": q(58, 70, 64), "c1": q(58, 70, 64), "c2": q(58, 70, 64),
        "b0": q(-3, 3, 64), "b1": q(-3, 3, 64), "b2": q(-3, 3, 64),
        "a3": q(150, 170, 1024), "wrk1": q(-20, 20, 1024),
    }
    bnd = np.zeros(shape)
    bnd[1:-1, 1:-1, 1:-1] = 1.0
    if random_bnd:
        bnd *= rng.integers(0, 2, size=shape)
    f["bnd"] = bnd
    return f


def quad_poly(rng):
    """p = c + sum alpha_d x_d + sum_{d<=e} beta_de x_d x_e, small integer coefficients."""
    return {"c": float(rng.integers(-5, 6)),
            "alpha": rng.integers(-4, 5, size=3).astype(np.float64),
            "beta": {de: float(rng.integers(-3, 4)) for de in
                     [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]}}


def poly_eval(P, X):
    v = P["c"] + sum(P["alpha"][d] * X[d] for d in range(3))
    for (d, e), b in P["beta"].items():
        v = v + b * X[d] * X[e]
    return v


def poly_grad(P, X, d):
    g = P["alpha"][d] + 2.0 * P["beta"][(d, d)] * X[d]
    for (u, v), b in P["beta"].items():
        if u != v:
            if u == d:
                g = g + b * X[v]
            elif v == d:
                g = g + b * X[u]
    return g


def poly_d2(P, d, e):
    if d == e:
        return 2.0 * P["beta"][(d, d)]
    return P["beta"][(min(d, e), max(d, e))]


def closed_form_s0_without_source(f, P, X):
    """s0 - wrk1 from the Taylor identities (exact for quadratic p)."""
    p = poly_eval(P, X)
    a = (f["a0"], f["a1"], f["a2"])
    c = (f["c0"], f["c1"], f["c2"])
    s = np.zeros_like(p)
    for d in range(3):
        s = s + (a[d] + c[d]) * p + (a[d] - c[d]) * poly_grad(P, X, d) \
            + 0.5 * (a[d] + c[d]) * poly_d2(P, d, d)
    # b0: (i,j) plane, b1: (j,k) plane, b2: (i,k) plane
    s = s + 4.0 * (f["b0"] * poly_d2(P, 0, 1) + f["b1"] * poly_d2(P, 1, 2) + f["b2"] * poly_d2(P, 0, 2))
    return s


def closed_form(f, P, shape, omega):
    X = grid(shape)
    p = poly_eval(P, X)
    s0 = closed_form_s0_without_source(f, P, X) + f["wrk1"]
    ss = (s0 * f["a3"] - p) * f["bnd"]
    inner = np.zeros(shape, bool)
    inner[1:-1, 1:-1, 1:-1] = True
    ss = np.where(inner, ss, 0.0)
    wrk2 = np.where(inner, p + omega * ss, p)
    return p, ss, wrk2


SMALL_SHAPES = list(itertools.product((3, 4, 5), repeat=3))


@pytest.mark.parametrize("shape", SMALL_SHAPES + [(6, 7, 9), (9, 5, 12), (11, 10, 8)])
def test_taylor_closed_form_bitwise(shape):
    rng = np.random.default_rng(hash(shape) % 2**32)
    for trial in range(3):
        f = dyadic_case(shape, rng, random_bnd=(trial == 2))
        P = quad_poly(rng)
        p, ss, wrk2 = closed_form(f, P, shape, 0.75)
        arrays = dict(f, p=p)
        p1, w1, hist = oracle.sweep(arrays, 1, 0.75)
        assert np.array_equal(p1, wrk2), "field differs from the Taylor closed form"
        inner = (slice(1, -1),) * 3
        assert np.array_equal(w1[inner], wrk2[inner])
        assert hist[0] == pytest.approx(math.fsum((ss * ss).ravel()), rel=1e-15, abs=0.0)


def test_closed_form_detects_planted_mistakes():
    """The pin is sharp: a one-sign change to the operator breaks it."""
    shape = (6, 7, 8)
    rng = np.random.default_rng(5)
    f = dyadic_case(shape, rng)
    P = quad_poly(rng)
    P["beta"][(0, 1)] = 2.0
    p, _, wrk2 = closed_form(f, P, shape, 0.75)
    good = oracle.sweep(dict(f, p=p), 1, 0.75)[0]
    assert np.array_equal(good, wrk2)
    # a b0 of the wrong sign is what a flipped bracket would produce
    bad = oracle.sweep(dict(f, p=p, b0=-f["b0"]), 1, 0.75)[0]
    assert not np.array_equal(bad, wrk2)
    # an a0/c0 swap is what a mirrored face pairing would produce
    P["alpha"][0] = 3.0
    p, _, wrk2 = closed_form(f, P, shape, 0.75)
    bad = oracle.sweep(dict(f, p=p, a0=f["c0"], c0=f["a0"]), 1, 0.75)[0]
    assert not np.array_equal(bad, wrk2)


def test_constant_field_is_fixed_point():
    shape = (7, 8, 9)
    rng = np.random.default_rng(3)
    f = dyadic_case(shape, rng)
    for n in ("a0", "a1", "c0", "c1"):
        f[n][:] = 1.0
    f["a2"][:] = 2.0
    f["c2"][:] = 2.0
    f["a3"][:] = 0.125
    f["wrk1"][:] = 0.0
    p = np.full(shape, 0.8125)
    for omega in (0.3, 0.8, 1.0):
        p1, _, hist = oracle.sweep(dict(f, p=p), 3, omega)
        assert np.array_equal(p1, p) and np.all(hist == 0.0)


def test_source_only():
    shape = (5, 6, 7)
    rng = np.random.default_rng(4)
    f = dyadic_case(shape, rng)
    p = np.zeros(shape)
    p1, _, hist = oracle.sweep(dict(f, p=p), 1, 0.75)
    exp = np.zeros(shape)
    exp[1:-1, 1:-1, 1:-1] = (0.75 * (f["wrk1"] * f["a3"]))[1:-1, 1:-1, 1:-1]
    assert np.array_equal(p1, exp)


def test_textbook_seven_point_average():
    shape = (9, 10, 11)
    rng = np.random.default_rng(11)
    p = rng.random(shape)
    ones = np.ones(shape)
    f = {n: ones.copy() for n in ("a0", "a1", "a2", "c0", "c1", "c2")}
    for n in ("b0", "b1", "b2", "wrk1"):
        f[n] = np.zeros(shape)
    f["a3"] = np.full(shape, 1.0 / 6.0)
    f["bnd"] = np.zeros(shape)
    f["bnd"][1:-1, 1:-1, 1:-1] = 1.0
    k = np.zeros((3, 3, 3))
    k[0, 1, 1] = k[2, 1, 1] = k[1, 0, 1] = k[1, 2, 1] = k[1, 1, 0] = k[1, 1, 2] = 1.0
    avg = ndimage.correlate(p, k, mode="constant") / 6.0
    p1, _, _ = oracle.sweep(dict(f, p=p), 1, 1.0)
    inner = (slice(1, -1),) * 3
    np.testing.assert_allclose(p1[inner], avg[inner], rtol=4e-16 * 8, atol=0)
    assert np.array_equal(p1[0], p[0]) and np.array_equal(p1[:, :, -1], p[:, :, -1])


def contraction_case(shape, rng, margin):
    f = {n: rng.uniform(0.9, 1.1, shape) for n in ("a0", "a1", "a2", "c0", "c1", "c2")}
    for n in ("b0", "b1", "b2"):
        f[n] = rng.uniform(-0.05, 0.05, shape)
    rowsum = sum(f[n] for n in ("a0", "a1", "a2", "c0", "c1", "c2")) \
        + 4.0 * sum(np.abs(f[n]) for n in ("b0", "b1", "b2"))
    f["a3"] = 1.0 / (rowsum + margin)
    f["bnd"] = np.zeros(shape)
    f["bnd"][1:-1, 1:-1, 1:-1] = 1.0
    rho_cells = (f["a3"] * rowsum)[1:-1, 1:-1, 1:-1]
    return f, float(rho_cells.max())


def test_fixed_point_recovered_at_contraction_rate():
    shape = (10, 9, 12)
    rng = np.random.default_rng(21)
    f, r = contraction_case(shape, rng, margin=2.0)
    P = quad_poly(rng)
    X = grid(shape)
    pstar = poly_eval(P, X)
    # choose the source so that pstar is the exact fixed point: a3*s0 == p
    f["wrk1"] = pstar / f["a3"] - closed_form_s0_without_source(f, P, X)
    omega = 0.8
    rho = (1 - omega) + omega * r
    p0 = pstar.copy()
    p0[1:-1, 1:-1, 1:-1] += rng.uniform(-1, 1, (8, 7, 10))
    e0 = np.abs(p0 - pstar).max()
    for n in (10, 40, 80):
        pn, _, _ = oracle.sweep(dict(f, p=p0), n, omega)
        err = np.abs(pn - pstar).max()
        assert err <= rho ** n * e0 + 1e-10, (n, err, rho ** n * e0)
    assert err < 1e-6


def test_monotone_decrease_config_distributions():
    shape = (12, 11, 14)
    f = inputs.fields(2002, shape)
    omega = 0.8
    p = f["p"]
    ssmax = []
    hist_all = []
    cur = dict(f)
    for it in range(25):
        p1, _, h = oracle.sweep(cur, 1, omega)
        ssmax.append(np.abs(p1 - cur["p"]).max() / omega)
        hist_all.append(h[0])
        cur = dict(cur, p=p1)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(ssmax, ssmax[1:]))
    assert all(b <= a for a, b in zip(hist_all, hist_all[1:]))
    # per-iteration history of one call equals the chained single sweeps
    _, _, hist = oracle.sweep(f, 25, omega)
    np.testing.assert_allclose(hist, hist_all, rtol=1e-15)
    del p


def test_history_is_residual_of_pre_update_field():
    shape = (8, 9, 10)
    f = inputs.fields(1, shape)
    p3, _, hist = oracle.sweep(f, 4, 0.8)
    assert hist[0] == oracle.residual(f)
    p2, _, _ = oracle.sweep(f, 3, 0.8)
    assert hist[3] == oracle.residual(dict(f, p=p2))
    assert oracle.residual(dict(f, p=p3)) < hist[3]


def test_omega_linearity():
    shape = (7, 8, 9)
    f = inputs.fields(7, shape)
    d1 = oracle.sweep(f, 1, 0.4)[0] - f["p"]
    d2 = oracle.sweep(f, 1, 0.8)[0] - f["p"]
    np.testing.assert_allclose(d2, 2 * d1, rtol=0, atol=1e-15)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry(axis):
    shape = (7, 8, 9)
    f = inputs.fields(2002, shape)
    face = {0: ("a0", "c0"), 1: ("a1", "c1"), 2: ("a2", "c2")}[axis]
    flip_b = {0: ("b0", "b2"), 1: ("b0", "b1"), 2: ("b1", "b2")}[axis]
    g = {n: np.flip(v, axis).copy() for n, v in f.items()}
    g[face[0]], g[face[1]] = g[face[1]], g[face[0]]
    for b in flip_b:
        g[b] = -g[b]
    pf, _, hf = oracle.sweep(f, 5, 0.8)
    pg, _, hg = oracle.sweep(g, 5, 0.8)
    np.testing.assert_allclose(np.flip(pg, axis), pf, rtol=0, atol=5e-15)
    np.testing.assert_allclose(hg, hf, rtol=1e-12)


def test_thread_count_independent():
    shape = (20, 13, 17)
    f = inputs.fields(2002, shape)
    p1, w1, h1 = oracle.sweep(f, 6, 0.8, nthreads=1)
    p4, w4, h4 = oracle.sweep(f, 6, 0.8, nthreads=4)
    assert np.array_equal(p1, p4) and np.array_equal(w1, w4) and np.array_equal(h1, h4)


def test_cells_matches_sweep():
    shape = (9, 10, 11)
    f = inputs.fields(1, shape)
    p1, _, _ = oracle.sweep(f, 1, 0.8)
    rng = np.random.default_rng(0)
    ijk = np.stack([rng.integers(1, s - 1, 50) for s in shape], 1)
    idx = (ijk[:, 0] * shape[1] + ijk[:, 1]) * shape[2] + ijk[:, 2]
    ss, w2 = oracle.cells(f, 0.8, idx)
    assert np.array_equal(w2, p1.ravel()[idx])
    with pytest.raises(ValueError):
        oracle.cells(f, 0.8, [0])


def test_bad_arguments():
    f = inputs.fields(1, (3, 3, 2))
    with pytest.raises(ValueError):
        oracle.sweep(f, 1, 0.8)
    f = inputs.fields(1, (3, 3, 3))
    with pytest.raises(ValueError):
        oracle.sweep(f, -1, 0.8)
    p1, _, h = oracle.sweep(f, 0, 0.8)
    assert np.array_equal(p1, f["p"]) and h.size == 0


def test_neighbourhood_blocks_reproduce_full_sweep():
    """Sampled-cell checking of large grids: the oracle run on a cell's own
    3x3x3 neighbourhood (values drawn at those positions) gives that cell's
    value of a full-grid sweep."""
    shape = (9, 11, 13)
    f = inputs.fields(2002, shape)
    p1, _, _ = oracle.sweep(f, 1, 0.8)
    rng = np.random.default_rng(1)
    cells = np.stack([rng.integers(1, s - 1, 40) for s in shape], 1)
    nb = inputs.neighbourhood(2002, shape, cells)
    for q, (i, j, k) in enumerate(cells):
        blk = {n: nb[n][q] for n in inputs.INPUTS}
        assert oracle.sweep(blk, 1, 0.8)[0][1, 1, 1] == p1[i, j, k]


@pytest.mark.parametrize("n", [2, 3])
def test_radius_n_blocks_reproduce_n_sweeps(n):
    """After n Jacobi iterations a cell depends only on its (2n+1)^3 block."""
    shape = (11, 12, 13)
    f = inputs.fields(7, shape)
    pn, _, _ = oracle.sweep(f, n, 0.8)
    rng = np.random.default_rng(2)
    cells = np.stack([rng.integers(n, s - n, 30) for s in shape], 1)
    nb = inputs.neighbourhood(7, shape, cells, radius=n)
    for q, (i, j, k) in enumerate(cells):
        blk = {f_: nb[f_][q] for f_ in inputs.INPUTS}
        assert oracle.sweep(blk, n, 0.8)[0][n, n, n] == pn[i, j, k]
