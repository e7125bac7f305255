"""Dense-matrix view of the oracle on grids of at most 8^3.

The operator is assembled from a table of the 19 (offset, coefficient, sign)
entries into a sparse matrix N, so one sweep is the mat-vec
wrk2 = p + omega * bnd * (a3 * (N p + wrk1) - p). This re-expresses the
stencil, so it is a consistency check of the iteration (interior/shell
split, copy-back, fixed point, convergence), not an independent pin of the
stencil itself (the Taylor closed forms are that).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_2002_12115_amd import inputs

# (di, dj, dk, coefficient, sign)
TABLE = [
    (1, 0, 0, "a0", 1), (0, 1, 0, "a1", 1), (0, 0, 1, "a2", 1),
    (1, 1, 0, "b0", 1), (1, -1, 0, "b0", -1), (-1, 1, 0, "b0", -1), (-1, -1, 0, "b0", 1),
    (0, 1, 1, "b1", 1), (0, -1, 1, "b1", -1), (0, 1, -1, "b1", -1), (0, -1, -1, "b1", 1),
    (1, 0, 1, "b2", 1), (-1, 0, 1, "b2", -1), (1, 0, -1, "b2", -1), (-1, 0, -1, "b2", 1),
    (-1, 0, 0, "c0", 1), (0, -1, 0, "c1", 1), (0, 0, -1, "c2", 1),
]


def assemble(f, shape):
    nx, ny, nz = shape
    n = nx * ny * nz
    rows, cols, vals = [], [], []
    idx = np.arange(n).reshape(shape)
    inner = idx[1:-1, 1:-1, 1:-1].ravel()
    ii, jj, kk = np.unravel_index(inner, shape)
    for di, dj, dk, name, sgn in TABLE:
        rows.append(inner)
        cols.append(idx[ii + di, jj + dj, kk + dk])
        vals.append(sgn * f[name].ravel()[inner])
    N = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return N, inner


@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 5, 6), (8, 8, 8), (5, 8, 7)])
def test_one_sweep_is_dense_matvec(shape):
    f = inputs.fields(2002, shape)
    N, inner = assemble(f, shape)
    p = f["p"].ravel()
    a3, bnd, w = (f[n].ravel() for n in ("a3", "bnd", "wrk1"))
    ss = np.zeros_like(p)
    ss[inner] = (bnd * (a3 * (N @ p + w) - p))[inner]
    exp = p + 0.8 * ss
    got, _, hist = oracle.sweep(f, 1, 0.8)
    np.testing.assert_allclose(got.ravel(), exp, rtol=0, atol=2e-15)
    assert hist[0] == pytest.approx(np.sum(ss * ss), rel=1e-13)


@pytest.mark.parametrize("shape", [(6, 6, 6), (8, 8, 8)])
def test_converges_to_direct_solve(shape):
    f = inputs.fields(7, shape)
    N, inner = assemble(f, shape)
    p0 = f["p"].ravel()
    a3, w = f["a3"].ravel(), f["wrk1"].ravel()
    m = inner.size
    sel = sp.csr_matrix((np.ones(m), (np.arange(m), inner)), shape=(m, p0.size))
    Nii = sel @ N @ sel.T
    # A p_int = a3 (N_bnd p_bnd + w) with A = I - D_a3 N_int
    pb = p0.copy()
    pb[inner] = 0.0
    D = sp.diags(a3[inner])
    A = sp.identity(m) - D @ Nii
    rhs = a3[inner] * ((N @ pb)[inner] + w[inner])
    pstar_int = spla.spsolve(A.tocsc(), rhs)
    pstar = p0.copy()
    pstar[inner] = pstar_int
    assert oracle.residual(dict(f, p=pstar.reshape(shape))) < 1e-26
    M = (1 - 0.8) * sp.identity(m) + 0.8 * (D @ Nii)
    rho = abs(M).sum(axis=1).max()
    assert rho < 1
    e0 = np.abs(p0 - pstar).max()
    for n in (5, 50, 200):
        pn, _, _ = oracle.sweep(f, n, 0.8)
        err = np.abs(pn.ravel() - pstar).max()
        assert err <= rho ** n * e0 + 1e-13
