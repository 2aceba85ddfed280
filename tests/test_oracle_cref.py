"""Pins of the C oracle (host timing code) against dense brute force and closed forms."""

import numpy as np

from gen import laplacian, random_sparse
from oracle import cref


def _dense(A):
    D = np.zeros((A.n, A.n))
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
    D[rows, A.col_idx] = A.vals
    return D


def test_c_forward_and_adjoint_dense():
    A = random_sparse(64, 5.0, seed=31, empty_row_frac=0.1)
    rng = np.random.default_rng(31)
    x, g = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    D = _dense(A)
    y = cref.spmv(A.row_ptr, A.col_idx, A.vals, x)
    assert np.allclose(y, D @ x, rtol=1e-13, atol=1e-15)
    gx, gv = cref.adjoint(A.row_ptr, A.col_idx, A.vals, x, g)
    assert np.allclose(gx, D.T @ g, rtol=1e-13, atol=1e-15)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
    assert np.array_equal(gv, g[rows] * x[A.col_idx])


def test_c_laplacian_ones():
    A = laplacian((17, 9, 5), "3d7", 6.0)
    y = cref.spmv(A.row_ptr, A.col_idx, A.vals, np.ones(A.n))
    z, yy, xx = np.meshgrid(np.arange(5), np.arange(9), np.arange(17), indexing="ij")
    nb = ((xx > 0).astype(int) + (xx < 16) + (yy > 0) + (yy < 8) + (z > 0) + (z < 4)).ravel()
    assert np.array_equal(y, 6.0 - nb)
    assert cref.threads() >= 1
    assert cref.time_forward(A.row_ptr, A.col_idx, A.vals, np.ones(A.n), 2) >= 0.0


def test_c_gather_adjoint_equals_scatter_and_dense():
    """The column-parallel gather form adds each column's terms in the scatter's order: bitwise equal; and both
    match the dense transpose product."""
    for seed, empty in ((32, 0.0), (33, 0.2)):
        A = random_sparse(500, 6.0, seed=seed, empty_row_frac=empty)
        rng = np.random.default_rng(seed)
        x, g = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
        gx_s, gv_s = cref.adjoint(A.row_ptr, A.col_idx, A.vals, x, g)
        gx_g, gv_g = cref.adjoint_gather(A.row_ptr, A.col_idx, A.vals, x, g)
        assert np.array_equal(gx_s, gx_g) and np.array_equal(gv_s, gv_g)
        assert np.allclose(gx_g, _dense(A).T @ g, rtol=1e-13, atol=1e-15)
    tp, tr, tq = cref.column_index(A.row_ptr, A.col_idx)
    assert np.array_equal(np.asarray(A.col_idx)[tq], np.repeat(np.arange(A.n), np.diff(tp)))
    cref.set_threads(1)
    try:
        assert cref.threads() == 1
        assert cref.time_adjoint_gather(A.row_ptr, A.col_idx, A.vals, x, g, 1) >= 0.0
    finally:
        cref.set_threads(max(1, __import__("os").cpu_count()))
