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
