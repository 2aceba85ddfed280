"""Pins of the FP64 SpMV oracle against facts outside itself."""

from fractions import Fraction

import numpy as np
import pytest

from gen import laplacian, random_sparse, workload_c2, stencil_pattern
from oracle import spmv as O
from oracle import bandk

U64 = 2.0 ** -53


def gamma(m):
    return m * U64 / (1 - m * U64)


def _dense_from_triplets(n, row_ptr, col_idx, vals):
    """Independent dense construction (vectorised scatter, not the oracle's loop)."""
    D = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    D[rows, np.asarray(col_idx, dtype=np.int64)] = vals
    return D


@pytest.mark.parametrize("seed", range(8))
def test_dense_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 65))
    A = random_sparse(n, avg_per_row=float(rng.uniform(0.5, 6)), seed=seed, empty_row_frac=0.15)
    x = rng.uniform(-1, 1, n)
    y = O.spmv(A.row_ptr, A.col_idx, A.vals, x)
    D = _dense_from_triplets(n, A.row_ptr, A.col_idx, A.vals)
    ref = D @ x
    scale = np.abs(D) @ np.abs(x)
    assert np.all(np.abs(y - ref) <= 2 * gamma(n) * scale + 1e-300)
    # a transposed operand would fail here (pattern is nonsymmetric)
    if not np.allclose(D, D.T):
        assert not np.allclose(y, D.T @ x)


@pytest.mark.parametrize("seed", range(5))
def test_exact_rational(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 17))
    A = random_sparse(n, avg_per_row=4.0, seed=100 + seed)
    x = rng.uniform(-1, 1, n)
    y = O.spmv(A.row_ptr, A.col_idx, A.vals, x)
    for i in range(n):
        exact = Fraction(0)
        scale = Fraction(0)
        m = 0
        for k in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
            a = Fraction(float(A.vals[k]))
            xv = Fraction(float(x[int(A.col_idx[k])]))
            exact += a * xv
            scale += abs(a) * abs(xv)
            m += 1
        err = abs(Fraction(float(y[i])) - exact)
        assert err <= Fraction(gamma(max(m, 1))) * scale


def _neighbour_count_2d(nx, ny):
    x, y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    return ((x > 0).astype(int) + (x < nx - 1) + (y > 0) + (y < ny - 1)).ravel()


def _neighbour_count_3d(s):
    z, y, x = np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij")
    return ((x > 0).astype(int) + (x < s - 1) + (y > 0) + (y < s - 1) + (z > 0) + (z < s - 1)).ravel()


def test_laplacian_times_ones_2d():
    A = laplacian((64, 64), "2d5", 4.0)
    y = O.spmv(A.row_ptr, A.col_idx, A.vals, np.ones(A.n))
    expected = 4.0 - _neighbour_count_2d(64, 64)
    assert np.array_equal(y, expected.astype(np.float64))


def test_laplacian_times_ones_3d_scrambled():
    w = workload_c2(seed=9, side=20)
    A = w["A"]
    y = O.spmv(A.row_ptr, A.col_idx, A.vals, np.ones(A.n))
    expected = 6.0 - _neighbour_count_3d(20)[A.meta["perm0"]]
    assert np.array_equal(y, expected.astype(np.float64))


def test_unit_vectors_give_columns():
    A = random_sparse(40, 3.0, seed=7, empty_row_frac=0.1)
    D = _dense_from_triplets(A.n, A.row_ptr, A.col_idx, A.vals)
    for j in range(A.n):
        e = np.zeros(A.n)
        e[j] = 1.0
        assert np.array_equal(O.spmv(A.row_ptr, A.col_idx, A.vals, e), D[:, j])


def test_empty_rows_are_exact_zero():
    A = random_sparse(50, 2.0, seed=3, empty_row_frac=0.4, with_diag=False)
    lengths = np.diff(A.row_ptr)
    assert (lengths == 0).any()
    y = O.spmv(A.row_ptr, A.col_idx, A.vals, np.random.default_rng(0).uniform(-1, 1, A.n))
    assert np.all(y[lengths == 0] == 0.0)
    assert O.spmv(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), np.zeros(0)).shape == (0,)


def test_multi_rhs_matches_columns():
    A = random_sparse(30, 4.0, seed=5)
    X = np.random.default_rng(1).uniform(-1, 1, (30, 8))
    Y = O.spmv(A.row_ptr, A.col_idx, A.vals, X)
    for c in range(8):
        assert np.array_equal(Y[:, c], O.spmv(A.row_ptr, A.col_idx, A.vals, X[:, c]))


@pytest.mark.parametrize("seed", range(4))
def test_csrk_traversal_equals_row_loop_bitwise(seed):
    rng = np.random.default_rng(seed)
    A = random_sparse(200, 5.0, seed=seed, empty_row_frac=0.05)
    # random grouping sizes
    sizes = []
    left = A.n
    while left:
        s = int(min(left, rng.integers(1, 9)))
        sizes.append(s)
        left -= s
    ssizes = []
    left = len(sizes)
    while left:
        s = int(min(left, rng.integers(1, 5)))
        ssizes.append(s)
        left -= s
    sr_ptr, ssr_ptr = bandk.group_from_sizes(sizes, ssizes)
    x = rng.uniform(-1, 1, A.n)
    y1, visits = O.spmv_csrk_traversal(ssr_ptr, sr_ptr, A.row_ptr, A.col_idx, A.vals, x)
    y2 = O.spmv(A.row_ptr, A.col_idx, A.vals, x)
    assert np.all(visits == 1)
    assert np.array_equal(y1, y2)


def test_row_abs_sum():
    A = random_sparse(20, 3.0, seed=2)
    x = np.random.default_rng(2).uniform(-1, 1, 20)
    D = _dense_from_triplets(20, A.row_ptr, A.col_idx, A.vals)
    assert np.allclose(O.row_abs_sum(A.row_ptr, A.col_idx, A.vals, x), np.abs(D) @ np.abs(x), rtol=1e-14)


def test_stencil_pattern_is_sorted_and_symmetric():
    rp, ci, dg = stencil_pattern((5, 4, 3), "3d27")
    n = 60
    D = _dense_from_triplets(n, rp, ci, np.ones(len(ci)))
    assert np.array_equal(D, D.T)
    for i in range(n):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)


def test_oracle_cg_against_dense_solve_and_finite_termination():
    """CG on an n x n SPD system reaches the exact solution in at most n steps (exact arithmetic); in FP64 it
    matches numpy.linalg.solve to rounding.  A planted sign error in the update would not converge."""
    from gen import laplacian
    from oracle import cg as OC
    A = laplacian((5, 4), "2d5", 4.0)
    D = np.zeros((A.n, A.n))
    for i in range(A.n):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i, A.col_idx[k]] += A.vals[k]
    b = np.random.default_rng(3).uniform(-1, 1, A.n)
    x, it, rel = OC.cg(A.row_ptr, A.col_idx, A.vals, b, rtol=1e-13, max_iter=4 * A.n)
    assert it <= A.n + 2 and rel <= 1e-13
    assert np.allclose(x, np.linalg.solve(D, b), rtol=0, atol=1e-11)
    assert np.linalg.norm(D @ x - b) <= 1e-12 * np.linalg.norm(b) * 10
