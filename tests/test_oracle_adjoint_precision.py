"""Pins of the adjoint and precision oracles."""

import numpy as np
import pytest
import torch

from gen import random_sparse
from oracle import adjoint as AD
from oracle import precision as P
from oracle import spmv as O


def _dense(A):
    D = np.zeros((A.n, A.n))
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
    D[rows, A.col_idx] = A.vals
    return D


@pytest.mark.parametrize("seed", range(4))
def test_dot_product_identity(seed):
    A = random_sparse(80, 4.0, seed=seed, empty_row_frac=0.1)
    rng = np.random.default_rng(seed)
    x, g = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    lhs = np.dot(g, O.spmv(A.row_ptr, A.col_idx, A.vals, x))
    rhs = np.dot(AD.grad_x(A.row_ptr, A.col_idx, A.vals, g), x)
    D = _dense(A)
    scale = np.abs(g) @ np.abs(D) @ np.abs(x)
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_grad_x_is_dense_transpose():
    A = random_sparse(50, 5.0, seed=11)
    g = np.random.default_rng(3).uniform(-1, 1, A.n)
    D = _dense(A)
    assert not np.allclose(D, D.T)
    assert np.allclose(AD.grad_x(A.row_ptr, A.col_idx, A.vals, g), D.T @ g, rtol=1e-13, atol=1e-15)


def test_finite_differences():
    A = random_sparse(60, 4.0, seed=21)
    rng = np.random.default_rng(21)
    x, g = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    gx = AD.grad_x(A.row_ptr, A.col_idx, A.vals, g)
    gv = AD.grad_vals(A.row_ptr, A.col_idx, x, g)
    for j in rng.choice(A.n, 30, replace=False):
        h = 1e-3 * max(1.0, abs(x[j]))
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (AD.loss(A.row_ptr, A.col_idx, A.vals, xp, g) - AD.loss(A.row_ptr, A.col_idx, A.vals, xm, g)) / (2 * h)
        assert abs(fd - gx[j]) <= 1e-9
    for k in rng.choice(A.nnz, 30, replace=False):
        h = 1e-3 * max(1.0, abs(A.vals[k]))
        vp, vm = A.vals.copy(), A.vals.copy()
        vp[k] += h
        vm[k] -= h
        fd = (AD.loss(A.row_ptr, A.col_idx, vp, x, g) - AD.loss(A.row_ptr, A.col_idx, vm, x, g)) / (2 * h)
        assert abs(fd - gv[k]) <= 1e-9


def test_multi_rhs_grad_vals_sums_columns():
    A = random_sparse(40, 3.0, seed=4)
    rng = np.random.default_rng(4)
    X, G = rng.uniform(-1, 1, (40, 8)), rng.uniform(-1, 1, (40, 8))
    gv = AD.grad_vals(A.row_ptr, A.col_idx, X, G)
    ref = sum(AD.grad_vals(A.row_ptr, A.col_idx, X[:, c], G[:, c]) for c in range(8))
    assert np.allclose(gv, ref, rtol=1e-14, atol=1e-15)
    gx = AD.grad_x(A.row_ptr, A.col_idx, A.vals, G)
    assert np.allclose(gx, _dense(A).T @ G, rtol=1e-13, atol=1e-15)


def test_bf16_rounding_by_hand():
    cases = {
        1.0: 0x3F80,
        1.0 + 2 ** -8: 0x3F80,            # tie between 0x3F80 and 0x3F81 -> even
        1.0 + 3 * 2 ** -8: 0x3F82,        # tie between 0x3F81 and 0x3F82 -> even
        1.0 + 2 ** -8 + 2 ** -20: 0x3F81,  # just above the tie -> up
        -2.0: 0xC000,
        0.0: 0x0000,
        float("inf"): 0x7F80,
        3.4028234663852886e38: 0x7F80,    # largest float32 (0x7F7FFFFF) rounds to infinity in bf16
        3.3895313892515355e38: 0x7F7F,    # largest finite bf16 is exact
    }
    for v, bits in cases.items():
        assert int(P.f32_to_bf16_bits(np.float32(v))) == bits, v
    assert np.isnan(P.bf16_bits_to_f64(P.f32_to_bf16_bits(np.float32("nan"))))


def test_bf16_matches_torch():
    v = np.random.default_rng(0).standard_normal(100000).astype(np.float32) * 10.0 ** np.random.default_rng(1).integers(-20, 20, 100000)
    v = v.astype(np.float32)
    ours = P.f32_to_bf16_bits(v)
    theirs = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, theirs)


def test_f32_matches_torch():
    v = np.random.default_rng(2).standard_normal(100000) * 1e3
    assert np.array_equal(P.to_f32(v), torch.from_numpy(v).to(torch.float32).numpy())


def test_forward_bound_holds_for_f32_accumulation():
    A = random_sparse(500, 20.0, seed=9)
    x = np.random.default_rng(9).uniform(-1, 1, A.n)
    v32 = P.to_f32(A.vals)
    x32 = x.astype(np.float32)
    # float32 row sums, left to right
    y32 = np.zeros(A.n, dtype=np.float32)
    for i in range(A.n):
        acc = np.float32(0)
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            acc = np.float32(acc + np.float32(v32[k] * x32[A.col_idx[k]]))
        y32[i] = acc
    y = O.spmv(A.row_ptr, A.col_idx, A.vals, x)
    scale = O.row_abs_sum(A.row_ptr, A.col_idx, A.vals, x)
    e = P.relative_errors(y32, y, scale)
    beta = P.forward_bound(np.diff(A.row_ptr), "f32", True, "f32")
    assert np.all(e <= beta)
    assert np.max(e) > 1e-9  # the bound is not vacuous for this case
