"""Generator checks: sizes and row-length histograms from closed forms."""

import numpy as np

from gen import workload_c1, workload_c3, stencil_pattern, drop_offdiagonals, diag_dominant_values, laplacian
import gen


def test_c1_sizes_and_values():
    w = workload_c1()
    A = w["A"]
    assert A.n == 4096 and A.nnz == 20224
    base = laplacian((64, 64), "2d5", 4.0)
    assert np.all(np.abs(A.vals - base.vals) <= 0.1)
    assert w["x"].min() >= -1 and w["x"].max() <= 1


def test_pattern_counts_closed_form():
    # 3D 7-point on s^3: 7 s^3 - 6 s^2; 27-point: (3s-2)^3; 2D 9-point: (3s-2)^2
    for s in (3, 7, 12):
        assert stencil_pattern((s, s, s), "3d7")[0][-1] == 7 * s ** 3 - 6 * s ** 2
        assert stencil_pattern((s, s, s), "3d27")[0][-1] == (3 * s - 2) ** 3
        assert stencil_pattern((s, s), "2d9")[0][-1] == (3 * s - 2) ** 2


def test_drop_rate_and_diag_dominance():
    rng = np.random.default_rng(0)
    rp, ci, dg = stencil_pattern((200, 200), "2d9")
    off_before = int((~dg).sum())
    rp2, ci2, dg2 = drop_offdiagonals(rp, ci, dg, rng, 0.1)
    kept = int((~dg2).sum())
    assert abs(kept / off_before - 0.9) < 0.01
    assert dg2.sum() == 200 * 200
    vals = diag_dominant_values(rp2, dg2, rng)
    rows = np.repeat(np.arange(40000), np.diff(rp2.astype(np.int64)))
    off = np.zeros(40000)
    np.add.at(off, rows[~dg2], np.abs(vals[~dg2]))
    assert np.allclose(vals[dg2], 1.1 * off)
    assert np.all((vals[~dg2] <= -0.5) & (vals[~dg2] >= -1.5))


def test_c3_small_side_variance():
    w = workload_c3(side=12)
    lengths = np.diff(w["A"].row_ptr.astype(np.int64))
    ec, ec2 = (10 * 3 + 2 * 2) / 12, (10 * 9 + 2 * 4) / 12
    assert abs(lengths.mean() - ec ** 3) < 1e-12
    assert abs(lengths.var() - (ec2 ** 3 - ec ** 6)) < 1e-9


def test_seeded_reproducible():
    a = workload_c1(seed=5)
    b = workload_c1(seed=5)
    c = workload_c1(seed=6)
    assert np.array_equal(a["A"].vals, b["A"].vals) and np.array_equal(a["x"], b["x"])
    assert not np.array_equal(a["A"].vals, c["A"].vals)


def test_c5_small_batch():
    w = gen.workload_c5(count=3, lo=4, hi=6, nrhs=8)
    assert len(w["As"]) == 3
    for A, X, s in zip(w["As"], w["xs"], w["sides"]):
        assert A.n == s ** 3 and X.shape == (A.n, 8)
        assert np.array_equal(X.astype(np.float32).astype(np.float64), X)


def test_rmat_pattern_properties():
    from gen.irregular import rmat_matrix
    A = rmat_matrix(12, 4.0, 5, symmetric=True)
    B = rmat_matrix(12, 4.0, 5, symmetric=True)
    assert np.array_equal(A.row_ptr, B.row_ptr) and np.array_equal(A.vals, B.vals)
    n, rp, ci = A.n, A.row_ptr.astype(np.int64), A.col_idx.astype(np.int64)
    rows = np.repeat(np.arange(n), np.diff(rp))
    key = rows * n + ci
    assert np.all(np.diff(key) > 0)  # sorted within rows, no duplicates
    assert set((ci * n + rows).tolist()) == set(key.tolist())  # symmetric pattern
    assert np.all(np.isin(np.arange(n) * (n + 1), key))  # every diagonal stored
    lengths = np.diff(rp)
    assert lengths.var() > 10 and lengths.max() > 20 * lengths.mean()  # the irregular class (variance above 10)
    diag = ci == rows
    off = np.bincount(rows, weights=np.where(diag, 0.0, np.abs(A.vals)), minlength=n)
    assert np.allclose(A.vals[diag], np.where(off > 0, 1.1 * off, 1.0))
    N = rmat_matrix(12, 4.0, 6, symmetric=False)
    rn = np.repeat(np.arange(N.n), np.diff(N.row_ptr))
    assert set((N.col_idx.astype(np.int64) * N.n + rn).tolist()) != set((rn * N.n + N.col_idx).tolist())
