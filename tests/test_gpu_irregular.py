"""GPU parity on irregular matrices: rows longer than a staging window (streamed in windows by their
super-row's wavefront) and rows longer than the long-row limit (split over a workgroup of their own)."""

import numpy as np
import pytest

from gen import CsrInput
from gen.irregular import rmat_matrix
from gpu_util import check_forward, params, say, to_dev
from oracle import adjoint as OA
from oracle import precision as OP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05096_amd import _capi as C  # noqa: E402
from paper_2203_05096_amd.matrix import CsrkBatch, CsrkMatrix  # noqa: E402

VEC = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32}
LONG_ROW = 1024  # rows longer than this get a workgroup of their own


def _mixed(seed, symmetric, n=6000):
    """Short rows (0..8 entries) mixed with rows of 40..200 (windows of a few rows), 509..520, 1023..1026, 3000
    and 5000 entries, and a column (7) present in every third row, so that A^T has a row of n / 3 entries too."""
    rng = np.random.default_rng(seed)
    special = {17: 509, 18: 510, 19: 511, 20: 520, 300: 1023, 301: 1024, 302: 1025, 303: 1026, 900: 3000,
               2500: min(5000, n - 1), 4000 % n: 700, 30: 40, 31: 60, 32: 100, 33: 200, 34: 150, 35: 90, 36: 33}
    ii, jj = [], []
    for i in range(n):
        k = special.get(i, int(rng.integers(0, 9)))
        cols = rng.choice(n, size=min(k, n), replace=False)
        if i % 3 == 0 and 7 not in cols:
            cols = np.append(cols, 7)
        ii.extend([i] * len(cols))
        jj.extend(cols.tolist())
    ii, jj = np.array(ii, np.int64), np.array(jj, np.int64)
    if symmetric:
        ii, jj = np.concatenate([ii, jj]), np.concatenate([jj, ii])
    key = np.unique(ii * n + jj)
    ii, jj = key // n, key % n
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(ii, minlength=n), out=rp[1:])
    vals = rng.uniform(-1, 1, len(jj))
    return CsrInput(f"mixed_{seed}_{'sym' if symmetric else 'nonsym'}", n, rp.astype(np.int32),
                    jj.astype(np.int32), vals, {})


def _build(A, store, p):
    return CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, p, store), store)


def _vec(v, store):
    return v if store == "f64" else v.astype(np.float32).astype(np.float64)


def _check_grad_x(gx, A, g, store, label):
    ref = OA.grad_x(A.row_ptr, A.col_idx, A.vals, g)
    scale = OA.grad_x(A.row_ptr, A.col_idx, np.abs(A.vals), np.abs(g))
    colcount = np.bincount(A.col_idx, minlength=A.n)
    beta = np.full(A.n, 1e-12) if store == "f64" else OP.forward_bound(np.maximum(colcount, 1), store, True, "f32")
    err = np.abs(gx - ref)
    assert np.all(err <= beta * scale), f"{label}: grad_x over bound by {np.max(err - beta * scale):.3e}"


def test_mixed_matrix_has_every_row_class():
    A = _mixed(1, False)
    lengths = np.diff(A.row_ptr)
    assert (lengths == 0).any() and ((lengths > 504) & (lengths <= LONG_ROW)).sum() >= 5
    assert (lengths == LONG_ROW).any() and (lengths > LONG_ROW).sum() >= 4
    assert ((lengths > LONG_ROW) & (lengths <= 4096)).any() and (lengths > 4096).any()  # both long-row classes
    assert np.bincount(A.col_idx, minlength=A.n).max() > 1024  # and a long row of A^T
    assert ((lengths >= 33) & (lengths <= 201)).sum() >= 7  # windows of a few rows: more lanes per row


@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", [(16, 4, 1, 4), (64, 2, 4, 2)])
def test_forward_long_rows(store, shape):
    A = _mixed(2, False)
    if store != "f64":
        A.vals = OP.stored_values(A.vals, store)
    x = _vec(np.random.default_rng(3).uniform(-1, 1, A.n), store)
    say("irregular forward", store, shape)
    M = _build(A, store, params(*shape))
    perm = M.structure()["perm"]
    xp = x[perm]
    y = M.spmv(to_dev(xp, VEC[store]))
    y2 = M.spmv(to_dev(xp, VEC[store]))
    torch.cuda.synchronize()
    assert torch.equal(y, y2)
    check_forward(y.double().cpu().numpy(), A, x, perm, store, store != "f64", label=f"irregular {store} {shape}")


@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("symmetric", [False, True])
@pytest.mark.parametrize("explicit_vals", [False, True])
def test_adjoint_long_rows(store, symmetric, explicit_vals):
    A = _mixed(4 + symmetric, symmetric)
    if store != "f64":
        A.vals = OP.stored_values(A.vals, store)
    rng = np.random.default_rng(7)
    x, g = _vec(rng.uniform(-1, 1, A.n), store), _vec(rng.uniform(-1, 1, A.n), store)
    say("irregular adjoint", store, symmetric, explicit_vals)
    M = _build(A, store, params(32, 4, lanes=2))
    assert (M.info["symmetry"] == 1.0) == symmetric and M.info["long_rows"] >= 4
    s = M.structure()
    perm, vmap = s["perm"], s["vmap"]
    dt = VEC[store]
    xd, gd = to_dev(x[perm], dt), to_dev(g[perm], dt)
    vals = M.values() if explicit_vals else None
    gx, gv = M.adjoint(xd, gd, vals=vals)
    gx_only, _ = M.adjoint(xd, gd, vals=vals, grad_vals=False)
    _, gv_only = M.adjoint(xd, gd, vals=vals, grad_x=False)
    torch.cuda.synchronize()
    gv_in = np.empty(A.nnz)
    gv_in[vmap] = gv.double().cpu().numpy()
    ref_gv = OA.grad_vals(A.row_ptr, A.col_idx, x, g)
    if store != "f64":
        ref_gv = ref_gv.astype(np.float32).astype(np.float64)
    assert np.array_equal(gv_in, ref_gv)
    assert torch.equal(gv_only, gv)
    for out, label in ((gx, "both"), (gx_only, "grad_x only")):
        gx_in = np.empty(A.n)
        gx_in[perm] = out.double().cpu().numpy()
        _check_grad_x(gx_in, A, g, "f64" if store == "f64" else "f32", f"{store} sym={symmetric} {label}")


def test_batched_long_rows_match_single():
    """The batched kernels keep long rows in their super-row's wavefront (streamed in windows)."""
    mats = [_mixed(10, True, n=3000), _mixed(11, False, n=2500), _mixed(12, False, n=4000)]
    Ms = [_build(A, "f64", params(32, 4, lanes=2)) for A in mats]
    B = CsrkBatch(Ms)
    rng = np.random.default_rng(13)
    xs = [to_dev(rng.uniform(-1, 1, M.n), torch.float64) for M in Ms]
    gs = [to_dev(rng.uniform(-1, 1, M.n), torch.float64) for M in Ms]
    say("irregular batched")
    ys = B.spmv(xs)
    gxs, gvs = B.adjoint(xs, gs)
    for M, A, xd, gd, y, gx, gv in zip(Ms, mats, xs, gs, ys, gxs, gvs):
        y1 = M.spmv(xd)
        gx1, gv1 = M.adjoint(xd, gd)
        torch.cuda.synchronize()
        perm = M.structure()["perm"]
        x_in = np.empty(M.n)
        x_in[perm] = xd.cpu().numpy()
        check_forward(y.cpu().numpy(), A, x_in, perm, "f64", False, label="batched irregular")
        assert torch.allclose(y, y1, rtol=0, atol=1e-12 * float(torch.abs(y1).max()))
        assert torch.equal(gv, gv1)
        assert torch.allclose(gx, gx1, rtol=0, atol=1e-12 * float(torch.abs(gx1).max()))
    B.close()


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_rmat_full_size(store):
    """R-MAT, n = 2^20, about 9.2 M nonzeros, row lengths up to ~23 k (1 351 rows above a window)."""
    A = rmat_matrix(20, 4.0, 21, symmetric=True)
    if store != "f64":
        A.vals = OP.stored_values(A.vals, store)
    rng = np.random.default_rng(22)
    x, g = _vec(rng.uniform(-1, 1, A.n), store), _vec(rng.uniform(-1, 1, A.n), store)
    say("rmat full", store)
    M = _build(A, store, C.csrk_tune(A.n, A.nnz, "mi355x"))
    s = M.structure()
    perm, vmap = s["perm"], s["vmap"]
    dt = VEC[store]
    xd, gd = to_dev(x[perm], dt), to_dev(g[perm], dt)
    y = M.spmv(xd)
    gx, gv = M.adjoint(xd, gd)
    torch.cuda.synchronize()
    check_forward(y.double().cpu().numpy(), A, x, perm, store, store != "f64", label=f"rmat {store}")
    gv_in = np.empty(A.nnz)
    gv_in[vmap] = gv.double().cpu().numpy()
    ref_gv = OA.grad_vals(A.row_ptr, A.col_idx, x, g)
    if store != "f64":
        ref_gv = ref_gv.astype(np.float32).astype(np.float64)
    assert np.array_equal(gv_in, ref_gv)
    gx_in = np.empty(A.n)
    gx_in[perm] = gx.double().cpu().numpy()
    _check_grad_x(gx_in, A, g, store, f"rmat {store}")
