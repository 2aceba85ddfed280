"""GPU parity of the adjoint (grad_x = A^T g, grad_vals = g_i x_j) and of the autograd wrapper."""

import numpy as np
import pytest

from gen import random_sparse, workload_c4
from gpu_util import params, say, to_dev
from oracle import adjoint as OA
from oracle import precision as OP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05096_amd import _capi as C  # noqa: E402
from paper_2203_05096_amd.matrix import CsrkMatrix, CsrkSpMV  # noqa: E402

VEC = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32}
U = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -24}


def _build(A, store, p):
    return CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, p, store), store)


def _adjoint(M, x, g):
    """x, g in input order (float64, (n,) or (n, k)); returns (grad_x in input order, grad_vals in input order)."""
    s = M.structure()
    perm, vmap = s["perm"], s["vmap"]
    xp, gp = x[perm], g[perm]
    if M.store != "f64":
        xp, gp = xp.astype(np.float32), gp.astype(np.float32)
    gx, gv = M.adjoint(to_dev(xp, VEC[M.store]), to_dev(gp, VEC[M.store]))
    torch.cuda.synchronize()
    gx_in = np.empty_like(np.asarray(gx.double().cpu().numpy()))
    gx_in[perm] = gx.double().cpu().numpy()
    gv_in = np.empty(len(vmap), dtype=np.float64)
    gv_in[vmap] = gv.double().cpu().numpy()
    return gx_in, gv_in


def _check_grad_x(gx, A, g, store, x_rounded, label):
    ref = OA.grad_x(A.row_ptr, A.col_idx, A.vals, g)
    scale = OA.grad_x(A.row_ptr, A.col_idx, np.abs(A.vals), np.abs(g))
    colcount = np.bincount(A.col_idx, minlength=A.n)
    if ref.ndim == 2:
        colcount = colcount[:, None]
    if store == "f64":
        beta = np.full(colcount.shape, 1e-12)
    else:
        beta = OP.forward_bound(np.maximum(colcount, 1), store, x_rounded, "f32")
    err = np.abs(gx - ref)
    assert np.all(err <= beta * scale), f"{label}: grad_x over bound by {np.max(err - beta * scale):.3e}"


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_adjoint_random_ragged(store):
    A = random_sparse(4000, 6.0, seed=12, empty_row_frac=0.1)
    if store == "f32":
        A.vals = A.vals.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(12)
    x, g = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    if store == "f32":
        x, g = x.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)
    say("adjoint ragged", store)
    M = _build(A, store, params(19, 4))
    gx, gv = _adjoint(M, x, g)
    ref_gv = OA.grad_vals(A.row_ptr, A.col_idx, x, g)
    if store == "f32":
        ref_gv = ref_gv.astype(np.float32).astype(np.float64)  # exact FP64 product rounded once = FP32 product
    assert np.array_equal(gv, ref_gv), "grad_vals must be bitwise equal"
    _check_grad_x(gx, A, g, store, False, f"ragged {store}")
    # dot-product identity on the GPU results: <g, A x> = <A^T g, x>
    from oracle import spmv as OS
    lhs = np.dot(g, OS.spmv(A.row_ptr, A.col_idx, A.vals, x))
    # grad_x[j] is within beta_j * sum_i |a_ij||g_i| (FP64: the stated 1e-12; FP32: gamma of column j's count),
    # so <grad_x, x> is within max_j beta_j * <|g|, |A| |x|>, plus the FP64 rounding of the two dot products
    colmax = int(np.bincount(A.col_idx, minlength=A.n).max())
    beta = 1e-12 if store == "f64" else float(OP.gamma(colmax, 2.0 ** -24))
    fp64 = float(OP.gamma(A.n + colmax, 2.0 ** -53))
    tol = (beta + 2 * fp64) * np.dot(np.abs(g), OS.spmv(A.row_ptr, A.col_idx, np.abs(A.vals), np.abs(x)))
    assert abs(lhs - np.dot(gx, x)) <= tol


@pytest.mark.parametrize("nrhs", [2, 8])
def test_adjoint_multi_rhs(nrhs):
    A = random_sparse(3000, 7.0, seed=nrhs)
    A.vals = A.vals.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(nrhs)
    X = rng.uniform(-1, 1, (A.n, nrhs)).astype(np.float32).astype(np.float64)
    G = rng.uniform(-1, 1, (A.n, nrhs)).astype(np.float32).astype(np.float64)
    say("adjoint mrhs", nrhs)
    M = _build(A, "f32", params(21, 4))
    gx, gv = _adjoint(M, X, G)
    _check_grad_x(gx, A, G, "f32", False, f"mrhs {nrhs}")
    ref = OA.grad_vals(A.row_ptr, A.col_idx, X, G)
    scale = OA.grad_vals(A.row_ptr, A.col_idx, np.abs(X), np.abs(G))
    beta = OP.gamma(nrhs, 2.0 ** -24)
    assert np.all(np.abs(gv - ref) <= beta * scale)


def test_adjoint_skips_outputs():
    A = random_sparse(500, 4.0, seed=3)
    M = _build(A, "f64", params(8, 2))
    s = M.structure()
    x = to_dev(np.random.default_rng(1).uniform(-1, 1, A.n), torch.float64)
    g = to_dev(np.random.default_rng(2).uniform(-1, 1, A.n), torch.float64)
    gx, gv = M.adjoint(x, g, grad_vals=False)
    assert gv is None and gx is not None
    gx2, gv2 = M.adjoint(x, g, grad_x=False)
    torch.cuda.synchronize()
    assert gx2 is None
    ref = OA.grad_vals(s["row_ptr"], s["col_idx"], x.cpu().numpy(), g.cpu().numpy())
    assert np.array_equal(gv2.cpu().numpy(), ref)


def test_c4_full_adjoint_and_finite_differences():
    w = workload_c4()
    A, x, g = w["A"], w["x"], w["g"]
    p = C.csrk_tune(A.n, A.nnz, "mi355x")
    say("c4 adjoint", p)
    M = _build(A, "f32", p)
    assert M.info["adjoint_union"] == 1  # nonsymmetric: one pass over the union pattern
    gx, gv = _adjoint(M, x, g)
    ref_gv = OA.grad_vals(A.row_ptr, A.col_idx, x, g).astype(np.float32).astype(np.float64)
    assert np.array_equal(gv, ref_gv)
    _check_grad_x(gx, A, g, "f32", False, "c4")
    # central finite differences of L = <g, A x> on sampled coordinates; L is bilinear, so only the
    # terms that touch the perturbed coordinate change: evaluate those exactly in FP64.
    rng = np.random.default_rng(0)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
    for j in rng.choice(A.n, 100, replace=False):
        ks = np.nonzero(A.col_idx == j)[0]
        h = 1e-3 * max(1.0, abs(x[j]))

        def local(xj):
            return np.sum(A.vals[ks] * g[rows[ks]] * xj)
        fd = (local(x[j] + h) - local(x[j] - h)) / (2 * h)
        scale = np.sum(np.abs(A.vals[ks] * g[rows[ks]]))
        # grad_x[j]: FP32 sum of the column's rounded products, gamma_{c_j}(2^-24); the FP64 difference
        # quotient of a linear function is exact up to its own rounding, (|x_j| + h) / h * gamma(c_j + 2, 2^-53)
        fd_err = (abs(x[j]) + h) / h * OP.gamma(len(ks) + 2, 2.0 ** -53)
        assert abs(fd - gx[j]) <= (OP.gamma(len(ks), 2.0 ** -24) + fd_err) * scale
    for k in rng.choice(A.nnz, 100, replace=False):
        h = 1e-3 * max(1.0, abs(A.vals[k]))
        fd = ((A.vals[k] + h) * g[rows[k]] * x[A.col_idx[k]] - (A.vals[k] - h) * g[rows[k]] * x[A.col_idx[k]]) / (2 * h)
        # grad_vals[k] is the FP32 rounding of g_i x_j (2^-24 relative); the quotient's own FP64 rounding as above
        fd_err = (abs(A.vals[k]) + h) / h * OP.gamma(4, 2.0 ** -53)
        assert abs(fd - gv[k]) <= (2.0 ** -24 + fd_err) * abs(g[rows[k]] * x[A.col_idx[k]])


@pytest.mark.parametrize("store", ["bf16", "f64"])
def test_c4_full_union_adjoint_other_precisions(store):
    """The full-size nonsymmetric c4 matrix through the union pass in BF16 and FP64 storage."""
    w = workload_c4()
    A, x, g = w["A"], w["x"], w["g"]
    if store == "bf16":
        A.vals = OP.stored_values(A.vals, store)
    p = C.csrk_tune(A.n, A.nnz, "mi355x")
    say("c4 union adjoint", store, p)
    M = _build(A, store, p)
    assert M.info["adjoint_union"] == 1
    gx, gv = _adjoint(M, x, g)
    ref_gv = OA.grad_vals(A.row_ptr, A.col_idx, x, g)
    if store != "f64":
        ref_gv = ref_gv.astype(np.float32).astype(np.float64)
    assert np.array_equal(gv, ref_gv)
    _check_grad_x(gx, A, g, "f32" if store != "f64" else "f64", False, f"c4 {store}")


def test_autograd_gradcheck_f64():
    A = random_sparse(40, 4.0, seed=8, empty_row_frac=0.1)
    M = _build(A, "f64", params(5, 2))
    vals = M.values().clone().requires_grad_(True)
    x = torch.randn(A.n, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda v, xx: CsrkSpMV.apply(M, v, xx), (vals, x), eps=1e-6, atol=1e-9)


def test_autograd_backward_matches_adjoint_f32():
    A = random_sparse(1000, 5.0, seed=9)
    M = _build(A, "f32", params(13, 3))
    vals = M.values().clone().requires_grad_(True)
    x = torch.rand(A.n, dtype=torch.float32, device="cuda").requires_grad_(True)
    y = CsrkSpMV.apply(M, vals, x)
    g = torch.rand_like(y)
    y.backward(g)
    gx, gv = M.adjoint(x.detach(), g, vals=vals.detach())
    torch.cuda.synchronize()
    assert torch.equal(vals.grad, gv)
    assert torch.equal(x.grad, gx)  # the same kernel on the same inputs: deterministic


@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("explicit_vals", [False, True])
def test_adjoint_symmetric_fused(store, explicit_vals):
    """Symmetric patterns take the one-pass path; values from the handle's transposed copy or passed in."""
    from gen import workload_c2
    A = workload_c2(seed=5, side=40)["A"]
    A.vals = A.vals * np.random.default_rng(5).uniform(0.5, 1.5, A.nnz)  # values not symmetric
    if store != "f64":
        A.vals = OP.stored_values(A.vals, store)
    rng = np.random.default_rng(6)
    x, g = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    if store != "f64":
        x, g = x.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)
    say("adjoint symmetric", store, explicit_vals)
    M = _build(A, store, params(48, 4, lanes=2))
    s = M.structure()
    perm, vmap = s["perm"], s["vmap"]
    xp, gp = x[perm], g[perm]
    dt = VEC[store]
    vals = M.values() if explicit_vals else None
    gx, gv = M.adjoint(to_dev(xp, dt), to_dev(gp, dt), vals=vals)
    torch.cuda.synchronize()
    gx_in = np.empty(A.n)
    gx_in[perm] = gx.double().cpu().numpy()
    gv_in = np.empty(A.nnz)
    gv_in[vmap] = gv.double().cpu().numpy()
    ref_gv = OA.grad_vals(A.row_ptr, A.col_idx, x, g)
    if store != "f64":
        ref_gv = ref_gv.astype(np.float32).astype(np.float64)
    assert np.array_equal(gv_in, ref_gv)
    _check_grad_x(gx_in, A, g, "f32" if store != "f64" else "f64", False, f"sym {store} {explicit_vals}")
    # partial outputs fall back to the two-phase path and agree bitwise with the fused pass
    gx2, _ = M.adjoint(to_dev(xp, dt), to_dev(gp, dt), vals=vals, grad_vals=False)
    _, gv2 = M.adjoint(to_dev(xp, dt), to_dev(gp, dt), vals=vals, grad_x=False)
    torch.cuda.synchronize()
    assert torch.equal(gv2, gv)
    _check_grad_x(np.asarray(gx2.double().cpu().numpy())[np.argsort(perm)], A, g,
                  "f32" if store != "f64" else "f64", False, "sym partial")


def _union_fits(s):
    """Whether every super-row of the structure s has <= 64 rows and <= 504 entries of the union pattern (its A'
    entries plus, per row i, the columns j with (j, i) in A' and (i, j) not in A')."""
    rp, ci, srp = s["row_ptr"].astype(np.int64), s["col_idx"].astype(np.int64), s["sr_ptr"].astype(np.int64)
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    lone = ~np.isin(ci * n + rows, rows * n + ci)  # (i, j) whose mirror (j, i) is absent
    extras = np.concatenate([[0], np.cumsum(np.bincount(ci[lone], minlength=n))])
    entries = (rp[srp[1:]] - rp[srp[:-1]]) + (extras[srp[1:]] - extras[srp[:-1]])
    return bool(np.all(np.diff(srp) <= 64) and np.all(entries <= 504))


@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("explicit_vals", [False, True])
@pytest.mark.parametrize("srs", [19, 32, 200])
def test_adjoint_nonsymmetric_union_and_two_phase(store, explicit_vals, srs):
    """Nonsymmetric patterns: super-rows that fit a window take one pass over the union pattern (A' + A'^T);
    super-rows of more than 64 rows (SRS 200) keep the pass over A' and then over A'^T.  Values from the
    handle's copies or passed in (through the union's source map, -1 where A' has no mirror entry)."""
    A = random_sparse(3000, 5.0, seed=90 + srs, empty_row_frac=0.05)
    if store != "f64":
        A.vals = OP.stored_values(A.vals, store)
    rng = np.random.default_rng(91)
    x, g = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    if store != "f64":
        x, g = x.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)
    say("adjoint nonsymmetric", store, explicit_vals, srs)
    M = _build(A, store, params(srs, 2, lanes=2, waves=2))
    s = M.structure()
    fits = _union_fits(s)
    assert fits == (srs <= 64)  # the cases meant for each path
    assert M.info["adjoint_union"] == int(fits)
    perm, vmap = s["perm"], s["vmap"]
    dt = VEC[store]
    vals = M.values() if explicit_vals else None
    gx, gv = M.adjoint(to_dev(x[perm], dt), to_dev(g[perm], dt), vals=vals)
    torch.cuda.synchronize()
    gx_in = np.empty(A.n)
    gx_in[perm] = gx.double().cpu().numpy()
    gv_in = np.empty(A.nnz)
    gv_in[vmap] = gv.double().cpu().numpy()
    ref_gv = OA.grad_vals(A.row_ptr, A.col_idx, x, g)
    if store != "f64":
        ref_gv = ref_gv.astype(np.float32).astype(np.float64)
    assert np.array_equal(gv_in, ref_gv)
    _check_grad_x(gx_in, A, g, "f32" if store != "f64" else "f64", False, f"nonsym {store} {explicit_vals} {srs}")
    # a single output runs the two-phase path; grad_vals agrees bit for bit
    _, gv2 = M.adjoint(to_dev(x[perm], dt), to_dev(g[perm], dt), vals=vals, grad_x=False)
    torch.cuda.synchronize()
    assert torch.equal(gv2, gv)


@pytest.mark.parametrize("nrhs", [4, 8])
@pytest.mark.parametrize("store", ["f32", "f64"])
def test_adjoint_multi_rhs_union_and_two_phase(nrhs, store):
    """A nonsymmetric pattern with blocks of right-hand sides, FP32 and FP64 storage: the union pass (SRS 21)
    and the two-phase walk (SRS 200, super-rows past 64 rows) against the oracle at the accumulation's bound."""
    A = random_sparse(3000, 6.0, seed=70 + nrhs, empty_row_frac=0.05)
    A.vals = OP.stored_values(A.vals, store)
    rng = np.random.default_rng(71)
    X = rng.uniform(-1, 1, (A.n, nrhs))
    G = rng.uniform(-1, 1, (A.n, nrhs))
    if store != "f64":
        X, G = X.astype(np.float32).astype(np.float64), G.astype(np.float32).astype(np.float64)
    ref = OA.grad_x(A.row_ptr, A.col_idx, A.vals, G)
    scale = OA.grad_x(A.row_ptr, A.col_idx, np.abs(A.vals), np.abs(G))
    colcount = np.maximum(np.bincount(A.col_idx, minlength=A.n), 1)[:, None]
    refv = OA.grad_vals(A.row_ptr, A.col_idx, X, G)
    scalev = OA.grad_vals(A.row_ptr, A.col_idx, np.abs(X), np.abs(G))
    beta = 1e-12 if store == "f64" else OP.gamma(colcount, 2.0 ** -24)
    betav = 1e-12 if store == "f64" else OP.gamma(nrhs, 2.0 ** -24)
    for srs, union in ((21, 1), (200, 0)):
        say("adjoint mrhs union/two-phase", store, nrhs, srs)
        M = _build(A, store, params(srs, 2, lanes=2, waves=2))
        assert M.info["adjoint_union"] == union
        gx, gv = _adjoint(M, X, G)
        assert np.all(np.abs(gx - ref) <= beta * scale), f"grad_x, SRS {srs}"
        assert np.all(np.abs(gv - refv) <= betav * scalev), f"grad_vals, SRS {srs}"
        M.close()


def _structured_nonsymmetric(kind, n, seed):
    """Hand-built nonsymmetric patterns: upper bidiagonal (every row but the first gets one extra in the union,
    its lower neighbour), a dense lower triangle (union rows are full), and an upper bidiagonal with empty rows
    (rows reached only through their extras)."""
    from gen import CsrInput
    rows = []
    for i in range(n):
        if kind == "bidiag":
            rows.append([j for j in (i, i + 1) if j < n])
        elif kind == "lower":
            rows.append(list(range(i + 1)))
        else:  # "holes": every third row stored empty
            rows.append([] if i % 3 == 1 else [j for j in (i, i + 1) if j < n])
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.array([j for r in rows for j in r], dtype=np.int32)
    vals = np.random.default_rng(seed).uniform(-1, 1, len(ci))
    return CsrInput(kind, n, rp, ci, vals, {"seed": seed})


@pytest.mark.parametrize("kind,n", [("bidiag", 1), ("bidiag", 2), ("bidiag", 65), ("bidiag", 300), ("lower", 40),
                                    ("holes", 200)])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_adjoint_union_structured(kind, n, nrhs):
    """The union pass on hand-built nonsymmetric patterns, FP64 (one column) and FP32 (blocks of three)."""
    A = _structured_nonsymmetric(kind, n, seed=n)
    store = "f64" if nrhs == 1 else "f32"
    if store == "f32":
        A.vals = OP.stored_values(A.vals, store)
    rng = np.random.default_rng(n + 1)
    shp = (A.n,) if nrhs == 1 else (A.n, nrhs)
    X, G = rng.uniform(-1, 1, shp), rng.uniform(-1, 1, shp)
    if store == "f32":
        X, G = X.astype(np.float32).astype(np.float64), G.astype(np.float32).astype(np.float64)
    say("adjoint union structured", kind, n, nrhs)
    M = _build(A, store, params(8, 2, lanes=2, waves=2))
    sym = bool(n == 1)  # a single diagonal entry is its own mirror
    assert M.info["adjoint_union"] == (0 if sym else 1)
    gx, gv = _adjoint(M, X, G)
    ref = OA.grad_x(A.row_ptr, A.col_idx, A.vals, G)
    scale = OA.grad_x(A.row_ptr, A.col_idx, np.abs(A.vals), np.abs(G))
    cc = np.maximum(np.bincount(A.col_idx, minlength=A.n), 1)
    cc = cc if nrhs == 1 else cc[:, None]
    beta = 1e-12 if store == "f64" else OP.gamma(cc, 2.0 ** -24)
    assert np.all(np.abs(gx - ref) <= beta * scale)
    refv = OA.grad_vals(A.row_ptr, A.col_idx, X, G)
    if nrhs == 1:
        assert np.array_equal(gv, refv)
    else:
        scalev = OA.grad_vals(A.row_ptr, A.col_idx, np.abs(X), np.abs(G))
        assert np.all(np.abs(gv - refv) <= OP.gamma(nrhs, 2.0 ** -24) * scalev)


def test_adjoint_deterministic():
    A = random_sparse(5000, 8.0, seed=31, symmetric_pattern=True)
    M = _build(A, "f64", params(32, 4))
    x = to_dev(np.random.default_rng(1).uniform(-1, 1, A.n), torch.float64)
    g = to_dev(np.random.default_rng(2).uniform(-1, 1, A.n), torch.float64)
    a = M.adjoint(x, g)
    b = M.adjoint(x, g)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def _long_rows(rng, symmetric):
    """n = 2500 rows of 1..7 entries, every 97th row with 1500 (past one LDS window); optionally symmetrised."""
    from gen import CsrInput
    n = 2500
    dense_rows = set(range(0, n, 97))
    ii, jj = [], []
    for i in range(n):
        k = 1500 if i in dense_rows else int(rng.integers(1, 8))
        cols = rng.choice(n, size=k, replace=False)
        ii.extend([i] * k)
        jj.extend(cols.tolist())
    ii, jj = np.array(ii), np.array(jj)
    if symmetric:
        ii, jj = np.concatenate([ii, jj]), np.concatenate([jj, ii])
    key = np.unique(ii * n + jj)
    ii, jj = key // n, key % n
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(ii, minlength=n), out=rp[1:])
    return CsrInput("longsym" if symmetric else "long", n, rp.astype(np.int32), jj.astype(np.int32),
                    rng.uniform(-1, 1, len(jj)).astype(np.float32).astype(np.float64), {})


@pytest.mark.parametrize("nrhs", [3, 8])
@pytest.mark.parametrize("symmetric", [False, True])
def test_adjoint_multi_rhs_long_rows(nrhs, symmetric):
    rng = np.random.default_rng(nrhs + 10 * symmetric)
    A = _long_rows(rng, symmetric)
    n = A.n
    X = rng.uniform(-1, 1, (n, nrhs)).astype(np.float32).astype(np.float64)
    G = rng.uniform(-1, 1, (n, nrhs)).astype(np.float32).astype(np.float64)
    say("adjoint mrhs long", nrhs, symmetric)
    M = _build(A, "f32", params(16, 4))
    gx, gv = _adjoint(M, X, G)
    _check_grad_x(gx, A, G, "f32", False, f"mrhs long {nrhs} {symmetric}")
    ref = OA.grad_vals(A.row_ptr, A.col_idx, X, G)
    scale = OA.grad_vals(A.row_ptr, A.col_idx, np.abs(X), np.abs(G))
    assert np.all(np.abs(gv - ref) <= OP.gamma(nrhs, 2.0 ** -24) * scale)


@pytest.mark.parametrize("nrhs", [2, 8])
@pytest.mark.parametrize("long_rows", [False, True])
def test_adjoint_multi_rhs_symmetric_f64(nrhs, long_rows):
    """FP64 storage, several right-hand sides, symmetric pattern: the one-pass multi-column adjoint (8-byte
    values staged per window; rows past one window take the row-slice walk) against the oracle."""
    rng = np.random.default_rng(90 + nrhs + long_rows)
    A = _long_rows(rng, True) if long_rows else random_sparse(4000, 9.0, seed=91 + nrhs, empty_row_frac=0.05,
                                                              symmetric_pattern=True)
    X, G = rng.uniform(-1, 1, (A.n, nrhs)), rng.uniform(-1, 1, (A.n, nrhs))
    say("adjoint mrhs symmetric f64", nrhs, long_rows)
    M = _build(A, "f64", C.csrk_tune_rhs(A.n, A.nnz, nrhs, "mi355x"))
    gx, gv = _adjoint(M, X, G)
    _check_grad_x(gx, A, G, "f64", False, f"mrhs f64 {nrhs} {long_rows}")
    ref = OA.grad_vals(A.row_ptr, A.col_idx, X, G)
    scale = OA.grad_vals(A.row_ptr, A.col_idx, np.abs(X), np.abs(G))
    assert np.all(np.abs(gv - ref) <= 1e-12 * scale)


def test_symmetric_values_share_the_forward_array():
    """A matrix equal to its transpose keeps one value array: info reports it, and the adjoint is unchanged."""
    from gen import laplacian
    L = laplacian((20, 18, 9), "3d7", 6.0)
    L.vals = L.vals.copy()
    L.vals[L.vals < 0] = -1.25  # still symmetric
    M = _build(L, "f64", params(16, 4))
    assert M.info["values_symmetric"] == 1
    rng = np.random.default_rng(71)
    x, g = rng.uniform(-1, 1, L.n), rng.uniform(-1, 1, L.n)
    gx, gv = _adjoint(M, x, g)
    assert np.array_equal(gv, OA.grad_vals(L.row_ptr, L.col_idx, x, g))
    _check_grad_x(gx, L, g, "f64", False, "symmetric values")
    A = random_sparse(800, 6.0, seed=72, symmetric_pattern=True)  # symmetric pattern, random values
    assert _build(A, "f64", params(16, 4)).info["values_symmetric"] == 0
    # values equal as numbers but not as bits: +0.0 mirrored by -0.0 keeps its own transposed copy
    Z = laplacian((6, 5), "2d5", 4.0)
    Z.vals = Z.vals.copy()
    rows = np.repeat(np.arange(Z.n), np.diff(Z.row_ptr))
    Z.vals[(Z.col_idx == rows + 1)] = 0.0
    Z.vals[(Z.col_idx == rows - 1)] = -0.0
    MZ = _build(Z, "f64", params(4, 2))
    assert MZ.info["values_symmetric"] == 0
    gx, gv = _adjoint(MZ, np.ones(Z.n), np.ones(Z.n))
    # and the adjoint through the copy agrees with the oracle
    _check_grad_x(gx, Z, np.ones(Z.n), "f64", False, "signed zeros")


def test_c2_full_adjoint_random_vectors_at_tuned_shape():
    """The benchmark's adjoint: the full 128^3 scrambled 7-point matrix at the tuned shape, fused path reading
    the forward's own values, random x and g: grad_vals bitwise, grad_x within 1e-12 sum |a||g|."""
    from gen import workload_c2
    w = workload_c2()
    A, x, g = w["A"], w["x"], w["g"]
    p = C.csrk_tune(A.n, A.nnz, "mi355x")
    say("c2 full adjoint", p)
    M = _build(A, "f64", p)
    assert M.info["values_symmetric"] == 1
    gx, gv = _adjoint(M, x, g)
    assert np.array_equal(gv, OA.grad_vals(A.row_ptr, A.col_idx, x, g))
    _check_grad_x(gx, A, g, "f64", False, "c2 full")


@pytest.mark.parametrize("nrhs", [3, 8])
@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("symmetric", [False, True])
@pytest.mark.parametrize("explicit_vals", [False, True])
def test_adjoint_multi_rhs_precisions(nrhs, store, symmetric, explicit_vals):
    """Blocks of right-hand sides in every storage type, symmetric (one fused pass when both outputs are wanted
    and the accumulation is FP32) and nonsymmetric patterns (one pass over the union pattern with FP32
    accumulation, else grad_vals then A'^T g), with the handle's values or values passed in."""
    A = random_sparse(2500, 7.0, seed=40 + nrhs, empty_row_frac=0.05, symmetric_pattern=symmetric)
    A.vals = OP.stored_values(A.vals, store)
    rng = np.random.default_rng(41 + nrhs)
    X = rng.uniform(-1, 1, (A.n, nrhs))
    G = rng.uniform(-1, 1, (A.n, nrhs))
    if store != "f64":
        X, G = X.astype(np.float32).astype(np.float64), G.astype(np.float32).astype(np.float64)
    say("adjoint mrhs", nrhs, store, symmetric, explicit_vals)
    M = _build(A, store, params(21, 4))
    assert M.info["adjoint_union"] == (0 if symmetric else 1)
    s = M.structure()
    perm, vmap = s["perm"], s["vmap"]
    dt = VEC[store]
    vals = M.values() if explicit_vals else None
    gx, gv = M.adjoint(to_dev(X[perm], dt), to_dev(G[perm], dt), vals=vals)
    torch.cuda.synchronize()
    gx_in = np.empty((A.n, nrhs))
    gx_in[perm] = gx.double().cpu().numpy()
    gv_in = np.empty(A.nnz)
    gv_in[vmap] = gv.double().cpu().numpy()
    # values and vectors are exact in the storage type: only the accumulation rounds
    ref = OA.grad_x(A.row_ptr, A.col_idx, A.vals, G)
    scale = OA.grad_x(A.row_ptr, A.col_idx, np.abs(A.vals), np.abs(G))
    colcount = np.maximum(np.bincount(A.col_idx, minlength=A.n), 1)[:, None]
    beta = np.full(colcount.shape, 1e-12) if store == "f64" else OP.gamma(colcount, 2.0 ** -24)
    assert np.all(np.abs(gx_in - ref) <= beta * scale), f"grad_x over bound by {np.max(np.abs(gx_in - ref) - beta * scale)}"
    refv = OA.grad_vals(A.row_ptr, A.col_idx, X, G)
    scalev = OA.grad_vals(A.row_ptr, A.col_idx, np.abs(X), np.abs(G))
    betav = 1e-12 if store == "f64" else OP.gamma(nrhs, 2.0 ** -24)
    assert np.all(np.abs(gv_in - refv) <= betav * scalev)
    # grad_vals does not depend on the values: the same with or without them, and bitwise per column block
    _, gv2 = M.adjoint(to_dev(X[perm], dt), to_dev(G[perm], dt), vals=vals, grad_x=False)
    torch.cuda.synchronize()
    assert torch.equal(gv2, gv)
