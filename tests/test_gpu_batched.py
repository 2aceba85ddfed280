"""GPU parity of the batched launches (many matrices, blocks of right-hand sides)."""

import concurrent.futures as cf

import numpy as np
import pytest

from gen import workload_c5
from gpu_util import check_forward, say, to_dev
from oracle import adjoint as OA
from oracle import precision as OP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05096_amd import _capi as C  # noqa: E402
from paper_2203_05096_amd.matrix import CsrkBatch, CsrkMatrix  # noqa: E402


def _build_all(mats, store="f32", nrhs=8):
    def one(A):
        p = C.csrk_tune_rhs(A.n, A.nnz, nrhs, "mi355x")
        return CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, p, store), store)
    with cf.ThreadPoolExecutor(8) as ex:
        return list(ex.map(one, mats))


def _permuted(Ms, arrays):
    out = []
    for M, a in zip(Ms, arrays):
        perm = M.structure()["perm"]
        out.append(to_dev(a[perm].astype(np.float32), torch.float32))
    return out


@pytest.fixture(scope="module")
def small_batch():
    w = workload_c5(seed=50, count=12, lo=4, hi=20, nrhs=8)
    Ms = _build_all(w["As"])
    return w, Ms


def test_batch_forward_equals_single_and_oracle(small_batch):
    w, Ms = small_batch
    xs = _permuted(Ms, w["xs"])
    B = CsrkBatch(Ms)
    ys = B.spmv(xs)
    for M, x, y, A, X in zip(Ms, xs, ys, w["As"], w["xs"]):
        y1 = M.spmv(x)
        torch.cuda.synchronize()
        assert torch.equal(y, y1), "batched and single launches share the kernel body: bitwise equal"
        check_forward(y.double().cpu().numpy(), A, X, M.structure()["perm"], "f32", False, label=A.name)


def test_batch_single_rhs(small_batch):
    w, Ms = small_batch
    xs = [x[:, 0].contiguous() for x in _permuted(Ms, w["xs"])]
    B = CsrkBatch(Ms)
    ys = B.spmv(xs)
    for M, x, y in zip(Ms, xs, ys):
        assert torch.equal(y, M.spmv(x))


def test_batch_adjoint(small_batch):
    w, Ms = small_batch
    xs, gs = _permuted(Ms, w["xs"]), _permuted(Ms, w["gs"])
    B = CsrkBatch(Ms)
    gxs, gvs = B.adjoint(xs, gs)
    torch.cuda.synchronize()
    for M, x, g, gx, gv, A, X, G in zip(Ms, xs, gs, gxs, gvs, w["As"], w["xs"], w["gs"]):
        gx1, gv1 = M.adjoint(x, g)
        torch.cuda.synchronize()
        assert torch.equal(gv, gv1), "grad_vals is deterministic"
        s = M.structure()
        ref = OA.grad_x(s["row_ptr"], s["col_idx"], s["vals"], g.double().cpu().numpy())
        scale = OA.grad_x(s["row_ptr"], s["col_idx"], np.abs(s["vals"]), np.abs(g.double().cpu().numpy()))
        beta = OP.gamma(8, 2.0 ** -24)
        assert np.all(np.abs(gx.double().cpu().numpy() - ref) <= beta * scale)
        refv = OA.grad_vals(s["row_ptr"], s["col_idx"], x.double().cpu().numpy(), g.double().cpu().numpy())
        scalev = OA.grad_vals(s["row_ptr"], s["col_idx"], np.abs(x.double().cpu().numpy()),
                              np.abs(g.double().cpu().numpy()))
        assert np.all(np.abs(gv.double().cpu().numpy() - refv) <= OP.gamma(8, 2.0 ** -24) * scalev)


def test_batch_argument_checks_before_launch(small_batch):
    """Mismatched lists and wrongly sized outputs are rejected in Python, before any pointer reaches the library."""
    w, Ms = small_batch
    xs, gs = _permuted(Ms, w["xs"]), _permuted(Ms, w["gs"])
    B = CsrkBatch(Ms)
    with pytest.raises(ValueError):
        B.spmv(xs[:-1])  # one right-hand-side block short
    with pytest.raises(ValueError):
        B.adjoint(xs, gs[:-1])
    short = [torch.empty(M.nnz - 1, device="cuda") for M in Ms]
    with pytest.raises(TypeError):
        B.adjoint(xs, gs, out_vals=short)
    with pytest.raises(ValueError):
        B.adjoint(xs, gs, out_x=[torch.empty_like(g)[:-1] for g in gs])
    M = Ms[0]
    with pytest.raises(TypeError):
        M.adjoint(xs[0], gs[0], out_vals=short[0])
    with pytest.raises(TypeError):
        M.to_permuted(torch.zeros(M.n - 1, device="cuda"))
    with pytest.raises(TypeError):
        M.spmv(xs[0].reshape(M.n, 2, 4).contiguous())
    gx, _ = B.adjoint(None, gs, grad_vals=False)  # x is not needed without grad_vals
    torch.cuda.synchronize()
    assert torch.equal(gx[0], M.adjoint(xs[0], gs[0], grad_vals=False)[0])


@pytest.fixture(scope="module")
def full_c5():
    w = workload_c5()
    say("c5 full build", len(w["As"]))
    Ms = _build_all(w["As"])
    return w, Ms


def test_c5_full_batch_ones_closed_form_and_sampled_parity(full_c5):
    w, Ms = full_c5
    B = CsrkBatch(Ms)
    ones = [torch.ones((M.n, 8), dtype=torch.float32, device="cuda") for M in Ms]
    ys = B.spmv(ones)
    torch.cuda.synchronize()
    for M, y, s in zip(Ms, ys, w["sides"]):
        s = int(s)
        z, yy, xx = np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij")
        cnt = ((xx > 0).astype(int) + (xx < s - 1) + (yy > 0) + (yy < s - 1) + (z > 0) + (z < s - 1)).ravel()
        exact = (6.0 - cnt)[M.structure()["perm"]]
        assert np.array_equal(y.cpu().numpy(), np.repeat(exact[:, None], 8, axis=1).astype(np.float32))
    xs = _permuted(Ms, w["xs"])
    ys = B.spmv(xs)
    torch.cuda.synchronize()
    for b in (0, 17, 63):
        M, A, X = Ms[b], w["As"][b], w["xs"][b]
        check_forward(ys[b].double().cpu().numpy(), A, X, M.structure()["perm"], "f32", False, label=f"c5[{b}]")


def test_c5_full_batch_adjoint_sampled_parity(full_c5):
    """The benchmark's batched adjoint at full size (64 matrices, 8 right-hand sides, FP32), one launch; matrices
    0, 17 and 63 against the oracle: grad_x per column within gamma_{c_j}(2^-24), grad_vals (a sum over the 8
    columns) within gamma_8(2^-24); every matrix's grad_vals equal to its single-matrix launch bit for bit."""
    w, Ms = full_c5
    B = CsrkBatch(Ms)
    xs, gs = _permuted(Ms, w["xs"]), _permuted(Ms, w["gs"])
    gxs, gvs = B.adjoint(xs, gs)
    torch.cuda.synchronize()
    for b in (0, 17, 63):
        say("c5 adjoint matrix", b)
        M, s = Ms[b], Ms[b].structure()
        X, G = xs[b].double().cpu().numpy(), gs[b].double().cpu().numpy()
        ref = OA.grad_x(s["row_ptr"], s["col_idx"], s["vals"], G)
        scale = OA.grad_x(s["row_ptr"], s["col_idx"], np.abs(s["vals"]), np.abs(G))
        colcount = np.maximum(np.bincount(s["col_idx"], minlength=M.n), 1)[:, None]
        assert np.all(np.abs(gxs[b].double().cpu().numpy() - ref) <= OP.gamma(colcount, 2.0 ** -24) * scale)
        refv = OA.grad_vals(s["row_ptr"], s["col_idx"], X, G)
        scalev = OA.grad_vals(s["row_ptr"], s["col_idx"], np.abs(X), np.abs(G))
        assert np.all(np.abs(gvs[b].double().cpu().numpy() - refv) <= OP.gamma(8, 2.0 ** -24) * scalev)
        gx1, gv1 = M.adjoint(xs[b], gs[b])
        torch.cuda.synchronize()
        assert torch.equal(gv1, gvs[b]) and torch.equal(gx1, gxs[b])


@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nrhs", [1, 8])
@pytest.mark.parametrize("explicit_vals", [False, True])
@pytest.mark.parametrize("patterns", ["mixed", "symmetric"])
def test_batch_adjoint_precisions_mixed_patterns(store, nrhs, explicit_vals, patterns):
    """A batch mixing symmetric and nonsymmetric patterns (or of symmetric patterns only, which takes the
    one-pass multi-column launch) in every storage type, one and eight right-hand sides, handle values or
    values passed in: each matrix against the oracle at its bound and against its own single-matrix launch."""
    from gen import random_sparse
    mats = [random_sparse(n, 6.0, seed=60 + i, empty_row_frac=0.05,
                          symmetric_pattern=(patterns == "symmetric" or i % 2 == 0))
            for i, n in enumerate((700, 1500, 90, 2300, 411))]
    rng = np.random.default_rng(61)
    for A in mats:
        A.vals = OP.stored_values(A.vals, store)
    Ms = [CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, C.csrk_tune_rhs(A.n, A.nnz, nrhs, "mi355x"), store),
                     store) for A in mats]
    B = CsrkBatch(Ms)
    dt = torch.float64 if store == "f64" else torch.float32
    Xs, Gs = [], []
    for A in mats:
        shp = (A.n,) if nrhs == 1 else (A.n, nrhs)
        X, G = rng.uniform(-1, 1, shp), rng.uniform(-1, 1, shp)
        if store != "f64":
            X, G = X.astype(np.float32).astype(np.float64), G.astype(np.float32).astype(np.float64)
        Xs.append(X)
        Gs.append(G)
    xs = [to_dev(X[M.structure()["perm"]], dt) for X, M in zip(Xs, Ms)]
    gs = [to_dev(G[M.structure()["perm"]], dt) for G, M in zip(Gs, Ms)]
    vals = [M.values() for M in Ms] if explicit_vals else None
    say("batch adjoint", store, nrhs, explicit_vals, patterns)
    gxs, gvs = B.adjoint(xs, gs, vals=vals)
    torch.cuda.synchronize()
    for i, (A, M) in enumerate(zip(mats, Ms)):
        s = M.structure()
        perm, vmap = s["perm"], s["vmap"]
        gx_in = np.empty(gxs[i].shape)
        gx_in[perm] = gxs[i].double().cpu().numpy()
        gv_in = np.empty(A.nnz)
        gv_in[vmap] = gvs[i].double().cpu().numpy()
        ref = OA.grad_x(A.row_ptr, A.col_idx, A.vals, Gs[i])
        scale = OA.grad_x(A.row_ptr, A.col_idx, np.abs(A.vals), np.abs(Gs[i]))
        cc = np.maximum(np.bincount(A.col_idx, minlength=A.n), 1)
        cc = cc if nrhs == 1 else cc[:, None]
        beta = 1e-12 if store == "f64" else OP.gamma(cc, 2.0 ** -24)
        assert np.all(np.abs(gx_in - ref) <= beta * scale), (i, store, nrhs)
        refv = OA.grad_vals(A.row_ptr, A.col_idx, Xs[i], Gs[i])
        if nrhs == 1:
            # one rounded product per entry: bitwise in every precision
            refv = refv if store == "f64" else refv.astype(np.float32).astype(np.float64)
            assert np.array_equal(gv_in, refv), (i, store)
        else:
            scalev = OA.grad_vals(A.row_ptr, A.col_idx, np.abs(Xs[i]), np.abs(Gs[i]))
            betav = 1e-12 if store == "f64" else OP.gamma(nrhs, 2.0 ** -24)
            assert np.all(np.abs(gv_in - refv) <= betav * scalev), (i, store)
        gx1, gv1 = M.adjoint(xs[i], gs[i], vals=None if vals is None else vals[i])
        torch.cuda.synchronize()
        assert torch.equal(gv1, gvs[i]), (i, "grad_vals differs from the single-matrix launch")


@pytest.mark.parametrize("nrhs", [1, 4])
@pytest.mark.parametrize("explicit_vals", [False, True])
@pytest.mark.parametrize("store", ["f32", "f64"])
def test_batch_adjoint_union(nrhs, explicit_vals, store):
    """A batch of nonsymmetric matrices that all have a union-pattern index, FP32 and FP64 storage: the batched
    adjoint takes one pass over each union (values from the handles' union copies or passed in) and matches the
    oracle."""
    from gen import random_sparse
    mats = [random_sparse(n, 5.0, seed=80 + i, empty_row_frac=0.05) for i, n in enumerate((900, 1700, 333))]
    for A in mats:
        A.vals = OP.stored_values(A.vals, store)
    p = {"k": 3, "srs": 16, "ssrs": 2, "lanes_per_row": 2, "waves_per_wg": 2, "reorder": "bandk"}
    Ms = [CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, p, store), store) for A in mats]
    assert all(M.info["adjoint_union"] == 1 for M in Ms)
    B = CsrkBatch(Ms)
    rng = np.random.default_rng(81)
    dt = torch.float64 if store == "f64" else torch.float32
    Xs, Gs = [], []
    for A in mats:
        shp = (A.n,) if nrhs == 1 else (A.n, nrhs)
        X, G = rng.uniform(-1, 1, shp), rng.uniform(-1, 1, shp)
        if store != "f64":
            X, G = X.astype(np.float32).astype(np.float64), G.astype(np.float32).astype(np.float64)
        Xs.append(X)
        Gs.append(G)
    xs = [to_dev(X[M.structure()["perm"]], dt) for X, M in zip(Xs, Ms)]
    gs = [to_dev(G[M.structure()["perm"]], dt) for G, M in zip(Gs, Ms)]
    vals = [M.values() for M in Ms] if explicit_vals else None
    say("batch adjoint union", store, nrhs, explicit_vals)
    gxs, gvs = B.adjoint(xs, gs, vals=vals)
    torch.cuda.synchronize()
    for i, (A, M) in enumerate(zip(mats, Ms)):
        s = M.structure()
        gx_in = np.empty(gxs[i].shape)
        gx_in[s["perm"]] = gxs[i].double().cpu().numpy()
        gv_in = np.empty(A.nnz)
        gv_in[s["vmap"]] = gvs[i].double().cpu().numpy()
        ref = OA.grad_x(A.row_ptr, A.col_idx, A.vals, Gs[i])
        scale = OA.grad_x(A.row_ptr, A.col_idx, np.abs(A.vals), np.abs(Gs[i]))
        cc = np.maximum(np.bincount(A.col_idx, minlength=A.n), 1)
        cc = cc if nrhs == 1 else cc[:, None]
        beta = 1e-12 if store == "f64" else OP.gamma(cc, 2.0 ** -24)
        assert np.all(np.abs(gx_in - ref) <= beta * scale), i
        refv = OA.grad_vals(A.row_ptr, A.col_idx, Xs[i], Gs[i])
        if nrhs == 1:
            # one rounded product per entry: bitwise in either precision
            refv = refv if store == "f64" else refv.astype(np.float32).astype(np.float64)
            assert np.array_equal(gv_in, refv), i
        else:
            scalev = OA.grad_vals(A.row_ptr, A.col_idx, np.abs(Xs[i]), np.abs(Gs[i]))
            betav = 1e-12 if store == "f64" else OP.gamma(nrhs, 2.0 ** -24)
            assert np.all(np.abs(gv_in - refv) <= betav * scalev), i
    B.close()

