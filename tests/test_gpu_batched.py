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


def test_c5_full_batch_ones_closed_form_and_sampled_parity():
    w = workload_c5()
    say("c5 full build", len(w["As"]))
    Ms = _build_all(w["As"])
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
