"""GPU conjugate gradients on the CSR-k product (FP64 vectors and reductions, product in the storage
precision) against the FP64 oracle CG and the FP64 true residual."""

import numpy as np
import pytest

from gen import laplacian
from gpu_util import params, say, to_dev
from oracle import cg as OCG
from oracle import precision as OP
from oracle import spmv as OS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05096_amd import _capi as C  # noqa: E402
from paper_2203_05096_amd.matrix import CsrkMatrix  # noqa: E402


def _spd(side=64):
    return laplacian((side, side), "2d5", 4.0)  # diagonal 4, off-diagonal -1: symmetric positive definite


def _solve(A, store, b, rtol, p=None, x0=None):
    M = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, p or C.csrk_tune(A.n, A.nnz, "mi355x"), store), store)
    perm = M.structure()["perm"]
    x0d = None if x0 is None else to_dev(x0[perm], torch.float64)
    x, it, rel = M.cg(to_dev(b[perm], torch.float64), x0=x0d, rtol=rtol, max_iter=5000, check_every=1)
    out = np.empty(A.n)
    out[perm] = x.cpu().numpy()
    return out, it, rel, M


def test_cg_f64_matches_oracle():
    A = _spd()
    b = np.random.default_rng(1).uniform(-1, 1, A.n)
    say("cg f64")
    x, it, rel, _ = _solve(A, "f64", b, 1e-10)
    xo, ito, relo = OCG.cg(A.row_ptr, A.col_idx, A.vals, b, rtol=1e-10)
    assert rel <= 1e-10 and abs(it - ito) <= 2, (it, ito)
    true = np.linalg.norm(b - OS.spmv(A.row_ptr, A.col_idx, A.vals, x)) / np.linalg.norm(b)
    assert true <= 1e-9
    assert np.max(np.abs(x - xo)) <= 1e-8 * np.max(np.abs(xo))


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_cg_reduced_precision_storage(store):
    """Values that the storage type cannot hold (4.1 / -0.9, still symmetric positive definite): the recurrence converges on the stored
    matrix; against the FP64 values the storage rounding remains, and the true residual is bounded by
    ||b - A_s x|| + || |A - A_s| |x| || (A_s the stored matrix), computed from the oracle in FP64."""
    A = _spd()
    A.vals = np.where(A.vals > 0, 4.1, -0.9)
    b = np.random.default_rng(2).uniform(-1, 1, A.n)
    rtol = 1e-6
    say("cg", store)
    x, it, rel, _ = _solve(A, store, b, rtol)
    assert rel <= rtol
    stored = OP.stored_values(A.vals, store)
    assert not np.array_equal(stored, A.vals)
    nb = np.linalg.norm(b)
    r_stored = np.linalg.norm(b - OS.spmv(A.row_ptr, A.col_idx, stored, x)) / nb
    r_true = np.linalg.norm(b - OS.spmv(A.row_ptr, A.col_idx, A.vals, x)) / nb
    pert = np.linalg.norm(OS.spmv(A.row_ptr, A.col_idx, np.abs(A.vals - stored), np.abs(x))) / nb
    # the recurrence residual drifts from the true one of the stored matrix by the FP32 rounding of the products
    # and of the direction vector: bounded here by 100x the recurrence tolerance
    assert r_stored <= 100 * rtol, r_stored
    assert r_true <= r_stored + pert * (1 + 1e-12), (r_true, r_stored, pert)


def test_cg_bf16_equals_f32_when_values_are_exact():
    """4 / -1 values are exact in BF16 and FP32: both storages feed the same FP32 products in the same order, so
    the two solves agree bit for bit."""
    A = _spd()
    b = np.random.default_rng(2).uniform(-1, 1, A.n)
    say("cg bf16 == f32")
    x32, it32, rel32, _ = _solve(A, "f32", b, 1e-6)
    x16, it16, rel16, _ = _solve(A, "bf16", b, 1e-6)
    assert it32 == it16 and rel32 == rel16 and np.array_equal(x32, x16)


def test_cg_deterministic_initial_guess_and_csr2():
    A = _spd(40)
    rng = np.random.default_rng(3)
    b, x0 = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    say("cg determinism")
    x1, it1, _, _ = _solve(A, "f64", b, 1e-9, x0=x0)
    x2, it2, _, _ = _solve(A, "f64", b, 1e-9, x0=x0)
    assert it1 == it2 and np.array_equal(x1, x2)
    x3, it3, rel3, _ = _solve(A, "f64", b, 1e-9, p=params(16, 2, lanes=1, waves=2, k=2))
    true = np.linalg.norm(b - OS.spmv(A.row_ptr, A.col_idx, A.vals, x3)) / np.linalg.norm(b)
    assert rel3 <= 1e-9 and true <= 1e-8


def test_cg_breakdown_and_arguments():
    A = laplacian((20, 20), "2d5", -4.0, off_value=1.0)  # negative definite: p'Ap < 0 at once
    b = np.ones(A.n)
    M = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, C.csrk_tune(A.n, A.nnz, "mi355x"), "f64"), "f64")
    say("cg breakdown")
    with pytest.raises(C.CsrkError) as e:
        M.cg(to_dev(b, torch.float64), rtol=1e-8, max_iter=50, check_every=1)
    assert e.value.name == "CSRK_ERR_UNSUPPORTED"
    bd = to_dev(b, torch.float64)
    xd = torch.zeros_like(bd)
    for args in ((0, bd.data_ptr(), xd.data_ptr(), 1e-8, 10, 1), (M.handle, bd.data_ptr(), xd.data_ptr(), 0.0, 10, 1),
                 (M.handle, bd.data_ptr(), xd.data_ptr(), 1e-8, 10, 0)):
        with pytest.raises(C.CsrkError) as e:
            C.csrk_cg(*args, torch.cuda.current_stream().cuda_stream)
        assert e.value.name == "CSRK_ERR_ARG"
    torch.cuda.synchronize()
