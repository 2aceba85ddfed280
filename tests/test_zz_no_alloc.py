"""csrk_cg_noalloc (work memory in the library's fixed per-device array, no device allocation) against csrk_cg
(work memory allocated per call) on the same inputs, through the C ABI: two solves in a row on one device, the
second on a smaller matrix, each compared bit for bit (same kernels, fixed-order reductions); and the rejection
of a handle whose work memory exceeds the array."""

import numpy as np
import pytest

from gen import diag_dominant_values, laplacian, stencil_pattern
from gen.stencils import CsrInput
from gpu_util import params, say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05096_amd import _capi as C  # noqa: E402
from paper_2203_05096_amd.matrix import CsrkMatrix  # noqa: E402


def _spd_3d27(side, seed):
    """3D 27-point pattern, diagonally dominant values (symmetric positive definite after symmetrising)."""
    row_ptr, col_idx, is_diag = stencil_pattern((side, side, side), "3d27")
    vals = diag_dominant_values(row_ptr, is_diag, np.random.default_rng(seed))
    n = side ** 3
    # symmetric values: (A + A^T) / 2 keeps diagonal dominance and makes A symmetric positive definite
    import scipy.sparse as sp
    M = sp.csr_matrix((vals, col_idx, row_ptr), shape=(n, n))
    M = ((M + M.T) * 0.5).tocsr()
    M.sort_indices()
    return CsrInput(f"spd3d27_{side}", n, M.indptr.astype(np.int32), M.indices.astype(np.int32),
                    M.data.astype(np.float64), {})


def _both(A, store, seed, rtol=1e-9, check_every=7):
    """Solves with csrk_cg and then csrk_cg_noalloc from the same x0; returns both results."""
    p = C.csrk_tune(A.n, A.nnz, "mi355x")
    M = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, p, store), store)
    rng = np.random.default_rng(seed)
    b = to_dev(rng.uniform(-1, 1, A.n), torch.float64)
    x0 = to_dev(rng.uniform(-0.1, 0.1, A.n), torch.float64)
    st = torch.cuda.current_stream().cuda_stream
    need = C.csrk_cg_noalloc_bytes(M.handle)
    assert 0 < need <= C.CG_NOALLOC_BYTES
    xa = x0.clone()
    it_a, rel_a = C.csrk_cg(M.handle, b.data_ptr(), xa.data_ptr(), rtol, 20000, check_every, st)
    xb = x0.clone()
    it_b, rel_b = C.csrk_cg_noalloc(M.handle, b.data_ptr(), xb.data_ptr(), rtol, 20000, check_every, st)
    torch.cuda.synchronize()
    M.close()
    return (xa.cpu().numpy(), it_a, rel_a), (xb.cpu().numpy(), it_b, rel_b)


@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
def test_cg_noalloc_matches_cg_two_calls(store):
    # first a larger solve, then a smaller one on the same device: the second reuses the array with the first's
    # contents still in it
    cases = [(_spd_3d27(28, 5), 11), (laplacian((37, 23), "2d5", 4.0), 12)]
    for A, seed in cases:
        say("cg_noalloc", store, A.name, "n", A.n)
        (xa, it_a, rel_a), (xb, it_b, rel_b) = _both(A, store, seed)
        assert it_a == it_b and it_a > 0, (it_a, it_b)
        assert rel_a == rel_b and rel_a <= 1e-9, (rel_a, rel_b)
        assert np.array_equal(xa, xb), f"{A.name}: max |diff| {np.max(np.abs(xa - xb)):.3e}"


def test_cg_noalloc_rejects_work_beyond_the_array():
    # a diagonal matrix of 2^22 rows needs 3 FP64 vectors of 32 MiB each: more than the 64 MiB array
    n = 1 << 22
    row_ptr = np.arange(n + 1, dtype=np.int32)
    col_idx = np.arange(n, dtype=np.int32)
    vals = np.full(n, 2.0)
    say("cg_noalloc reject n", n)
    M = CsrkMatrix(C.csrk_build(row_ptr, col_idx, vals, params(64, 2, 1, 2, reorder="none"), "f64"), "f64")
    assert C.csrk_cg_noalloc_bytes(M.handle) > C.CG_NOALLOC_BYTES
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    st = torch.cuda.current_stream().cuda_stream
    with pytest.raises(C.CsrkError) as e:
        C.csrk_cg_noalloc(M.handle, b.data_ptr(), x.data_ptr(), 1e-8, 10, 1, st)
    assert e.value.name == "CSRK_ERR_ARG" and "csrk_cg" in str(e.value)
    assert torch.count_nonzero(x).item() == 0  # rejected before any device work
    M.close()
