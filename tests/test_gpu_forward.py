"""GPU parity of the CSR-k forward product against the FP64 oracle (through the C ABI)."""

import numpy as np
import pytest

from gen import laplacian, random_sparse, workload_c1, workload_c2, workload_c3, workload_c4
from gpu_util import check_forward, params, say, to_dev
from oracle import precision as OP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05096_amd import _capi as C  # noqa: E402
from paper_2203_05096_amd.matrix import CsrkMatrix  # noqa: E402

VEC = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32}


def _build(A, store, p):
    return CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, p, store), store)


def _run(M, x_host, plain=False):
    """x_host in input order (float64); returns GPU y in permuted space as float64 numpy."""
    s = M.structure()
    xp = x_host[s["perm"]]
    if M.store != "f64":
        xp = xp.astype(np.float32)
    xd = to_dev(xp, VEC[M.store])
    y = M.spmv_plain(xd) if plain else M.spmv(xd)
    torch.cuda.synchronize()
    return y.double().cpu().numpy(), s["perm"]


def test_library_is_native():
    assert C.lib() is not None and torch.cuda.is_available()


def test_c1_f64_parity():
    w = workload_c1()
    A, x = w["A"], w["x"]
    for p in (C.csrk_tune(A.n, A.nnz, "mi355x"), params(8, 8), params(7, 15, lanes=4, waves=2),
              C.csrk_tune(A.n, A.nnz, "volta"), C.csrk_tune(A.n, A.nnz, "ampere")):
        say("c1 f64", p)
        M = _build(A, "f64", p)
        y, perm = _run(M, x)
        check_forward(y, A, x, perm, "f64", False, label=f"c1 {p}")


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("waves", [1, 4, 16])
def test_lanes_waves_shapes(lanes, waves):
    A = random_sparse(3000, 9.0, seed=lanes * 31 + waves, empty_row_frac=0.05)
    x = np.random.default_rng(lanes).uniform(-1, 1, A.n)
    say("shape", lanes, waves)
    M = _build(A, "f64", params(37, 5, lanes=lanes, waves=waves))
    y, perm = _run(M, x)
    check_forward(y, A, x, perm, "f64", False, label=f"L={lanes} W={waves}")


@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("reorder", ["bandk", "rcm", "none"])
def test_random_ragged_all_precisions(store, reorder):
    A = random_sparse(5003, 6.0, seed=7, empty_row_frac=0.1)
    x = np.random.default_rng(8).uniform(-1, 1, A.n)
    say("ragged", store, reorder)
    M = _build(A, store, params(23, 3, lanes=2, waves=4, reorder=reorder))
    vals_stored = OP.stored_values(A.vals, store)
    y, perm = _run(M, x)
    # the stored matrix, with x rounded like the kernel's input, must meet the accumulation bound
    check_forward(y, A, x, perm, store, store != "f64", label=f"{store} {reorder}")
    if store != "f64":
        # against the stored values and the rounded x, only accumulation error remains
        xr = x.astype(np.float32).astype(np.float64)
        check_forward(y, A, xr, perm, "f32", False, vals=vals_stored, label=f"{store} {reorder} (stored values)")


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_csr2_forward_and_adjoint(store):
    """k = 2 (one grouping level) and k = 4, 5 (levels above the super-super-row shape the ordering only):
    the same kernels over each structure."""
    from oracle import adjoint as OA
    A = random_sparse(4001, 7.0, seed=19, empty_row_frac=0.05, symmetric_pattern=False)
    rng = np.random.default_rng(20)
    x, g = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    if store != "f64":
        A.vals = OP.stored_values(A.vals, store)
        x, g = x.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)
    for p in (params(24, 2, lanes=2, waves=2, k=2), params(64, 4, lanes=1, waves=4, k=2),
              params(16, 2, lanes=2, waves=2, k=4), params(8, 3, lanes=1, waves=3, k=5)):
        say("csr-k", store, p)
        M = _build(A, store, p)
        assert M.info["params"]["k"] == p["k"]
        y, perm = _run(M, x)
        check_forward(y, A, x, perm, store, False, label=f"csr2 {store}")
        s = M.structure()
        dt = VEC[store]
        gx, gv = M.adjoint(to_dev(x[s["perm"]], dt), to_dev(g[s["perm"]], dt))
        torch.cuda.synchronize()
        gv_in = np.empty(A.nnz)
        gv_in[s["vmap"]] = gv.double().cpu().numpy()
        ref = OA.grad_vals(A.row_ptr, A.col_idx, x, g)
        if store != "f64":
            ref = ref.astype(np.float32).astype(np.float64)
        assert np.array_equal(gv_in, ref)
        gx_in = np.empty(A.n)
        gx_in[s["perm"]] = gx.double().cpu().numpy()
        gref = OA.grad_x(A.row_ptr, A.col_idx, A.vals, g)
        scale = OA.grad_x(A.row_ptr, A.col_idx, np.abs(A.vals), np.abs(g))
        # values, x and g are exact in the storage type: FP64 takes the stated 1e-12; FP32 sums the c_j rounded
        # products of column j in FP32, within gamma_{c_j}(2^-24) (Higham, ch. 3)
        colcount = np.maximum(np.bincount(A.col_idx, minlength=A.n), 1)
        tol = np.full(A.n, 1e-12) if store == "f64" else OP.gamma(colcount, 2.0 ** -24)
        assert np.all(np.abs(gx_in - gref) <= tol * scale)


def test_long_rows_exceed_staging_window():
    # rows of 3000 nonzeros (longer than a wavefront's LDS window) next to short rows
    n = 4000
    rng = np.random.default_rng(3)
    rows = []
    for i in range(n):
        k = 3000 if i % 97 == 0 else int(rng.integers(0, 9))
        rows.append(np.sort(rng.choice(n, size=k, replace=False)))
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    from gen import CsrInput
    A = CsrInput("long", n, rp.astype(np.int32), np.concatenate(rows).astype(np.int32),
                 rng.uniform(-1, 1, int(rp[-1])), {})
    x = rng.uniform(-1, 1, n)
    for store in ("f64", "f32", "bf16"):
        say("long rows", store)
        M = _build(A, store, params(16, 4, lanes=4))
        y, perm = _run(M, x)
        check_forward(y, A, x, perm, store, store != "f64", label=f"long {store}")


def test_empty_rows_give_exact_zero():
    A = random_sparse(700, 2.0, seed=5, empty_row_frac=0.5, with_diag=False)
    x = np.random.default_rng(5).uniform(-1, 1, A.n)
    M = _build(A, "f64", params(9, 3))
    y, perm = _run(M, x)
    empty = np.diff(A.row_ptr)[perm] == 0
    assert empty.any() and np.all(y[empty] == 0.0)
    # every row empty
    from gen import CsrInput
    Z = CsrInput("zero", 50, np.zeros(51, np.int32), np.zeros(0, np.int32), np.zeros(0), {})
    M = _build(Z, "f32", params(4, 4))
    y, _ = _run(M, x[:50])
    assert np.all(y == 0.0)


def test_tiny_sizes():
    for n in (1, 2, 63, 64, 65):
        A = random_sparse(n, 3.0, seed=n)
        x = np.random.default_rng(n).uniform(-1, 1, n)
        say("tiny", n)
        M = _build(A, "f64", params(3, 2))
        y, perm = _run(M, x)
        check_forward(y, A, x, perm, "f64", False, label=f"n={n}")


def test_c2_full_laplacian_ones_bitwise_and_parity():
    w = workload_c2()
    A = w["A"]
    p = C.csrk_tune(A.n, A.nnz, "mi355x")
    say("c2 full", p)
    M = _build(A, "f64", p)
    ones = np.ones(A.n)
    y1, perm = _run(M, ones)
    nb = A.meta["dims"][0]
    z, yy, xx = np.meshgrid(np.arange(nb), np.arange(nb), np.arange(nb), indexing="ij")
    cnt = ((xx > 0).astype(int) + (xx < nb - 1) + (yy > 0) + (yy < nb - 1) + (z > 0) + (z < nb - 1)).ravel()
    exact = (6.0 - cnt)[A.meta["perm0"]]
    assert np.array_equal(y1, exact[perm])
    x = w["x"]
    y, perm = _run(M, x)
    rel = check_forward(y, A, x, perm, "f64", False, label="c2")
    say("c2 max rel err", rel)
    # determinism: a second launch is bitwise identical
    y2, _ = _run(M, x)
    assert np.array_equal(y, y2)
    # plain-CSR baseline kernel on the same arrays
    yp, _ = _run(M, x, plain=True)
    check_forward(yp, A, x, perm, "f64", False, label="c2 plain")


@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
def test_c3_full_precisions(store):
    w = workload_c3()
    A, x = w["A"], w["x"]
    p = C.csrk_tune(A.n, A.nnz, "mi355x")
    say("c3 full", store, p)
    M = _build(A, store, p)
    y, perm = _run(M, x)
    rel = check_forward(y, A, x, perm, store, store != "f64", label=f"c3 {store}")
    say("c3", store, "max rel err", rel)


def test_c4_full_f32():
    w = workload_c4()
    A, x = w["A"], w["x"]
    p = C.csrk_tune(A.n, A.nnz, "mi355x")
    say("c4 full", p)
    M = _build(A, "f32", p)
    y, perm = _run(M, x)
    check_forward(y, A, x, perm, "f32", False, label="c4")


@pytest.mark.parametrize("nrhs", [2, 3, 8, 65])
@pytest.mark.parametrize("store", ["f64", "f32"])
def test_multi_rhs(nrhs, store):
    A = random_sparse(2000, 7.0, seed=nrhs, empty_row_frac=0.05)
    X = np.random.default_rng(nrhs).uniform(-1, 1, (A.n, nrhs))
    if store != "f64":
        X = X.astype(np.float32).astype(np.float64)
    say("mrhs", nrhs, store)
    M = _build(A, store, params(21, 4, lanes=1))
    Y, perm = _run(M, X)
    check_forward(Y, A, X, perm, store, False, label=f"nrhs={nrhs}")
    Yp, _ = _run(M, X, plain=True)
    check_forward(Yp, A, X, perm, store, False, label=f"plain nrhs={nrhs}")


def test_vals_override_and_permute_roundtrip():
    A = random_sparse(1500, 5.0, seed=21)
    x = np.random.default_rng(21).uniform(-1, 1, A.n)
    M = _build(A, "f64", params(11, 3))
    s = M.structure()
    # pass doubled values explicitly (CSR-k order)
    v2 = to_dev(2.0 * s["vals"], torch.float64)
    xd = M.to_permuted(to_dev(x, torch.float64))
    assert np.array_equal(xd.cpu().numpy(), x[s["perm"]])
    y = M.spmv(xd, vals=v2)
    back = M.from_permuted(y)
    torch.cuda.synchronize()
    check_forward(back.cpu().numpy(), A, x, np.arange(A.n), "f64", False, vals=2.0 * A.vals, label="vals override")
    # multi-column permute round trip, 4-byte elements
    X = np.random.default_rng(0).uniform(-1, 1, (A.n, 3)).astype(np.float32)
    Xd = to_dev(X, torch.float32)
    assert np.array_equal(M.from_permuted(M.to_permuted(Xd)).cpu().numpy(), X)


def test_bf16_values_are_round_to_nearest_even():
    A = random_sparse(800, 4.0, seed=2)
    M = _build(A, "bf16", params(8, 2))
    s = M.structure()
    got = M.values().view(torch.int16).cpu().numpy().view(np.uint16)
    want = OP.f32_to_bf16_bits(OP.to_f32(s["vals"]))
    assert np.array_equal(got, want)
    M32 = _build(A, "f32", params(8, 2))
    assert np.array_equal(M32.values().cpu().numpy(), OP.to_f32(s["vals"]))


def test_argument_errors():
    A = random_sparse(100, 3.0, seed=1)
    M = _build(A, "f64", params(8, 2))
    x = to_dev(np.zeros(A.n), torch.float64)
    y = to_dev(np.zeros(A.n), torch.float64)
    v = to_dev(np.zeros(A.nnz + 2), torch.float64)
    # every call below is rejected on the host before any launch
    with pytest.raises(C.CsrkError) as e:
        C.csrk_spmv(M.handle, None, x.data_ptr(), x.data_ptr(), 1, None)
    assert e.value.name == "CSRK_ERR_ARG"  # y aliases x
    with pytest.raises(C.CsrkError) as e:
        C.csrk_spmv(M.handle, None, x.data_ptr(), None, 1, None)
    assert e.value.name == "CSRK_ERR_ARG"  # null y
    with pytest.raises(C.CsrkError) as e:
        C.csrk_spmv(M.handle, v.data_ptr() + 8, x.data_ptr(), y.data_ptr(), 1, None)
    assert e.value.name == "CSRK_ERR_ARG"  # misaligned values
    with pytest.raises(C.CsrkError) as e:
        C.csrk_spmv(M.handle, None, x.data_ptr(), y.data_ptr(), 0, None)
    assert e.value.name == "CSRK_ERR_ARG"  # nrhs < 1
    with pytest.raises(TypeError):
        M.spmv(x.float())


def _long_row_matrix(n=3000, long_len=2000, every=89, seed=3):
    from gen import CsrInput
    rng = np.random.default_rng(seed)
    rows = [np.sort(rng.choice(n, size=(long_len if i % every == 0 else int(rng.integers(0, 9))), replace=False))
            for i in range(n)]
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    return CsrInput("long", n, rp.astype(np.int32), np.concatenate(rows).astype(np.int32),
                    rng.uniform(-1, 1, int(rp[-1])), {})


@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nrhs", [4, 8])
def test_multi_rhs_long_rows(store, nrhs):
    A = _long_row_matrix()
    X = np.random.default_rng(nrhs).uniform(-1, 1, (A.n, nrhs))
    if store != "f64":
        X = X.astype(np.float32).astype(np.float64)
    say("mrhs long rows", store, nrhs)
    M = _build(A, store, params(16, 4))
    Y, perm = _run(M, X)
    check_forward(Y, A, X, perm, store, False, label=f"long mrhs {store} {nrhs}")


def test_multi_rhs_misaligned_block_uses_scalar_columns():
    A = random_sparse(1200, 6.0, seed=44)
    X = np.random.default_rng(44).uniform(-1, 1, (A.n, 8)).astype(np.float32).astype(np.float64)
    M = _build(A, "f32", params(16, 4))
    perm = M.structure()["perm"]
    # a block starting 4 bytes into an allocation: 16-byte column slices are not aligned
    raw = torch.zeros(A.n * 8 + 1, dtype=torch.float32, device="cuda")
    raw[1:] = to_dev(X[perm], torch.float32).reshape(-1)
    xd = raw[1:].view(A.n, 8)
    assert xd.data_ptr() % 16 != 0
    yraw = torch.zeros(A.n * 8 + 1, dtype=torch.float32, device="cuda")
    yd = yraw[1:].view(A.n, 8)
    M.spmv(xd, yd)
    torch.cuda.synchronize()
    check_forward(yd.double().cpu().numpy(), A, X, perm, "f32", False, label="misaligned mrhs")
    # the aligned launch gives the same numbers up to summation order (bitwise: same order)
    y2 = M.spmv(to_dev(X[perm], torch.float32).contiguous())
    torch.cuda.synchronize()
    assert torch.equal(y2, yd)


def test_value_array_beyond_2gib():
    """3D 7-point Laplacian on 340^3 points: 274 M nonzeros, so the FP64 value array (2.2 GB) and every
    byte offset past 2^31 are exercised.  A.1 and the adjoint at ones are exact small integers (checked
    bitwise on every row); a random x is checked against the oracle on sampled rows."""
    from gen import laplacian
    from oracle import spmv as OS
    A = laplacian((340, 340, 340), "3d7", 6.0)
    assert A.nnz * 8 > 2 ** 31
    p = C.csrk_tune(A.n, A.nnz, "mi355x")
    p["reorder"] = "none"  # the input order is already banded; this keeps the host build short
    say("2 GiB values", A.n, A.nnz, p)
    M = _build(A, "f64", p)
    deg = np.diff(A.row_ptr).astype(np.float64)
    exact = 7.0 - deg  # 6 - (number of neighbours), and the row holds the diagonal plus its neighbours
    ones = torch.ones(A.n, dtype=torch.float64, device="cuda")
    y = M.from_permuted(M.spmv(M.to_permuted(ones)))
    assert np.array_equal(y.cpu().numpy(), exact)
    gx, gv = M.adjoint(M.to_permuted(ones), M.to_permuted(ones))
    assert np.array_equal(M.from_permuted(gx).cpu().numpy(), exact)  # symmetric: A^T 1 = A 1
    assert bool(torch.all(gv == 1.0))
    del gx, gv
    rng = np.random.default_rng(340)
    x = rng.uniform(-1, 1, A.n)
    yd = M.from_permuted(M.spmv(M.to_permuted(to_dev(x, torch.float64)))).cpu().numpy()
    rows = np.sort(rng.choice(A.n, 4000, replace=False))
    rows = np.concatenate([rows, [0, A.n - 1]])
    lo, hi = A.row_ptr[rows].astype(np.int64), A.row_ptr[rows + 1].astype(np.int64)
    idx = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
    rp = np.concatenate([[0], np.cumsum(hi - lo)])
    ref = OS.spmv(rp, A.col_idx[idx], A.vals[idx], x)
    scale = OS.row_abs_sum(rp, A.col_idx[idx], A.vals[idx], x)
    assert np.all(np.abs(yd[rows] - ref) <= 1e-12 * scale)


@pytest.mark.parametrize("in_dtype,store", [("f32", "f32"), ("bf16", "bf16"), ("f32", "bf16"), ("bf16", "f64")])
def test_build_from_reduced_precision_input(in_dtype, store):
    """Values handed over as FP32 or BF16 (in_dtype) are stored as if they had come in FP64: the device values
    equal those of an FP64 build of the same numbers, and the storage type's rounding of them."""
    A = random_sparse(2000, 6.0, seed=41, empty_row_frac=0.05)
    v64 = OP.stored_values(A.vals, in_dtype)
    v_in = v64.astype(np.float32) if in_dtype == "f32" else \
        (v64.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    p = params(16, 4, lanes=2, waves=4)
    say("input dtype", in_dtype, store)
    M = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, v_in, p, store, in_dtype=in_dtype), store)
    M64 = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, v64, p, store), store)
    a, b = M.values(), M64.values()
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int16) if store == "bf16" else a, b.view(torch.int16) if store == "bf16" else b)
    expect = OP.stored_values(v64, store)[M.structure()["vmap"]]
    assert np.array_equal(a.double().cpu().numpy(), expect)


def test_bandwidth_probes():
    """The read probe touches every 16-byte word once (the xor of its per-workgroup checksums is the xor of the
    buffer); the copy probe copies exactly; sizes must be multiples of 16."""
    n16 = 4096 * 256 * 4 * 2 + 12345  # whole unrolled sweeps plus a ragged tail
    g = torch.Generator(device="cuda").manual_seed(7)
    buf = torch.randint(-2 ** 31, 2 ** 31 - 1, (n16 * 4,), generator=g, device="cuda", dtype=torch.int64)
    buf = buf.to(torch.int32)
    part = torch.zeros(4096, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    C.csrk_probe_read(buf.data_ptr(), n16 * 16, part.data_ptr(), st)
    dst = torch.empty_like(buf)
    C.csrk_probe_copy(buf.data_ptr(), dst.data_ptr(), n16 * 16, st)
    torch.cuda.synchronize()
    assert torch.equal(dst, buf)
    words = buf.cpu().numpy().view(np.uint32)
    assert int(np.bitwise_xor.reduce(part.cpu().numpy().astype(np.uint64))) == int(np.bitwise_xor.reduce(words))
    with pytest.raises(C.CsrkError):
        C.csrk_probe_read(buf.data_ptr(), 24, part.data_ptr(), st)
    with pytest.raises(C.CsrkError):
        C.csrk_probe_copy(buf.data_ptr() + 4, dst.data_ptr(), 32, st)
