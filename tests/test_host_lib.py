"""CPU tests of libcsrk.so: exports, the size model, bit-exact structure vs the oracle, error statuses.

These call only host entry points (no GPU needed).
"""

import math
import os

import numpy as np
import pytest

from gen import laplacian, random_sparse, workload_c1, workload_c2, workload_c4
from oracle import bandk as OB
from oracle import stats as OS
from oracle import tune as OT
from paper_2203_05096_amd import _capi as C


@pytest.fixture(scope="module")
def lib():
    return C.lib()


def test_exports_every_header_symbol(lib):
    names = C.header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(C._SIGS), "binding and header disagree"


def test_status_strings(lib):
    for s, name in C.STATUS.items():
        assert C.csrk_status_string(s).startswith(name)
    assert C.csrk_status_string(2) == "unknown csrk_status"  # no status 2: non-square input is a column range error


def _golden_vectors(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "paper_tune_vectors.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line and not line.startswith("alt"):
                p = line.split()
                rows.append((float(p[0]), *map(int, p[1:])))
    return rows


def test_tune_paper_vectors(golden_dir):
    for r, case, vs, vr, as_, ar in _golden_vectors(golden_dir):
        n = 10 ** 6
        nnz = int(round(r * n))
        v = C.csrk_tune(n, nnz, "volta")
        a = C.csrk_tune(n, nnz, "ampere")
        assert (v["ssrs"], v["srs"]) == (vs, vr), r
        assert (a["ssrs"], a["srs"]) == (as_, ar), r


def test_tune_matches_oracle_over_range():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        n = int(rng.integers(1, 10 ** 6))
        nnz = int(rng.integers(1, 60 * n))
        for model in ("volta", "ampere"):
            p = C.csrk_tune(n, nnz, model)
            assert (p["ssrs"], p["srs"]) == OT.paper_tune(n, nnz, model)[:2], (n, nnz, model)


def test_tune_errors():
    for n, nnz in ((0, 5), (5, 0), (-1, 3)):
        with pytest.raises(C.CsrkError) as e:
            C.csrk_tune(n, nnz, "volta")
        assert e.value.name == "CSRK_ERR_ARG"
    with pytest.raises(C.CsrkError):
        C.csrk_tune(10, 10, 7)
    p = C.csrk_tune(4096, 20224, "mi355x")
    assert p["k"] == 3 and p["srs"] >= 1 and p["ssrs"] >= 1


def _path(n):
    rp, ci = [0], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
        rp.append(len(ci))
    return np.array(rp), np.array(ci)


def _params(srs, ssrs, reorder="bandk", k=3):
    return {"k": k, "srs": srs, "ssrs": ssrs, "lanes_per_row": 1, "waves_per_wg": 4, "reorder": reorder}


def _lib_structure(row_ptr, col_idx, vals, srs, ssrs, reorder="bandk", k=3):
    h = C.csrk_build_host(row_ptr, col_idx, vals, _params(srs, ssrs, reorder, k))
    try:
        return C.csrk_copy_structure(h), C.csrk_get_info(h)
    finally:
        C.csrk_destroy(h)


def _assert_same_as_oracle(A_rp, A_ci, A_vals, srs, ssrs, reorder="bandk", k=3):
    s, info = _lib_structure(A_rp, A_ci, A_vals, srs, ssrs, reorder, k)
    perm, sr_ptr, ssr_ptr = OB.build_grouping(A_rp, A_ci, srs, ssrs, reorder, k)
    rp2, ci2, v2, vmap = OB.apply_permutation(A_rp, A_ci, A_vals, perm)
    assert np.array_equal(s["perm"], perm)
    assert np.array_equal(s["sr_ptr"], sr_ptr)
    assert np.array_equal(s["ssr_ptr"], ssr_ptr)
    assert np.array_equal(s["row_ptr"], rp2)
    assert np.array_equal(s["col_idx"], ci2)
    assert np.array_equal(s["vals"].view(np.uint64), np.asarray(v2, dtype=np.float64).view(np.uint64))
    assert np.array_equal(s["vmap"], vmap)
    return s, info


def test_worked_example_path12(golden_dir):
    rp, ci = _path(12)
    s, _ = _assert_same_as_oracle(rp, ci, np.arange(len(ci), dtype=np.float64), 2, 2)
    assert s["perm"].tolist() == list(range(11, -1, -1))


@pytest.mark.parametrize("seed,sym,srs,ssrs,empty", [(0, True, 4, 3, 0.1), (1, False, 8, 2, 0.0),
                                                     (2, False, 3, 7, 0.3), (3, True, 1, 1, 0.0),
                                                     (4, False, 16, 16, 0.05), (5, True, 5, 1, 0.2),
                                                     (6, False, 64, 8, 0.0), (7, True, 2, 64, 0.5)])
def test_bitexact_random(seed, sym, srs, ssrs, empty):
    A = random_sparse(400, 4.0, seed=seed, empty_row_frac=empty, symmetric_pattern=sym)
    _assert_same_as_oracle(A.row_ptr, A.col_idx, A.vals, srs, ssrs)


@pytest.mark.parametrize("k,seed,sym,srs,ssrs", [(4, 0, True, 4, 3), (4, 1, False, 8, 2), (5, 2, False, 3, 3),
                                                 (6, 3, True, 2, 2), (8, 4, False, 2, 2), (4, 5, True, 1, 1)])
def test_bitexact_general_k(k, seed, sym, srs, ssrs):
    """CSR-k for k >= 4 (Section 2.2): Band-k with k - 1 coarsening levels, every level bit for bit with the
    oracle, including the levels above the super-super-row (csrk_level_ptr)."""
    A = random_sparse(500, 4.0, seed=seed, empty_row_frac=0.1, symmetric_pattern=sym)
    _assert_same_as_oracle(A.row_ptr, A.col_idx, A.vals, srs, ssrs, "bandk", k)
    up = OB.upper_levels(A.row_ptr, A.col_idx, srs, ssrs, "bandk", k)
    h = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, _params(srs, ssrs, "bandk", k))
    try:
        assert np.array_equal(C.csrk_level_ptr(h, 1), C.csrk_copy_structure(h)["sr_ptr"])
        for lvl, ref in enumerate(up, start=3):
            assert np.array_equal(C.csrk_level_ptr(h, lvl), ref)
        with pytest.raises(C.CsrkError):
            C.csrk_level_ptr(h, k)
        with pytest.raises(C.CsrkError):
            C.csrk_level_ptr(h, 0)
    finally:
        C.csrk_destroy(h)


def test_general_k_path16_golden(golden_dir):
    """The hand-derived k = 4 example (tests/golden/bandk_path16_k4.txt) through the library."""
    rp, ci = _path(16)
    s, _ = _assert_same_as_oracle(rp, ci, np.arange(len(ci), dtype=np.float64), 2, 2, "bandk", 4)
    assert s["perm"].tolist() == list(range(15, -1, -1))
    h = C.csrk_build_host(rp, ci, None, _params(2, 2, "bandk", 4))
    try:
        assert C.csrk_level_ptr(h, 3).tolist() == [0, 2, 4]
    finally:
        C.csrk_destroy(h)


@pytest.mark.parametrize("reorder", ["rcm", "none"])
def test_general_k_other_orders(reorder):
    A = random_sparse(300, 5.0, seed=19, empty_row_frac=0.1)
    _assert_same_as_oracle(A.row_ptr, A.col_idx, A.vals, 6, 3, reorder, 5)
    h = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, _params(6, 3, reorder, 5))
    try:
        for lvl, ref in enumerate(OB.upper_levels(A.row_ptr, A.col_idx, 6, 3, reorder, 5), start=3):
            assert np.array_equal(C.csrk_level_ptr(h, lvl), ref)
    finally:
        C.csrk_destroy(h)


def test_general_k_irregular_split_keeps_upper_levels():
    """On an irregular matrix the super-row split refines the SR and SSR levels; the level above the SSR keeps
    its row ranges (each of its units starts where it started, now counted in the new SSRs)."""
    from gen.irregular import rmat_matrix
    A = rmat_matrix(scale=12, edge_factor=8, seed=3)
    k, srs, ssrs = 4, 64, 2
    up = OB.upper_levels(A.row_ptr, A.col_idx, srs, ssrs, "bandk", k)[0]
    _, sr0, ssr0 = OB.build_grouping(A.row_ptr, A.col_idx, srs, ssrs, "bandk", k)
    h = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, _params(srs, ssrs, "bandk", k))
    try:
        s = C.csrk_copy_structure(h)
        lib_up = C.csrk_level_ptr(h, 3)
        assert len(s["sr_ptr"]) > len(sr0)  # the split happened
        rows_ref = sr0[ssr0[up]]
        rows_lib = s["sr_ptr"][s["ssr_ptr"][lib_up]]
        assert np.array_equal(rows_ref, rows_lib)
    finally:
        C.csrk_destroy(h)


def _union_reference(s):
    """The union-pattern layout built directly from its description (csrk_copy_union in include/csrk.h)."""
    rp, ci, srp = s["row_ptr"].astype(np.int64), s["col_idx"].astype(np.int64), s["sr_ptr"].astype(np.int64)
    n = len(rp) - 1
    pos = {}
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            pos[(i, int(ci[k]))] = k
    extras = [[] for _ in range(n)]  # row i: columns j with (j, i) in A' and (i, j) not
    for (i, j), k in pos.items():
        if (j, i) not in pos:
            extras[j].append((i, k))
    erow = np.zeros(n + 1, np.int64)
    for i in range(n):
        extras[i].sort()
        erow[i + 1] = erow[i] + len(extras[i])
    u_col, u_src, begin, end = [], [], [], []
    for t in range(len(srp) - 1):
        r0, r1 = srp[t], srp[t + 1]
        if r1 - r0 > 64 or (rp[r1] - rp[r0]) + (erow[r1] - erow[r0]) > 504:
            return None
        begin.append(len(u_col))
        for i in range(r0, r1):
            for k in range(rp[i], rp[i + 1]):
                u_col.append(int(ci[k]))
                u_src.append(pos.get((int(ci[k]), i), -1))
        for i in range(r0, r1):
            for j, k in extras[i]:
                u_col.append(j)
                u_src.append(k)
        end.append(len(u_col))
        while (len(u_col) - begin[-1] - (rp[r1] - rp[r0])) % 8:
            u_col.append(int(r0))
            u_src.append(-1)
    return {"u_col": u_col, "u_src": u_src, "erow_ptr": erow.tolist(), "sr_begin": begin, "sr_end": end}


@pytest.mark.parametrize("seed,srs,ssrs,sym", [(1, 8, 2, False), (2, 19, 4, False), (3, 48, 2, False),
                                               (4, 100, 2, False), (5, 16, 2, True)])
def test_union_index_layout(seed, srs, ssrs, sym):
    """The union pattern of a nonsymmetric A' (one-pass adjoint): every array as the layout describes it, or no
    union when the pattern is symmetric or a super-row does not fit one window."""
    A = random_sparse(700, 4.0, seed=seed, empty_row_frac=0.1, symmetric_pattern=sym)
    h = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, _params(srs, ssrs))
    try:
        s = C.csrk_copy_structure(h)
        got = C.csrk_copy_union(h)
    finally:
        C.csrk_destroy(h)
    ref = None if sym else _union_reference(s)
    if ref is None:
        assert got is None
        return
    assert got is not None
    for key in ("u_col", "u_src", "erow_ptr", "sr_begin", "sr_end"):
        assert got[key].tolist() == ref[key], key
    # the A' part of super-row t sits at a multiple-of-8 offset from its A' positions
    off = got["sr_begin"] - s["row_ptr"][s["sr_ptr"][:-1]]
    assert np.all(off % 8 == 0) and np.all(np.diff(off) >= 0)


@pytest.mark.parametrize("kind", ["bidiag", "lower", "holes"])
def test_union_index_structured(kind):
    """Hand-built nonsymmetric patterns (upper bidiagonal, dense lower triangle, rows reached only through
    their extras): the union layout exactly as described."""
    n = 40 if kind == "lower" else 150
    rows = []
    for i in range(n):
        if kind == "bidiag":
            rows.append([j for j in (i, i + 1) if j < n])
        elif kind == "lower":
            rows.append(list(range(i + 1)))
        else:
            rows.append([] if i % 3 == 1 else [j for j in (i, i + 1) if j < n])
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.array([j for r in rows for j in r], dtype=np.int32)
    h = C.csrk_build_host(rp, ci, np.ones(len(ci)), _params(8, 2))
    try:
        s = C.csrk_copy_structure(h)
        got = C.csrk_copy_union(h)
    finally:
        C.csrk_destroy(h)
    ref = _union_reference(s)
    assert ref is not None and got is not None
    for key in ("u_col", "u_src", "erow_ptr", "sr_begin", "sr_end"):
        assert got[key].tolist() == ref[key], key


def test_union_index_c4_fits():
    """The 2D 9-point matrix with 10% of its off-diagonals dropped gets a union at its tuned sizes."""
    A = workload_c4()["A"]
    h = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, C.csrk_tune(A.n, A.nnz, "mi355x"))
    try:
        u = C.csrk_copy_union(h)
        assert u is not None
        extras, nsr = int(u["erow_ptr"][-1]), len(u["sr_begin"])
        assert A.nnz + extras <= len(u["u_col"]) <= A.nnz + extras + 7 * nsr  # padding: < 8 per super-row
    finally:
        C.csrk_destroy(h)


def test_level_ptr_k2_and_k3():
    """k = 2 and 3 have levels 1 and 2 (for k = 2 level 2 is the launch grouping of the super-rows)."""
    A = random_sparse(400, 4.0, seed=21)
    for k in (2, 3):
        h = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, _params(7, 3, "bandk", k))
        try:
            s = C.csrk_copy_structure(h)
            assert np.array_equal(C.csrk_level_ptr(h, 1), s["sr_ptr"])
            assert np.array_equal(C.csrk_level_ptr(h, 2), s["ssr_ptr"])
            with pytest.raises(C.CsrkError):
                C.csrk_level_ptr(h, 3)
        finally:
            C.csrk_destroy(h)


def test_from_groups_rejects_k4():
    rp, ci = _path(8)
    with pytest.raises(C.CsrkError):
        C.csrk_build_from_groups(rp, ci, None, np.arange(8), [4, 4], [2], _params(4, 2, "bandk", 4))


@pytest.mark.parametrize("reorder", ["rcm", "none"])
def test_bitexact_other_orders(reorder):
    A = random_sparse(300, 5.0, seed=9, empty_row_frac=0.1)
    _assert_same_as_oracle(A.row_ptr, A.col_idx, A.vals, 6, 3, reorder)


def test_bitexact_c1_and_stats():
    A = workload_c1()["A"]
    for srs, ssrs in ((8, 8), (64, 8), (15, 7), (7, 15)):
        s, info = _assert_same_as_oracle(A.row_ptr, A.col_idx, A.vals, srs, ssrs)
    st = OS.row_stats(A.row_ptr)
    assert info["n"] == A.n and info["nnz"] == A.nnz
    assert abs(info["rdensity"] - st["r"]) < 1e-12 and abs(info["row_variance"] - st["var"]) < 1e-12
    assert info["max_row"] == st["max"] and info["symmetry"] == 1.0
    assert info["bandwidth"] == OB.bandwidth(s["row_ptr"], s["col_idx"])
    assert info["bandwidth_input"] == 64 and info["on_device"] == 0


def test_bitexact_medium_scrambled_3d():
    w = workload_c2(seed=3, side=24)
    A = w["A"]
    _assert_same_as_oracle(A.row_ptr, A.col_idx, A.vals, 14, 7)
    _assert_same_as_oracle(A.row_ptr, A.col_idx, A.vals, 64, 8)


def test_bitexact_nonsymmetric_drop():
    from gen import stencil_pattern, drop_offdiagonals
    rng = np.random.default_rng(4)
    rp, ci, dg = stencil_pattern((48, 40), "2d9")
    rp, ci, dg = drop_offdiagonals(rp, ci, dg, rng, 0.1)
    vals = rng.uniform(-1, 1, len(ci))
    _, info = _assert_same_as_oracle(rp, ci, vals, 18, 9)
    assert abs(info["symmetry"] - OS.pattern_symmetry(rp, ci)) < 1e-12


@pytest.mark.slow
def test_bitexact_c2_full_size():
    """The full 3D 7-point 128^3 scrambled workload: library vs oracle, bit for bit."""
    w = workload_c2()
    A = w["A"]
    p = C.csrk_tune(A.n, A.nnz, "mi355x")
    _assert_same_as_oracle(A.row_ptr, A.col_idx, A.vals, p["srs"], p["ssrs"])


def test_from_groups_fig1(golden_dir):
    # 9 rows, sizes of the paper's Fig. 1 example, identity ordering, tridiagonal pattern
    rp, ci = _path(9)
    h = C.csrk_build_from_groups(rp, ci, np.ones(len(ci)), np.arange(9), [2, 3, 2, 2], [2, 2], _params(1, 1))
    s = C.csrk_copy_structure(h)
    C.csrk_destroy(h)
    assert s["sr_ptr"].tolist() == [0, 2, 5, 7, 9] and s["ssr_ptr"].tolist() == [0, 2, 4]


def test_from_groups_errors():
    rp, ci = _path(5)
    bad = [([0, 1, 2, 3, 3], [2, 3], [2]), (np.arange(5), [2, 2], [2]), (np.arange(5), [2, 3], [1]),
           (np.arange(5), [0, 5], [2])]
    for perm, srz, ssrz in bad:
        with pytest.raises(C.CsrkError) as e:
            C.csrk_build_from_groups(rp, ci, None, perm, srz, ssrz, _params(1, 1))
        assert e.value.name == "CSRK_ERR_ARG"


@pytest.mark.parametrize("in_dtype", ["f32", "bf16"])
def test_build_input_dtypes_widen_exactly(in_dtype):
    """FP32 and BF16 input values are kept exactly in the FP64 master copy (same structure as an FP64 build)."""
    from oracle import precision as OP
    A = random_sparse(300, 5.0, seed=21, empty_row_frac=0.05)
    v64 = OP.stored_values(A.vals, in_dtype)  # the values representable in the input type, as float64
    if in_dtype == "f32":
        v_in = v64.astype(np.float32)
    else:
        v_in = (v64.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    h = C.csrk_build_host(A.row_ptr, A.col_idx, v_in, _params(8, 4), in_dtype=in_dtype)
    h64 = C.csrk_build_host(A.row_ptr, A.col_idx, v64, _params(8, 4))
    try:
        s, s64 = C.csrk_copy_structure(h), C.csrk_copy_structure(h64)
        for k in s:
            assert np.array_equal(s[k], s64[k]), k
        assert np.array_equal(s["vals"], v64[s["vmap"]])
    finally:
        C.csrk_destroy(h)
        C.csrk_destroy(h64)


# ---------------------------------------------------------------- the library's super-row budget
#
# For heavy irregular matrices the library cuts super-rows whose nonzeros exceed a budget into consecutive
# pieces (its own refinement for the GPU kernels; the paper leaves irregular load balance open).  The oracle
# does not model it; these tests check the library's output against the paper's grouping (the oracle's) by
# invariants, and against a hand-worked example.  The budget rule and the long-row threshold are the
# library's, as its header states them.

LIB_LONG_ROW = 1024


def _lib_budget(n, nnz, srs):
    return max(2048, -(-(4 * srs * nnz) // n))


def _lengths_matrix(lengths, n):
    """Row i holds lengths[i] distinct columns (row i itself first, then 0, 1, 2, ... skipping i)."""
    rows, cols = [], []
    for i, L in enumerate(lengths):
        c = [i] + [j for j in range(L + 1) if j != i][:L - 1] if L else []
        rows += [i] * len(c)
        cols += sorted(c)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(np.asarray(rows, np.int64), minlength=n), out=rp[1:])
    return rp.astype(np.int32), np.asarray(cols, np.int32)


def test_budget_split_worked_example():
    # SRS 8, SSRS 2, input order.  Rows 0..7 have 1000, 1000, 1000, 100, 1000, 3000, 1, 1 nonzeros; the other
    # 3992 rows one each: nnz = 11094, B = max(2048, ceil(4 * 8 * 11094 / 4000)) = 2048.  SR 0 costs
    # 4102 (the 3000-entry row is long and costs 0): greedy pieces {0,1} (2000), {2,3} (1100; row 4 would give
    # 2100), {4..7} (1002).  SSR 0 = SR 0 + SR 1 becomes 4 pieces, regrouped two at a time.
    n = 4000
    rp, ci = _lengths_matrix([1000, 1000, 1000, 100, 1000, 3000, 1, 1] + [1] * (n - 8), n)
    assert int(rp[-1]) == 11094 and _lib_budget(n, 11094, 8) == 2048
    s, _ = _lib_structure(rp, ci, None, 8, 2, "none")
    assert np.array_equal(s["perm"], np.arange(n))
    assert np.array_equal(s["sr_ptr"], OB.running_counts([2, 2, 4, 8] + [8] * 498))
    assert np.array_equal(s["ssr_ptr"], OB.running_counts([2, 2] + [2] * 249))


def _check_budget_refinement(A, srs, ssrs, reorder, k=3):
    """The library's grouping refines the oracle's: same permutation and matrix; super-rows only cut, each piece
    within the budget or a single row, greedy; every SSR start kept; pieces regrouped at most SSRS at a time."""
    s, info = _lib_structure(A.row_ptr, A.col_idx, A.vals, srs, ssrs, reorder, k)
    perm, sr0, ssr0 = OB.build_grouping(A.row_ptr, A.col_idx, srs, ssrs, reorder, k)
    rp2, ci2, v2, vmap = OB.apply_permutation(A.row_ptr, A.col_idx, A.vals, perm)
    assert np.array_equal(s["perm"], perm)
    assert np.array_equal(s["row_ptr"], rp2) and np.array_equal(s["col_idx"], ci2)
    assert np.array_equal(s["vals"].view(np.uint64), np.asarray(v2, dtype=np.float64).view(np.uint64))
    assert np.array_equal(s["vmap"], vmap)
    sr, ssr = s["sr_ptr"].astype(np.int64), s["ssr_ptr"].astype(np.int64)
    budget = _lib_budget(A.n, A.nnz, srs)
    L = np.diff(A.row_ptr.astype(np.int64))[perm]
    cost = np.where(L > LIB_LONG_ROW, 0, L)
    c = np.concatenate([[0], np.cumsum(cost)])
    sr_cost = c[sr[1:]] - c[sr[:-1]]
    assert sr[0] == 0 and sr[-1] == A.n and ssr[0] == 0 and ssr[-1] == len(sr) - 1
    assert np.all((sr_cost <= budget) | (np.diff(sr) == 1))
    assert np.all(np.diff(sr) >= 1) and np.all(np.diff(sr) <= srs)
    assert set(sr0.tolist()) <= set(sr.tolist())  # pieces only cut existing super-rows
    assert set(sr0[ssr0].tolist()) <= set(sr[ssr].tolist())  # every SSR start (in rows) is kept
    assert np.all(np.diff(ssr) >= 1) and np.all(np.diff(ssr) <= ssrs)
    ends = set(sr0.tolist())
    for t in range(len(sr) - 1):  # greedy: a piece plus the next row of its super-row would exceed the budget
        b = int(sr[t + 1])
        if b not in ends:
            assert sr_cost[t] + cost[b] > budget
    # a super-row of the oracle's grouping within the budget is never cut
    c0 = c[sr0[1:]] - c[sr0[:-1]]
    kept = set(zip(sr0[:-1][c0 <= budget].tolist(), sr0[1:][c0 <= budget].tolist()))
    assert kept <= set(zip(sr[:-1].tolist(), sr[1:].tolist()))
    # the product through the refined structure equals plain CSR of the input
    from oracle import spmv as OSP
    x = np.random.default_rng(1).uniform(-1, 1, A.n)
    y2, visits = OSP.spmv_csrk_traversal(s["ssr_ptr"], s["sr_ptr"], s["row_ptr"], s["col_idx"], s["vals"], x[perm])
    assert np.all(visits == 1)
    y = np.empty(A.n)
    y[perm] = y2
    ref = OSP.spmv(A.row_ptr, A.col_idx, A.vals, x)
    assert np.all(np.abs(y - ref) <= 1e-12 * OSP.row_abs_sum(A.row_ptr, A.col_idx, A.vals, x))
    return s, info, sr0


@pytest.mark.parametrize("reorder", ["bandk", "rcm", "none"])
@pytest.mark.parametrize("symmetric", [True, False])
def test_irregular_budget_split_refines_oracle_grouping(reorder, symmetric):
    """R-MAT rows (power-law lengths): heavy super-rows are cut by the library's nonzero budget."""
    from gen.irregular import rmat_matrix
    A = rmat_matrix(13, 6.0, 17, symmetric=symmetric)
    s, info, sr0 = _check_budget_refinement(A, 64, 4, reorder)
    assert info["nsr"] > len(sr0) - 1  # at least one super-row was split


@pytest.mark.parametrize("seed,sym,srs,group", [(0, True, 4, 3), (1, False, 8, 2), (3, True, 1, 1),
                                                (6, False, 64, 8), (7, True, 2, 64)])
def test_bitexact_csr2(seed, sym, srs, group):
    A = random_sparse(400, 4.0, seed=seed, empty_row_frac=0.1, symmetric_pattern=sym)
    _assert_same_as_oracle(A.row_ptr, A.col_idx, A.vals, srs, group, k=2)


def test_bitexact_csr2_irregular_and_3d():
    from gen.irregular import rmat_matrix
    A = rmat_matrix(12, 6.0, 4, symmetric=False)
    _check_budget_refinement(A, 32, 4, "bandk", k=2)
    L = laplacian((12, 11, 10), "3d7", 6.0)
    _assert_same_as_oracle(L.row_ptr, L.col_idx, L.vals, 16, 2, k=2)


def test_info_counts_long_rows():
    from gen.irregular import rmat_matrix
    A = rmat_matrix(14, 8.0, 3, symmetric=True)
    h = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, None)
    try:
        info = C.csrk_get_info(h)
        expect = int((np.diff(A.row_ptr) > 1024).sum())
        assert expect > 0 and info["long_rows"] == expect and info["max_row"] == int(np.diff(A.row_ptr).max())
    finally:
        C.csrk_destroy(h)


def test_validation_statuses():
    rp, ci = _path(6)
    rp = np.asarray(rp)
    ci = np.asarray(ci)
    bad_start = rp.copy()
    bad_start[0] = 1
    decreasing = rp.copy()
    decreasing[3] = decreasing[2] - 1
    cases = [
        (bad_start, ci, "CSRK_ERR_BAD_ROWPTR"),
        (decreasing, ci, "CSRK_ERR_BAD_ROWPTR"),
        (rp, np.r_[ci[:-1], 6], "CSRK_ERR_COL_RANGE"),
        (rp, np.r_[ci[:-1], -1], "CSRK_ERR_COL_RANGE"),
        (rp, np.r_[ci[:2], ci[1], ci[3:]], "CSRK_ERR_DUPLICATE"),
    ]
    for r, c, status in cases:
        with pytest.raises(C.CsrkError) as e:
            C.csrk_build_host(r, c, None, _params(2, 2))
        assert e.value.name == status, (r, c)
    # row_ptr[n] != nnz, through the raw entry point
    import ctypes
    r32 = np.ascontiguousarray(rp, np.int32)
    c32 = np.ascontiguousarray(ci, np.int32)
    h = ctypes.c_void_p()
    st = C.lib().csrk_build_host(6, len(ci) + 1, r32.ctypes.data_as(C._i32p), c32.ctypes.data_as(C._i32p), None,
                                 C.F64, None, ctypes.byref(h))
    assert C.STATUS[st] == "CSRK_ERR_BAD_ROWPTR"
    st = C.lib().csrk_build_host(6, len(ci), None, c32.ctypes.data_as(C._i32p), None, C.F64, None, ctypes.byref(h))
    assert C.STATUS[st] == "CSRK_ERR_ARG"
    v = np.ones(len(ci))
    st = C.lib().csrk_build_host(6, len(ci), r32.ctypes.data_as(C._i32p), c32.ctypes.data_as(C._i32p), v.ctypes.data,
                                 7, None, ctypes.byref(h))
    assert C.STATUS[st] == "CSRK_ERR_ARG" and "dtype" in C.csrk_last_error_detail()
    with pytest.raises(C.CsrkError) as e:
        C.csrk_build_host(rp, ci, None, _params(0, 2))
    assert e.value.name == "CSRK_ERR_ARG"
    with pytest.raises(C.CsrkError) as e:
        C.csrk_build_host(rp, ci, None, dict(_params(2, 2), lanes_per_row=3))
    assert e.value.name == "CSRK_ERR_ARG"
    assert "lanes_per_row" in C.csrk_last_error_detail()


def test_unsorted_columns_accepted():
    rp, ci = _path(10)
    ci2 = ci.copy()
    for i in range(10):  # reverse each row
        ci2[rp[i]:rp[i + 1]] = ci[rp[i]:rp[i + 1]][::-1]
    vals = np.arange(len(ci), dtype=np.float64)
    vals2 = vals.copy()
    for i in range(10):
        vals2[rp[i]:rp[i + 1]] = vals[rp[i]:rp[i + 1]][::-1]
    a, _ = _lib_structure(rp, ci, vals, 3, 2)
    b, _ = _lib_structure(rp, ci2, vals2, 3, 2)
    for k in ("perm", "row_ptr", "col_idx", "vals", "sr_ptr", "ssr_ptr"):
        assert np.array_equal(a[k], b[k]), k


def test_empty_and_degenerate():
    h = C.csrk_build_host(np.zeros(1, np.int32), np.zeros(0, np.int32), None, _params(4, 4))
    info = C.csrk_get_info(h)
    assert info["n"] == 0 and info["nsr"] == 0 and info["nssr"] == 0
    C.csrk_destroy(h)
    # a single row without entries
    h = C.csrk_build_host(np.zeros(2, np.int32), np.zeros(0, np.int32), None, _params(4, 4))
    s = C.csrk_copy_structure(h)
    assert s["sr_ptr"].tolist() == [0, 1] and s["ssr_ptr"].tolist() == [0, 1]
    C.csrk_destroy(h)
    # diagonal matrix: no graph edges
    n = 33
    _assert_same_as_oracle(np.arange(n + 1), np.arange(n), np.linspace(1, 2, n), 4, 3)


def test_device_calls_need_device_arrays():
    rp, ci = _path(8)
    h = C.csrk_build_host(rp, ci, np.ones(len(ci)), _params(2, 2))
    with pytest.raises(C.CsrkError) as e:
        C.csrk_spmv(h, None, 1 << 20, 2 << 20, 1, None)
    assert e.value.name == "CSRK_ERR_UNSUPPORTED"
    with pytest.raises(C.CsrkError) as e:
        C.csrk_device_vals(h)
    assert e.value.name == "CSRK_ERR_UNSUPPORTED"
    C.csrk_destroy(h)


def test_upload_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rp, ci = _path(8)
    with pytest.raises(C.CsrkError) as e:
        C.csrk_build(rp, ci, np.ones(len(ci)), _params(2, 2), "f64")
    assert e.value.name == "CSRK_ERR_DEVICE"


def test_mi355x_model_shape():
    import math
    from paper_2203_05096_amd import autotune as T
    assert [T.snap_srs(v) for v in (-5, 1, 2, 3, 5, 7, 10, 14, 28, 40, 52, 57, 61, 71, 80, 81)] == \
        [1, 1, 2, 3, 4, 6, 8, 12, 24, 32, 48, 64, 64, 64, 64, 96]
    assert T.snap_srs(5, floor=7) == 8 and T.snap_srs(3, floor=3) == 3 and T.snap_srs(-40, floor=10) == 12
    for r in (1.0, 2.2, 4.9375, 6.953125, 8.19, 13.7, 26.46, 80.0, 300.0, 1000.0):
        n = 10 ** 6
        p = C.csrk_tune(n, int(round(r * n)), "mi355x")
        srs = T.snap_srs(math.floor(124.21 - 32.80 * math.log(r) + 0.5), math.ceil(256.0 / r))
        assert (p["srs"], p["ssrs"], p["waves_per_wg"]) == (srs, 2, 2), r
        assert p["lanes_per_row"] == (1 if r <= 6 else 2 if r <= 24 else 4 if r <= 48 else 8 if r <= 96 else 16)
        assert p["reorder"] == 0 and p["k"] == 3


def test_autotune_fit_and_evaluate():
    from paper_2203_05096_amd import autotune as T
    res = []
    for name, r, srs, ssrs in (("a", 5.0, 64, 2), ("b", 10.0, 48, 3), ("c", 25.0, 32, 4)):
        sr = T.SweepResult(name, 1000, int(1000 * r), r)
        for s_ in (16, 32, 48, 64):
            for ss in (2, 3, 4):
                sr.trials.append(T.Trial(s_, ss, 1, ss, "bandk", 10.0 + abs(s_ - srs) + 5 * abs(ss - ssrs)))
        res.append(sr)
    f = T.fit(res)
    a, b = f["srs"]
    assert abs((a - b * math.log(5.0)) - 64) < 6 and b > 0
    ev = T.evaluate(res, f)
    assert all(e["ratio"] >= 1.0 for e in ev) and ev[0]["model_srs"] in (48, 64)
    assert all(e["model_ssrs"] in (2, 4) for e in ev)


def test_tune_rhs():
    for n, nnz in ((4096, 20224), (10 ** 6, 26463592), (2097152, 14581760)):
        one = C.csrk_tune(n, nnz, "mi355x")
        assert C.csrk_tune_rhs(n, nnz, 1, "mi355x") == one
        many = C.csrk_tune_rhs(n, nnz, 8, "mi355x")
        # half the one-column super-row, snapped to the {2^i, 1.5 * 2^i} set, four per workgroup
        half = one["srs"] // 2
        snapped = min((c for i in range(12) for c in (2 ** i, 3 * 2 ** i // 2) if c >= 1),
                      key=lambda c: (abs(c - half), c))
        assert (many["srs"], many["lanes_per_row"]) == (snapped, one["lanes_per_row"])
        assert many["ssrs"] == many["waves_per_wg"] == 4
        assert C.csrk_tune_rhs(n, nnz, 8, "ampere") == C.csrk_tune(n, nnz, "ampere")
    with pytest.raises(C.CsrkError) as e:
        C.csrk_tune_rhs(100, 500, 0, "mi355x")
    assert e.value.name == "CSRK_ERR_ARG"


def test_autotune_helpers_match_library_model():
    from paper_2203_05096_amd import autotune as T
    assert [T.nearest_pow2(v) for v in range(0, 13)] == [1, 1, 2, 2, 4, 4, 4, 8, 8, 8, 8, 8, 8]
    assert T.nearest_pow2(24) == 16 and T.nearest_pow2(25) == 32
    for r in (1.0, 5.0, 6.0, 6.01, 13.7, 24.0, 24.5, 48.0, 60.0, 96.0, 97.0, 400.0):
        n = 100000
        p = C.csrk_tune(n, int(round(r * n)), "mi355x")
        assert p["lanes_per_row"] == T.lanes_rule(int(round(r * n)) / n), r


def test_spmv_host_matches_oracle_bitwise():
    """The CPU kernel sums each row left to right, as the oracle does: bitwise equal results."""
    from oracle import spmv as OS
    from gen.irregular import rmat_matrix
    for A, p in ((random_sparse(3000, 6.0, seed=41, empty_row_frac=0.1), _params(16, 4)),
                 (rmat_matrix(12, 4.0, 5), _params(32, 2)),
                 (random_sparse(500, 3.0, seed=42), _params(8, 3, k=2))):
        h = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, p)
        try:
            s = C.csrk_copy_structure(h)
            x = np.random.default_rng(43).uniform(-1, 1, A.n)
            for threads in (1, 3, 0):
                y = C.csrk_spmv_host(h, x[s["perm"]], nthreads=threads)
                ref = OS.spmv(s["row_ptr"], s["col_idx"], s["vals"], x[s["perm"]])
                assert np.array_equal(y.view(np.uint64), ref.view(np.uint64))
        finally:
            C.csrk_destroy(h)
    assert C.STATUS[C.lib().csrk_spmv_host(None, None, None, 0)] == "CSRK_ERR_ARG"


# ---------------------------------------------------------------- host CPU tuning (CSR-2, Section 4.2)

def test_host_cpu_constant_time_model():
    """The paper's constant-time CPU choice: CSR-2 with SRS = 96 for every matrix; ssrs 1 (a super-row is one
    unit of the host kernel's parallel loop)."""
    for n, nnz in ((10, 10), (4096, 20224), (2097152, 14581760), (10 ** 6, 80 * 10 ** 6)):
        p = C.csrk_tune(n, nnz, "host_cpu")
        assert (p["k"], p["srs"], p["ssrs"], p["reorder"]) == (2, 96, 1, 0)
    with pytest.raises(C.CsrkError):
        C.csrk_tune(0, 5, "host_cpu")


def test_host_sweep_set_and_sweep():
    from paper_2203_05096_amd import host_tune as HT
    paper = [8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 3072]
    assert HT.srs_set_cpu() == paper == OT.sweep_set_cpu()
    A = laplacian((30, 30, 20), "3d7", 6.0)
    r = HT.sweep_host(A, srs_list=[8, 96, 384], reps=3, warmup=1, nthreads=2)
    assert [s for s, _ in r["trials"]] == [8, 96, 384]
    assert r["best_us"] == min(us for _, us in r["trials"]) and r["constant_time_srs"] == 96
    assert r["constant_time_us"] == dict(r["trials"])[96] and r["constant_over_best"] >= 1.0
    # every swept structure computes the same product (CSR-2 built with the host parameters)
    x = np.random.default_rng(3).uniform(-1, 1, A.n)
    from oracle import spmv as OSP
    ref = OSP.spmv(A.row_ptr, A.col_idx, A.vals, x)
    for srs in (8, 3072):
        h = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, HT.host_params(srs))
        try:
            s = C.csrk_copy_structure(h)
            assert np.all(np.diff(s["ssr_ptr"]) == 1)  # one super-row per parallel unit
            y = np.empty(A.n)
            y[s["perm"]] = C.csrk_spmv_host(h, x[s["perm"]], nthreads=3)
            assert np.all(np.abs(y - ref) <= 1e-12 * OSP.row_abs_sum(A.row_ptr, A.col_idx, A.vals, x))
        finally:
            C.csrk_destroy(h)
