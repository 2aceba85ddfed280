"""Pins of the Band-k (BandK-v1) and grouping oracle."""

import os

import numpy as np
import pytest

from gen import laplacian, random_sparse, workload_c1
from oracle import bandk as B
from oracle import spmv as O


def _read_golden(path):
    out = {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            out[key] = [int(v) for v in vals]
    return out


def _path(n):
    rp, ci = [0], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
        rp.append(len(ci))
    return np.array(rp), np.array(ci)


def _star(leaves):
    """Vertex 0 joined to 1..leaves."""
    n = leaves + 1
    rows = [[0] + list(range(1, n))] + [[0, i] for i in range(1, n)]
    rp = np.cumsum([0] + [len(r) for r in rows])
    return rp, np.concatenate([sorted(r) for r in rows])


def test_fig1_pointer_encoding(golden_dir):
    g = _read_golden(os.path.join(golden_dir, "fig1_pointers.txt"))
    sr_ptr, ssr_ptr = B.group_from_sizes(g["sr_sizes"], g["ssr_sizes"])
    assert sr_ptr.tolist() == g["sr_ptr"]
    assert ssr_ptr.tolist() == g["ssr_ptr"]
    assert len(ssr_ptr) - 1 == g["num_ssr"][0]


def test_worked_example_path12(golden_dir):
    g = _read_golden(os.path.join(golden_dir, "bandk_path12.txt"))
    rp, ci = _path(g["n"][0])
    perm, sr_ptr, ssr_ptr = B.bandk_v1(rp, ci, g["srs"][0], g["ssrs"][0])
    assert perm.tolist() == g["perm"]
    assert sr_ptr.tolist() == g["sr_ptr"]
    assert ssr_ptr.tolist() == g["ssr_ptr"]


def test_cm_star_by_hand():
    # degrees: centre 4, leaves 1.  Start = leaf 1 (smallest degree, then id);
    # then the centre; then leaves 2, 3, 4 (equal weight and degree -> by id).
    rp, ci = _star(4)
    G = B.graph_from_csr(rp, ci)
    assert B.cuthill_mckee(G) == [1, 0, 2, 3, 4]
    assert B.reverse_cuthill_mckee(G) == [4, 3, 2, 0, 1]


def test_cm_prefers_heavier_edges():
    # weighted graph by hand: 0-1 (w1), 0-2 (w5), 0-3 (w3); degrees 3,1,1,1
    G = B.LevelGraph(4, np.array([0, 3, 4, 5, 6]), np.array([1, 2, 3, 0, 0, 0]),
                     np.array([1, 5, 3, 1, 5, 3]), np.arange(4))
    # start = vertex 1 (degree 1, lowest id), then 0, then 0's neighbours by weight: 2 (5), 3 (3)
    assert B.cuthill_mckee(G) == [1, 0, 2, 3]


def test_quotient_weights_by_hand():
    # 2x4 grid, x fastest: rows 0..3 on y=0, 4..7 on y=1; aggregates {0,1,4,5} and {2,3,6,7}
    L = laplacian((4, 2), "2d5", 4.0)
    G = B.graph_from_csr(L.row_ptr, L.col_idx)
    agg = np.array([0, 0, 1, 1, 0, 0, 1, 1])
    Q = B.quotient(G, agg, np.array([0, 2]))
    # crossing fine edges: 1-2 and 5-6 -> weight 2
    assert Q.n == 2 and Q.adj.tolist() == [1, 0] and Q.wgt.tolist() == [2, 2]


def test_apply_permutation_by_hand():
    # A = [[1,2,0],[0,3,4],[5,0,6]]; perm (new->old) = [2,0,1]
    rp = np.array([0, 2, 4, 6])
    ci = np.array([0, 1, 1, 2, 0, 2])
    va = np.array([1., 2., 3., 4., 5., 6.])
    r2, c2, v2, vm = B.apply_permutation(rp, ci, va, [2, 0, 1])
    # A'[i',j'] = A[p[i'], p[j']]: row0 = old row2 -> (old col0 -> new 1, old col2 -> new 0) = [(0,6),(1,5)]
    # row1 = old row0: cols 0->1, 1->2 = [(1,1),(2,2)]; row2 = old row1: cols 1->2, 2->0 = [(0,4),(2,3)]
    assert r2.tolist() == [0, 2, 4, 6]
    assert c2.tolist() == [0, 1, 1, 2, 0, 2]
    assert v2.tolist() == [6., 5., 1., 2., 4., 3.]
    assert vm.tolist() == [5, 4, 0, 1, 3, 2]


def test_unit_sizes_reduce_to_rcm():
    A = workload_c1()["A"]
    perm, sr_ptr, ssr_ptr = B.bandk_v1(A.row_ptr, A.col_idx, 1, 1)
    rcm = B.reverse_cuthill_mckee(B.graph_from_csr(A.row_ptr, A.col_idx))
    assert perm.tolist() == rcm
    assert sr_ptr.tolist() == list(range(A.n + 1))
    assert ssr_ptr.tolist() == list(range(A.n + 1))


def _check_structure(n, perm, sr_ptr, ssr_ptr, srs, ssrs):
    assert sorted(perm.tolist()) == list(range(n))
    assert sr_ptr[0] == 0 and sr_ptr[-1] == n
    assert ssr_ptr[0] == 0 and ssr_ptr[-1] == len(sr_ptr) - 1
    if n:
        assert np.all(np.diff(sr_ptr) >= 1) and np.all(np.diff(sr_ptr) <= srs)
        assert np.all(np.diff(ssr_ptr) >= 1) and np.all(np.diff(ssr_ptr) <= ssrs)


@pytest.mark.parametrize("seed,sym,srs,ssrs", [(0, True, 4, 3), (1, False, 8, 2), (2, False, 3, 7),
                                               (3, True, 1, 5), (4, False, 16, 16), (5, True, 5, 1)])
def test_invariants_random(seed, sym, srs, ssrs):
    A = random_sparse(300, 3.0, seed=seed, empty_row_frac=0.1, symmetric_pattern=sym)
    perm, sr_ptr, ssr_ptr = B.bandk_v1(A.row_ptr, A.col_idx, srs, ssrs)
    _check_structure(A.n, perm, sr_ptr, ssr_ptr, srs, ssrs)
    r2, c2, v2, vm = B.apply_permutation(A.row_ptr, A.col_idx, A.vals, perm)
    x = np.random.default_rng(seed).uniform(-1, 1, A.n)
    y_perm = O.spmv(r2, c2, v2, x[perm])
    y = O.spmv(A.row_ptr, A.col_idx, A.vals, x)
    scale = O.row_abs_sum(A.row_ptr, A.col_idx, A.vals, x)
    assert np.all(np.abs(y_perm - y[perm]) <= 1e-12 * scale[perm])
    assert np.array_equal(A.vals[vm], v2)
    again = B.bandk_v1(A.row_ptr, A.col_idx, srs, ssrs)
    assert np.array_equal(again[0], perm) and np.array_equal(again[1], sr_ptr)


def test_diagonal_matrix_all_isolated():
    n = 37
    rp = np.arange(n + 1)
    ci = np.arange(n)
    va = np.random.default_rng(0).uniform(1, 2, n)
    perm, sr_ptr, ssr_ptr = B.bandk_v1(rp, ci, 4, 3)
    _check_structure(n, perm, sr_ptr, ssr_ptr, 4, 3)
    r2, c2, v2, _ = B.apply_permutation(rp, ci, va, perm)
    x = np.random.default_rng(1).uniform(-1, 1, n)
    assert np.array_equal(O.spmv(r2, c2, v2, x[perm]), (va * x)[perm])


def test_chunked_variants():
    p, sr, ssr = B.reorder_none(10, 3, 2)
    assert p.tolist() == list(range(10)) and sr.tolist() == [0, 3, 6, 9, 10] and ssr.tolist() == [0, 2, 4]
    rp, ci = _path(6)
    p, sr, ssr = B.reorder_rcm(rp, ci, 4, 4)
    assert p.tolist() == [5, 4, 3, 2, 1, 0] and sr.tolist() == [0, 4, 6] and ssr.tolist() == [0, 2]


def test_empty_matrix():
    perm, sr_ptr, ssr_ptr = B.bandk_v1(np.zeros(1, np.int32), np.zeros(0, np.int32), 4, 4)
    assert len(perm) == 0 and sr_ptr.tolist() == [0] and ssr_ptr.tolist() == [0]


def test_band_close_to_rcm_on_grid():
    A = laplacian((32, 32), "2d5", 4.0)
    perm, _, _ = B.bandk_v1(A.row_ptr, A.col_idx, 8, 4)
    r2, c2, _, _ = B.apply_permutation(A.row_ptr, A.col_idx, A.vals, perm)
    rcm = B.reverse_cuthill_mckee(B.graph_from_csr(A.row_ptr, A.col_idx))
    r3, c3, _, _ = B.apply_permutation(A.row_ptr, A.col_idx, A.vals, rcm)
    # reported, loosely bounded: the paper calls Band-k's band "slightly wider" than RCM's
    assert B.bandwidth(r3, c3) <= B.bandwidth(r2, c2) <= 4 * B.bandwidth(r3, c3)


# ---------------------------------------------------------------- CSR-2 (k = 2)

def test_csr2_worked_example_path12():
    # Path 0-1-...-11, SRS 2: CM(G0) = 0..11 gives SRs {0,1} (id 0), {2,3} (id 2), ..., {10,11} (id 10); G1 is
    # a path; RCM(G1) = 10, 8, ..., 0.  Expanding SR 10: row 11 first (degree 1), then 10; in SR 8 row 9 comes
    # first (weight 1 to the emitted row 10), then 8; and so on.  Groups of 2 SRs for the launch.
    rp, ci = _path(12)
    perm, sr_ptr, ssr_ptr = B.bandk_k2(rp, ci, 2, 2)
    assert perm.tolist() == list(range(11, -1, -1))
    assert sr_ptr.tolist() == list(range(0, 13, 2)) and ssr_ptr.tolist() == [0, 2, 4, 6]


def test_csr2_srs1_is_rcm_and_invariants():
    A = random_sparse(300, 5.0, seed=8, symmetric_pattern=True)
    perm, sr_ptr, ssr_ptr = B.bandk_k2(A.row_ptr, A.col_idx, 1, 3)
    assert perm.tolist() == list(B.reverse_cuthill_mckee(B.graph_from_csr(A.row_ptr, A.col_idx)))
    perm, sr_ptr, ssr_ptr = B.bandk_k2(A.row_ptr, A.col_idx, 7, 3)
    assert sorted(perm.tolist()) == list(range(A.n))
    assert sr_ptr[0] == 0 and sr_ptr[-1] == A.n and np.all(np.diff(sr_ptr) >= 1) and np.all(np.diff(sr_ptr) <= 7)
    assert ssr_ptr[-1] == len(sr_ptr) - 1 and np.all(np.diff(ssr_ptr)[:-1] == 3)
    x = np.random.default_rng(1).uniform(-1, 1, A.n)
    rp2, ci2, v2, _ = B.apply_permutation(A.row_ptr, A.col_idx, A.vals, perm)
    y2 = O.spmv(rp2, ci2, v2, x[perm])
    y = np.empty(A.n)
    y[perm] = y2
    assert np.allclose(y, O.spmv(A.row_ptr, A.col_idx, A.vals, x), rtol=0, atol=1e-12)


# ------------------------------------------------------------------ CSR-k for k >= 4 (Section 2.2: any k)

def test_worked_example_path16_k4(golden_dir):
    g = _read_golden(os.path.join(golden_dir, "bandk_path16_k4.txt"))
    rp, ci = _path(g["n"][0])
    perm, ptrs = B.bandk_levels(rp, ci, g["sizes"])
    assert perm.tolist() == g["perm"]
    assert [p.tolist() for p in ptrs] == [g["level1_ptr"], g["level2_ptr"], g["level3_ptr"]]


@pytest.mark.parametrize("srs,ssrs", [(4, 3), (1, 1), (7, 2)])
def test_levels_reduce_to_k3_and_k2(srs, ssrs):
    """Two and three levels of the general walk are the k = 3 and k = 2 forms (pinned separately)."""
    for A in (workload_c1()["A"], random_sparse(400, 3.0, seed=srs, empty_row_frac=0.1)):
        perm, ptrs = B.bandk_levels(A.row_ptr, A.col_idx, [srs, ssrs])
        p3 = B.bandk_v1(A.row_ptr, A.col_idx, srs, ssrs)
        assert np.array_equal(perm, p3[0]) and np.array_equal(ptrs[0], p3[1]) and np.array_equal(ptrs[1], p3[2])
        perm2, ptrs2 = B.bandk_levels(A.row_ptr, A.col_idx, [srs])
        p2 = B.bandk_k2(A.row_ptr, A.col_idx, srs, ssrs)
        assert np.array_equal(perm2, p2[0]) and np.array_equal(ptrs2[0], p2[1])


def test_levels_unit_sizes_reduce_to_rcm():
    A = workload_c1()["A"]
    perm, ptrs = B.bandk_levels(A.row_ptr, A.col_idx, [1, 1, 1, 1])
    assert perm.tolist() == B.reverse_cuthill_mckee(B.graph_from_csr(A.row_ptr, A.col_idx))
    assert all(p.tolist() == list(range(A.n + 1)) for p in ptrs)


@pytest.mark.parametrize("seed,sym,sizes", [(0, True, [4, 3, 2]), (1, False, [8, 2, 3, 2]), (2, False, [3, 5, 5]),
                                            (3, True, [2, 2, 2, 2, 2])])
def test_levels_invariants_random(seed, sym, sizes):
    A = random_sparse(300, 3.0, seed=seed, empty_row_frac=0.1, symmetric_pattern=sym)
    perm, ptrs = B.bandk_levels(A.row_ptr, A.col_idx, sizes)
    assert sorted(perm.tolist()) == list(range(A.n))
    units = A.n
    for p, t in zip(ptrs, sizes):
        assert p[0] == 0 and p[-1] == units
        assert np.all(np.diff(p) >= 1) and np.all(np.diff(p) <= t)
        units = len(p) - 1
    assert units >= 1
    r2, c2, v2, vm = B.apply_permutation(A.row_ptr, A.col_idx, A.vals, perm)
    x = np.random.default_rng(seed).uniform(-1, 1, A.n)
    y = O.spmv(A.row_ptr, A.col_idx, A.vals, x)
    scale = O.row_abs_sum(A.row_ptr, A.col_idx, A.vals, x)
    assert np.all(np.abs(O.spmv(r2, c2, v2, x[perm]) - y[perm]) <= 1e-12 * scale[perm])


def test_upper_levels_chunk_the_level_below():
    A = random_sparse(500, 4.0, seed=9)
    for reorder in ("rcm", "none"):
        _, _, ssr_ptr = B.build_grouping(A.row_ptr, A.col_idx, 5, 3, reorder, 3)
        up = B.upper_levels(A.row_ptr, A.col_idx, 5, 3, reorder, 5)
        assert len(up) == 2
        assert up[0][-1] == len(ssr_ptr) - 1 and np.all(np.diff(up[0]) == np.minimum(3, (len(ssr_ptr) - 1) - up[0][:-1]))
        assert up[1][-1] == len(up[0]) - 1

