"""Pins of the paper's size model (hand-computed vectors) and of the row statistics (closed forms)."""

import os

import numpy as np
import pytest

from gen import laplacian, stencil_pattern, workload_c1
from oracle import stats as S
from oracle import tune as T


def _vectors(golden_dir):
    rows, alt = [], []
    with open(os.path.join(golden_dir, "paper_tune_vectors.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            parts = line.split()
            if parts[0] == "alt":
                alt.append([float(parts[1])] + [int(v) for v in parts[2:]])
            else:
                rows.append([float(parts[0])] + [int(v) for v in parts[1:]])
    return rows, alt


def _n_nnz(r):
    # an (n, nnz) pair with nnz / n == r exactly in binary floating point for the listed r
    n = 10 ** 6
    return n, int(round(r * n))


def test_paper_vectors(golden_dir):
    rows, _ = _vectors(golden_dir)
    for r, case, vs, vr, as_, ar in rows:
        n, nnz = _n_nnz(r)
        assert T.case_of(nnz / n) == case
        assert T.paper_tune(n, nnz, "volta")[:2] == (vs, vr), r
        assert T.paper_tune(n, nnz, "ampere")[:2] == (as_, ar), r


def test_alternative_srss_reading(golden_dir):
    _, alt = _vectors(golden_dir)
    for r, case, vs, vr, as_, ar in alt:
        n, nnz = _n_nnz(r)
        assert T.paper_tune(n, nnz, "volta", srss_reading="srs")[:2] == (vs, vr)
        assert T.paper_tune(n, nnz, "ampere", srss_reading="srs")[:2] == (as_, ar)


def test_round_half_up():
    assert T.round_half_up(12.5) == 13 and T.round_half_up(-0.5) == 0 and T.round_half_up(2.4999) == 2


def test_case_boundaries():
    assert [T.case_of(r) for r in (8, 8.0001, 16, 16.0001, 32, 32.0001)] == [1, 2, 2, 3, 3, 4]


def test_tune_rejects_bad_sizes():
    with pytest.raises(ValueError):
        T.paper_tune(0, 5, "volta")
    with pytest.raises(ValueError):
        T.paper_tune(5, 0, "ampere")


def test_sweep_sets():
    assert T.sweep_set_gpu() == [4, 6, 8, 12, 16, 24, 32, 48]
    cpu = T.sweep_set_cpu()
    assert cpu[0] == 8 and cpu[-1] == 3072 and len(cpu) == 18


def test_fit_log_model_recovers_line():
    rs = np.array([2.0, 5.0, 9.0, 20.0, 40.0])
    a, b = T.fit_log_model(rs, 9.0 - 1.5 * np.log(rs))
    assert abs(a - 9.0) < 1e-12 and abs(b - 1.5) < 1e-12


def test_row_stats_closed_forms():
    s1 = S.row_stats(workload_c1()["A"].row_ptr)
    # 64x64 5-point grid: 62^2 rows of 5, 4*62 of 4, 4 of 3
    mean = (62 * 62 * 5 + 4 * 62 * 4 + 4 * 3) / 4096
    var = (62 * 62 * 25 + 4 * 62 * 16 + 4 * 9) / 4096 - mean ** 2
    assert s1["r"] == mean == 4.9375 and abs(s1["var"] - var) < 1e-12 and s1["max"] == 5
    for side, regular in ((30, False), (60, True)):
        rp, _, _ = stencil_pattern((side, side, side), "3d27")
        s3 = S.row_stats(rp)
        # per-axis neighbour count is 3 inside, 2 on the two faces; row length is the product
        ec, ec2 = ((side - 2) * 3 + 2 * 2) / side, ((side - 2) * 9 + 2 * 4) / side
        assert abs(s3["r"] - ec ** 3) < 1e-12 and abs(s3["var"] - (ec2 ** 3 - ec ** 6)) < 1e-9
        assert s3["regular"] == regular


def test_pattern_symmetry():
    L = laplacian((6, 5), "2d5", 4.0)
    assert S.pattern_symmetry(L.row_ptr, L.col_idx) == 1.0
    # [[x, x], [0, x]]: one off-diagonal entry, mirror absent -> 0
    assert S.pattern_symmetry(np.array([0, 2, 3]), np.array([0, 1, 1])) == 0.0
