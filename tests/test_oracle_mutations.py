"""Mutation check of the oracle's pins: plausible mistakes planted in the oracle (on the CPU, for the duration
of one check) must make at least one of its pins fail.

Each case replaces one oracle function with a wrong version (a dropped term, a wrong sign or index, a transposed
operand, a wrong rounding, a wrong tie-break or boundary) and runs the pin tests that guard it; the case passes
when a pin raises.  The correct oracle passes the same pins in the ordinary test modules."""

import math
import os

import numpy as np
import pytest

import oracle.adjoint as AD
import oracle.bandk as B
import oracle.precision as P
import oracle.spmv as O
import oracle.stats as S
import oracle.tune as T
import test_oracle_adjoint_precision as TA
import test_oracle_bandk as TB
import test_oracle_spmv as TS
import test_oracle_tune_stats as TT

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(row_ptr):
    return np.repeat(np.arange(len(row_ptr) - 1), np.diff(np.asarray(row_ptr, dtype=np.int64)))


# ---------------------------------------------------------------- planted mistakes

def spmv_drops_last_term(row_ptr, col_idx, vals, x):
    x = np.asarray(x, dtype=np.float64)
    rp = np.asarray(row_ptr, dtype=np.int64)
    y = np.zeros((len(rp) - 1,) + x.shape[1:])
    for i in range(len(rp) - 1):
        for k in range(int(rp[i]), max(int(rp[i + 1]) - 1, int(rp[i]))):
            y[i] += vals[k] * x[col_idx[k]]
    return y


def spmv_transposed(row_ptr, col_idx, vals, x):
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros((len(row_ptr) - 1,) + x.shape[1:])
    np.add.at(y, np.asarray(col_idx), (np.asarray(vals)[:, None] if x.ndim > 1 else np.asarray(vals))
              * x[_rows(row_ptr)])
    return y


def spmv_column_shifted(row_ptr, col_idx, vals, x):
    x = np.asarray(x, dtype=np.float64)
    n = len(row_ptr) - 1
    c = (np.asarray(col_idx, dtype=np.int64) + 1) % max(n, 1)
    y = np.zeros((n,) + x.shape[1:])
    np.add.at(y, _rows(row_ptr), (np.asarray(vals)[:, None] if x.ndim > 1 else np.asarray(vals)) * x[c])
    return y


def spmv_empty_rows_pick_next_value(row_ptr, col_idx, vals, x):
    """The np.add.reduceat pitfall: an empty segment returns the element at its start instead of 0."""
    x = np.asarray(x, dtype=np.float64)
    prods = np.asarray(vals) * x[np.asarray(col_idx)]
    rp = np.asarray(row_ptr, dtype=np.int64)
    if len(prods) == 0:
        return np.zeros(len(rp) - 1)
    return np.add.reduceat(prods, np.minimum(rp[:-1], len(prods) - 1))


def grad_x_sign(row_ptr, col_idx, vals, g):
    out = np.zeros(len(row_ptr) - 1)
    np.add.at(out, np.asarray(col_idx), -np.asarray(vals) * np.asarray(g)[_rows(row_ptr)])
    return out


def grad_x_untransposed(row_ptr, col_idx, vals, g):
    out = np.zeros(len(row_ptr) - 1)
    np.add.at(out, _rows(row_ptr), np.asarray(vals) * np.asarray(g)[np.asarray(col_idx)])
    return out


def grad_vals_swapped(row_ptr, col_idx, x, g):
    return np.asarray(g)[np.asarray(col_idx)] * np.asarray(x)[_rows(row_ptr)]


def bf16_truncates(v32):
    f = np.atleast_1d(np.asarray(v32, dtype=np.float32))
    out = (f.view(np.uint32) >> 16).astype(np.uint16)
    return out if np.ndim(v32) else out[0]


def round_half_even(v):
    return int(round(v))


def case_of_strict(r):
    return 1 if r < 8 else 2 if r < 16 else 3 if r < 32 else 4


def row_stats_sample_variance(row_ptr):
    lengths = np.diff(np.asarray(row_ptr, dtype=np.int64)).astype(np.float64)
    r = lengths.mean()
    var = float(np.sum((lengths - r) ** 2) / max(len(lengths) - 1, 1))
    return {"n": len(lengths), "nnz": int(lengths.sum()), "r": float(r), "var": var, "max": int(lengths.max()),
            "regular": var <= 10.0}


def rcm_not_reversed(G):
    return B.cuthill_mckee(G)


def quotient_unit_weights(G, agg, ident):
    Q = _orig_quotient(G, agg, ident)
    return B.LevelGraph(Q.n, Q.xadj, Q.adj, np.ones_like(Q.wgt), Q.ident)


def apply_permutation_maps_columns_by_perm(row_ptr, col_idx, vals, perm):
    perm = np.asarray(perm, dtype=np.int64)
    rp = np.asarray(row_ptr, dtype=np.int64)
    lengths = np.diff(rp)[perm]
    new_ptr = np.zeros(len(perm) + 1, dtype=np.int64)
    np.cumsum(lengths, out=new_ptr[1:])
    new_row = np.repeat(np.arange(len(perm)), lengths)
    src = rp[perm][new_row] + (np.arange(new_ptr[-1]) - new_ptr[new_row])
    new_col = perm[np.asarray(col_idx)[src]]  # should be iperm
    o = np.lexsort((new_col, new_row))
    return new_ptr, new_col[o], np.asarray(vals)[src[o]], src[o]


_orig_quotient = B.quotient


# ---------------------------------------------------------------- cases: (module, name, mutant, pins)

CASES = [
    ("spmv: dropped term", O, "spmv", spmv_drops_last_term,
     [lambda: TS.test_dense_brute_force(0), TS.test_laplacian_times_ones_2d]),
    ("spmv: transposed operand", O, "spmv", spmv_transposed, [lambda: TS.test_dense_brute_force(1)]),
    ("spmv: column index off by one", O, "spmv", spmv_column_shifted, [TS.test_unit_vectors_give_columns]),
    ("spmv: empty rows not zero", O, "spmv", spmv_empty_rows_pick_next_value, [TS.test_empty_rows_are_exact_zero]),
    ("grad_x: wrong sign", AD, "grad_x", grad_x_sign, [lambda: TA.test_dot_product_identity(0)]),
    ("grad_x: A g instead of A^T g", AD, "grad_x", grad_x_untransposed, [TA.test_grad_x_is_dense_transpose]),
    ("grad_vals: row and column swapped", AD, "grad_vals", grad_vals_swapped, [TA.test_finite_differences]),
    ("bf16: truncation instead of round to nearest even", P, "f32_to_bf16_bits", bf16_truncates,
     [TA.test_bf16_rounding_by_hand, TA.test_bf16_matches_torch]),
    ("tune: halves rounded to even", T, "round_half_up", round_half_even,
     [TT.test_round_half_up, lambda: TT.test_paper_vectors(GOLDEN)]),
    ("tune: case boundaries to the upper case", T, "case_of", case_of_strict,
     [TT.test_case_boundaries, lambda: TT.test_paper_vectors(GOLDEN)]),
    ("stats: sample variance", S, "row_stats", row_stats_sample_variance, [TT.test_row_stats_closed_forms]),
    ("Band-k: coarse order not reversed", B, "reverse_cuthill_mckee", rcm_not_reversed,
     [lambda: TB.test_worked_example_path12(GOLDEN), TB.test_cm_star_by_hand]),
    ("Band-k: quotient weights not summed", B, "quotient", quotient_unit_weights, [TB.test_quotient_weights_by_hand]),
    ("permutation: columns mapped by perm instead of its inverse", B, "apply_permutation",
     apply_permutation_maps_columns_by_perm, [TB.test_apply_permutation_by_hand]),
]


@pytest.mark.parametrize("label,module,name,mutant,pins", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_fails_a_pin(monkeypatch, label, module, name, mutant, pins):
    monkeypatch.setattr(module, name, mutant)
    caught = []
    for pin in pins:
        try:
            pin()
        except AssertionError:
            caught.append(pin)
    assert caught, f"no pin caught the planted mistake: {label}"


def test_pins_pass_on_the_oracle():
    """The same pins, unmodified oracle: none fails (so a failure above is the mutant's)."""
    for _, _, _, _, pins in CASES:
        for pin in pins:
            pin()
    assert math.isfinite(T.round_half_up(2.5))
