"""Oracle: the sparse matrix-vector product in FP64 — TEST INFRASTRUCTURE ONLY.

Definition (Section 1): for every row i, y_i is the sum over the row's stored
nonzeros of a_ij * x_j.  Storage (Section 2.1): CSR with ``row_ptr`` holding
the running count of nonzeros per row, ``col_idx`` and ``vals`` the column and
value of each nonzero.

CSR-k (Section 2.2, Fig. 1) keeps exactly this storage and adds
``sr_ptr`` (running count of rows per super-row) and ``ssr_ptr`` (running
count of super-rows per super-super-row).  Its CPU kernel walks
super-super-rows, then their super-rows, then their rows, and forms each row's
sum from zero, one term after the other, storing it to y.

Pins (tests/test_oracle_spmv.py): dense brute force, exact rational
arithmetic, the Laplacian times the ones vector, A e_j = column j, empty rows
give exactly 0, and the CSR-k traversal equals the plain row loop bit for bit.
"""

from __future__ import annotations

import numpy as np


def spmv(row_ptr, col_idx, vals, x) -> np.ndarray:
    """y = A x in FP64; each row is summed left to right starting from 0.0.

    ``x`` may be (n,) or (n, nrhs) (row-major block of right-hand sides); the
    result has the same trailing shape.  Rows without nonzeros give exactly 0.
    """
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = len(row_ptr) - 1
    y = np.zeros((n,) + x.shape[1:], dtype=np.float64)
    if n == 0 or row_ptr[-1] == 0:
        return y
    prods = vals * x[col_idx] if x.ndim == 1 else vals[:, None] * x[col_idx]
    lengths = np.diff(row_ptr)
    # Visit term j of every row that has one, for j = 0, 1, ...: this adds each
    # row's terms in storage order, vectorised across rows.
    order = np.argsort(-lengths, kind="stable")
    neg_sorted = -lengths[order]
    for j in range(int(-neg_sorted[0])):
        count = int(np.searchsorted(neg_sorted, -j, side="left"))  # rows with more than j terms
        rows = order[:count]
        y[rows] += prods[row_ptr[rows] + j]
    return y


def spmv_csrk_traversal(ssr_ptr, sr_ptr, row_ptr, col_idx, vals, x):
    """The CSR-k (k=3) traversal in pure Python loops, for small cases.

    Super-super-row t covers super-rows ssr_ptr[t] .. ssr_ptr[t+1]-1; super-row
    s covers rows sr_ptr[s] .. sr_ptr[s+1]-1; each row's sum starts at 0.0 and
    adds its terms in storage order (Section 2.2, CPU kernel for CSR-3).

    Returns ``(y, visits)`` where ``visits[i]`` counts how often row i was
    written, so a test can check that the grouping covers every row once.
    """
    n = len(row_ptr) - 1
    y = np.zeros(n, dtype=np.float64)
    visits = np.zeros(n, dtype=np.int64)
    rp = [int(v) for v in row_ptr]
    ci = [int(v) for v in col_idx]
    va = [float(v) for v in vals]
    xv = [float(v) for v in x]
    for t in range(len(ssr_ptr) - 1):
        for s in range(int(ssr_ptr[t]), int(ssr_ptr[t + 1])):
            for i in range(int(sr_ptr[s]), int(sr_ptr[s + 1])):
                acc = 0.0
                for k in range(rp[i], rp[i + 1]):
                    acc += va[k] * xv[ci[k]]
                y[i] = acc
                visits[i] += 1
    return y, visits


def row_abs_sum(row_ptr, col_idx, vals, x) -> np.ndarray:
    """sum_j |a_ij| |x_j| per row (the scale of the forward error bound), FP64."""
    return spmv(row_ptr, col_idx, np.abs(np.asarray(vals, dtype=np.float64)), np.abs(np.asarray(x, dtype=np.float64)))

