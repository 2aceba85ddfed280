"""Oracle: the adjoint of y = A x — TEST INFRASTRUCTURE ONLY.

Not in the paper; plain definitions of the two gradients of L = g^T A x:

* grad_x = A^T g: for every stored a_ij, grad_x[j] += a_ij * g_i (a scatter
  over the stored entries in storage order, FP64);
* grad_vals[k] = g_i * x_j for the k-th stored entry (i, j); with a block of
  right-hand sides it is the sum over the columns c of g_{i,c} x_{j,c}.

Pins (tests/test_oracle_adjoint.py): the dot-product identity
<g, A x> = <A^T g, x>, central finite differences of the bilinear form L, and
the dense transpose on small cases.
"""

from __future__ import annotations

import numpy as np


def row_of_entry(row_ptr) -> np.ndarray:
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    return np.repeat(np.arange(len(row_ptr) - 1, dtype=np.int64), np.diff(row_ptr))


def grad_x(row_ptr, col_idx, vals, g) -> np.ndarray:
    """A^T g by scattering a_ij * g_i into position j, FP64."""
    g = np.asarray(g, dtype=np.float64)
    vals = np.asarray(vals, dtype=np.float64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    rows = row_of_entry(row_ptr)
    n = len(row_ptr) - 1
    out = np.zeros((n,) + g.shape[1:], dtype=np.float64)
    contrib = vals * g[rows] if g.ndim == 1 else vals[:, None] * g[rows]
    np.add.at(out, col_idx, contrib)
    return out


def grad_vals(row_ptr, col_idx, x, g) -> np.ndarray:
    """g_i * x_j per stored entry (summed over right-hand-side columns), FP64."""
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    rows = row_of_entry(row_ptr)
    cols = np.asarray(col_idx, dtype=np.int64)
    if x.ndim == 1:
        return g[rows] * x[cols]
    return np.sum(g[rows] * x[cols], axis=1)


def loss(row_ptr, col_idx, vals, x, g) -> float:
    """L = <g, A x> evaluated entry by entry (used by the finite-difference pin)."""
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    rows = row_of_entry(row_ptr)
    cols = np.asarray(col_idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    if x.ndim == 1:
        return float(np.sum(vals * g[rows] * x[cols]))
    return float(np.sum(vals[:, None] * g[rows] * x[cols]))
