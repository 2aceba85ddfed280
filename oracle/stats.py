"""Oracle: matrix statistics of Section 5.3 — TEST INFRASTRUCTURE ONLY.

* row density r = NNZ / N (Section 4.1);
* variance of the number of nonzeros per row, sigma^2, and the regular /
  irregular split at sigma^2 <= 10 (Section 5.3; the abstract);
* maximum nonzeros in a row (MAX of Table 1);
* pattern symmetry SY: the fraction of off-diagonal stored entries (i, j)
  whose mirror (j, i) is also stored (Table 1, Section 5.3).
"""

from __future__ import annotations

import numpy as np


def row_stats(row_ptr):
    lengths = np.diff(np.asarray(row_ptr, dtype=np.int64)).astype(np.float64)
    n = len(lengths)
    if n == 0:
        return {"n": 0, "nnz": 0, "r": 0.0, "var": 0.0, "max": 0, "regular": True}
    r = lengths.sum() / n
    var = float(np.mean((lengths - r) ** 2))
    return {"n": n, "nnz": int(lengths.sum()), "r": float(r), "var": var, "max": int(lengths.max()),
            "regular": var <= 10.0}


def pattern_symmetry(row_ptr, col_idx) -> float:
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    n = len(row_ptr) - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    off = rows != col_idx
    if not off.any():
        return 1.0
    fwd = rows[off] * n + col_idx[off]
    mirror = col_idx[off] * n + rows[off]
    return float(np.isin(mirror, fwd).mean())
