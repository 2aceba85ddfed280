"""Irregular sparse matrices (power-law row lengths), seeded.

The paper's test suite has an irregular class (row-length variance above 10:
web, citation, social and circuit graphs, Table 1) on which CSR-3 loses most,
because long rows end up summed serially (Section 7, GPU performance).  These matrices are
not available here; R-MAT graphs stand in for them: recursive quadrant
sampling with probabilities (a, b, c, d) gives a heavy-tailed degree
distribution with a few very long rows and many short ones.
"""

from __future__ import annotations

import numpy as np

from .stencils import CsrInput, _streams


def rmat_pattern(scale: int, edge_factor: float, rng, a: float = 0.57, b: float = 0.19, c: float = 0.19,
                 symmetric: bool = False, diagonal: bool = True):
    """CSR pattern of an R-MAT graph on n = 2^scale vertices with about edge_factor * n sampled edges.

    Duplicate edges are merged; with ``symmetric`` the pattern is A | A^T; with ``diagonal`` every row
    gets its diagonal entry.  Returns (row_ptr int32[n+1], col_idx int32[nnz], is_diag bool[nnz]),
    columns sorted within rows.
    """
    n = 1 << scale
    m = int(round(edge_factor * n))
    rows = np.zeros(m, dtype=np.int64)
    cols = np.zeros(m, dtype=np.int64)
    cum = np.array([a, a + b, a + b + c])
    for level in range(scale):
        u = rng.random(m)
        q = np.searchsorted(cum, u, side="right")  # 0..3: quadrant
        bit = np.int64(1) << (scale - 1 - level)
        rows += np.where(q >= 2, bit, 0)
        cols += np.where((q == 1) | (q == 3), bit, 0)
    if symmetric:
        rows, cols = np.concatenate([rows, cols]), np.concatenate([cols, rows])
    if diagonal:
        d = np.arange(n, dtype=np.int64)
        rows, cols = np.concatenate([rows, d]), np.concatenate([cols, d])
    key = np.unique(rows * n + cols)
    r, cidx = key // n, key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr.astype(np.int32), cidx.astype(np.int32), r == cidx


def rmat_matrix(scale: int = 20, edge_factor: float = 4.0, seed: int = 21, symmetric: bool = True,
                name: str | None = None) -> CsrInput:
    """R-MAT pattern with diagonally dominant values: off-diagonals -U[0.5, 1.5], diagonal 1.1 * row
    sum of |off-diagonals| (0 where a row has no off-diagonal: then 1.0)."""
    rp, rv = _streams(seed, 2)
    row_ptr, col_idx, is_diag = rmat_pattern(scale, edge_factor, rp, symmetric=symmetric)
    nnz = int(row_ptr[-1])
    vals = -rv.uniform(0.5, 1.5, size=nnz)
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    off = np.where(is_diag, 0.0, np.abs(vals))
    rsum = np.bincount(rows, weights=off, minlength=len(row_ptr) - 1)
    vals[is_diag] = np.where(rsum[rows[is_diag]] > 0, 1.1 * rsum[rows[is_diag]], 1.0)
    n = len(row_ptr) - 1
    return CsrInput(name or f"rmat_s{scale}_e{edge_factor:g}{'_sym' if symmetric else ''}", n, row_ptr, col_idx,
                    vals, {"scale": scale, "edge_factor": edge_factor, "symmetric": symmetric, "seed": seed})


def workload_irregular(seed: int = 21, scale: int = 20, edge_factor: float = 4.0, symmetric: bool = True):
    """R-MAT stand-in for the paper's irregular class: n = 2^20, about 9 nonzeros per row after
    symmetrisation and the diagonal, row-length variance in the hundreds; x, g ~ U[-1, 1]; float64."""
    A = rmat_matrix(scale, edge_factor, seed, symmetric)
    rx, rg = _streams(seed + 1, 2)
    return {"name": "irregular", "A": A, "x": rx.uniform(-1.0, 1.0, A.n), "g": rg.uniform(-1.0, 1.0, A.n),
            "dtype": "f64", "nrhs": 1}
