"""Oracle: conjugate gradients in FP64 — TEST INFRASTRUCTURE ONLY.

The paper names CG on PDE matrices as the application of its format (Section 1
and the conclusions) but gives no solver.  This is the textbook method
(Hestenes and Stiefel, 1952) written out: r0 = b - A x0, p0 = r0; per step
alpha = (r.r) / (p.A p), x += alpha p, r -= alpha A p, beta = (r_new.r_new) /
(r.r), p = r + beta p; stop when ||r|| <= rtol ||b||.  Every product uses the
plain CSR oracle.
"""

from __future__ import annotations

import numpy as np

from .spmv import spmv


def cg(row_ptr, col_idx, vals, b, x0=None, rtol: float = 1e-8, max_iter: int = 10000):
    """Returns (x, iterations, ||r|| / ||b||) with r the recurrence residual."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - spmv(row_ptr, col_idx, vals, x)
    p = r.copy()
    rr = float(r @ r)
    bnorm = float(np.sqrt(b @ b)) or 1.0
    it = 0
    while np.sqrt(rr) > rtol * bnorm and it < max_iter:
        q = spmv(row_ptr, col_idx, vals, p)
        alpha = rr / float(p @ q)
        x += alpha * p
        r -= alpha * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, float(np.sqrt(rr)) / bnorm
