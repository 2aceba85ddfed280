"""Oracle: the paper's constant-time super-row size model — TEST INFRASTRUCTURE ONLY.

Section 4.1 of the paper, step by step:

1. rdensity r = NNZ / N.
2. Case by r: 1 for r <= 8, 2 for 8 < r <= 16, 3 for 16 < r <= 32, 4 for r > 32
   (each boundary belongs to the lower case, as the case list states "<=").
3. Initial sizes from a logarithmic fit: SSRS = round(a_s - b_s ln r),
   SRS = round(a_r - b_r ln r), where round() is to nearest with halves
   going toward +infinity.  Volta: (8.900, 1.25), (10.146, 1.50);
   Ampere: (9.175, 1.32), (20.500, 3.50).
4. Per-case adjustment, applied line after line (each line sees the previous
   line's result).  Where the paper writes "SRSS" we read SSRS: every other
   adjusting line derives SRS from SSRS.
5. Both sizes are clamped to at least 1 (the paper is silent; Volta's SSRS
   would reach 0 for r above about 830).

SSRS is the number of super-rows per super-super-row and SRS the number of
rows per super-row.  The model is pinned by hand-computed values in
tests/golden/paper_tune_vectors.txt.
"""

from __future__ import annotations

import math

CONSTANTS = {
    "volta": (8.900, 1.25, 10.146, 1.50),
    "ampere": (9.175, 1.32, 20.500, 3.50),
}


def round_half_up(v: float) -> int:
    """Nearest integer, halves toward +infinity."""
    return int(math.floor(v + 0.5))


def case_of(r: float) -> int:
    if r <= 8:
        return 1
    if r <= 16:
        return 2
    if r <= 32:
        return 3
    return 4


def raw_sizes(r: float, model: str):
    a_s, b_s, a_r, b_r = CONSTANTS[model]
    return a_s - b_s * math.log(r), a_r - b_r * math.log(r)


def paper_tune(n: int, nnz: int, model: str, srss_reading: str = "ssrs"):
    """(SSRS, SRS, case) for the Volta or Ampere model.

    ``srss_reading`` selects how the paper's "SRSS" is read: "ssrs" (default)
    or "srs" (the alternative kept for comparison).
    """
    if n <= 0 or nnz <= 0:
        raise ValueError("n and nnz must be positive")
    r = nnz / n
    c = case_of(r)
    s_raw, r_raw = raw_sizes(r, model)
    ssrs = round_half_up(s_raw)
    srs = round_half_up(r_raw)
    if model == "volta":
        if c == 2:
            ssrs = round_half_up(ssrs * 1.5)
            srs = (ssrs if srss_reading == "ssrs" else srs) * 2
        elif c == 3:
            ssrs = ssrs * 4
            srs = ssrs // 2
        elif c == 4:
            ssrs = ssrs * 5
            srs = ssrs // 2
    elif model == "ampere":
        if c == 2:
            srs = (ssrs if srss_reading == "ssrs" else srs) * 4
        elif c == 3:
            ssrs = round_half_up(ssrs * 2.5)
            srs = ssrs * 3
        elif c == 4:
            ssrs = ssrs * 2
            srs = ssrs * 2
    else:
        raise ValueError(model)
    return max(1, ssrs), max(1, srs), c


def sweep_set_gpu():
    """The paper's GPU sweep values {2^i, 1.5 * 2^i}, i = 2..5."""
    return sorted({2 ** i for i in range(2, 6)} | {3 * 2 ** (i - 1) for i in range(2, 6)})


def sweep_set_cpu():
    """The paper's CPU SRS sweep values {2^i, 1.5 * 2^i}, i = 3..11."""
    return sorted({2 ** i for i in range(3, 12)} | {3 * 2 ** (i - 1) for i in range(3, 12)})


def fit_log_model(rs, best):
    """Least-squares fit best ~ a - b ln r (the paper's logarithmic regression).  Returns (a, b)."""
    import numpy as np
    L = np.log(np.asarray(rs, dtype=np.float64))
    y = np.asarray(best, dtype=np.float64)
    M = np.stack([np.ones_like(L), -L], axis=1)
    (a, b), *_ = np.linalg.lstsq(M, y, rcond=None)
    return float(a), float(b)
