"""Oracle: reduced-precision value storage and its error bound — TEST INFRASTRUCTURE ONLY.

Not in the paper (its precision is unstated; its format discussion uses 32-bit
values as the example, Section 2.1).  Definitions used here:

* FP64 -> FP32: IEEE round to nearest, ties to even.
* FP32 -> BF16: keep the upper 16 bits of the FP32 pattern after rounding to
  nearest, ties to even, on the 16 discarded bits; NaN stays NaN.  BF16 storage
  of an FP64 value is BF16(FP32(v)), two rounding steps.
* Forward error of a row computed from stored values (unit roundoff u_v),
  right-hand side rounded to the vector type (u_x) and an inner product
  accumulated in a type with unit roundoff u_acc over m terms: standard
  inner-product analysis (Higham, Accuracy and Stability of Numerical
  Algorithms, ch. 3) gives
      |y_hat_i - y_i| <= beta_i * sum_j |a_ij| |x_j|,
      beta_i = (1 + u_v)(1 + u_x)(1 + gamma_m(u_acc)) - 1,
      gamma_m(u) = m u / (1 - m u).

Pins (tests/test_oracle_precision.py): hand-worked rounding cases including
ties, and agreement with torch's own float32/bfloat16 conversions.
"""

from __future__ import annotations

import numpy as np

UNIT_ROUNDOFF = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -8}


def to_f32(v) -> np.ndarray:
    return np.asarray(v, dtype=np.float64).astype(np.float32)


def f32_to_bf16_bits(v32) -> np.ndarray:
    """uint16 BF16 patterns of float32 values, round to nearest even."""
    f = np.atleast_1d(np.asarray(v32, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    is_nan = np.isnan(f)
    lsb = (u >> 16) & 1
    rounded = (u + 0x7FFF + lsb) >> 16
    out = (rounded & 0xFFFF).astype(np.uint16)
    out[is_nan] = ((u[is_nan] >> 16) | 0x40).astype(np.uint16)
    return out if np.ndim(v32) else out[0]


def bf16_bits_to_f64(bits) -> np.ndarray:
    u = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def to_bf16_as_f64(v) -> np.ndarray:
    """Value of BF16(FP32(v)) as float64."""
    return bf16_bits_to_f64(f32_to_bf16_bits(to_f32(v)))


def stored_values(vals, dtype: str) -> np.ndarray:
    """The values a matrix holds after storage in ``dtype``, as float64."""
    if dtype == "f64":
        return np.asarray(vals, dtype=np.float64).copy()
    if dtype == "f32":
        return to_f32(vals).astype(np.float64)
    if dtype == "bf16":
        return to_bf16_as_f64(vals)
    raise ValueError(dtype)


def gamma(m, u: float):
    m = np.asarray(m, dtype=np.float64)
    return m * u / (1.0 - m * u)


def forward_bound(row_lengths, store: str, x_rounded: bool, acc: str) -> np.ndarray:
    """beta_i per row (relative to sum_j |a_ij||x_j|), see the module notes."""
    u_v = UNIT_ROUNDOFF[store] if store != "bf16" else (1 + 2.0 ** -24) * (1 + 2.0 ** -8) - 1
    u_x = UNIT_ROUNDOFF["f32"] if x_rounded else 0.0
    return (1 + u_v) * (1 + u_x) * (1 + gamma(row_lengths, UNIT_ROUNDOFF[acc])) - 1


def relative_errors(y_hat, y_ref, scale) -> np.ndarray:
    """|y_hat - y_ref| / scale per entry (0 where scale is 0 and the values agree)."""
    y_hat = np.asarray(y_hat, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    diff = np.abs(y_hat - y_ref)
    out = np.zeros_like(diff)
    nz = scale > 0
    out[nz] = diff[nz] / scale[nz]
    out[~nz] = np.where(diff[~nz] == 0, 0.0, np.inf)
    return out
