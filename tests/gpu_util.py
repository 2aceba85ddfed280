"""Helpers shared by the GPU parity tests (not a test module)."""

import sys

import numpy as np

from oracle import precision as OP
from oracle import spmv as OS


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def params(srs, ssrs, lanes=1, waves=4, reorder="bandk", k=3):
    return {"k": int(k), "srs": int(srs), "ssrs": int(ssrs), "lanes_per_row": int(lanes), "waves_per_wg": int(waves),
            "reorder": reorder}


def to_dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def forward_bound(row_ptr, store, x_rounded):
    lengths = np.diff(np.asarray(row_ptr, dtype=np.int64))
    if store == "f64":
        # stated tolerance for the FP64 path: 1e-12 relative to sum |a_ij||x_j|
        return np.full(len(lengths), 1e-12)
    return OP.forward_bound(np.maximum(lengths, 1), store, x_rounded, "f32")


def check_forward(y_perm, A, x, perm, store, x_rounded, vals=None, label=""):
    """y_perm: GPU result in permuted space (numpy); compares with the FP64 oracle on the input order."""
    vals = A.vals if vals is None else vals
    y_ref = OS.spmv(A.row_ptr, A.col_idx, vals, x)
    scale = OS.row_abs_sum(A.row_ptr, A.col_idx, vals, x)
    beta = forward_bound(A.row_ptr, store, x_rounded)
    if y_ref.ndim == 2:
        beta = beta[:, None]
    err = np.abs(np.asarray(y_perm, dtype=np.float64) - y_ref[perm])
    lim = beta[perm] * scale[perm]
    bad = err > lim
    assert not bad.any(), f"{label}: {int(bad.sum())} rows over the bound; worst excess {np.max(err - lim):.3e}"
    rel = np.where(scale[perm] > 0, err / np.where(scale[perm] > 0, scale[perm], 1), 0)
    return float(rel.max()) if rel.size else 0.0
