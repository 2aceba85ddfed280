"""ctypes access to the C oracle (spmv_ref.c) — TEST INFRASTRUCTURE ONLY."""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spmv_ref.c")
LIB = os.path.join(HERE, "libspmv_ref.so")

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


def build() -> str:
    """Compile the C oracle (portable -O3, OpenMP)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99", SRC, "-o", LIB + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.oracle_spmv_f64.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.oracle_spmv_adjoint_f64.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p]
        L.oracle_spmv_adjoint_gather_f64.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _i32p, _i32p, _i32p,
                                                     _f64p, _f64p, _f64p, _f64p]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_time_adjoint_gather_f64.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _i32p, _i32p, _i32p,
                                                     _f64p, _f64p, _f64p, _f64p, ctypes.c_int]
        L.oracle_time_adjoint_gather_f64.restype = ctypes.c_double
        L.oracle_time_spmv_f64.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p, ctypes.c_int]
        L.oracle_time_spmv_f64.restype = ctypes.c_double
        L.oracle_time_adjoint_f64.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p,
                                              ctypes.c_int]
        L.oracle_time_adjoint_f64.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _prep(row_ptr, col_idx, vals):
    return (np.ascontiguousarray(row_ptr, dtype=np.int32), np.ascontiguousarray(col_idx, dtype=np.int32),
            np.ascontiguousarray(vals, dtype=np.float64))


def spmv(row_ptr, col_idx, vals, x) -> np.ndarray:
    rp, ci, va = _prep(row_ptr, col_idx, vals)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = len(rp) - 1
    y = np.empty(n, dtype=np.float64)
    lib().oracle_spmv_f64(n, _p(rp, _i32p), _p(ci, _i32p), _p(va, _f64p), _p(x, _f64p), _p(y, _f64p))
    return y


def adjoint(row_ptr, col_idx, vals, x, g):
    rp, ci, va = _prep(row_ptr, col_idx, vals)
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    n = len(rp) - 1
    gx = np.empty(n, dtype=np.float64)
    gv = np.empty(len(ci), dtype=np.float64)
    lib().oracle_spmv_adjoint_f64(n, _p(rp, _i32p), _p(ci, _i32p), _p(va, _f64p), _p(x, _f64p), _p(g, _f64p),
                                  _p(gx, _f64p), _p(gv, _f64p))
    return gx, gv


def column_index(row_ptr, col_idx):
    """(t_ptr, t_row, t_pos): the entries of each column by increasing row, as (row, position)."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    n = len(rp) - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    pos = np.argsort(ci, kind="stable")  # stable: within a column, entries stay in row order
    t_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(ci, minlength=n), out=t_ptr[1:])
    return t_ptr.astype(np.int32), rows[pos].astype(np.int32), pos.astype(np.int32)


def adjoint_gather(row_ptr, col_idx, vals, x, g):
    """The adjoint by columns (gather form, OpenMP); equals ``adjoint`` bit for bit."""
    rp, ci, va = _prep(row_ptr, col_idx, vals)
    tp, tr, tq = column_index(rp, ci)
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    n = len(rp) - 1
    gx = np.empty(n, dtype=np.float64)
    gv = np.empty(len(ci), dtype=np.float64)
    lib().oracle_spmv_adjoint_gather_f64(n, _p(rp, _i32p), _p(ci, _i32p), _p(va, _f64p), _p(tp, _i32p),
                                         _p(tr, _i32p), _p(tq, _i32p), _p(x, _f64p), _p(g, _f64p), _p(gx, _f64p),
                                         _p(gv, _f64p))
    return gx, gv


def threads() -> int:
    return int(lib().oracle_threads())


def set_threads(t: int):
    lib().oracle_set_threads(int(t))


def time_forward(row_ptr, col_idx, vals, x, reps: int) -> float:
    rp, ci, va = _prep(row_ptr, col_idx, vals)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(len(rp) - 1, dtype=np.float64)
    return float(lib().oracle_time_spmv_f64(len(rp) - 1, _p(rp, _i32p), _p(ci, _i32p), _p(va, _f64p),
                                            _p(x, _f64p), _p(y, _f64p), reps))


def time_adjoint(row_ptr, col_idx, vals, x, g, reps: int) -> float:
    rp, ci, va = _prep(row_ptr, col_idx, vals)
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    n = len(rp) - 1
    gx = np.empty(n, dtype=np.float64)
    gv = np.empty(len(ci), dtype=np.float64)
    return float(lib().oracle_time_adjoint_f64(n, _p(rp, _i32p), _p(ci, _i32p), _p(va, _f64p), _p(x, _f64p),
                                               _p(g, _f64p), _p(gx, _f64p), _p(gv, _f64p), reps))


def time_adjoint_gather(row_ptr, col_idx, vals, x, g, reps: int, index=None) -> float:
    """Wall seconds of `reps` runs of the gather adjoint; ``index`` = column_index(...) if already built."""
    rp, ci, va = _prep(row_ptr, col_idx, vals)
    tp, tr, tq = index if index is not None else column_index(rp, ci)
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    n = len(rp) - 1
    gx = np.empty(n, dtype=np.float64)
    gv = np.empty(len(ci), dtype=np.float64)
    return float(lib().oracle_time_adjoint_gather_f64(n, _p(rp, _i32p), _p(ci, _i32p), _p(va, _f64p),
                                                      _p(tp, _i32p), _p(tr, _i32p), _p(tq, _i32p), _p(x, _f64p),
                                                      _p(g, _f64p), _p(gx, _f64p), _p(gv, _f64p), reps))
