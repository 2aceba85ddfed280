"""ctypes binding of libcsrk.so: one Python function per C entry point, same names.

Argument marshalling only (NumPy host arrays, raw device pointers, stream
handles); every step of the computation runs in the library.  Loading fails
loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libcsrk.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "csrk.h")

F64, F32, BF16 = 0, 1, 2
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}
MODELS = {"mi355x": 0, "volta": 1, "ampere": 2, "host_cpu": 3}
REORDERS = {"bandk": 0, "rcm": 1, "none": 2}
STATUS = {0: "CSRK_OK", 1: "CSRK_ERR_ARG", 3: "CSRK_ERR_BAD_ROWPTR", 4: "CSRK_ERR_COL_RANGE",
          5: "CSRK_ERR_DUPLICATE", 6: "CSRK_ERR_ALLOC", 7: "CSRK_ERR_DEVICE", 8: "CSRK_ERR_UNSUPPORTED"}


class csrk_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("srs", ctypes.c_int32), ("ssrs", ctypes.c_int32),
                ("lanes_per_row", ctypes.c_int32), ("waves_per_wg", ctypes.c_int32), ("reorder", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class csrk_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("nsr", ctypes.c_int32), ("nssr", ctypes.c_int32),
                ("rdensity", ctypes.c_double), ("row_variance", ctypes.c_double), ("max_row", ctypes.c_int32),
                ("bandwidth_input", ctypes.c_int32), ("bandwidth", ctypes.c_int32), ("symmetry", ctypes.c_double),
                ("max_sr_nnz", ctypes.c_int32), ("max_ssr_rows", ctypes.c_int32), ("on_device", ctypes.c_int32),
                ("store", ctypes.c_int32), ("long_rows", ctypes.c_int32), ("values_symmetric", ctypes.c_int32),
                ("params", csrk_params), ("adjoint_union", ctypes.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "params"}
        d["params"] = self.params.as_dict()
        return d


class CsrkError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {detail}")


_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_h = ctypes.c_void_p

_SIGS = {
    "csrk_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "csrk_last_error_detail": ([], ctypes.c_char_p),
    "csrk_tune": ([ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(csrk_params)], ctypes.c_int),
    "csrk_tune_rhs": ([ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(csrk_params)],
                      ctypes.c_int),
    "csrk_spmv_host": ([_h, _f64p, _f64p, ctypes.c_int32], ctypes.c_int),
    "csrk_cg": ([_h, _vp, _vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.POINTER(ctypes.c_int32),
                 ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "csrk_cg_noalloc": ([_h, _vp, _vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _vp,
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "csrk_cg_noalloc_bytes": ([_h, _i64p], ctypes.c_int),
    "csrk_build_host": ([ctypes.c_int32, ctypes.c_int64, _i32p, _i32p, _vp, ctypes.c_int,
                         ctypes.POINTER(csrk_params), ctypes.POINTER(_h)], ctypes.c_int),
    "csrk_build_from_groups": ([ctypes.c_int32, ctypes.c_int64, _i32p, _i32p, _vp, ctypes.c_int, _i32p, ctypes.c_int32,
                                _i32p, ctypes.c_int32, _i32p, ctypes.POINTER(csrk_params), ctypes.POINTER(_h)],
                               ctypes.c_int),
    "csrk_upload": ([_h, ctypes.c_int], ctypes.c_int),
    "csrk_build": ([ctypes.c_int32, ctypes.c_int64, _i32p, _i32p, _vp, ctypes.c_int, ctypes.c_int,
                    ctypes.POINTER(csrk_params), ctypes.POINTER(_h)], ctypes.c_int),
    "csrk_set_launch": ([_h, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "csrk_get_info": ([_h, ctypes.POINTER(csrk_info)], ctypes.c_int),
    "csrk_copy_structure": ([_h, _i32p, _i32p, _i32p, _f64p, _i64p, _i32p, _i32p], ctypes.c_int),
    "csrk_copy_union": ([_h, ctypes.POINTER(ctypes.c_int64), _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "csrk_level_ptr": ([_h, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _vp], ctypes.c_int),
    "csrk_device_vals": ([_h, ctypes.POINTER(_vp)], ctypes.c_int),
    "csrk_copy_device_vals": ([_h, _vp, _vp], ctypes.c_int),
    "csrk_spmv": ([_h, _vp, _vp, _vp, ctypes.c_int32, _vp], ctypes.c_int),
    "csrk_spmv_plain": ([_h, _vp, _vp, _vp, ctypes.c_int32, _vp], ctypes.c_int),
    "csrk_spmv_adjoint": ([_h, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp], ctypes.c_int),
    "csrk_permute": ([_h, ctypes.c_int32, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp], ctypes.c_int),
    "csrk_destroy": ([_h], ctypes.c_int),
    "csrk_batch_create": ([ctypes.POINTER(_h), ctypes.c_int32, ctypes.POINTER(_h)], ctypes.c_int),
    "csrk_batch_spmv": ([_h, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int32, _vp],
                        ctypes.c_int),
    "csrk_batch_spmv_adjoint": ([_h, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                 ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int32, _vp], ctypes.c_int),
    "csrk_batch_set_launch": ([_h, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "csrk_batch_destroy": ([_h], ctypes.c_int),
    "csrk_probe_read": ([_vp, ctypes.c_int64, _vp, _vp], ctypes.c_int),
    "csrk_probe_copy": ([_vp, _vp, ctypes.c_int64, _vp], ctypes.c_int),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libcsrk.so not built ({LIB_PATH}); run __graft_entry__.build() "
                              "or python -m paper_2203_05096_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/csrk.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(csrk_[a-z_]+)\s*\(", text)))


def _check(status: int, where: str):
    if status != 0:
        raise CsrkError(status, where, lib().csrk_last_error_detail().decode())


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


_IN_DTYPE = {np.dtype(np.float64): F64, np.dtype(np.float32): F32, np.dtype(np.uint16): BF16}


def _vals(a, in_dtype=None):
    """(contiguous value array, csrk_dtype): float64 -> F64, float32 -> F32, uint16 (BF16 bit patterns) -> BF16;
    other types are converted to float64.  ``in_dtype`` ("f64", "f32", "bf16") forces the type."""
    if a is None:
        return None, F64
    if in_dtype is not None:
        dt = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16}[in_dtype]
        return np.ascontiguousarray(a, dtype=dt), DTYPES[in_dtype]
    a = np.asarray(a)
    if a.dtype in _IN_DTYPE:
        return np.ascontiguousarray(a), _IN_DTYPE[a.dtype]
    return np.ascontiguousarray(a, dtype=np.float64), F64


def _params(p):
    if p is None:
        return None
    if isinstance(p, csrk_params):
        return p
    q = csrk_params()
    d = dict(p)
    if isinstance(d.get("reorder"), str):
        d["reorder"] = REORDERS[d["reorder"]]
    d.setdefault("k", 3)
    for f, _ in csrk_params._fields_:
        setattr(q, f, int(d[f]))
    return q


# ----------------------------------------------------------------- entry points

def csrk_status_string(status: int) -> str:
    return lib().csrk_status_string(status).decode()


def csrk_last_error_detail() -> str:
    return lib().csrk_last_error_detail().decode()


def csrk_tune(n: int, nnz: int, model: str = "mi355x") -> dict:
    p = csrk_params()
    _check(lib().csrk_tune(int(n), int(nnz), MODELS[model] if isinstance(model, str) else int(model), ctypes.byref(p)),
           "csrk_tune")
    return p.as_dict()


def csrk_tune_rhs(n: int, nnz: int, nrhs: int, model: str = "mi355x") -> dict:
    p = csrk_params()
    _check(lib().csrk_tune_rhs(int(n), int(nnz), int(nrhs), MODELS[model] if isinstance(model, str) else int(model),
                               ctypes.byref(p)), "csrk_tune_rhs")
    return p.as_dict()


def _vptr(a):
    return None if a is None else a.ctypes.data


def csrk_build_host(row_ptr, col_idx, vals=None, params=None, in_dtype=None) -> int:
    rp, ci = _i32(row_ptr), _i32(col_idx)
    va, vt = _vals(vals, in_dtype)
    h = _h()
    p = _params(params)
    _check(lib().csrk_build_host(len(rp) - 1, int(rp[-1]) if len(rp) else 0, _ptr(rp, _i32p), _ptr(ci, _i32p),
                                 _vptr(va), vt, ctypes.byref(p) if p is not None else None, ctypes.byref(h)),
           "csrk_build_host")
    return h.value


def csrk_build_from_groups(row_ptr, col_idx, vals, perm, sr_sizes, ssr_sizes, params=None, in_dtype=None) -> int:
    rp, ci = _i32(row_ptr), _i32(col_idx)
    va, vt = _vals(vals, in_dtype)
    pm, srz, ssrz = _i32(perm), _i32(sr_sizes), _i32(ssr_sizes)
    h = _h()
    p = _params(params)
    _check(lib().csrk_build_from_groups(len(rp) - 1, int(rp[-1]), _ptr(rp, _i32p), _ptr(ci, _i32p), _vptr(va), vt,
                                        _ptr(pm, _i32p), len(srz), _ptr(srz, _i32p), len(ssrz), _ptr(ssrz, _i32p),
                                        ctypes.byref(p) if p is not None else None, ctypes.byref(h)),
           "csrk_build_from_groups")
    return h.value


def csrk_upload(h: int, store: str = "f64"):
    _check(lib().csrk_upload(h, DTYPES[store]), "csrk_upload")


def csrk_build(row_ptr, col_idx, vals, params=None, store: str = "f64", in_dtype=None) -> int:
    """Host build + upload.  ``vals``: float64, float32 or uint16 (BF16 bit patterns) array, or None."""
    rp, ci = _i32(row_ptr), _i32(col_idx)
    va, vt = _vals(vals, in_dtype)
    h = _h()
    p = _params(params)
    _check(lib().csrk_build(len(rp) - 1, int(rp[-1]), _ptr(rp, _i32p), _ptr(ci, _i32p), _vptr(va), vt, DTYPES[store],
                            ctypes.byref(p) if p is not None else None, ctypes.byref(h)), "csrk_build")
    return h.value


def csrk_set_launch(h: int, lanes_per_row: int, waves_per_wg: int):
    _check(lib().csrk_set_launch(h, int(lanes_per_row), int(waves_per_wg)), "csrk_set_launch")


def csrk_get_info(h: int) -> dict:
    i = csrk_info()
    _check(lib().csrk_get_info(h, ctypes.byref(i)), "csrk_get_info")
    return i.as_dict()


def csrk_copy_structure(h: int) -> dict:
    info = csrk_get_info(h)
    n, nnz, nsr, nssr = info["n"], info["nnz"], info["nsr"], info["nssr"]
    out = {"perm": np.empty(n, np.int32), "row_ptr": np.empty(n + 1, np.int32), "col_idx": np.empty(nnz, np.int32),
           "vals": np.empty(nnz, np.float64), "vmap": np.empty(nnz, np.int64), "sr_ptr": np.empty(nsr + 1, np.int32),
           "ssr_ptr": np.empty(nssr + 1, np.int32)}
    _check(lib().csrk_copy_structure(h, _ptr(out["perm"], _i32p), _ptr(out["row_ptr"], _i32p),
                                     _ptr(out["col_idx"], _i32p), _ptr(out["vals"], _f64p), _ptr(out["vmap"], _i64p),
                                     _ptr(out["sr_ptr"], _i32p), _ptr(out["ssr_ptr"], _i32p)), "csrk_copy_structure")
    return out


def csrk_copy_union(h: int):
    """The union-pattern index of a nonsymmetric handle as numpy arrays, or None when it has none."""
    nu = ctypes.c_int64(0)
    _check(lib().csrk_copy_union(h, ctypes.byref(nu), None, None, None, None, None), "csrk_copy_union")
    if nu.value == 0:
        return None
    info = csrk_get_info(h)
    out = {"u_col": np.empty(nu.value, np.int32), "u_src": np.empty(nu.value, np.int32),
           "erow_ptr": np.empty(info["n"] + 1, np.int32), "sr_begin": np.empty(info["nsr"], np.int32),
           "sr_end": np.empty(info["nsr"], np.int32)}
    ptr = lambda a: a.ctypes.data_as(_vp)  # noqa: E731
    _check(lib().csrk_copy_union(h, ctypes.byref(nu), ptr(out["u_col"]), ptr(out["u_src"]), ptr(out["erow_ptr"]),
                                 ptr(out["sr_begin"]), ptr(out["sr_end"])), "csrk_copy_union")
    return out


def csrk_level_ptr(h: int, level: int) -> np.ndarray:
    """Pointer array of grouping level `level` (1 = sr_ptr, 2 = ssr_ptr, 3 .. k-1 higher levels)."""
    count = ctypes.c_int32(0)
    _check(lib().csrk_level_ptr(h, level, ctypes.byref(count), None), "csrk_level_ptr")
    out = np.empty(count.value + 1, dtype=np.int32)
    _check(lib().csrk_level_ptr(h, level, ctypes.byref(count), out.ctypes.data_as(_vp)), "csrk_level_ptr")
    return out


def csrk_device_vals(h: int) -> int:
    p = _vp()
    _check(lib().csrk_device_vals(h, ctypes.byref(p)), "csrk_device_vals")
    return p.value


def csrk_copy_device_vals(h: int, dst_dev, stream):
    _check(lib().csrk_copy_device_vals(h, dst_dev, stream), "csrk_copy_device_vals")


def csrk_spmv(h: int, vals_dev, x_dev, y_dev, nrhs: int, stream):
    _check(lib().csrk_spmv(h, vals_dev, x_dev, y_dev, int(nrhs), stream), "csrk_spmv")


def csrk_spmv_host(h: int, x, y=None, nthreads: int = 0):
    """y' = A' x' on the host CPU; x (and y) float64 arrays of length n in permuted space."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if y is None:
        y = np.empty_like(x)
    if y.dtype != np.float64 or not y.flags.c_contiguous or y.shape != x.shape:
        raise ValueError("y must be a contiguous float64 array shaped like x")
    _check(lib().csrk_spmv_host(h, x.ctypes.data_as(_f64p), y.ctypes.data_as(_f64p), int(nthreads)), "csrk_spmv_host")
    return y


def csrk_cg(h: int, b_dev, x_dev, rtol: float, max_iter: int, check_every: int, stream):
    """Runs csrk_cg; returns (iterations, relative recurrence residual)."""
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    _check(lib().csrk_cg(h, b_dev, x_dev, float(rtol), int(max_iter), int(check_every), stream, ctypes.byref(it),
                         ctypes.byref(rr)), "csrk_cg")
    return it.value, rr.value


def csrk_cg_noalloc(h: int, b_dev, x_dev, rtol: float, max_iter: int, check_every: int, stream):
    """Runs csrk_cg_noalloc (work memory in the library's fixed per-device array); returns (iterations, relative
    recurrence residual)."""
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    _check(lib().csrk_cg_noalloc(h, b_dev, x_dev, float(rtol), int(max_iter), int(check_every), stream,
                                 ctypes.byref(it), ctypes.byref(rr)), "csrk_cg_noalloc")
    return it.value, rr.value


def csrk_cg_noalloc_bytes(h: int) -> int:
    """Device work memory csrk_cg_noalloc needs for this handle, in bytes."""
    b = ctypes.c_int64(0)
    _check(lib().csrk_cg_noalloc_bytes(h, ctypes.byref(b)), "csrk_cg_noalloc_bytes")
    return b.value


CG_NOALLOC_BYTES = 64 << 20  # CSRK_CG_NOALLOC_BYTES


def csrk_spmv_plain(h: int, vals_dev, x_dev, y_dev, nrhs: int, stream):
    _check(lib().csrk_spmv_plain(h, vals_dev, x_dev, y_dev, int(nrhs), stream), "csrk_spmv_plain")


def csrk_spmv_adjoint(h: int, vals_dev, x_dev, g_dev, grad_x_dev, grad_vals_dev, nrhs: int, stream):
    _check(lib().csrk_spmv_adjoint(h, vals_dev, x_dev, g_dev, grad_x_dev, grad_vals_dev, int(nrhs), stream),
           "csrk_spmv_adjoint")


def csrk_permute(h: int, direction: int, in_dev, out_dev, nrhs: int, elem_bytes: int, stream):
    _check(lib().csrk_permute(h, int(direction), in_dev, out_dev, int(nrhs), int(elem_bytes), stream), "csrk_permute")


def csrk_destroy(h: int):
    _check(lib().csrk_destroy(h), "csrk_destroy")


def _ptr_array(ptrs):
    if ptrs is None:
        return None
    return (_vp * len(ptrs))(*[p if p else None for p in ptrs])


def csrk_batch_create(handles) -> int:
    arr = (_h * len(handles))(*handles)
    b = _h()
    _check(lib().csrk_batch_create(arr, len(handles), ctypes.byref(b)), "csrk_batch_create")
    return b.value


def csrk_batch_spmv(b: int, vals, x, y, nrhs: int, stream):
    _check(lib().csrk_batch_spmv(b, _ptr_array(vals), _ptr_array(x), _ptr_array(y), int(nrhs), stream),
           "csrk_batch_spmv")


def csrk_batch_spmv_adjoint(b: int, vals, x, g, grad_x, grad_vals, nrhs: int, stream):
    _check(lib().csrk_batch_spmv_adjoint(b, _ptr_array(vals), _ptr_array(x), _ptr_array(g), _ptr_array(grad_x),
                                         _ptr_array(grad_vals), int(nrhs), stream), "csrk_batch_spmv_adjoint")


def csrk_batch_set_launch(b: int, blocks_per_cu: int = 0, waves_per_wg: int = 0):
    _check(lib().csrk_batch_set_launch(b, int(blocks_per_cu), int(waves_per_wg)), "csrk_batch_set_launch")


def csrk_batch_destroy(b: int):
    _check(lib().csrk_batch_destroy(b), "csrk_batch_destroy")


def csrk_probe_read(buf_dev, nbytes: int, part_dev, stream):
    _check(lib().csrk_probe_read(buf_dev, int(nbytes), part_dev, stream), "csrk_probe_read")


def csrk_probe_copy(src_dev, dst_dev, nbytes: int, stream):
    _check(lib().csrk_probe_copy(src_dev, dst_dev, int(nbytes), stream), "csrk_probe_copy")
