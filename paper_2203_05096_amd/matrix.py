"""Torch-facing wrappers of the CSR-k library: CsrkMatrix, CsrkSpMV, CsrkBatch.

PyTorch supplies device memory and streams; every computation runs in
libcsrk.so (host preprocessing in C++, products in HIP kernels).  Vectors are
torch tensors on the GPU in the matrix's permuted row order; ``to_permuted`` /
``from_permuted`` move them between input and permuted order.
"""

from __future__ import annotations

import numpy as np
import torch

from . import _capi as C

_VEC_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32}
_VAL_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}
_GRADV_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32}


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


class CsrkMatrix:
    """A square sparse matrix in CSR-k form, resident on the current GPU.

    Build with :meth:`from_csr`.  ``params`` is a dict of csrk_params fields
    (``srs``, ``ssrs``, ``lanes_per_row``, ``waves_per_wg``, ``reorder``) or
    None for the constant-time model of ``model``.
    """

    def __init__(self, handle: int, store: str):
        self.handle = handle
        self.store = store
        self.info = C.csrk_get_info(handle)
        self.n = self.info["n"]
        self.nnz = self.info["nnz"]
        self.params = self.info["params"]
        self.vec_dtype = _VEC_DTYPE[store]
        self.val_dtype = _VAL_DTYPE[store]

    @classmethod
    def from_csr(cls, row_ptr, col_idx, vals, store: str = "f64", model: str = "mi355x", params=None,
                 nrhs: int = 1):
        """``nrhs``: width of the right-hand-side blocks the matrix will mostly be used with (tuning only)."""
        if not torch.cuda.is_available():
            raise RuntimeError("CsrkMatrix needs a GPU")
        if params is None:
            params = C.csrk_tune_rhs(len(row_ptr) - 1, int(np.asarray(row_ptr)[-1]), nrhs, model)
        h = C.csrk_build(row_ptr, col_idx, vals, params, store)
        return cls(h, store)

    # ---------------------------------------------------------------- data
    def structure(self) -> dict:
        """Host copy of perm, row_ptr, col_idx, vals (FP64 master), vmap, sr_ptr, ssr_ptr."""
        return C.csrk_copy_structure(self.handle)

    def values(self) -> torch.Tensor:
        """A new tensor holding the stored values (CSR-k order, storage dtype)."""
        t = torch.empty(self.nnz, dtype=self.val_dtype, device="cuda")
        C.csrk_copy_device_vals(self.handle, t.data_ptr(), _stream())
        return t

    def _check_vec(self, t, name, nrhs=None):
        if t.device.type != "cuda" or t.dtype != self.vec_dtype or not t.is_contiguous() or t.dim() not in (1, 2):
            raise TypeError(f"{name} must be a contiguous {self.vec_dtype} CUDA tensor of shape (n,) or (n, nrhs)")
        if t.shape[0] != self.n:
            raise ValueError(f"{name} has {t.shape[0]} rows, matrix has {self.n}")
        k = 1 if t.dim() == 1 else t.shape[1]
        if nrhs is not None and k != nrhs:
            raise ValueError(f"{name} has {k} columns, expected {nrhs}")
        return k

    def _check_vals(self, vals):
        if vals is None:
            return None
        if vals.dtype != self.val_dtype or vals.device.type != "cuda" or not vals.is_contiguous() or \
                vals.numel() != self.nnz:
            raise TypeError(f"vals must be a contiguous {self.val_dtype} CUDA tensor of {self.nnz} elements")
        return vals.data_ptr()

    def _check_grad_vals(self, t):
        dt = _GRADV_DTYPE[self.store]
        if t.dtype != dt or t.device.type != "cuda" or not t.is_contiguous() or t.numel() != self.nnz:
            raise TypeError(f"grad_vals output must be a contiguous {dt} CUDA tensor of {self.nnz} elements")
        return t

    # ---------------------------------------------------------------- products
    def spmv(self, x: torch.Tensor, y: torch.Tensor | None = None, vals: torch.Tensor | None = None) -> torch.Tensor:
        """y' = A' x' (permuted space); x is (n,) or (n, nrhs)."""
        nrhs = self._check_vec(x, "x")
        if y is None:
            y = torch.empty_like(x)
        self._check_vec(y, "y", nrhs)
        C.csrk_spmv(self.handle, self._check_vals(vals), _ptr(x), _ptr(y), nrhs, _stream())
        return y

    def cg(self, b: torch.Tensor, x0: torch.Tensor | None = None, rtol: float = 1e-8, max_iter: int = 10000,
           check_every: int = 10):
        """Conjugate gradients for A' x = b (permuted space, float64 device vectors); returns (x, iterations,
        relative residual)."""
        for t, name in ((b, "b"), (x0, "x0")):
            if t is None:
                continue
            if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous() or t.shape != (self.n,):
                raise TypeError(f"{name} must be a contiguous float64 CUDA vector of length {self.n}")
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        it, rel = C.csrk_cg(self.handle, _ptr(b), _ptr(x), rtol, max_iter, check_every, _stream())
        return x, it, rel

    def spmv_plain(self, x, y=None, vals=None):
        """Same product with the plain CSR kernel (no super-row levels)."""
        nrhs = self._check_vec(x, "x")
        if y is None:
            y = torch.empty_like(x)
        self._check_vec(y, "y", nrhs)
        C.csrk_spmv_plain(self.handle, self._check_vals(vals), _ptr(x), _ptr(y), nrhs, _stream())
        return y

    def adjoint(self, x, g, vals=None, grad_x: bool = True, grad_vals: bool = True, out_x=None, out_vals=None):
        """(A'^T g', g'_i x'_j per stored entry); either part may be skipped."""
        nrhs = self._check_vec(g, "g")
        if grad_vals:
            self._check_vec(x, "x", nrhs)
        gx = None
        gv = None
        if grad_x:
            gx = out_x if out_x is not None else torch.empty_like(g)
            self._check_vec(gx, "grad_x", nrhs)
        if grad_vals:
            gv = self._check_grad_vals(out_vals) if out_vals is not None else \
                torch.empty(self.nnz, dtype=_GRADV_DTYPE[self.store], device="cuda")
        C.csrk_spmv_adjoint(self.handle, self._check_vals(vals), _ptr(x) if grad_vals else None, _ptr(g), _ptr(gx),
                            _ptr(gv), nrhs, _stream())
        return gx, gv

    def _permute(self, v: torch.Tensor, direction: int) -> torch.Tensor:
        if v.device.type != "cuda" or v.dim() not in (1, 2) or v.shape[0] != self.n or v.element_size() not in (4, 8):
            raise TypeError(f"expected a CUDA tensor of shape ({self.n},) or ({self.n}, k) with 4- or 8-byte elements")
        v = v.contiguous()
        out = torch.empty_like(v)
        C.csrk_permute(self.handle, direction, _ptr(v), _ptr(out), 1 if v.dim() == 1 else v.shape[1],
                       v.element_size(), _stream())
        return out

    def to_permuted(self, v: torch.Tensor) -> torch.Tensor:
        """v' = v[perm] (input order to the matrix's row order)."""
        return self._permute(v, 0)

    def from_permuted(self, v: torch.Tensor) -> torch.Tensor:
        """v[perm] = v' (the matrix's row order back to input order)."""
        return self._permute(v, 1)

    def close(self):
        if self.handle:
            C.csrk_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CsrkSpMV(torch.autograd.Function):
    """y = A x with A's stored values as a differentiable tensor.

    ``CsrkSpMV.apply(M, vals, x)``: vals in CSR-k order (M.values()), x in
    permuted space.  Backward calls the library's adjoint (grad_x = A^T g,
    grad_vals = g_i x_j).  Gradients of BF16-stored values are returned in
    float32 and are not supported by autograd (use M.adjoint directly).
    """

    @staticmethod
    def forward(ctx, M: CsrkMatrix, vals: torch.Tensor, x: torch.Tensor):
        ctx.M = M
        ctx.save_for_backward(vals, x)
        return M.spmv(x.contiguous(), vals=vals)

    @staticmethod
    def backward(ctx, gy):
        vals, x = ctx.saved_tensors
        M = ctx.M
        need_vals, need_x = ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        gx, gv = M.adjoint(x, gy.contiguous(), vals=vals, grad_x=need_x, grad_vals=need_vals)
        if gv is not None and gv.dtype != vals.dtype:
            raise NotImplementedError("value gradients for BF16 storage are not supported by autograd")
        return None, gv, gx


class CsrkBatch:
    """Many CSR-k matrices (same storage type) multiplied in one launch."""

    def __init__(self, mats):
        self.mats = list(mats)
        self.store = self.mats[0].store
        self.handle = C.csrk_batch_create([m.handle for m in self.mats])

    def _same_count(self, **lists):
        for name, v in lists.items():
            if v is not None and len(v) != len(self.mats):
                raise ValueError(f"{name} has {len(v)} entries, the batch has {len(self.mats)} matrices")

    def spmv(self, xs, ys=None, vals=None):
        self._same_count(xs=xs, ys=ys, vals=vals)
        nrhs = 1 if xs[0].dim() == 1 else xs[0].shape[1]
        if ys is None:
            ys = [torch.empty_like(x) for x in xs]
        for m, x, y in zip(self.mats, xs, ys):
            m._check_vec(x, "x", nrhs)
            m._check_vec(y, "y", nrhs)
        vp = None if vals is None else [m._check_vals(v) for m, v in zip(self.mats, vals)]
        C.csrk_batch_spmv(self.handle, vp, [_ptr(x) for x in xs], [_ptr(y) for y in ys], nrhs, _stream())
        return ys

    def adjoint(self, xs, gs, vals=None, grad_x=True, grad_vals=True, out_x=None, out_vals=None):
        self._same_count(xs=xs if grad_vals else None, gs=gs, vals=vals, out_x=out_x, out_vals=out_vals)
        nrhs = 1 if gs[0].dim() == 1 else gs[0].shape[1]
        gxs = None
        gvs = None
        if grad_x:
            gxs = out_x if out_x is not None else [torch.empty_like(g) for g in gs]
        if grad_vals:
            gvs = out_vals if out_vals is not None else [
                torch.empty(m.nnz, dtype=_GRADV_DTYPE[m.store], device="cuda") for m in self.mats]
        for i, m in enumerate(self.mats):
            m._check_vec(gs[i], "g", nrhs)
            if grad_vals:
                m._check_vec(xs[i], "x", nrhs)
                m._check_grad_vals(gvs[i])
            if grad_x:
                m._check_vec(gxs[i], "grad_x", nrhs)
        vp = None if vals is None else [m._check_vals(v) for m, v in zip(self.mats, vals)]
        C.csrk_batch_spmv_adjoint(self.handle, vp, [_ptr(x) for x in xs] if grad_vals else None,
                                  [_ptr(g) for g in gs],
                                  None if gxs is None else [_ptr(t) for t in gxs],
                                  None if gvs is None else [_ptr(t) for t in gvs], nrhs, _stream())
        return gxs, gvs

    def close(self):
        if self.handle:
            C.csrk_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
