"""Benchmark of the CSR-k hot path on one MI355X.

One step = the CSR-k forward product y = A x followed by its adjoint
(grad_x = A^T g, grad_vals = g_i x_j) on one workload.  The headline workload
is the largest single-GPU one: 64 3D 7-point Laplacians with sides drawn from
16..96 (17.5 M rows, 120.8 M nonzeros), each with a block of 8 right-hand
sides, FP32 values and vectors, one batched launch per direction.  The other
workloads are measured in the same run and reported under extras.configs:
the 3D 7-point 128^3 scrambled Laplacian (FP64), the 3D 27-point 100^3
stencil in FP64 / FP32 / BF16 storage, the 2D 9-point 2048^2 stencil with 10%
of off-diagonals dropped (FP32, nonsymmetric) and an R-MAT graph of 2^20 rows
(FP64, irregular).

Timing (the paper's Section 5.4 protocol, with a cache flush): the
reordering, grouping, size choice and upload run before any timing; data
stays resident on the GPU; W untimed warm-up steps, then exactly K timed
steps, each preceded by a 1 GiB read that evicts the L2s and the 256 MB
Infinity Cache, with HIP events on the launch stream around each kernel.
Reported per kernel: mean, min and standard deviation over the K runs; the
mean is the headline.  Warm back-to-back times (the iterative-solver steady
state) are reported beside them, labelled.  Prints one JSON line (the last
line of stdout).

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload all|c2|c3|c4|c5|irr] [--store f64|f32|bf16]
                    [--no-cpu] [--no-extras] [--copy-calibration]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "SpMV GFLOP/s + achieved HBM GB/s (% of peak), CSR-k vs plain CSR, fwd+adj"
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2203_05096_amd", "csrc", "device", f)
                  for f in sorted(os.listdir(os.path.join(ROOT, "paper_2203_05096_amd", "csrc", "device")))
                  if f.endswith((".hip", ".hpp"))]
VAL_BYTES = {"f64": 8, "f32": 4, "bf16": 2}
VEC_BYTES = {"f64": 8, "f32": 4, "bf16": 4}
WORKLOAD_NAMES = {"c2": "3d7pt_128cube_scrambled", "c3": "3d27pt_100cube", "c4": "2d9pt_2048sq_drop10",
                  "c5": "batch64_3d7pt_sides16to96_8rhs", "irr": "rmat_2pow20_rows_sym"}
DEFAULT_STORE = {"c2": "f64", "c3": "f64", "c4": "f32", "c5": "f32", "irr": "f64"}
HEADLINE = "c5"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def fwd_bytes(n, nnz, nsr, nssr, val_bytes=8, vec_bytes=8, nrhs=1):
    """Algorithmic bytes of one forward launch: vals + col_idx per nonzero; row_ptr, x, y per row; SR/SSR pointers."""
    return nnz * (val_bytes + 4) + n * (4 + 2 * vec_bytes * nrhs) + 4 * (nsr + nssr)


def adj_bytes(n, nnz, nsr, nssr, val_bytes=8, vec_bytes=8, nrhs=1):
    """Algorithmic bytes of one adjoint launch: col_idx, vals read and grad_vals written per nonzero;
    row_ptr, g, x read and grad_x written per row; SR/SSR pointers."""
    gv_bytes = 8 if val_bytes == 8 else 4
    return nnz * (4 + val_bytes + gv_bytes) + n * (4 + 3 * vec_bytes * nrhs) + 4 * (nsr + nssr)


def profiled_traffic(workload, store, direction):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) recorded in profiles/ for this kernel source,
    workload and direction, else None."""
    path = os.path.join(PROFILES, f"hbm_traffic_{WORKLOAD_NAMES[workload]}_{store}.txt")
    try:
        text = "".join(line for line in open(path) if not line.startswith("#"))
        rec = json.loads(text)
        if rec["kernel_source_sha256"] != kernel_source_hash():
            return None
        return int(rec["per_launch"][direction]["fetch_bytes"] + rec["per_launch"][direction]["write_bytes"])
    except (OSError, ValueError, KeyError):
        return None


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor()


def stats(ts):
    a = np.asarray(ts, dtype=np.float64) * 1e3  # ms -> us
    return {"mean": round(float(a.mean()), 2), "min": round(float(a.min()), 2), "std": round(float(a.std()), 2)}


def measure(torch, W, steps, warmup, flush):
    """Warm-up steps, then `steps` flushed steps (1 GiB read, then forward and adjoint with events around each on
    the launch stream), then `steps` warm back-to-back steps (wall clock, and events per kernel)."""
    for _ in range(warmup):
        W.fwd()
        W.adj()
    torch.cuda.synchronize()
    E = torch.cuda.Event
    ev = [(E(enable_timing=True), E(enable_timing=True), E(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b, c in ev:
        flush()
        a.record()
        W.fwd()
        b.record()
        W.adj()
        c.record()
    torch.cuda.synchronize()
    wall_flushed = (time.perf_counter() - t0) * 1e3 / steps
    f_fl = [a.elapsed_time(b) for a, b, _ in ev]
    a_fl = [b.elapsed_time(c) for _, b, c in ev]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        W.fwd()
        W.adj()
    torch.cuda.synchronize()
    wall_warm = (time.perf_counter() - t0) * 1e3 / steps
    ev = [(E(enable_timing=True), E(enable_timing=True), E(enable_timing=True)) for _ in range(steps)]
    for a, b, c in ev:
        a.record()
        W.fwd()
        b.record()
        W.adj()
        c.record()
    torch.cuda.synchronize()
    f_w = [a.elapsed_time(b) for a, b, _ in ev]
    a_w = [b.elapsed_time(c) for _, b, c in ev]
    fs, as_ = stats(f_fl), stats(a_fl)
    out = {"step_ms_flushed": round((fs["mean"] + as_["mean"]) / 1e3, 5),
           "wall_ms_per_step_flushed_incl_flush": round(wall_flushed, 5),
           "step_ms_warm_wall": round(wall_warm, 5)}
    for name, flushed, warm, nbytes, flops in (("forward", fs, f_w, W.fb, W.flops_fwd),
                                               ("adjoint", as_, a_w, W.ab, W.flops_adj)):
        us = flushed["mean"]
        out[name] = {"flushed_us": flushed, "warm_us": stats(warm)["mean"], "bytes": nbytes,
                     "GBs": round(nbytes / us / 1e3, 1), "GFLOPs": round(flops / us / 1e3, 1),
                     "frac_of_peak": round(nbytes / us / 1e3 / HBM_PEAK_GBS, 4)}
    out["GFLOPs_step"] = round((W.flops_fwd + W.flops_adj) / (fs["mean"] + as_["mean"]) / 1e3, 2)
    return out


def flushed_mean_us(torch, fn, flush, reps=20, warmup=3):
    for _ in range(warmup):
        fn()
    E = torch.cuda.Event
    ts = []
    for _ in range(reps):
        flush()
        a, b = E(enable_timing=True), E(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return stats(ts)


# ------------------------------------------------------------------------------------------ CPU oracle leg

def cpu_baseline(w, budget_s=12.0):
    """The C oracle (FP64 CSR; forward over rows and adjoint over columns, both OpenMP static) on a bounded sample
    of the headline workload: (matrix, right-hand-side column) products in input order, about budget_s of CPU
    work; GFLOP/s of forward + adjoint (2 and 3 flops per nonzero)."""
    from oracle import cref
    cref.lib()
    cores = cref.threads()
    flops = t_fwd = t_adj = 0.0
    used = 0
    mats = w["As"] if "As" in w else [w["A"]]
    xs = w["xs"] if "xs" in w else [w["x"]]
    gs = w["gs"] if "gs" in w else [w["g"]]
    order = np.argsort([-A.nnz for A in mats], kind="stable")  # largest matrices first
    for b in order:
        A = mats[b]
        X, G = xs[b].reshape(A.n, -1), gs[b].reshape(A.n, -1)
        index = cref.column_index(A.row_ptr, A.col_idx)
        for c in range(X.shape[1]):
            x, g = np.ascontiguousarray(X[:, c]), np.ascontiguousarray(G[:, c])
            cref.time_forward(A.row_ptr, A.col_idx, A.vals, x, 1)  # warm-up
            t_fwd += cref.time_forward(A.row_ptr, A.col_idx, A.vals, x, 5) / 5
            t_adj += cref.time_adjoint_gather(A.row_ptr, A.col_idx, A.vals, x, g, 3, index) / 3
            flops += 5.0 * A.nnz
            used += 1
            if 6 * t_fwd + 4 * t_adj > budget_s:
                break
        if 6 * t_fwd + 4 * t_adj > budget_s:
            break
    return {"value": round(flops / (t_fwd + t_adj) / 1e9, 3), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"{used} (matrix, right-hand side) products of the headline workload in input order, largest "
                      f"matrices first: forward (OpenMP over rows, {cores} threads) {t_fwd * 1e3:.2f} ms + adjoint "
                      f"(OpenMP over columns, gather form, {cores} threads) {t_adj * 1e3:.2f} ms",
            "cpu": cpu_model()}


def cpu_oracle_study(C, A, x, g, perm_bandk):
    """The C oracle on one matrix: forward and adjoint, input order and Band-k order, 1 thread and all threads
    (5 warm-ups and the mean of 20 forward runs; mean of 5 adjoint runs)."""
    from oracle import cref
    allc = cref.threads()
    out = {}
    rp2, ci2, v2 = None, None, None
    s = None
    for order in ("input", "bandk"):
        if order == "input":
            rp, ci, va, xx, gg = A.row_ptr, A.col_idx, A.vals, x, g
        else:
            if s is None:
                s = perm_bandk()
            rp, ci, va = s["row_ptr"], s["col_idx"], s["vals"]
            xx, gg = x[s["perm"]], g[s["perm"]]
        index = cref.column_index(rp, ci)
        for t in (1, allc):
            cref.set_threads(t)
            cref.time_forward(rp, ci, va, xx, 5)
            f = cref.time_forward(rp, ci, va, xx, 20) / 20
            a = cref.time_adjoint_gather(rp, ci, va, xx, gg, 5, index) / 5
            out[f"{order}_order_{t}_threads"] = {"forward_ms": round(f * 1e3, 3), "adjoint_ms": round(a * 1e3, 3),
                                                 "forward_GFLOPs": round(2 * A.nnz / f / 1e9, 3),
                                                 "adjoint_GFLOPs": round(3 * A.nnz / a / 1e9, 3)}
        cref.set_threads(allc)
    out["cpu"] = cpu_model()
    return out


# ------------------------------------------------------------------------------------------ library legs

class Single:
    """One CSR-k matrix."""

    def __init__(self, torch, C, CsrkMatrix, A, x, g, store, M=None, params=None):
        self.C, self.A, self.store = C, A, store
        self.params = params or C.csrk_tune(A.n, A.nnz, "mi355x")
        t = time.perf_counter()
        self.M = M or CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, self.params, store), store)
        self.build_s = time.perf_counter() - t
        self.info = self.M.info
        self.nsr, self.nssr = self.info["nsr"], self.info["nssr"]
        perm = self.M.structure()["perm"]
        dt = torch.float64 if store == "f64" else torch.float32
        self.xd = torch.from_numpy(x[perm]).to(dtype=dt).cuda()
        self.gd = torch.from_numpy(g[perm]).to(dtype=dt).cuda()
        self.y = torch.empty_like(self.xd)
        self.gx = torch.empty_like(self.xd)
        self.gv = torch.empty(A.nnz, dtype=dt, device="cuda")
        self.lib = C.lib()
        self.h, self.stream = self.M.handle, torch.cuda.current_stream().cuda_stream
        self.ptrs = [t.data_ptr() for t in (self.xd, self.y, self.gd, self.gx, self.gv)]
        vb, xb = VAL_BYTES[store], VEC_BYTES[store]
        self.fb = fwd_bytes(A.n, A.nnz, self.nsr, self.nssr, vb, xb)
        self.ab = adj_bytes(A.n, A.nnz, self.nsr, self.nssr, vb, xb)
        self.flops_fwd, self.flops_adj = 2.0 * A.nnz, 3.0 * A.nnz

    # The timed loops call the C entry points directly with pre-marshalled pointers, so host-side Python
    # overhead stays far below the kernel time.
    def fwd(self):
        px, py = self.ptrs[0], self.ptrs[1]
        if self.lib.csrk_spmv(self.h, None, px, py, 1, self.stream):
            raise RuntimeError(self.C.csrk_last_error_detail())

    def adj(self, gx=True, gv=True):
        px, _, pg, pgx, pgv = self.ptrs
        if self.lib.csrk_spmv_adjoint(self.h, None, px, pg, pgx if gx else None, pgv if gv else None, 1,
                                      self.stream):
            raise RuntimeError(self.C.csrk_last_error_detail())

    def accuracy(self, torch, x):
        """Forward error of y against an FP64 product computed with scipy.sparse on the input order (values
        rounded to the storage type first, so the figure is the kernel's rounding only), relative to
        sum_j |a_ij||x_j| per row; also against the FP64 values (storage rounding included)."""
        import scipy.sparse as sp
        A = self.A
        self.fwd()
        torch.cuda.synchronize()
        perm = self.M.structure()["perm"]
        y = np.empty(A.n)
        y[perm] = self.y.double().cpu().numpy()
        vals = A.vals
        if self.store != "f64":
            v32 = A.vals.astype(np.float32)
            if self.store == "bf16":
                u = v32.view(np.uint32).astype(np.uint64)
                u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16  # round to nearest even (finite values)
                v32 = u.astype(np.uint32).view(np.float32)
            vals = v32.astype(np.float64)
        xr = x if self.store == "f64" else x.astype(np.float32).astype(np.float64)
        M = sp.csr_matrix((vals, A.col_idx, A.row_ptr), shape=(A.n, A.n))
        M64 = sp.csr_matrix((A.vals, A.col_idx, A.row_ptr), shape=(A.n, A.n))
        scale = abs(M64) @ np.abs(xr)
        scale[scale == 0] = 1.0
        e_kernel = np.abs(y - M @ xr) / scale
        e_total = np.abs(y - M64 @ xr) / scale
        return {"max_rel_err_vs_stored_values": float(e_kernel.max()), "rms_rel_err_vs_stored_values":
                float(np.sqrt(np.mean(e_kernel ** 2))), "max_rel_err_vs_fp64_values": float(e_total.max()),
                "rms_rel_err_vs_fp64_values": float(np.sqrt(np.mean(e_total ** 2))),
                "reference": "scipy.sparse FP64 product, error / sum_j |a_ij||x_j| per row"}

    def config(self):
        return {"n": self.A.n, "nnz": self.A.nnz, "csrk_params": self.params, "nsr": self.nsr, "nssr": self.nssr,
                "bandwidth_after_reorder": self.info["bandwidth"], "build_seconds": round(self.build_s, 2)}

    def close(self):
        self.M.close()


class Batch:
    """Many CSR-k matrices with blocks of right-hand sides in one launch per direction."""

    def __init__(self, torch, C, CsrkMatrix, CsrkBatch, mats, xs, gs, store, nrhs):
        import concurrent.futures as cf
        self.C, self.store, self.nrhs = C, store, nrhs

        def one(A):
            p = C.csrk_tune_rhs(A.n, A.nnz, nrhs, "mi355x")
            return C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, p)
        t = time.perf_counter()
        with cf.ThreadPoolExecutor(16) as ex:
            hs = list(ex.map(one, mats))
        self.Ms = []
        for h in hs:
            C.csrk_upload(h, store)
            self.Ms.append(CsrkMatrix(h, store))
        self.build_s = time.perf_counter() - t
        self.B = CsrkBatch(self.Ms)
        dt = torch.float64 if store == "f64" else torch.float32
        self.xs, self.gs, self.ys, self.gxs, self.gvs = [], [], [], [], []
        for M, X, G in zip(self.Ms, xs, gs):
            perm = M.structure()["perm"]
            self.xs.append(torch.from_numpy(X[perm]).to(dtype=dt).cuda())
            self.gs.append(torch.from_numpy(G[perm]).to(dtype=dt).cuda())
            self.ys.append(torch.empty_like(self.xs[-1]))
            self.gxs.append(torch.empty_like(self.xs[-1]))
            self.gvs.append(torch.empty(M.nnz, dtype=dt, device="cuda"))
        vb, xb = VAL_BYTES[store], VEC_BYTES[store]
        self.fb = sum(fwd_bytes(M.n, M.nnz, M.info["nsr"], M.info["nssr"], vb, xb, nrhs) for M in self.Ms)
        self.ab = sum(adj_bytes(M.n, M.nnz, M.info["nsr"], M.info["nssr"], vb, xb, nrhs) for M in self.Ms)
        self.n, self.nnz = sum(M.n for M in self.Ms), sum(M.nnz for M in self.Ms)
        self.flops_fwd, self.flops_adj = 2.0 * self.nnz * nrhs, 3.0 * self.nnz * nrhs
        self.lib = C.lib()
        self.h, self.stream = self.B.handle, torch.cuda.current_stream().cuda_stream
        arr = C._ptr_array
        self.px = arr([t.data_ptr() for t in self.xs])
        self.py = arr([t.data_ptr() for t in self.ys])
        self.pg = arr([t.data_ptr() for t in self.gs])
        self.pgx = arr([t.data_ptr() for t in self.gxs])
        self.pgv = arr([t.data_ptr() for t in self.gvs])

    def fwd(self):
        if self.lib.csrk_batch_spmv(self.h, None, self.px, self.py, self.nrhs, self.stream):
            raise RuntimeError(self.C.csrk_last_error_detail())

    def adj(self, gx=True, gv=True):
        if self.lib.csrk_batch_spmv_adjoint(self.h, None, self.px, self.pg, self.pgx if gx else None,
                                            self.pgv if gv else None, self.nrhs, self.stream):
            raise RuntimeError(self.C.csrk_last_error_detail())

    def config(self):
        p = self.Ms[0].params
        return {"matrices": len(self.Ms), "n_total": self.n, "nnz_total": self.nnz, "nrhs": self.nrhs,
                "csrk_params_first": p, "build_seconds": round(self.build_s, 2)}

    def close(self):
        self.B.close()
        for M in self.Ms:
            M.close()


def plain_csr_study(torch, C, CsrkMatrix, W, x, flush):
    """The metric's comparison: the plain CSR kernel on the input order, the RCM order and the Band-k order,
    beside the CSR-k forward on the same orders (flushed means)."""
    A, store = W.A, W.store
    out = {}
    for name, reorder in (("input_order", "none"), ("rcm", "rcm"), ("bandk", None)):
        if reorder is None:
            Mp, xp = W.M, W.xd
        else:
            q = dict(W.params, reorder=reorder)
            Mp = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, q, store), store)
            xp = torch.from_numpy(x[Mp.structure()["perm"]]).to(dtype=W.xd.dtype).cuda()
        yp = torch.empty_like(xp)
        pm = flushed_mean_us(torch, lambda: Mp.spmv_plain(xp, yp), flush)
        km = flushed_mean_us(torch, lambda: Mp.spmv(xp, yp), flush)
        out[name] = {"plain_forward_us": pm, "plain_forward_GFLOPs": round(2 * A.nnz / pm["mean"] / 1e3, 1),
                     "csrk_forward_us": km, "csrk_forward_GFLOPs": round(2 * A.nnz / km["mean"] / 1e3, 1),
                     "bandwidth": Mp.info["bandwidth"]}
        if Mp is not W.M:
            Mp.close()
    return out


def cg_study(torch, C, CsrkMatrix, A, b, rtol=1e-8):
    """csrk_cg on the (symmetric positive definite) matrix with each value storage: iterations, solve time and
    the final relative residual, both the solver's recurrence one and ||b - A x|| / ||b|| with the FP64
    matrix (scipy.sparse product)."""
    import scipy.sparse as sp
    A64 = sp.csr_matrix((A.vals, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    h0 = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, C.csrk_tune(A.n, A.nnz, "mi355x"))
    perm = C.csrk_copy_structure(h0)["perm"]
    C.csrk_destroy(h0)
    out = {}
    for store in ("f64", "f32", "bf16"):
        M = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, C.csrk_tune(A.n, A.nnz, "mi355x"), store), store)
        bd = torch.from_numpy(np.ascontiguousarray(b[perm])).cuda()
        M.cg(bd, rtol=1e-2, max_iter=5, check_every=5)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xd, it, rel = M.cg(bd, rtol=rtol, max_iter=20000, check_every=25)
        ms = (time.perf_counter() - t0) * 1e3
        x = np.empty(A.n)
        x[perm] = xd.cpu().numpy()
        true = float(np.linalg.norm(b - A64 @ x) / np.linalg.norm(b))
        out[store] = {"iterations": it, "ms": round(ms, 2), "ms_per_iteration": round(ms / max(it, 1), 4),
                      "recurrence_rel_residual": rel, "true_rel_residual_fp64_matrix": true}
        M.close()
    out["note"] = f"rtol {rtol}, b = the workload's x vector, x0 = 0, convergence checked every 25 iterations"
    return out


def cpu_csrk_study(C, A, x, W):
    """The library's host CPU kernel (csrk_spmv_host) on this matrix, FP64, all host threads: CSR-2 tuned per
    matrix over the paper's SRS set against the constant-time SRS = 96 (Section 4.2); the GPU handle's CSR-3
    structure; and plain CSR (one row per unit) in input order and in Band-k order."""
    from paper_2203_05096_amd import host_tune as HT
    sw = HT.sweep_host(A)
    out = {"csr2_tuned": {"srs": sw["best_srs"], "us": round(sw["best_us"], 1)},
           "csr2_constant_time_srs96_us": round(sw["constant_time_us"], 1),
           "csr2_constant_over_tuned": round(sw["constant_over_best"], 3),
           "csr2_sweep_us": {str(s): round(us, 1) for s, us in sw["trials"]}}
    out["csr3_gpu_structure_us"] = round(HT.time_host(W.M.handle, x[W.M.structure()["perm"]]), 1)
    for name, reorder in (("plain_input_order_us", "none"), ("plain_bandk_order_us", "bandk")):
        if reorder == "none":
            p = {"k": 3, "srs": 1, "ssrs": 1, "lanes_per_row": 1, "waves_per_wg": 1, "reorder": "none"}
            h = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, p)
        else:  # Band-k rows, regrouped one row per super-row
            s = W.M.structure()
            ones = np.ones(A.n, np.int32)
            h = C.csrk_build_from_groups(A.row_ptr, A.col_idx, A.vals, s["perm"], ones, ones,
                                         dict(W.params, srs=1, ssrs=1))
        out[name] = round(HT.time_host(h, x[C.csrk_copy_structure(h)["perm"]]), 1)
        C.csrk_destroy(h)
    out["threads"] = sw["threads"]
    out["note"] = ("FP64 forward on the host, csrk_spmv_host with the OpenMP default thread count; 5 warm-ups, "
                   "mean of 20 runs")
    return out


def probe_bandwidth(torch, C):
    """Attainable HBM rates on this machine: the library's streaming-read and copy probes (16-byte non-temporal
    accesses over 4 GiB) and torch's sum / copy_ of a 2 GiB tensor, event-timed."""
    out = {}
    big = torch.ones(1 << 29, dtype=torch.float64, device="cuda")  # 4 GiB
    dst = torch.empty_like(big)
    part = torch.empty(1 << 16, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    nb = big.numel() * 8
    E = torch.cuda.Event
    for name, fn, moved in (("probe_read_GBs", lambda: C.csrk_probe_read(big.data_ptr(), nb, part.data_ptr(), st), nb),
                            ("probe_copy_GBs", lambda: C.csrk_probe_copy(big.data_ptr(), dst.data_ptr(), nb, st),
                             2 * nb)):
        fn()
        a, b = E(enable_timing=True), E(enable_timing=True)
        a.record()
        for _ in range(10):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[name] = round(moved * 10 / (a.elapsed_time(b) * 1e-3) / 1e9, 1)
    half = big[: 1 << 28]
    dst2 = dst[: 1 << 28]
    for name, fn, moved in (("torch_read_GBs", lambda: half.sum(), half.numel() * 8),
                            ("torch_copy_GBs", lambda: dst2.copy_(half), 2 * half.numel() * 8)):
        fn()
        a, b = E(enable_timing=True), E(enable_timing=True)
        a.record()
        for _ in range(10):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[name] = round(moved * 10 / (a.elapsed_time(b) * 1e-3) / 1e9, 1)
    del big, dst, part
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=["all"] + sorted(WORKLOAD_NAMES), default="all",
                    help="all: the headline workload plus every other one in extras.configs")
    ap.add_argument("--store", choices=["f64", "f32", "bf16"], default=None,
                    help="storage type of a single named workload (default: its own)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle and host-kernel legs")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the comparisons (plain CSR, CSR-2, CG, bandwidth probes, accuracy)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 1 GiB device copies (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    from paper_2203_05096_amd import _capi as C
    from paper_2203_05096_amd.matrix import CsrkBatch, CsrkMatrix

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    C.lib()  # fail loudly if the HIP library is missing
    head = HEADLINE if args.workload == "all" else args.workload
    if args.workload == "all":
        plan = [("c5", "f32"), ("c2", "f64"), ("c3", "f64"), ("c3", "f32"), ("c3", "bf16"), ("c4", "f32"),
                ("irr", "f64")]
    else:
        plan = [(head, args.store or DEFAULT_STORE[head])]
    head_store = plan[0][1]

    flush_buf = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB

    def flush():
        # a read-only pass over 1 GiB evicts the L2s and the 256 MB Infinity Cache without leaving dirty lines
        # behind for the timed kernel to write back
        flush_buf.sum()

    results, extras, head_W, head_w = {}, {}, None, None
    cache = {}
    for name, store in plan:
        if name not in cache:
            log(f"generating workload {name}")
            cache = {name: gen.WORKLOADS[name]()}  # one workload's host data at a time
        w = cache[name]
        if name == "c5":
            W = Batch(torch, C, CsrkMatrix, CsrkBatch, w["As"], w["xs"], w["gs"], store, w["nrhs"])
        else:
            W = Single(torch, C, CsrkMatrix, w["A"], w["x"], w["g"], store)
        log(f"{name} {store}: built in {W.build_s:.2f}s: {W.config()}")
        m = measure(torch, W, args.steps, args.warmup, flush)
        m["config"] = W.config()
        key = f"{name}_{store}"
        log(f"{key}: forward {m['forward']['flushed_us']} us, adjoint {m['adjoint']['flushed_us']} us (flushed); "
            f"warm {m['forward']['warm_us']} / {m['adjoint']['warm_us']} us")
        if not args.no_extras and isinstance(W, Single):
            if name in ("c2", "c4", "irr") or (name == "c3" and store == "f64"):
                m["plain_csr"] = plain_csr_study(torch, C, CsrkMatrix, W, w["x"], flush)
            if name == "c3" or name == "c4":
                m["accuracy"] = W.accuracy(torch, w["x"])
            if name == "c2":
                q = dict(W.params, k=2)
                M2 = CsrkMatrix(C.csrk_build(w["A"].row_ptr, w["A"].col_idx, w["A"].vals, q, store), store)
                x2 = torch.from_numpy(w["x"][M2.structure()["perm"]]).to(dtype=W.xd.dtype).cuda()
                y2 = torch.empty_like(x2)
                m["csr2_forward_us"] = flushed_mean_us(torch, lambda: M2.spmv(x2, y2), flush)
                M2.close()
                m["cg"] = cg_study(torch, C, CsrkMatrix, w["A"], w["x"])
        if name == "c2" and not args.no_cpu:
            log("host CPU kernel and oracle studies on c2")
            m["cpu_csrk"] = cpu_csrk_study(C, w["A"], w["x"], W)
            m["cpu_oracle"] = cpu_oracle_study(C, w["A"], w["x"], w["g"], lambda: W.M.structure())
        results[key] = m
        if name == head and store == head_store:
            head_W, head_key = W, key
            head_cfg = W.config()
            if not args.no_cpu:
                log("timing the CPU oracle on a sample of the headline workload")
                cpu = cpu_baseline(w)
        else:
            W.close()
        torch.cuda.synchronize()
    del flush_buf

    if not args.no_extras:
        extras["hbm_calibration"] = probe_bandwidth(torch, C)
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        extras["copy_calibration"] = "3 x copy of 1 GiB (read 1 GiB, write 1 GiB per dispatch)"

    h = results[head_key]
    dom = "adjoint" if h["adjoint"]["flushed_us"]["mean"] >= h["forward"]["flushed_us"]["mean"] else "forward"
    d = h[dom]
    achieved = d["bytes"] / d["flushed_us"]["mean"] / 1e3
    extras["configs"] = results
    extras["protocol"] = (f"{args.warmup} warm-up steps, then {args.steps} steps each preceded by a 1 GiB read "
                          "(L2s and Infinity Cache flushed); HIP events on the launch stream around each kernel; "
                          "value, ms_per_step and roofline use the flushed means; warm back-to-back times are in "
                          "extras.configs[*].step_ms_warm_wall and warm_us")
    out = {
        "metric": METRIC,
        "value": h["GFLOPs_step"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["step_ms_flushed"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head_store,
        "data": "synthetic",
        "config": dict({"workload": f"{WORKLOAD_NAMES[head]}_forward_adjoint_{head_store}"}, **head_cfg),
        "forward": h["forward"],
        "adjoint": h["adjoint"],
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic(head, head_store, dom), "algorithmic_bytes": d["bytes"],
                     "duration_us": d["flushed_us"]["mean"]},
        "cpu_baseline": None if args.no_cpu else cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
