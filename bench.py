"""Benchmark of the CSR-k hot path on one MI355X.

One step = the CSR-k forward product y = A x followed by its adjoint
(grad_x = A^T g, grad_vals = g_i x_j).  The default workload is the 3D
7-point Laplacian of a 128^3 grid (n = 2,097,152, nnz = 14,581,760) whose grid
points were relabelled at random, stored in FP64.  The reordering, grouping,
size choice and upload run before the timed region, as the paper times only
the kernels on data already on the GPU.  Prints one JSON line (the last line
of stdout).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c3|c4|c5|irr] [--store f64|f32|bf16]
                    [--no-cpu] [--no-extras] [--copy-calibration]

Other workloads: c3 = 3D 27-point 100^3 (precision study), c4 = 2D 9-point
2048^2 with 10% of off-diagonals dropped (nonsymmetric, FP32), c5 = 64 3D
7-point Laplacians of uneven size with 8 right-hand sides each, in one
batched launch per direction (FP32), irr = an R-MAT graph of 2^20
rows (power-law row lengths, the paper's irregular class; FP64).
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_csrk_3d7pt128_f64.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2203_05096_amd", "csrc", "device", "kernels.hip")
VAL_BYTES = {"f64": 8, "f32": 4, "bf16": 2}
VEC_BYTES = {"f64": 8, "f32": 4, "bf16": 4}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fwd_bytes(n, nnz, nsr, nssr, val_bytes=8, vec_bytes=8, nrhs=1):
    """Algorithmic bytes of one forward launch: vals + col_idx per nonzero; row_ptr, x, y per row; SR/SSR pointers."""
    return nnz * (val_bytes + 4) + n * (4 + 2 * vec_bytes * nrhs) + 4 * (nsr + nssr)


def adj_bytes(n, nnz, nsr, nssr, val_bytes=8, vec_bytes=8, nrhs=1):
    """Algorithmic bytes of one adjoint launch: col_idx, vals read and grad_vals written per nonzero;
    row_ptr, g, x read and grad_x written per row; SR/SSR pointers."""
    gv_bytes = 8 if val_bytes == 8 else 4
    return nnz * (4 + val_bytes + gv_bytes) + n * (4 + 3 * vec_bytes * nrhs) + 4 * (nsr + nssr)


def profiled_traffic(kernel_prefix, workload, store):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) recorded for this kernel source, else None."""
    if workload != "c2" or store != "f64":
        return None
    try:
        text = "".join(line for line in open(TRAFFIC_FILE) if not line.startswith("#"))
        rec = json.loads(text)
        if rec["kernel_source_sha256"] != hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest():
            return None
        for name, k in rec["kernels"].items():
            if name.startswith(kernel_prefix):
                return int(k["fetch_bytes"] + k["write_bytes"])
    except (OSError, ValueError, KeyError):
        return None
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


def timed_launches(torch, fns, steps, warmup):
    """Runs `warmup` untimed steps of the callables in `fns`, then exactly `steps` timed steps (wall clock,
    bracketed by device synchronisation, no events inside), then `steps` more with an event pair around
    every launch for the per-kernel means (events on the current stream, which is the launch stream).
    Returns wall ms/step and per-fn mean event ms."""
    for _ in range(warmup):
        for f in fns:
            f()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for f in fns:
            f()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
          for _ in fns]
    for s in range(steps):
        for i, f in enumerate(fns):
            ev[i][s][0].record()
            f()
            ev[i][s][1].record()
    torch.cuda.synchronize()
    per = [float(np.mean([a.elapsed_time(b) for a, b in ev[i]])) for i in range(len(fns))]
    return wall, per


def flushed_ms(torch, fn, flush, reps=20):
    """Mean event time of fn with the L2s and the 256 MB Infinity Cache flushed before every run."""
    ts = []
    for _ in range(reps):
        flush()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.mean(ts)), float(np.min(ts))


def cpu_baseline(mats, xs, gs, budget_s=12.0):
    """The C oracle (FP64 CSR, OpenMP static over rows for the forward, serial scatter for the adjoint) on the
    same matrices in their input order, one right-hand-side column at a time, on a bounded sample
    (about budget_s of CPU work); reported in GFLOP/s."""
    from oracle import cref
    cref.lib()
    flops = t_fwd = t_adj = 0.0
    used = 0
    for A, X, G in zip(mats, xs, gs):
        X = X.reshape(A.n, -1)
        G = G.reshape(A.n, -1)
        for c in range(X.shape[1]):
            x = np.ascontiguousarray(X[:, c])
            g = np.ascontiguousarray(G[:, c])
            reps_f = reps_a = 1
            if used == 0:  # repeat the first product until it alone fills a quarter of the budget each way
                reps_f = max(1, int((budget_s / 4) / max(cref.time_forward(A.row_ptr, A.col_idx, A.vals, x, 1),
                                                         1e-4)))
                reps_a = max(1, int((budget_s / 4) / max(cref.time_adjoint(A.row_ptr, A.col_idx, A.vals, x, g, 1),
                                                         1e-4)))
            t_fwd += cref.time_forward(A.row_ptr, A.col_idx, A.vals, x, reps_f) / reps_f
            t_adj += cref.time_adjoint(A.row_ptr, A.col_idx, A.vals, x, g, reps_a) / reps_a
            flops += 5.0 * A.nnz
            used += 1
            if t_fwd + t_adj > budget_s / 2:
                break
        if t_fwd + t_adj > budget_s / 2:
            break
    return {"value": round(flops / (t_fwd + t_adj) / 1e9, 3), "unit": "GFLOP/s", "cores": cref.threads(),
            "kind": "oracle",
            "sample": f"{used} (matrix, right-hand side) products in input order: forward (OpenMP static over "
                      f"rows) {t_fwd * 1e3:.2f} ms + adjoint (serial scatter) {t_adj * 1e3:.2f} ms",
            "cpu": cpu_model()}


def cg_study(torch, C, CsrkMatrix, A, b, rtol=1e-8):
    """csrk_cg on the (symmetric positive definite) matrix with each value storage: iterations, solve time and
    the final relative residual, both the solver's recurrence one and ||b - A x|| / ||b|| with the FP64
    matrix (scipy.sparse product)."""
    import scipy.sparse as sp
    A64 = sp.csr_matrix((A.vals, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    out = {}
    for store in ("f64", "f32", "bf16"):
        M = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, C.csrk_tune(A.n, A.nnz, "mi355x"), store), store)
        perm = M.structure()["perm"]
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


def cpu_csrk(C, A, x, W, reps=20):
    """The library's host CPU kernel (csrk_spmv_host, OpenMP over super-super-rows) on this matrix: the
    Band-k structure of the GPU handle, and plain CSR (one row per super-row, one super-row per
    super-super-row) in input order and in Band-k order.  FP64, all host threads; mean of `reps` runs
    after 3 warm-ups."""
    def t(h, xp):
        y = np.empty_like(xp)
        for _ in range(3):
            C.csrk_spmv_host(h, xp, y)
        t0 = time.perf_counter()
        for _ in range(reps):
            C.csrk_spmv_host(h, xp, y)
        return (time.perf_counter() - t0) / reps * 1e6
    out = {"csrk_bandk_us": round(t(W.M.handle, x[W.M.structure()["perm"]]), 1)}
    for name, reorder in (("plain_input_order_us", "none"), ("plain_bandk_order_us", "bandk")):
        if reorder == "none":
            p = {"k": 3, "srs": 1, "ssrs": 1, "lanes_per_row": 1, "waves_per_wg": 1, "reorder": "none"}
            h = C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, p)
        else:  # Band-k rows, regrouped one row per super-row
            s = W.M.structure()
            n = A.n
            ones = np.ones(n, np.int32)
            h = C.csrk_build_from_groups(A.row_ptr, A.col_idx, A.vals, s["perm"], ones, ones,
                                         dict(W.params, srs=1, ssrs=1))
        out[name] = round(t(h, x[C.csrk_copy_structure(h)["perm"]]), 1)
        C.csrk_destroy(h)
    out["threads"] = os.cpu_count()
    out["note"] = "FP64 forward on the host, csrk_spmv_host with the OpenMP default thread count"
    return out


class Single:
    """One CSR-k matrix (workloads c2, c3, c4)."""

    def __init__(self, torch, C, CsrkMatrix, A, x, g, store):
        self.C, self.A, self.store = C, A, store
        p = C.csrk_tune(A.n, A.nnz, "mi355x")
        t = time.perf_counter()
        self.M = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, p, store), store)
        self.build_s = time.perf_counter() - t
        self.params = p
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

    # The timed loop calls the C entry points directly with pre-marshalled pointers, so host-side
    # Python overhead stays far below the kernel time.
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


class Batch:
    """Many CSR-k matrices with blocks of right-hand sides in one launch (workload c5)."""

    def __init__(self, torch, C, CsrkMatrix, CsrkBatch, mats, xs, gs, store, nrhs):
        import concurrent.futures as cf
        self.C, self.store, self.nrhs = C, store, nrhs

        def one(A):
            p = C.csrk_tune_rhs(A.n, A.nnz, nrhs, "mi355x")
            return CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, p, store), store)
        t = time.perf_counter()
        with cf.ThreadPoolExecutor(16) as ex:
            self.Ms = list(ex.map(one, mats))
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
        return {"matrices": len(self.Ms), "n_total": self.n, "nnz_total": self.nnz, "nrhs": self.nrhs,
                "csrk_params_first": self.Ms[0].params, "build_seconds": round(self.build_s, 2)}


WORKLOAD_NAMES = {"c2": "3d7pt_128cube_scrambled_forward_adjoint", "c3": "3d27pt_100cube_forward_adjoint",
                  "c4": "2d9pt_2048sq_drop10_forward_adjoint", "c5": "batch64_3d7pt_sides16to96_8rhs_forward_adjoint",
                  "irr": "rmat_2pow20_rows_sym_forward_adjoint"}
DEFAULT_STORE = {"c2": "f64", "c3": "f64", "c4": "f32", "c5": "f32", "irr": "f64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=sorted(WORKLOAD_NAMES), default="c2")
    ap.add_argument("--store", choices=["f64", "f32", "bf16"], default=None)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip plain-CSR, flushed and calibration measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each box has one MI355X); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    store = args.store or DEFAULT_STORE[args.workload]

    import torch
    import gen
    from paper_2203_05096_amd import _capi as C
    from paper_2203_05096_amd.matrix import CsrkBatch, CsrkMatrix

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    C.lib()  # fail loudly if the HIP library is missing
    log(f"generating workload {args.workload}")
    w = gen.WORKLOADS[args.workload]()
    if args.workload == "c5":
        W = Batch(torch, C, CsrkMatrix, CsrkBatch, w["As"], w["xs"], w["gs"], store, w["nrhs"])
        mats, xs, gs = w["As"], w["xs"], w["gs"]
    else:
        W = Single(torch, C, CsrkMatrix, w["A"], w["x"], w["g"], store)
        mats, xs, gs = [w["A"]], [w["x"]], [w["g"]]
    log(f"built in {W.build_s:.2f}s: {W.config()}")

    torch.cuda.synchronize()
    wall_ms, (fwd_ms, adj_ms) = timed_launches(torch, [W.fwd, W.adj], args.steps, args.warmup)
    value = (W.flops_fwd + W.flops_adj) / (wall_ms * 1e-3) / 1e9
    fwd_gbs = W.fb / (fwd_ms * 1e-3) / 1e9
    adj_gbs = W.ab / (adj_ms * 1e-3) / 1e9
    dom = ("forward", fwd_ms, W.fb, fwd_gbs, "k_spmv_csrk") if fwd_ms >= adj_ms else \
        ("adjoint", adj_ms, W.ab, adj_gbs, "k_adjoint_csrk")
    log(f"step {wall_ms:.4f} ms; forward {fwd_ms * 1e3:.1f} us {fwd_gbs:.0f} GB/s; "
        f"adjoint {adj_ms * 1e3:.1f} us {adj_gbs:.0f} GB/s")

    extras = {}
    if not args.no_extras:
        flush_buf = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB

        def flush():
            # a read-only pass over 1 GiB evicts the L2s and the 256 MB Infinity Cache without leaving
            # dirty lines behind for the timed kernel to write back
            flush_buf.sum()

        fm, _ = flushed_ms(torch, W.fwd, flush)
        am, _ = flushed_ms(torch, W.adj, flush)
        extras["flushed"] = {"forward_us": round(fm * 1e3, 2), "forward_GBs": round(W.fb / (fm * 1e-3) / 1e9, 1),
                             "adjoint_us": round(am * 1e3, 2), "adjoint_GBs": round(W.ab / (am * 1e-3) / 1e9, 1),
                             "note": "L2 and Infinity Cache flushed (1 GiB read) before each launch, 20 runs"}
        _, (gxm, gvm) = timed_launches(torch, [lambda: W.adj(gv=False), lambda: W.adj(gx=False)], 50, 5)
        extras["adjoint_parts"] = {"grad_x_only_us": round(gxm * 1e3, 2), "grad_vals_only_us": round(gvm * 1e3, 2)}
        del flush_buf
        # attainable HBM bandwidth on this machine: a streaming read (reduction) and a copy of 2 GiB
        big = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        big2 = torch.empty_like(big)
        _, (rd, cp) = timed_launches(torch, [lambda: big.sum(), lambda: big2.copy_(big)], 10, 2)
        extras["hbm_calibration"] = {"read_GBs": round(big.numel() * 8 / (rd * 1e-3) / 1e9, 1),
                                     "copy_GBs": round(2 * big.numel() * 8 / (cp * 1e-3) / 1e9, 1),
                                     "note": "torch sum / copy_ of a 2 GiB float64 tensor, event-timed"}
        del big, big2
        if isinstance(W, Single):
            A, x = W.A, w["x"]
            plain = {}
            for name, reorder in (("input_order", "none"), ("rcm", "rcm"), ("bandk", None)):
                if reorder is None:
                    Mp, xp = W.M, W.xd
                else:
                    q = dict(W.params, reorder=reorder)
                    Mp = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, q, store), store)
                    xp = torch.from_numpy(x[Mp.structure()["perm"]]).to(dtype=W.xd.dtype).cuda()
                yp = torch.empty_like(xp)
                _, (pm,) = timed_launches(torch, [lambda: Mp.spmv_plain(xp, yp)], 50, 5)
                entry = {"plain_forward_us": round(pm * 1e3, 2),
                         "plain_forward_GFLOPs": round(2 * A.nnz / pm / 1e6, 1)}
                if reorder is not None:
                    _, (km,) = timed_launches(torch, [lambda: Mp.spmv(xp, yp)], 50, 5)
                    entry["csrk_forward_us"] = round(km * 1e3, 2)
                    entry["bandwidth"] = Mp.info["bandwidth"]
                plain[name] = entry
                if Mp is not W.M:
                    Mp.close()
            extras["plain_csr"] = plain
            # CSR-2 (one grouping level) on the same matrix, same sizes
            q = dict(W.params, k=2)
            M2 = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, q, store), store)
            x2 = torch.from_numpy(x[M2.structure()["perm"]]).to(dtype=W.xd.dtype).cuda()
            y2 = torch.empty_like(x2)
            _, (k2,) = timed_launches(torch, [lambda: M2.spmv(x2, y2)], 50, 5)
            extras["csr2_forward_us"] = round(k2 * 1e3, 2)
            M2.close()
            extras["cpu_csrk"] = cpu_csrk(C, A, x, W)
            if args.workload == "c2":
                extras["cg"] = cg_study(torch, C, CsrkMatrix, A, w["x"])
    if isinstance(W, Single):
        extras["accuracy"] = W.accuracy(torch, w["x"])
        log(f"accuracy {extras['accuracy']}")
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        extras["copy_calibration"] = "3 x copy of 1 GiB (read 1 GiB, write 1 GiB per dispatch)"

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle")
        cpu = cpu_baseline(mats, xs, gs)

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": store,
        "data": "synthetic",
        "config": dict({"workload": f"{WORKLOAD_NAMES[args.workload]}_{store}"}, **W.config()),
        "forward": {"us": round(fwd_ms * 1e3, 2), "GFLOPs": round(W.flops_fwd / fwd_ms / 1e6, 1),
                    "GBs": round(fwd_gbs, 1), "bytes": W.fb},
        "adjoint": {"us": round(adj_ms * 1e3, 2), "GFLOPs": round(W.flops_adj / adj_ms / 1e6, 1),
                    "GBs": round(adj_gbs, 1), "bytes": W.ab},
        "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": round(dom[3], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(dom[3] / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic(dom[4], args.workload, store), "algorithmic_bytes": dom[2]},
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
