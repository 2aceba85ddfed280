"""Benchmark of the CSR-k hot path on one MI355X.

One step = the CSR-k forward product y = A x followed by its adjoint
(grad_x = A^T g, grad_vals = g_i x_j), on the 3D 7-point Laplacian of a
128^3 grid (n = 2,097,152, nnz = 14,581,760) whose rows were relabelled at
random, stored in FP64.  The reordering, grouping, size choice and upload run
before the timed region, as the paper times only the kernels on data already
on the GPU.  Prints one JSON line (the last line of stdout).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
"""

from __future__ import annotations

import argparse
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fwd_bytes(n, nnz, nsr, nssr, val_bytes=8, vec_bytes=8, nrhs=1):
    """Algorithmic bytes of one forward launch: vals + col_idx per nonzero; row_ptr, x, y per row; SR/SSR pointers."""
    return nnz * (val_bytes + 4) + n * (4 + 2 * vec_bytes * nrhs) + 4 * (nsr + nssr)


def adj_bytes(n, nnz, nsr, nssr, val_bytes=8, vec_bytes=8, gv_bytes=8, nrhs=1):
    """Algorithmic bytes of one adjoint launch: col_idx, vals read and grad_vals written per nonzero;
    row_ptr, g, x read and grad_x written per row; SR/SSR pointers."""
    return nnz * (4 + val_bytes + gv_bytes) + n * (4 + 3 * vec_bytes * nrhs) + 4 * (nsr + nssr)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_csrk_3d7pt128_f64.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2203_05096_amd", "csrc", "device", "kernels.hip")


def profiled_traffic(kernel_prefix):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) recorded for this kernel source, else None."""
    import hashlib
    try:
        text = "".join(l for l in open(TRAFFIC_FILE) if not l.startswith("#"))
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
    """Runs `steps` steps of the callables in `fns` after `warmup` steps; returns wall ms/step and per-fn
    mean event ms (events on the current stream, which is the launch stream)."""
    for _ in range(warmup):
        for f in fns:
            f()
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
          for _ in fns]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        for i, f in enumerate(fns):
            ev[i][s][0].record()
            f()
            ev[i][s][1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
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


def cpu_baseline(A, x, g, budget_s=12.0):
    """The C oracle (FP64 CSR, OpenMP static over rows for the forward, serial scatter for the adjoint) on
    the same matrix in its input order; runs until ~budget_s of CPU work."""
    from oracle import cref
    cref.lib()
    t1 = cref.time_forward(A.row_ptr, A.col_idx, A.vals, x, 1)
    rf = max(1, int((budget_s / 2) / max(t1, 1e-4)))
    tf = cref.time_forward(A.row_ptr, A.col_idx, A.vals, x, rf) / rf
    t1 = cref.time_adjoint(A.row_ptr, A.col_idx, A.vals, x, g, 1)
    ra = max(1, int((budget_s / 2) / max(t1, 1e-4)))
    ta = cref.time_adjoint(A.row_ptr, A.col_idx, A.vals, x, g, ra) / ra
    flops = 5.0 * A.nnz
    return {"value": round(flops / (tf + ta) / 1e9, 3), "unit": "GFLOP/s", "cores": cref.threads(), "kind": "oracle",
            "sample": f"full matrix in input order: forward x{rf} (OpenMP static over rows) + adjoint x{ra} "
                      f"(serial scatter); forward {tf * 1e3:.2f} ms, adjoint {ta * 1e3:.2f} ms per call",
            "cpu": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip plain-CSR and flushed measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each box has one MI355X); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from gen import workload_c2
    from paper_2203_05096_amd import _capi as C
    from paper_2203_05096_amd.matrix import CsrkMatrix

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    C.lib()  # fail loudly if the HIP library is missing
    log("generating workload")
    w = workload_c2()
    A, x, g = w["A"], w["x"], w["g"]
    p = C.csrk_tune(A.n, A.nnz, "mi355x")
    t = time.perf_counter()
    M = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, p, "f64"), "f64")
    build_s = time.perf_counter() - t
    info = M.info
    log(f"built in {build_s:.2f}s: params {p}, nsr {info['nsr']} nssr {info['nssr']} band {info['bandwidth']}")
    s = M.structure()
    perm = s["perm"]
    xd = torch.from_numpy(x[perm]).cuda()
    gd = torch.from_numpy(g[perm]).cuda()
    y = torch.empty_like(xd)
    gx = torch.empty_like(xd)
    gv = torch.empty(A.nnz, dtype=torch.float64, device="cuda")

    # The timed loop calls the C entry points directly with pre-marshalled pointers, so host-side
    # Python overhead stays far below the kernel time.
    lib = C.lib()
    h, stream = M.handle, torch.cuda.current_stream().cuda_stream
    px, py, pg, pgx, pgv = xd.data_ptr(), y.data_ptr(), gd.data_ptr(), gx.data_ptr(), gv.data_ptr()

    def fwd():
        if lib.csrk_spmv(h, None, px, py, 1, stream):
            raise RuntimeError(C.csrk_last_error_detail())

    def adj():
        if lib.csrk_spmv_adjoint(h, None, px, pg, pgx, pgv, 1, stream):
            raise RuntimeError(C.csrk_last_error_detail())

    torch.cuda.synchronize()
    wall_ms, (fwd_ms, adj_ms) = timed_launches(torch, [fwd, adj], args.steps, args.warmup)
    nsr, nssr = info["nsr"], info["nssr"]
    fb = fwd_bytes(A.n, A.nnz, nsr, nssr)
    ab = adj_bytes(A.n, A.nnz, nsr, nssr)
    flops_step = 5.0 * A.nnz
    value = flops_step / (wall_ms * 1e-3) / 1e9
    fwd_gbs = fb / (fwd_ms * 1e-3) / 1e9
    adj_gbs = ab / (adj_ms * 1e-3) / 1e9
    dom = ("forward", fwd_ms, fb, fwd_gbs, "k_spmv_csrk") if fwd_ms >= adj_ms else \
        ("adjoint", adj_ms, ab, adj_gbs, "k_adjoint_csrk")
    log(f"step {wall_ms:.4f} ms; forward {fwd_ms * 1e3:.1f} us {fwd_gbs:.0f} GB/s; "
        f"adjoint {adj_ms * 1e3:.1f} us {adj_gbs:.0f} GB/s")

    extras = {}
    if not args.no_extras:
        flush_buf = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB

        def flush():
            # a read-only pass over 1 GiB evicts the L2s and the 256 MB Infinity Cache without leaving
            # dirty lines behind for the timed kernel to write back
            flush_buf.sum()

        fm, fmin = flushed_ms(torch, fwd, flush)
        am, amin = flushed_ms(torch, adj, flush)
        extras["flushed"] = {"forward_us": round(fm * 1e3, 2), "forward_GBs": round(fb / (fm * 1e-3) / 1e9, 1),
                             "adjoint_us": round(am * 1e3, 2), "adjoint_GBs": round(ab / (am * 1e-3) / 1e9, 1),
                             "note": "L2 and Infinity Cache flushed (1 GiB read) before each launch, 20 runs"}

        def adj_gx_only():
            if lib.csrk_spmv_adjoint(h, None, px, pg, pgx, None, 1, stream):
                raise RuntimeError(C.csrk_last_error_detail())

        def adj_gv_only():
            if lib.csrk_spmv_adjoint(h, None, px, pg, None, pgv, 1, stream):
                raise RuntimeError(C.csrk_last_error_detail())

        _, (gxm, gvm) = timed_launches(torch, [adj_gx_only, adj_gv_only], 50, 5)
        extras["adjoint_parts"] = {"grad_x_only_us": round(gxm * 1e3, 2), "grad_vals_only_us": round(gvm * 1e3, 2)}
        # attainable HBM bandwidth on this machine: a streaming read (reduction) and a copy of 2 GiB
        big = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        big2 = torch.empty_like(big)
        _, (rd, cp) = timed_launches(torch, [lambda: big.sum(), lambda: big2.copy_(big)], 10, 2)
        extras["hbm_calibration"] = {"read_GBs": round(big.numel() * 8 / (rd * 1e-3) / 1e9, 1),
                                     "copy_GBs": round(2 * big.numel() * 8 / (cp * 1e-3) / 1e9, 1),
                                     "note": "torch sum / copy_ of a 2 GiB float64 tensor, event-timed"}
        del big, big2
        plain = {}
        for name, reorder in (("input_order", "none"), ("rcm", "rcm"), ("bandk", None)):
            if reorder is None:
                Mp = M
                xp = xd
            else:
                q = dict(p, reorder=reorder)
                Mp = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, q, "f64"), "f64")
                xp = torch.from_numpy(x[Mp.structure()["perm"]]).cuda()
            yp = torch.empty_like(xp)
            _, (pm,) = timed_launches(torch, [lambda: Mp.spmv_plain(xp, yp)], 50, 5)
            entry = {"plain_forward_us": round(pm * 1e3, 2), "plain_forward_GFLOPs": round(2 * A.nnz / pm / 1e6, 1)}
            if reorder is not None:
                _, (km,) = timed_launches(torch, [lambda: Mp.spmv(xp, yp)], 50, 5)
                entry["csrk_forward_us"] = round(km * 1e3, 2)
                entry["bandwidth"] = Mp.info["bandwidth"]
            plain[name] = entry
            if Mp is not M:
                Mp.close()
        extras["plain_csr"] = plain
        del flush_buf
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
        cpu = cpu_baseline(A, x, g)

    out = {
        "metric": "SpMV GFLOP/s + achieved HBM GB/s (% of peak), CSR-k vs plain CSR, fwd+adj",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3d7pt_128cube_scrambled_fp64_forward_adjoint", "n": A.n, "nnz": A.nnz,
                   "csrk_params": p, "nsr": nsr, "nssr": nssr, "bandwidth_after_reorder": info["bandwidth"],
                   "build_seconds": round(build_s, 2)},
        "forward": {"us": round(fwd_ms * 1e3, 2), "GFLOPs": round(2 * A.nnz / fwd_ms / 1e6, 1),
                    "GBs": round(fwd_gbs, 1), "bytes": fb},
        "adjoint": {"us": round(adj_ms * 1e3, 2), "GFLOPs": round(3 * A.nnz / adj_ms / 1e6, 1),
                    "GBs": round(adj_gbs, 1), "bytes": ab},
        "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": round(dom[3], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(dom[3] / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(dom[4]),
                     "algorithmic_bytes": dom[2]},
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
