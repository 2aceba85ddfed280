"""Autotuner for the CSR-k group sizes and kernel launch shape, and the fit of the size model.

The paper (Section 4.1) times every (SSRS, SRS) pair of a small set on a suite
of matrices, keeps the best pair per matrix, and fits SSRS and SRS separately
as a - b ln(rdensity) (logarithmic regression, each fitted independently), then
rounds to nearest with halves up.  This module does the same on the GPU at
hand: for each matrix it builds the CSR-k structure for every (SRS, SSRS) in
the sweep (host builds run in parallel threads), times the forward kernel for
every (lanes per row, waves per workgroup) launch shape, and returns the best;
``fit`` turns the per-matrix optima into the model's constants and
``evaluate`` compares the model's pick with the sweep optimum.

Timing follows the paper's methodology (Section 5.4): data resident on the GPU,
kernel time only, the mean of repeated back-to-back runs after warm-up runs.

    python -m paper_2203_05096_amd.autotune --scale 1.0 --out results.json
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import itertools
import json
import math
import sys
import time
from dataclasses import asdict, dataclass, field

import numpy as np
import torch

from . import _capi as C
from .matrix import CsrkMatrix

# Candidate sizes: the paper's {2^i, 1.5 * 2^i} pattern (Section 4.1), over the
# range where a super-row fills a wavefront's staging window; SSRS counts
# super-rows per workgroup.
SRS_SWEEP = (16, 24, 32, 48, 64, 96, 128)
SSRS_SWEEP = (2, 4, 8)
LANES_SWEEP = (1, 2, 4)
WAVES_SWEEP = (2, 4, 8)


@dataclass
class Trial:
    srs: int
    ssrs: int
    lanes: int
    waves: int
    reorder: str
    us: float


@dataclass
class SweepResult:
    name: str
    n: int
    nnz: int
    rdensity: float
    trials: list = field(default_factory=list)

    @property
    def best(self) -> Trial:
        return min(self.trials, key=lambda t: t.us)

    def best_for(self, srs=None, ssrs=None):
        ts = [t for t in self.trials if (srs is None or t.srs == srs) and (ssrs is None or t.ssrs == ssrs)]
        return min(ts, key=lambda t: t.us) if ts else None


def time_forward(M: CsrkMatrix, x: torch.Tensor, y: torch.Tensor, reps: int = 20, warmup: int = 5) -> float:
    """Mean event time (microseconds) of the CSR-k forward kernel over `reps` back-to-back runs."""
    lib = C.lib()
    h, st = M.handle, torch.cuda.current_stream().cuda_stream
    px, py = x.data_ptr(), y.data_ptr()
    nrhs = 1 if x.dim() == 1 else x.shape[1]
    for _ in range(warmup):
        lib.csrk_spmv(h, None, px, py, nrhs, st)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        if lib.csrk_spmv(h, None, px, py, nrhs, st):
            raise RuntimeError(C.csrk_last_error_detail())
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e3 / reps


def sweep(A, store: str = "f64", srs_list=SRS_SWEEP, ssrs_list=SSRS_SWEEP, lanes_list=LANES_SWEEP,
          waves_list=WAVES_SWEEP, reorder: str = "bandk", nrhs: int = 1, reps: int = 20, seed: int = 0,
          name: str | None = None, threads: int = 8) -> SweepResult:
    """Times every combination on matrix A (an object with row_ptr, col_idx, vals)."""
    n, nnz = len(A.row_ptr) - 1, int(A.row_ptr[-1])
    res = SweepResult(name or getattr(A, "name", "matrix"), n, nnz, nnz / max(n, 1))
    dt = torch.float64 if store == "f64" else torch.float32
    g = torch.Generator(device="cuda").manual_seed(seed)
    shape = (n,) if nrhs == 1 else (n, nrhs)
    x = torch.rand(shape, generator=g, device="cuda", dtype=dt) * 2 - 1
    y = torch.empty_like(x)

    def build(sizes):
        srs, ssrs = sizes
        p = {"k": 3, "srs": srs, "ssrs": ssrs, "lanes_per_row": lanes_list[0], "waves_per_wg": waves_list[0],
             "reorder": reorder}
        return sizes, C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, p)

    with cf.ThreadPoolExecutor(threads) as ex:
        for (srs, ssrs), h in ex.map(build, itertools.product(srs_list, ssrs_list)):
            C.csrk_upload(h, store)
            M = CsrkMatrix(h, store)
            for lanes, waves in itertools.product(lanes_list, waves_list):
                C.csrk_set_launch(M.handle, lanes, waves)
                res.trials.append(Trial(srs, ssrs, lanes, waves, reorder, time_forward(M, x, y, reps)))
            M.close()
    return res


def fit(results) -> dict:
    """Log-regression of the best SSRS and the best SRS against ln(rdensity), each fitted on its own
    (Section 4.1); returns the constants and the per-matrix picks."""
    rs = np.array([r.rdensity for r in results])
    best_srs = np.array([r.best.srs for r in results], dtype=np.float64)
    best_ssrs = np.array([r.best.ssrs for r in results], dtype=np.float64)
    L = np.log(rs)
    M = np.stack([np.ones_like(L), -L], axis=1)
    (a_r, b_r), *_ = np.linalg.lstsq(M, best_srs, rcond=None)
    (a_s, b_s), *_ = np.linalg.lstsq(M, best_ssrs, rcond=None)
    return {"ssrs": (float(a_s), float(b_s)), "srs": (float(a_r), float(b_r)),
            "points": [(r.name, r.rdensity, r.best.srs, r.best.ssrs, r.best.lanes, r.best.waves, r.best.us)
                       for r in results]}


def model_pick(a_b: tuple, r: float) -> int:
    """round-half-up(a - b ln r), clamped to >= 1 (the paper's rounding, Section 4.1)."""
    a, b = a_b
    return max(1, int(math.floor(a - b * math.log(r) + 0.5)))


def nearest(v, grid):
    return min(grid, key=lambda g: (abs(g - v), g))


def evaluate(results, consts: dict) -> list:
    """For each matrix: the model's (SRS, SSRS) snapped to the sweep grid, its best time over launch shapes,
    and the ratio to the sweep optimum."""
    out = []
    for r in results:
        srs_grid = sorted({t.srs for t in r.trials})
        ssrs_grid = sorted({t.ssrs for t in r.trials})
        srs = nearest(model_pick(consts["srs"], r.rdensity), srs_grid)
        ssrs = nearest(model_pick(consts["ssrs"], r.rdensity), ssrs_grid)
        pick = r.best_for(srs, ssrs)
        out.append({"name": r.name, "rdensity": r.rdensity, "model_srs": srs, "model_ssrs": ssrs,
                    "model_us": pick.us, "best": asdict(r.best), "ratio": pick.us / r.best.us})
    return out


def main(argv=None):
    import os
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--scale", type=float, default=1.0, help="grid scale of the tuning suite")
    ap.add_argument("--store", default="f64")
    ap.add_argument("--out", default=None)
    ap.add_argument("--threads", type=int, default=16)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import gen
    suite = gen.tuning_suite(scale=args.scale)
    results = []
    for A in suite:
        t = time.time()
        r = sweep(A, args.store, threads=args.threads)
        results.append(r)
        print(f"{A.name}: n={r.n} r={r.rdensity:.2f} best {asdict(r.best)} ({time.time() - t:.1f}s)", flush=True)
    consts = fit(results)
    ev = evaluate(results, consts)
    report = {"store": args.store, "scale": args.scale, "fit": consts, "evaluation": ev,
              "trials": {r.name: [asdict(t) for t in r.trials] for r in results}}
    print(json.dumps({"fit": consts, "evaluation": ev}, indent=1), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(report, f)


if __name__ == "__main__":
    main()
