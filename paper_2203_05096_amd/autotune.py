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
The objective is the forward product alone (the paper's) or the forward plus
its adjoint (this project's step).

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

# Candidate sizes: the paper's {2^i, 1.5 * 2^i} pattern (Section 4.1) for SRS,
# over the range where a super-row fills a wavefront's staging window.  SSRS
# counts super-rows per workgroup and is swept over powers of two: with one
# super-row per wavefront (waves = SSRS, the default launch) workgroups of 3
# or 6 wavefronts measured 5-8% slower than 2 or 4 on every matrix of the
# tuning suite.
SRS_SWEEP = (16, 24, 32, 48, 64, 96, 128)
SSRS_SWEEP = (2, 4, 8)
LANES_SWEEP = (1, 2, 4)
WAVES_SWEEP = None  # None: waves per workgroup = SSRS


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
    objective: str = "forward"  # what the trial times measure: "forward" or "step" (forward + adjoint)

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


def time_step(M: CsrkMatrix, x, g, y, gx, gv, reps: int = 20, warmup: int = 5) -> float:
    """Mean event time (microseconds) of one forward launch followed by one adjoint launch."""
    lib = C.lib()
    h, st = M.handle, torch.cuda.current_stream().cuda_stream
    px, pg, py, pgx, pgv = x.data_ptr(), g.data_ptr(), y.data_ptr(), gx.data_ptr(), gv.data_ptr()
    nrhs = 1 if x.dim() == 1 else x.shape[1]

    def once():
        if lib.csrk_spmv(h, None, px, py, nrhs, st) or lib.csrk_spmv_adjoint(h, None, px, pg, pgx, pgv, nrhs, st):
            raise RuntimeError(C.csrk_last_error_detail())
    for _ in range(warmup):
        once()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        once()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e3 / reps


def sweep(A, store: str = "f64", srs_list=SRS_SWEEP, ssrs_list=SSRS_SWEEP, lanes_list=LANES_SWEEP,
          waves_list=WAVES_SWEEP, reorder: str = "bandk", nrhs: int = 1, reps: int = 40, seed: int = 0,
          name: str | None = None, threads: int = 8, objective: str = "forward", on_trial=None) -> SweepResult:
    """Times every combination on matrix A (an object with row_ptr, col_idx, vals).  objective is
    "forward" (the paper's) or "step" (forward + adjoint); waves_list None ties the waves per
    workgroup to SSRS.  on_trial(M, x, y, trial), if given, is called after each timing with the
    matrix and the permuted-space input and output of its last timed product (a caller's check
    that every candidate computes the same product)."""
    n, nnz = len(A.row_ptr) - 1, int(A.row_ptr[-1])
    res = SweepResult(name or getattr(A, "name", "matrix"), n, nnz, nnz / max(n, 1), objective=objective)
    dt = torch.float64 if store == "f64" else torch.float32
    g = torch.Generator(device="cuda").manual_seed(seed)
    shape = (n,) if nrhs == 1 else (n, nrhs)
    x = torch.rand(shape, generator=g, device="cuda", dtype=dt) * 2 - 1
    y = torch.empty_like(x)
    if objective == "step":
        gvec = torch.rand(shape, generator=g, device="cuda", dtype=dt) * 2 - 1
        gx = torch.empty_like(x)
        gv = torch.empty(nnz, device="cuda", dtype=dt)

    def build(sizes):
        srs, ssrs = sizes
        p = {"k": 3, "srs": srs, "ssrs": ssrs, "lanes_per_row": lanes_list[0],
             "waves_per_wg": min(ssrs, 16) if waves_list is None else waves_list[0], "reorder": reorder}
        return sizes, C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, p)

    combos = list(itertools.product(srs_list, ssrs_list))
    with cf.ThreadPoolExecutor(threads) as ex:
        # `threads` host builds at a time, so at most that many structures are held at once
        for (srs, ssrs), h in (r for i in range(0, len(combos), threads) for r in ex.map(build, combos[i:i + threads])):
            C.csrk_upload(h, store)
            M = CsrkMatrix(h, store)
            for lanes, waves in itertools.product(lanes_list, [min(ssrs, 16)] if waves_list is None else waves_list):
                C.csrk_set_launch(M.handle, lanes, waves)
                us = time_forward(M, x, y, reps) if objective == "forward" else \
                    time_step(M, x, gvec, y, gx, gv, reps)
                res.trials.append(Trial(srs, ssrs, lanes, waves, reorder, us))
                if on_trial is not None:
                    torch.cuda.synchronize()
                    on_trial(M, x, y, res.trials[-1])
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


def nearest_pow2(v: int) -> int:
    """Nearest power of two, ties toward the smaller (the MI355X model's SSRS snap)."""
    if v <= 1:
        return 1
    lo = 1 << (int(v).bit_length() - 1)
    return lo if v - lo <= 2 * lo - v else 2 * lo


def snap_srs(v: int, floor: int = 1) -> int:
    """Nearest size of the {2^i, 3 * 2^(i-1)} set (ties toward the smaller), at least ``floor``: the MI355X
    model's SRS snap."""
    cands = sorted({c for i in range(41) for c in (1 << i, 3 * (1 << i) // 2)})
    best = min(cands, key=lambda c: (abs(c - v), c))
    return best if best >= floor else next(c for c in cands if c >= floor)


def lanes_rule(r: float) -> int:
    """Lanes per row of the MI355X model: a row per lane for short rows, wider groups as rows lengthen."""
    return 1 if r <= 6 else 2 if r <= 24 else 4 if r <= 48 else 8 if r <= 96 else 16


def nearest(v, grid):
    return min(grid, key=lambda g: (abs(g - v), g))


def evaluate(results, consts: dict) -> list:
    """For each matrix: the model's shape (fitted SRS snapped onto the size set, power-of-two SSRS, both then
    matched to the sweep grid; lanes by rdensity; waves = SSRS), its time, and the ratio to the sweep optimum."""
    out = []
    for r in results:
        srs_grid = sorted({t.srs for t in r.trials})
        ssrs_grid = sorted({t.ssrs for t in r.trials})
        lanes_grid = sorted({t.lanes for t in r.trials})
        srs = nearest(snap_srs(model_pick(consts["srs"], r.rdensity), math.ceil(256.0 / r.rdensity)), srs_grid)
        ssrs = nearest(nearest_pow2(model_pick(consts["ssrs"], r.rdensity)), ssrs_grid)
        lanes = nearest(lanes_rule(r.rdensity), lanes_grid)
        same = [t for t in r.trials if (t.srs, t.ssrs, t.lanes) == (srs, ssrs, lanes)]
        pick = min(same, key=lambda t: t.us) if same else r.best_for(srs, ssrs)
        out.append({"name": r.name, "rdensity": r.rdensity, "model_srs": srs, "model_ssrs": ssrs,
                    "model_lanes": pick.lanes, "model_us": pick.us, "best": asdict(r.best),
                    "ratio": pick.us / r.best.us})
    return out


def load(path: str) -> list:
    """Sweep results from a report written by ``--out``."""
    with open(path) as f:
        rep = json.load(f)
    pts = {p[0]: p for p in rep["fit"]["points"]}
    out = []
    for name, trials in rep["trials"].items():
        ts = [Trial(**t) for t in trials]
        n = next((e for e in rep["evaluation"] if e["name"] == name), None)
        res = SweepResult(name, 0, 0, pts[name][1] if name in pts else n["rdensity"])
        res.trials = ts
        out.append(res)
    return out


def markdown(groups: dict, consts: dict, command: str) -> str:
    """A summary table per storage type: best shape, model shape, ratio."""
    a_r, b_r = consts["srs"]
    a_s, b_s = consts["ssrs"]
    lines = [f"Fit (Section 4.1 form, each size regressed on ln r separately, over all sweeps below): "
             f"SRS = {a_r:.2f} - {b_r:.2f} ln r; SSRS = {a_s:.3f} - ({b_s:.4f}) ln r, rounded half up, then "
             f"snapped to the nearest power of two.", "", "Command:", "", "    " + command, ""]
    for store, results in groups.items():
        lines += [f"### {store}", "",
                  "| matrix | rdensity | best (SRS, SSRS, lanes) | best us | model (SRS, SSRS, lanes) | model us |"
                  " model / best |", "|---|---|---|---|---|---|---|"]
        for e in evaluate(results, consts):
            b = e["best"]
            lines.append(f"| {e['name']} | {e['rdensity']:.2f} | ({b['srs']}, {b['ssrs']}, {b['lanes']}) | "
                         f"{b['us']:.1f} | ({e['model_srs']}, {e['model_ssrs']}, {e['model_lanes']}) | "
                         f"{e['model_us']:.1f} | {e['ratio']:.3f} |")
        lines.append("")
    return "\n".join(lines)


def time_params(A, p: dict, store: str = "f64", reps: int = 40, objective: str = "forward") -> float:
    """Event time (microseconds) of one parameter set on matrix A: the forward, or forward + adjoint."""
    dt = torch.float64 if store == "f64" else torch.float32
    n, nnz = len(A.row_ptr) - 1, int(A.row_ptr[-1])
    M = CsrkMatrix(C.csrk_build(A.row_ptr, A.col_idx, A.vals, p, store), store)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.rand(n, generator=g, device="cuda", dtype=dt) * 2 - 1
    y = torch.empty_like(x)
    if objective == "forward":
        us = time_forward(M, x, y, reps)
    else:
        gv = torch.empty(nnz, device="cuda", dtype=dt)
        us = time_step(M, x, torch.rand(n, generator=g, device="cuda", dtype=dt), y, torch.empty_like(x), gv, reps)
    M.close()
    return us


def grid_markdown(res: SweepResult, picks: dict, command: str) -> str:
    """The (SRS x SSRS) grid of one matrix (best over lanes per cell), its optimum, and each model's pick timed
    on the same matrix."""
    srs_l = sorted({t.srs for t in res.trials})
    ssrs_l = sorted({t.ssrs for t in res.trials})
    b = res.best
    lines = [f"Matrix {res.name}: n = {res.n:,}, nnz = {res.nnz:,}, rdensity {res.rdensity:.3f}.", "",
             "Command:", "", "    " + command, "",
             f"{'Forward' if res.objective == 'forward' else 'Forward + adjoint'} kernel time in us per (SRS, SSRS) "
             "cell, the best over lanes per row; waves per workgroup = min(SSRS, 16):", "",
             "| SRS \\ SSRS | " + " | ".join(str(v) for v in ssrs_l) + " |",
             "|---|" + "---|" * len(ssrs_l)]
    for srs in srs_l:
        cells = []
        for ssrs in ssrs_l:
            t = res.best_for(srs, ssrs)
            cells.append(f"{t.us:.1f}" if t else "")
        lines.append(f"| {srs} | " + " | ".join(cells) + " |")
    lines += ["", f"Optimum: SRS {b.srs}, SSRS {b.ssrs}, lanes {b.lanes}, waves {b.waves}: {b.us:.1f} us.", "",
              "| model | (SRS, SSRS, lanes, waves) | us | model / optimum |", "|---|---|---|---|"]
    for name, (p, us) in picks.items():
        lines.append(f"| {name} | ({p['srs']}, {p['ssrs']}, {p['lanes_per_row']}, {p['waves_per_wg']}) | {us:.1f} | "
                     f"{us / b.us:.3f} |")
    return "\n".join(lines) + "\n"


@dataclass
class BatchTrial:
    srs: int
    ssrs: int
    blocks_per_cu: int
    fwd_us: float
    adj_us: float

    @property
    def us(self) -> float:
        return self.fwd_us + self.adj_us


def sweep_batch(mats, store: str = "f32", nrhs: int = 8, srs_list=(32, 48, 64, 96), ssrs_list=(4, 8, 16),
                blocks_list=(0, 16, 64), reps: int = 20, warmup: int = 5, seed: int = 0, threads: int = 16,
                extra=()) -> list:
    """The batched multi-right-hand-side objective: for every (SRS, SSRS) every matrix of the batch is rebuilt
    with those sizes (one super-row per wavefront: waves = SSRS, at most 16) and, for every grid size in
    workgroups per CU (0: one workgroup per (matrix, SSR) item, the library's default), the forward and the
    adjoint launches are timed (mean event time of `reps` back-to-back
    runs after `warmup`).  ``extra``: further (srs, ssrs, blocks_per_cu) points to time (a model's pick)."""
    from .matrix import CsrkBatch
    dt = torch.float64 if store == "f64" else torch.float32
    g = torch.Generator(device="cuda").manual_seed(seed)
    trials = []
    wanted = {}
    for srs, ssrs in itertools.product(srs_list, ssrs_list):
        wanted[(srs, ssrs)] = set(blocks_list)
    for srs, ssrs, blocks in extra:
        wanted.setdefault((srs, ssrs), set()).add(blocks)
    lib = C.lib()
    st = torch.cuda.current_stream().cuda_stream
    for (srs, ssrs), blocks_set in wanted.items():
        def build(A):
            p = C.csrk_tune_rhs(len(A.row_ptr) - 1, int(A.row_ptr[-1]), nrhs, "mi355x")
            p.update(srs=srs, ssrs=ssrs, waves_per_wg=min(ssrs, 16))
            return C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, p)
        with cf.ThreadPoolExecutor(threads) as ex:
            hs = list(ex.map(build, mats))
        Ms = []
        for h in hs:
            C.csrk_upload(h, store)
            Ms.append(CsrkMatrix(h, store))
        B = CsrkBatch(Ms)
        shape = lambda M: (M.n, nrhs) if nrhs > 1 else (M.n,)  # noqa: E731
        X = [torch.rand(shape(M), generator=g, device="cuda", dtype=dt) * 2 - 1 for M in Ms]
        G = [torch.rand(shape(M), generator=g, device="cuda", dtype=dt) * 2 - 1 for M in Ms]
        Y = [torch.empty_like(x) for x in X]
        GX = [torch.empty_like(x) for x in X]
        GV = [torch.empty(M.nnz, device="cuda", dtype=dt) for M in Ms]
        arr = C._ptr_array
        px, py, pg = arr([t.data_ptr() for t in X]), arr([t.data_ptr() for t in Y]), arr([t.data_ptr() for t in G])
        pgx, pgv = arr([t.data_ptr() for t in GX]), arr([t.data_ptr() for t in GV])
        fwd = lambda: lib.csrk_batch_spmv(B.handle, None, px, py, nrhs, st)  # noqa: E731
        adj = lambda: lib.csrk_batch_spmv_adjoint(B.handle, None, px, pg, pgx, pgv, nrhs, st)  # noqa: E731
        for blocks in sorted(blocks_set):
            C.csrk_batch_set_launch(B.handle, blocks, 0)
            times = []
            for f in (fwd, adj):
                for _ in range(warmup):
                    if f():
                        raise RuntimeError(C.csrk_last_error_detail())
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(reps):
                    f()
                b.record()
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b) * 1e3 / reps)
            trials.append(BatchTrial(srs, ssrs, blocks, times[0], times[1]))
            print(f"batch SRS {srs} SSRS {ssrs} blocks/CU {blocks or 'one per item'}: forward {times[0]:.1f} us, adjoint "
                  f"{times[1]:.1f} us", flush=True)
        B.close()
        for M in Ms:
            M.close()
    return trials


def batch_markdown(trials, model: tuple, command: str, label: str) -> str:
    """The batched sweep: every point, the optimum, and the model's pick against it."""
    best = min(trials, key=lambda t: t.us)
    pick = next((t for t in trials if (t.srs, t.ssrs, t.blocks_per_cu) == model), None)
    lines = [f"Batched multi-right-hand-side sweep on {label}: forward + adjoint launch times (mean of back-to-back "
             "runs, event-timed), one point per (SRS, SSRS, workgroups per CU); waves per workgroup = SSRS.", "",
             "Command:", "", "    " + command, "",
             "| SRS | SSRS | workgroups/CU | forward us | adjoint us | step us | / optimum |",
             "|---|---|---|---|---|---|---|"]
    for t in sorted(trials, key=lambda t: (t.srs, t.ssrs, t.blocks_per_cu)):
        mark = " **optimum**" if t is best else (" model" if t is pick else "")
        lines.append(f"| {t.srs} | {t.ssrs} | {t.blocks_per_cu or 'one per item'} | {t.fwd_us:.1f} | {t.adj_us:.1f} | {t.us:.1f} | "
                     f"{t.us / best.us:.3f}{mark} |")
    lines += ["", f"Optimum: SRS {best.srs}, SSRS {best.ssrs}, workgroups per CU {best.blocks_per_cu or 'one per item'}: "
                  f"{best.us:.1f} us per step."]
    if pick is not None:
        lines.append(f"Model pick (SRS {model[0]}, SSRS {model[1]}, workgroups per CU {model[2] or 'one per item'}): "
                     f"{pick.us:.1f} us, "
                     f"{pick.us / best.us:.3f} x the optimum.")
    return "\n".join(lines) + "\n"


def main(argv=None):
    import os
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--scale", type=float, default=1.0, help="grid scale of the tuning suite")
    ap.add_argument("--store", default="f64")
    ap.add_argument("--out", default=None)
    ap.add_argument("--threads", type=int, default=16)
    ap.add_argument("--objective", choices=["forward", "step"], default="step")
    ap.add_argument("--from-json", nargs="+", default=None,
                    help="fit and evaluate earlier --out reports together instead of sweeping")
    ap.add_argument("--markdown", default=None, help="with --from-json or --workload: write a summary table here")
    ap.add_argument("--workload", default=None, help="sweep one named workload of gen (e.g. c2) instead of the suite")
    ap.add_argument("--srs", default=None, help="comma-separated SRS values (with --workload)")
    ap.add_argument("--ssrs", default=None, help="comma-separated SSRS values (with --workload)")
    ap.add_argument("--lanes", default="1,2,4", help="comma-separated lanes per row (with --workload)")
    ap.add_argument("--batch", default=None, help="sweep a batched workload of gen (e.g. c5): SRS x SSRS x grid")
    ap.add_argument("--blocks", default="0,16,64",
                    help="comma-separated workgroups per CU (with --batch; 0 = one workgroup per work item)")
    args = ap.parse_args(argv)
    if args.batch:
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import gen
        w = gen.WORKLOADS[args.batch]()
        ints = lambda v, d: tuple(int(t) for t in v.split(",")) if v else d  # noqa: E731
        mats, nrhs = w["As"], w["nrhs"]
        p = C.csrk_tune_rhs(mats[0].n, mats[0].nnz, nrhs, "mi355x")
        model = (p["srs"], p["ssrs"], 0)  # the library's default grid: one workgroup per work item
        trials = sweep_batch(mats, w["dtype"], nrhs, ints(args.srs, (32, 48, 64, 96)), ints(args.ssrs, (4, 8, 16)),
                             ints(args.blocks, (0, 16, 64)), extra=[model])
        cmd = "python -m paper_2203_05096_amd.autotune " + " ".join(argv if argv is not None else sys.argv[1:])
        text = batch_markdown(trials, model, cmd, f"{args.batch} ({len(mats)} matrices, {nrhs} right-hand sides, "
                                                  f"{w['dtype']})")
        print(text, flush=True)
        if args.markdown:
            with open(args.markdown, "w") as f:
                f.write(text)
        return
    if args.workload:
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import gen
        A = gen.WORKLOADS[args.workload]()["A"]
        ints = lambda v, d: tuple(int(t) for t in v.split(",")) if v else d  # noqa: E731
        res = sweep(A, args.store, srs_list=ints(args.srs, SRS_SWEEP), ssrs_list=ints(args.ssrs, SSRS_SWEEP),
                    lanes_list=ints(args.lanes, LANES_SWEEP), threads=args.threads, objective=args.objective,
                    name=args.workload)
        n, nnz = len(A.row_ptr) - 1, int(A.row_ptr[-1])
        picks = {}
        for model in ("mi355x", "volta", "ampere"):
            p = C.csrk_tune(n, nnz, model)
            p["waves_per_wg"] = min(p["waves_per_wg"], 16)
            picks[model] = (p, time_params(A, p, args.store, objective=args.objective))
        cmd = "python -m paper_2203_05096_amd.autotune " + " ".join(argv if argv is not None else sys.argv[1:])
        text = grid_markdown(res, picks, cmd)
        print(text, flush=True)
        if args.markdown:
            with open(args.markdown, "w") as f:
                f.write(text)
        return
    if args.from_json:
        groups = {}
        for p in args.from_json:
            with open(p) as f:
                store = json.load(f).get("store", p)
            groups[f"{store} ({os.path.basename(p)})"] = load(p)
        consts = fit([r for g in groups.values() for r in g])
        text = markdown(groups, consts, "python -m paper_2203_05096_amd.autotune --from-json " +
                        " ".join(args.from_json))
        print(text)
        if args.markdown:
            with open(args.markdown, "w") as f:
                f.write(text + "\n")
        return
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import gen
    suite = gen.tuning_suite(scale=args.scale)
    results = []
    for A in suite:
        t = time.time()
        r = sweep(A, args.store, threads=args.threads, objective=args.objective)
        results.append(r)
        print(f"{A.name}: n={r.n} r={r.rdensity:.2f} best {asdict(r.best)} ({time.time() - t:.1f}s)", flush=True)
    consts = fit(results)
    ev = evaluate(results, consts)
    report = {"store": args.store, "scale": args.scale, "objective": args.objective, "fit": consts, "evaluation": ev,
              "trials": {r.name: [asdict(t) for t in r.trials] for r in results}}
    print(json.dumps({"fit": consts, "evaluation": ev}, indent=1), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(report, f)


if __name__ == "__main__":
    main()
