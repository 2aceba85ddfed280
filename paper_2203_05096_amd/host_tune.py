"""Per-matrix tuning of the host CPU kernel (CSR-2), and its constant-time fallback.

On CPUs the paper runs CSR-2 and finds that the best super-row size does not
follow simple matrix statistics, so it tunes each matrix over a set of
representative sizes between 8 and 3072, the union over i = 3..11 of
{2^i, 1.5 * 2^i}; when constant-time tuning is preferred, one size for every
matrix, SRS = 96 (a geometric mean of the per-matrix optima), is "good enough"
(Section 4.2).  ``sweep_host`` does the per-matrix search with this library's
host kernel (``csrk_spmv_host``); ``csrk_tune(..., "host_cpu")`` is the
constant-time choice.  Timing follows Section 5.4: 5 untimed warm-up runs,
then the arithmetic mean of 20 runs.

No GPU is used: the structures are host-only builds.

    python -m paper_2203_05096_amd.host_tune --workload c2 [--threads 0]
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import sys
import time

import numpy as np

from . import _capi as C


def srs_set_cpu() -> list:
    """{2^i, 1.5 * 2^i} for i = 3..11, ascending (8 .. 3072)."""
    return sorted({2 ** i for i in range(3, 12)} | {3 * 2 ** (i - 1) for i in range(3, 12)})


def host_params(srs: int) -> dict:
    """CSR-2 with Band-k ordering; each super-row is one unit of the host kernel's parallel loop."""
    return {"k": 2, "srs": int(srs), "ssrs": 1, "lanes_per_row": 1, "waves_per_wg": 4, "reorder": "bandk"}


def time_host(h: int, x_perm: np.ndarray, reps: int = 20, warmup: int = 5, nthreads: int = 0) -> float:
    """Mean wall time in microseconds of csrk_spmv_host over `reps` runs after `warmup` untimed runs."""
    y = np.empty_like(x_perm)
    for _ in range(warmup):
        C.csrk_spmv_host(h, x_perm, y, nthreads)
    t0 = time.perf_counter()
    for _ in range(reps):
        C.csrk_spmv_host(h, x_perm, y, nthreads)
    return (time.perf_counter() - t0) / reps * 1e6


def sweep_host(A, srs_list=None, reps: int = 20, warmup: int = 5, nthreads: int = 0, build_threads: int = 4,
               seed: int = 0) -> dict:
    """Times the CSR-2 host kernel for every SRS of the set on matrix A (row_ptr, col_idx, vals).  Structures are
    built `build_threads` at a time; timing runs one structure at a time.  Returns the trials, the optimum,
    the constant-time choice's time and the ratio of the two."""
    srs_list = list(srs_list or srs_set_cpu())
    x = np.random.default_rng(seed).uniform(-1, 1, len(A.row_ptr) - 1)

    def build(srs):
        return srs, C.csrk_build_host(A.row_ptr, A.col_idx, A.vals, host_params(srs))

    trials = []
    with cf.ThreadPoolExecutor(build_threads) as ex:
        for i in range(0, len(srs_list), build_threads):
            # every build of the chunk finishes before any timing starts: builds running beside the timed
            # kernel would take cores from it
            built = list(ex.map(build, srs_list[i:i + build_threads]))
            for j, (srs, h) in enumerate(built):
                try:
                    perm = C.csrk_copy_structure(h)["perm"]
                    trials.append((srs, time_host(h, x[perm], reps, warmup, nthreads)))
                finally:
                    C.csrk_destroy(h)
                    built[j] = (srs, None)
    best = min(trials, key=lambda t: t[1])
    fixed = C.csrk_tune(len(A.row_ptr) - 1, int(A.row_ptr[-1]), "host_cpu")
    at_fixed = next((us for srs, us in trials if srs == fixed["srs"]), None)
    return {"trials": trials, "best_srs": best[0], "best_us": best[1], "constant_time_srs": fixed["srs"],
            "constant_time_us": at_fixed, "constant_over_best": None if at_fixed is None else at_fixed / best[1],
            "threads": nthreads if nthreads > 0 else os.cpu_count()}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--threads", type=int, default=0, help="host kernel threads (0: the OpenMP default)")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import gen
    w = gen.WORKLOADS[args.workload]()
    A = w["A"] if "A" in w else w["As"][0]
    r = sweep_host(A, nthreads=args.threads)
    print("| SRS | us |\n|---|---|")
    for srs, us in r["trials"]:
        print(f"| {srs} | {us:.1f} |")
    print(f"\nbest SRS {r['best_srs']} ({r['best_us']:.1f} us); SRS {r['constant_time_srs']}: "
          f"{r['constant_time_us']:.1f} us ({r['constant_over_best']:.3f} x best)")


if __name__ == "__main__":
    main()
