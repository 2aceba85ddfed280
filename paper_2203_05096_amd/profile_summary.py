"""Summaries of rocprofv3 output for profiles/: kernel traces, HBM traffic and counters per kernel.

    # per-kernel durations from `rocprofv3 --kernel-trace --stats --output-format csv -d DIR -o kt -- ...`
    python -m paper_2203_05096_amd.profile_summary trace DIR --title T --command "rocprofv3 ..." > out.md

    # HBM bytes per launch from one FETCH_SIZE run and one WRITE_SIZE run of the same command (with
    # bench.py --copy-calibration, whose 1 GiB copies scale the counters to bytes)
    python -m paper_2203_05096_amd.profile_summary traffic FETCH_DIR WRITE_DIR --workload c5 --store f32 \\
        --command "..." > profiles/hbm_traffic_<workload>_<store>.txt

    # mean of every collected counter per kernel (any --pmc run)
    python -m paper_2203_05096_amd.profile_summary counters DIR [DIR ...] --title T --command "..." > out.md

Only reads CSV files; nothing here touches the GPU.
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEVICE = os.path.join(ROOT, "paper_2203_05096_amd", "csrc", "device")
WORKLOAD_NAMES = {"c2": "3d7pt_128cube_scrambled", "c3": "3d27pt_100cube", "c4": "2d9pt_2048sq_drop10",
                  "c5": "batch64_3d7pt_sides16to96_8rhs", "irr": "rmat_2pow20_rows_sym"}
COPY_KERNEL = "__amd_rocclr_copyBuffer"
GIB = 1 << 30


def kernel_source_hash() -> str:
    """sha256 over the device sources (the same digest bench.py compares before reporting traffic)."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(DEVICE)):
        if f.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(DEVICE, f), "rb").read())
    return h.hexdigest()


def _rows(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    for p in files:
        with open(p, newline="") as f:
            yield from csv.DictReader(f)


def short(name: str) -> str:
    """Kernel name without the argument list (template arguments kept)."""
    name = name.replace("csrk::dev::(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i].replace("csrk::dev::(anonymous namespace)::", "")
    return name.replace("csrk::dev::(anonymous namespace)::", "")


def trace(args):
    rows = list(_rows(args.dir, "kernel_stats.csv"))
    lines = [f"# Kernel trace: {args.title}", "", "Command (repository root, one MI355X):", "", "    " + args.command, "",
             f"Device source sha256: `{kernel_source_hash()}`", "",
             "| kernel | calls | average us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    print("\n".join(lines))


def _per_kernel(dirs, counter=None):
    """{kernel: {counter: [values per dispatch]}} from counter_collection CSVs."""
    acc = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        for r in _rows(d, "counter_collection.csv"):
            if counter is not None and r["Counter_Name"] != counter:
                continue
            acc[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return acc


def traffic(args):
    fetch = _per_kernel([args.fetch_dir], "FETCH_SIZE")
    write = _per_kernel([args.write_dir], "WRITE_SIZE")
    # calibration: the largest copy dispatches (1 GiB read + 1 GiB written each)
    cf = max(fetch[COPY_KERNEL]["FETCH_SIZE"]) if COPY_KERNEL in fetch else None
    cw = max(write[COPY_KERNEL]["WRITE_SIZE"]) if COPY_KERNEL in write else None
    if not cf or not cw:
        raise SystemExit("no calibration copy dispatches (run bench.py with --copy-calibration)")
    fs, ws = GIB / (cf * 1024), GIB / (cw * 1024)
    per = {}
    for direction, prefixes in (("forward", ("k_batch_forward", "k_spmv_csrk<", "k_spmv_csrk_mrhs")),
                                ("adjoint", ("k_batch_adjoint", "k_adjoint_csrk"))):
        names = [k for k in fetch if k.startswith(prefixes)]
        if not names:
            continue
        k = max(names, key=lambda n: len(fetch[n]["FETCH_SIZE"]))
        f = sum(fetch[k]["FETCH_SIZE"]) / len(fetch[k]["FETCH_SIZE"])
        w = sum(write[k]["WRITE_SIZE"]) / len(write[k]["WRITE_SIZE"]) if k in write else 0.0
        per[direction] = {"kernel": k, "dispatches": len(fetch[k]["FETCH_SIZE"]), "raw_fetch_KiB": round(f, 1),
                          "raw_write_KiB": round(w, 1), "fetch_bytes": int(f * 1024 * fs),
                          "write_bytes": int(w * 1024 * ws)}
    head = [f"# HBM traffic per launch, workload {args.workload} ({WORKLOAD_NAMES[args.workload]}), {args.store}.",
            "# Counters from two rocprofv3 runs of the same command (one counter each), repository root, one MI355X:"]
    head += [f"#   {c}" for c in args.command]
    head += [f"# Scaling: the largest {COPY_KERNEL} dispatch (1 GiB read, 1 GiB written, bench.py --copy-calibration)",
             f"# reported FETCH_SIZE {cf:.0f} KiB and WRITE_SIZE {cw:.0f} KiB, so bytes = counter * 1024 * scale.",
             "# Summarised by: python -m paper_2203_05096_amd.profile_summary traffic ...",
             "# kernel_source_sha256 identifies the device sources profiled; bench.py reports traffic only while it "
             "matches."]
    rec = {"kernel_source_sha256": kernel_source_hash(), "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
           "per_launch": per}
    print("\n".join(head))
    print(json.dumps(rec, indent=1))


def counters(args):
    acc = _per_kernel(args.dirs)
    names = sorted({c for k in acc for c in acc[k]})
    lines = [f"# Counters: {args.title}", "", "Commands (repository root, one MI355X):", ""]
    lines += ["    " + c for c in args.command]
    lines += ["", f"Device source sha256: `{kernel_source_hash()}`", "", "Mean per dispatch:", "",
              "| kernel | dispatches | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    kept = []
    for k in sorted(acc, key=lambda k: -len(next(iter(acc[k].values())))):
        if args.match and not any(m in k for m in args.match):
            continue
        kept.append(k)
        n = max(len(v) for v in acc[k].values())
        cells = []
        for c in names:
            v = acc[k].get(c)
            cells.append(f"{sum(v) / len(v):.4g}" if v else "")
        lines.append(f"| `{k}` | {n} | " + " | ".join(cells) + " |")
    # ratios that do not depend on the counters' units
    mean = lambda k, c: sum(acc[k][c]) / len(acc[k][c]) if acc[k].get(c) else None  # noqa: E731
    rows = []
    for k in kept:
        hit, miss = mean(k, "TCC_HIT_sum"), mean(k, "TCC_MISS_sum")
        wait, alive = mean(k, "SQ_WAIT_ANY"), mean(k, "SQ_WAVE_CYCLES")
        conf, lds = mean(k, "SQ_LDS_BANK_CONFLICT"), mean(k, "SQ_ACTIVE_INST_LDS")
        cells = [f"{hit / (hit + miss):.2f}" if hit is not None and miss else "",
                 f"{miss * 128 / 1e6:.0f}" if miss is not None else "",
                 f"{wait / alive:.2f}" if wait is not None and alive else "",
                 f"{conf / lds:.2f}" if conf is not None and lds else ""]
        rows.append(f"| `{k}` | " + " | ".join(cells) + " |")
    if rows:
        lines += ["", "Ratios: L2 hit rate TCC_HIT / (TCC_HIT + TCC_MISS); L2 misses x 128 B (MB, the line size); "
                      "share of wavefront time spent waiting SQ_WAIT_ANY / SQ_WAVE_CYCLES; LDS bank-conflict cycles "
                      "per active LDS cycle.", "",
                  "| kernel | L2 hit | L2 misses x 128 B (MB) | wait share | LDS conflicts / LDS active |",
                  "|---|---|---|---|---|", *rows]
    # per-CU busy shares: TA / TD / TCP counters are summed over the 256 CUs, GRBM_GUI_ACTIVE over the 8 XCDs
    rows = []
    for k in kept:
        act = mean(k, "GRBM_GUI_ACTIVE")
        if not act:
            continue
        share = lambda c: mean(k, c) / 256 / (act / 8) if mean(k, c) is not None else None  # noqa: E731
        vals = [share(c) for c in ("TA_TA_BUSY_sum", "TD_TD_BUSY_sum", "TCP_PENDING_STALL_CYCLES_sum")]
        if all(v is None for v in vals):
            continue
        rows.append(f"| `{k}` | " + " | ".join("" if v is None else f"{v:.2f}" for v in vals) + " |")
    if rows:
        lines += ["", "Vector-memory pipeline, share of the active cycles per CU (counters summed over the 256 CUs, "
                      "GRBM_GUI_ACTIVE over the 8 XCDs): texture-address unit busy, texture-data unit busy, L1 "
                      "waiting for L2 data.", "",
                  "| kernel | TA busy | TD busy | L1 pending on L2 |", "|---|---|---|---|", *rows]
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    f = sub.add_parser("traffic")
    f.add_argument("fetch_dir")
    f.add_argument("write_dir")
    f.add_argument("--workload", required=True, choices=sorted(WORKLOAD_NAMES))
    f.add_argument("--store", required=True)
    f.add_argument("--command", required=True, action="append")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--title", required=True)
    c.add_argument("--command", required=True, action="append")
    c.add_argument("--match", action="append", default=None, help="only kernels whose name contains this")
    args = ap.parse_args(argv)
    {"trace": trace, "traffic": traffic, "counters": counters}[args.mode](args)


if __name__ == "__main__":
    sys.exit(main())
