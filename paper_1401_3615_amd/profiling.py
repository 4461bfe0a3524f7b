"""Summaries of rocprofv3 output for the backprojection kernels.

    python -m paper_1401_3615_amd.profiling stats KERNEL_STATS_CSV [--top N]
        Markdown table of a `rocprofv3 --kernel-trace --stats` run.

    python -m paper_1401_3615_amd.profiling traffic --fetch DIR --write DIR
            --kernel SUBSTR --copy SUBSTR --copy-bytes N --out FILE.json
        HBM bytes per launch of one kernel from two `rocprofv3 --pmc` runs
        (FETCH_SIZE, then WRITE_SIZE; both in KiB per dispatch), each scaled by
        what the same counter reads for a plain elementwise kernel that moves a
        known number of bytes (read N, write N).  The result records the
        SHA-256 of the kernel source it was taken on, so a reader can tell
        when it no longer describes the code.

    python -m paper_1401_3615_amd.profiling counters DIR --kernel SUBSTR
        Per-dispatch averages of every counter of one kernel in a --pmc run.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(PKG, "csrc", "fdk_kernels.hip")


def kernel_source_sha256() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def short_name(name: str) -> str:
    """Kernel name without the return type, namespaces and argument list."""
    n = name.strip()
    if n.endswith(")"):
        depth = 0
        for i in range(len(n) - 1, -1, -1):
            if n[i] == ")":
                depth += 1
            elif n[i] == "(":
                depth -= 1
                if depth == 0:
                    n = n[:i]
                    break
    for pre in ("void ", "fdk::", "(anonymous namespace)::"):
        n = n.replace(pre, "")
    return n.strip()


def read_stats(path: str) -> list[dict]:
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append({"name": r["Name"], "calls": int(r["Calls"]),
                         "total_ns": float(r["TotalDurationNs"]), "avg_ns": float(r["AverageNs"]),
                         "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"]),
                         "pct": float(r["Percentage"])})
    return rows


# kernels of this library (the rest of a trace is torch's input generation)
OWN_KERNELS = r"^(bp_|fp_|window_kernel|stage_|fold_|filter_kernel|unstage|absmax|convert|finalize|zero_u32|fill|"\
              r"reset_counter|sumsq|max_kernel|scalar_kernel|cgls_|residual_kernel|sirt_|inv_floor|band_gather)"


def stats_markdown(path: str, top: int = 15, match: str | None = None) -> str:
    rows = read_stats(path)
    if match:
        rows = [r for r in rows if re.search(match, short_name(r["name"]))]
    rows = sorted(rows, key=lambda r: -r["total_ns"])[:top]
    out = ["| kernel | calls | avg ms | min ms | max ms | total ms | % |", "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{short_name(r['name'])}` | {r['calls']} | {r['avg_ns'] / 1e6:.3f} | "
                   f"{r['min_ns'] / 1e6:.3f} | {r['max_ns'] / 1e6:.3f} | {r['total_ns'] / 1e6:.1f} | "
                   f"{r['pct']:.1f} |")
    return "\n".join(out)


def counter_means(outdir: str, kernel_substr: str) -> dict[str, float]:
    """Mean per dispatch of every counter recorded for kernels matching kernel_substr."""
    files = glob.glob(os.path.join(outdir, "**", "*counter_collection*.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection CSV under {outdir}")
    total = defaultdict(float)
    dispatches = defaultdict(set)
    for path in files:
        with open(path) as f:
            for r in csv.DictReader(f):
                if kernel_substr not in r["Kernel_Name"]:
                    continue
                total[r["Counter_Name"]] += float(r["Counter_Value"])
                dispatches[r["Counter_Name"]].add((path, r.get("Dispatch_Id", r.get("Correlation_Id", ""))))
    if not total:
        raise KeyError(f"no dispatch of a kernel matching {kernel_substr!r} in {outdir}")
    return {k: total[k] / len(dispatches[k]) for k in total}


def traffic(fetch_dir: str, write_dir: str, kernel: str, copy: str, copy_bytes: int) -> dict:
    kib = 1024.0
    f_k = counter_means(fetch_dir, kernel)["FETCH_SIZE"] * kib
    f_c = counter_means(fetch_dir, copy)["FETCH_SIZE"] * kib
    w_k = counter_means(write_dir, kernel)["WRITE_SIZE"] * kib
    w_c = counter_means(write_dir, copy)["WRITE_SIZE"] * kib
    f_scale, w_scale = copy_bytes / f_c, copy_bytes / w_c
    return {
        "kernel": kernel,
        "kernel_source_sha256": kernel_source_sha256(),
        "fetch_bytes_raw": f_k, "write_bytes_raw": w_k,
        "copy_kernel": copy, "copy_bytes_each_way": copy_bytes,
        "copy_fetch_bytes_raw": f_c, "copy_write_bytes_raw": w_c,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "hbm_read_bytes_per_launch": f_k * f_scale,
        "hbm_write_bytes_per_launch": w_k * w_scale,
        "hbm_bytes_per_launch": f_k * f_scale + w_k * w_scale,
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_1401_3615_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=15)
    s.add_argument("--own", action="store_true", help="only kernels of this library")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--out")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--kernel", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_markdown(a.csv, a.top, OWN_KERNELS if a.own else None))
    elif a.cmd == "traffic":
        res = traffic(a.fetch, a.write, a.kernel, a.copy, a.copy_bytes)
        txt = json.dumps(res, indent=1)
        if a.out:
            with open(a.out, "w") as f:
                f.write(txt + "\n")
        print(txt)
    else:
        print(json.dumps(counter_means(a.dir, a.kernel), indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
