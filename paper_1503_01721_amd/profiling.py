"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1503_01721_amd.profiling trace --dir OUT --command CMD --title T --out FILE
    python -m paper_1503_01721_amd.profiling traffic --fetch DIR --write DIR --copy-fetch DIR \\
        --copy-write DIR --kernel PATTERN --orientation dose|price --algorithmic BYTES \\
        --workload W --storage S --layout L --command CMD --out FILE
    python -m paper_1503_01721_amd.profiling counters --dir DIR [--dir DIR ...] --kernel PATTERN \\
        [--kernel PATTERN ...] --title T --command CMD --out FILE

`trace` turns a `--kernel-trace --stats` directory into a table of kernels
(calls, average/min/max duration).  `traffic` turns two `--pmc FETCH_SIZE`
and `--pmc WRITE_SIZE` runs of the benchmark, plus the same counters over a
plain 1 GiB device copy, into HBM bytes per launch of one kernel: the
counters' KiB are scaled by what they read for the copy of known size.
`counters` tabulates the mean of every counter of one or more `--pmc` runs per
launch of each named kernel.  The
traffic file carries the hash of the product kernels' sources (their code:
comments and the layout of white space do not enter it); bench.py reports
its figure only while that code is unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PRODUCT_SOURCES = ("spmv_device.hpp", "spmv.hip", "spmv_panel.hip", "common.hpp", "ddc_host.cpp")


def code_only(text: str) -> str:
    """C++ source without its comments, runs of white space as one blank
    (string and character literals kept whole)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def products_source_sha() -> str:
    """Hash of the product kernels' code (comments excluded)."""
    h = hashlib.sha256()
    for name in PRODUCT_SOURCES:
        with open(os.path.join(ROOT, "paper_1503_01721_amd", "csrc", name), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def _one(pattern):
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    return files[0]


def trace_table(d):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "**", "*kernel_stats.csv")))))
    out = ["# percent  calls   avg_us    min_us    max_us  kernel"]
    for r in rows:
        out.append(f"{float(r['Percentage']):8.2f} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} "
                   f"{float(r['MinNs']) / 1e3:9.2f} {float(r['MaxNs']) / 1e3:9.2f}  {r['Name'][:120]}")
    return out


def counter_mean(d, counter, match):
    vals = []
    for r in csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))):
        if r["Counter_Name"] == counter and match in r["Kernel_Name"]:
            vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} sample for a kernel matching {match!r} in {d}")
    return statistics.fmean(vals), len(vals)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--dir", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--note", action="append", default=[])
    t.add_argument("--out", required=True)
    f = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy-fetch", "copy-write", "kernel", "orientation", "workload", "storage",
              "layout", "command", "out"):
        f.add_argument("--" + k, required=True)
    f.add_argument("--algorithmic", type=float, required=True)
    f.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    c = sub.add_parser("counters")
    c.add_argument("--dir", action="append", required=True)
    c.add_argument("--kernel", action="append", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", action="append", required=True)
    c.add_argument("--note", action="append", default=[])
    c.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.what == "counters":
        lines = [f"# rocprofv3 counters, mean per launch: {a.title}", "#",
                 "# commands (from /tmp with TMPDIR=/tmp, one run per counter set):",
                 *[f"#   rocprofv3 --pmc {cmd}" for cmd in a.command], *[f"# {n}" for n in a.note], "#"]
        for k in a.kernel:
            lines.append(f"kernel: {k}")
            for d in a.dir:
                names = sorted({r["Counter_Name"] for r in csv.DictReader(
                    open(_one(os.path.join(d, "**", "*counter_collection.csv"))))})
                for n in names:
                    try:
                        v, cnt = counter_mean(d, n, k)
                    except SystemExit:
                        continue
                    lines.append(f"  {n:24s} {v:14.5g}  (mean of {cnt} launches)")
    elif a.what == "trace":
        lines = [f"# rocprofv3 kernel trace: {a.title}", "#", "# command (from /tmp with TMPDIR=/tmp, library built in place):",
                 f"#   {a.command}", *[f"# {n}" for n in a.note], "#", *trace_table(a.dir)]
    else:
        fetch, n_f = counter_mean(a.fetch, "FETCH_SIZE", a.kernel)
        write, n_w = counter_mean(a.write, "WRITE_SIZE", a.kernel)
        cf, _ = counter_mean(a.copy_fetch, "FETCH_SIZE", "copyBuffer")
        cw, _ = counter_mean(a.copy_write, "WRITE_SIZE", "copyBuffer")
        rs = a.copy_bytes / (cf * 1024)          # bytes per counted KiB, from the copy
        ws = a.copy_bytes / (cw * 1024)
        rb, wb = fetch * 1024 * rs, write * 1024 * ws
        lines = [f"# HBM bytes per launch from rocprofv3 counters: {a.orientation} product, "
                 f"{a.workload}, {a.storage}, {a.layout} layout",
                 "#", "# commands (from /tmp with TMPDIR=/tmp):",
                 f"#   rocprofv3 --pmc FETCH_SIZE -f csv -d <out> -o pmc -- {a.command}",
                 f"#   rocprofv3 --pmc WRITE_SIZE -f csv -d <out> -o pmc -- {a.command}",
                 "#   rocprofv3 --pmc FETCH_SIZE|WRITE_SIZE -f csv -d <out> -o pmc -- python3 <repo>/bench.py --copy-calibration",
                 f"# kernel: {a.kernel}",
                 f"# calibration: 1 GiB device copy, FETCH_SIZE {cf:.1f} KiB -> read scale {rs:.3f}; "
                 f"WRITE_SIZE {cw:.1f} KiB -> write scale {ws:.3f}",
                 f"# FETCH_SIZE {fetch:.1f} KiB (mean of {n_f} launches), WRITE_SIZE {write:.1f} KiB (mean of {n_w})",
                 f"# read {rb / 1e9:.4f} GB + written {wb / 1e9:.4f} GB per launch; algorithmic "
                 f"{a.algorithmic / 1e9:.4f} GB (the layout's own index width; traffic "
                 f"{(rb + wb) / a.algorithmic:.3f} x the algorithmic bytes)",
                 f"products_source_sha256_16 = {products_source_sha()}",
                 f"hbm_read_bytes_per_launch = {rb:.0f}",
                 f"hbm_write_bytes_per_launch = {wb:.0f}",
                 f"hbm_bytes_per_launch = {rb + wb:.0f}"]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
