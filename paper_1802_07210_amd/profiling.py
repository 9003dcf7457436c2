"""Summaries of rocprofv3 output for the committed profiles.

Two commands, each reading the CSV output of rocprofv3 runs
(``--output-format csv``):

  stats    kernel-trace statistics (``--kernel-trace --stats``) as a markdown
           table: calls, mean / min / max duration and share of kernel time
           per kernel.
  traffic  HBM bytes per launch of one kernel from two counter runs of the
           benchmark (``--pmc FETCH_SIZE``, then ``--pmc WRITE_SIZE``; KiB
           per dispatch) and the same two counters on a plain copy kernel of
           known size (``bench.py --mode calib``), which give the factor from
           counter units to bytes. Writes a JSON record (bytes per launch and a
           hash of the kernel source the counters were taken on) and a
           markdown summary.
  valu     instruction counts per launch and per wavefront of every kernel of
           one counter run (``--pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU
           SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_WAVE_CYCLES SQ_WAIT_INST_ANY``):
           a JSON record per kernel (with the kernel-source hash) and a
           markdown table. With a kernel's duration they give its share of
           the chip's VALU issue rate (a wave64 instruction holds a 16-lane
           SIMD for 4 cycles: 256 CUs x 4 SIMDs x 2.4 GHz / 4 = 614.4 G
           wavefront instructions per second).

Usage:
  python -m paper_1802_07210_amd.profiling stats DIR OUT.md --cmd "..."
  python -m paper_1802_07210_amd.profiling traffic --kernel NAME \\
      --fetch DIR --write DIR --calib-fetch DIR --calib-write DIR \\
      --copy-bytes N --json OUT.json --md OUT.md --cmd "..."
  python -m paper_1802_07210_amd.profiling valu DIR --workload W \
      --json OUT.json --md OUT.md --cmd "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1802_07210_amd", "csrc")
# the kernels' source and the headers compiled into them
KERNEL_SOURCES = [os.path.join(CSRC, n) for n in ("elas_kernels.hip", "elas_internal.h", "elas_wave.h")]


def kernel_source_hash() -> str:
    """First 16 hex digits of the SHA-256 over the kernels' source files."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _one(dirpath: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(dirpath, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {dirpath}")
    return hits[-1]


def _col(row: dict, *names: str) -> str:
    for n in names:
        for k in row:
            if k.lower() == n.lower():
                return row[k]
    raise KeyError(f"none of {names} in {list(row)}")


def short_name(name: str) -> str:
    """Kernel name without namespaces and arguments (k_dense2, k_mesh, ...)."""
    base = name.replace("(anonymous namespace)::", "").split("(")[0]
    return base.split("::")[-1].strip()


def kernel_stats(dirpath: str):
    rows = list(csv.DictReader(open(_one(dirpath, "kernel_stats.csv"))))
    out = []
    for r in rows:
        out.append({
            "name": short_name(_col(r, "Name", "KERNEL_NAME")),
            "calls": int(_col(r, "Calls")),
            "total_ns": float(_col(r, "TotalDurationNs")),
            "mean_ns": float(_col(r, "AverageNs")),
            "min_ns": float(_col(r, "MinNs")),
            "max_ns": float(_col(r, "MaxNs")),
            "pct": float(_col(r, "Percentage")),
        })
    return out


def cmd_stats(args):
    st = kernel_stats(args.dir)
    lines = [f"# rocprofv3 kernel statistics: {args.title}", "",
             "Command (from the repository root on the GPU host):", "",
             "```", args.cmd, "```", "",
             "| kernel | calls | mean us | min us | max us | share of kernel time % |",
             "|---|---:|---:|---:|---:|---:|"]
    for r in sorted(st, key=lambda r: -r["total_ns"]):
        lines.append(f"| {r['name']} | {r['calls']} | {r['mean_ns'] / 1e3:.2f} | "
                     f"{r['min_ns'] / 1e3:.2f} | {r['max_ns'] / 1e3:.2f} | {r['pct']:.2f} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(args.out)


def counter_means(dirpath: str, counter: str):
    """Mean counter value per dispatch, per kernel short name."""
    vals = {}
    for r in csv.DictReader(open(_one(dirpath, "counter_collection.csv"))):
        if _col(r, "Counter_Name") != counter:
            continue
        vals.setdefault(short_name(_col(r, "Kernel_Name")), []).append(
            float(_col(r, "Counter_Value")))
    return {k: (statistics.fmean(v), len(v)) for k, v in vals.items()}


def _copy_kernel(means: dict):
    """The calibration copy (torch's neg kernel; failing that, the kernel with
    the largest counter per dispatch)."""
    named = [k for k in means if "neg" in k]
    return named[0] if named else max(means, key=lambda k: means[k][0])


def cmd_traffic(args):
    fetch = counter_means(args.fetch, "FETCH_SIZE")
    write = counter_means(args.write, "WRITE_SIZE")
    cf = counter_means(args.calib_fetch, "FETCH_SIZE")
    cw = counter_means(args.calib_write, "WRITE_SIZE")
    kf, kw = _copy_kernel(cf), _copy_kernel(cw)
    # counters are in KiB; the factor maps counter KiB to true bytes
    f_fetch = args.copy_bytes / (cf[kf][0] * 1024.0)
    f_write = args.copy_bytes / (cw[kw][0] * 1024.0)
    if args.kernel not in fetch or args.kernel not in write:
        raise SystemExit(f"{args.kernel} not among {sorted(fetch)}")
    fb = fetch[args.kernel][0] * 1024.0 * f_fetch
    wb = write[args.kernel][0] * 1024.0 * f_write
    sha = kernel_source_hash()
    rec = {"kernel": args.kernel, "workload": args.workload,
           "bytes_per_launch": round(fb + wb), "fetch_bytes": round(fb), "write_bytes": round(wb),
           "fetch_kib_raw": fetch[args.kernel][0], "write_kib_raw": write[args.kernel][0],
           "dispatches": [fetch[args.kernel][1], write[args.kernel][1]],
           "calib_copy_kernel": [kf, kw], "calib_copy_bytes": args.copy_bytes,
           "calib_factor_fetch": f_fetch, "calib_factor_write": f_write,
           "source_sha256_16": sha}
    with open(args.json, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    lines = [f"# HBM traffic per launch: {args.kernel}, {args.workload}", "",
             "Commands (from the repository root on the GPU host):", "",
             "```", args.cmd, "```", "",
             "Counters are KiB per dispatch, averaged over the kernel's dispatches, and",
             "scaled by a plain copy kernel of known size read through the same counter.", "",
             "| quantity | value |", "|---|---:|",
             f"| FETCH_SIZE, KiB per dispatch (raw) | {fetch[args.kernel][0]:.1f} |",
             f"| WRITE_SIZE, KiB per dispatch (raw) | {write[args.kernel][0]:.1f} |",
             f"| copy kernel ({kf}) FETCH_SIZE KiB / true KiB | "
             f"{cf[kf][0]:.1f} / {args.copy_bytes / 1024:.1f} |",
             f"| copy kernel ({kw}) WRITE_SIZE KiB / true KiB | "
             f"{cw[kw][0]:.1f} / {args.copy_bytes / 1024:.1f} |",
             f"| scale factor fetch / write | {f_fetch:.4f} / {f_write:.4f} |",
             f"| fetched bytes per launch | {fb:,.0f} |",
             f"| written bytes per launch | {wb:,.0f} |",
             f"| HBM traffic per launch | {fb + wb:,.0f} |",
             f"| kernel source sha256 (first 16 hex) | {sha} |", "",
             "All kernels of the run (raw KiB per dispatch, fetch / write):", "",
             "| kernel | FETCH_SIZE | WRITE_SIZE |", "|---|---:|---:|"]
    for k in sorted(set(fetch) | set(write)):
        lines.append(f"| {k} | {fetch.get(k, (float('nan'),))[0]:.1f} | "
                     f"{write.get(k, (float('nan'),))[0]:.1f} |")
    with open(args.md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps(rec))


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD",
               "SQ_WAVE_CYCLES", "SQ_WAIT_INST_ANY")
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4   # wavefront instructions per second


def valu_record(dirpath: str) -> dict:
    """Per kernel: the mean of each SQ counter per dispatch (device totals)."""
    means = {c: counter_means(dirpath, c) for c in SQ_COUNTERS}
    out = {}
    for k in means["SQ_WAVES"]:
        if not all(k in means[c] for c in SQ_COUNTERS):
            continue
        rec = {c.lower(): means[c][k][0] for c in SQ_COUNTERS}
        rec["dispatches"] = means["SQ_WAVES"][k][1]
        out[k] = rec
    return out


def cmd_valu(args):
    rec = valu_record(args.dir)
    sha = kernel_source_hash()
    with open(args.json, "w") as f:
        json.dump({"workload": args.workload, "valu_issue_peak_per_s": VALU_ISSUE_PEAK,
                   "kernels": rec, "source_sha256_16": sha}, f, indent=1)
        f.write("\n")
    lines = [f"# Instruction counts per launch: {args.workload}", "",
             "Command (from the repository root on the GPU host):", "",
             "```", args.cmd, "```", "",
             "SQ counters are device totals per dispatch, averaged over the kernel's",
             "dispatches. A wave64 VALU instruction holds a 16-lane SIMD for 4 cycles,",
             f"so the chip issues at most {VALU_ISSUE_PEAK / 1e9:.1f} G wavefront VALU "
             "instructions per second;",
             "a kernel's VALU instructions per launch over that rate is the floor of its",
             "duration from instruction issue alone.", "",
             "| kernel | waves | VALU / wave | SALU / wave | LDS / wave | VMEM rd / wave | "
             "VALU per launch | VALU issue floor (us) |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(rec, key=lambda k: -rec[k]["sq_insts_valu"]):
        r = rec[k]
        w = max(r["sq_waves"], 1.0)
        lines.append(f"| {k} | {r['sq_waves']:.0f} | {r['sq_insts_valu'] / w:.1f} | "
                     f"{r['sq_insts_salu'] / w:.1f} | {r['sq_insts_lds'] / w:.1f} | "
                     f"{r['sq_insts_vmem_rd'] / w:.1f} | {r['sq_insts_valu']:,.0f} | "
                     f"{r['sq_insts_valu'] / VALU_ISSUE_PEAK * 1e6:.2f} |")
    lines += ["", f"Kernel source sha256 (first 16 hex): {sha}"]
    with open(args.md, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("out")
    a.add_argument("--cmd", required=True)
    a.add_argument("--title", default="")
    a.set_defaults(fn=cmd_stats)
    b = sub.add_parser("traffic")
    b.add_argument("--kernel", required=True)
    b.add_argument("--workload", default="")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--calib-fetch", required=True)
    b.add_argument("--calib-write", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--json", required=True)
    b.add_argument("--md", required=True)
    b.add_argument("--cmd", required=True)
    b.set_defaults(fn=cmd_traffic)
    c = sub.add_parser("valu")
    c.add_argument("dir")
    c.add_argument("--workload", default="")
    c.add_argument("--json", required=True)
    c.add_argument("--md", required=True)
    c.add_argument("--cmd", required=True)
    c.set_defaults(fn=cmd_valu)
    args = ap.parse_args(argv)
    args.fn(args)


if __name__ == "__main__":
    main(sys.argv[1:])
