"""Summarises rocprofv3 output into short text files for profiles/.

Mode `traffic` (default): HBM byte counters of one kernel.

Input: four counter-collection CSV files written by `rocprofv3 --pmc ...
--output-format csv`: FETCH_SIZE and WRITE_SIZE of a plain device copy of known
size (`bench.py --copy-calibration MIB`), and FETCH_SIZE and WRITE_SIZE of the
kernel. Each counter is scaled by (bytes the copy moved) / (what the counter
read for it); the result is the kernel's HBM traffic per launch. The summary
records the SHA-256 of the kernel's source files so that a reader can tell
whether the kernel changed after the counters were taken.

python -m paper_2311_05322_amd.pmc_summary --copy-mib 1024 \\
    --copy-fetch C_F.csv --copy-write C_W.csv --fetch K_F.csv --write K_W.csv \\
    --kernel k_lu_update --command "..." --out profiles/x.md

Mode `stats`: the kernel statistics CSV of `rocprofv3 --kernel-trace --stats
--output-format csv` as a markdown table (namespaces and argument lists
dropped from the names), with the command and a note.

python -m paper_2311_05322_amd.pmc_summary stats --csv prof/x_kernel_stats.csv \\
    --title "..." --command "..." [--note "..."] --out profiles/y.md

Mode `counters`: any counters of `rocprofv3 --pmc` runs (one or more
counter-collection CSV files), averaged per kernel, as one markdown table.

python -m paper_2311_05322_amd.pmc_summary counters --csv a.csv --csv b.csv \\
    --title "..." --command "..." --out profiles/z.md
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = {"k_lu_update": ["csrc/k_dense.hip", "csrc/mx_device.h"],
           "k_lu_update_list": ["csrc/k_dense.hip", "csrc/mx_device.h"],
           "k_trsm": ["csrc/k_dense.hip", "csrc/mx_device.h"],
           "k_trsm_lower": ["csrc/k_dense.hip", "csrc/mx_device.h"],
           "k_trsm_upper": ["csrc/k_dense.hip", "csrc/mx_device.h"],
           "k_spmm": ["csrc/k_operator.hip", "csrc/mx_device.h"],
           "k_spmm_bcast": ["csrc/k_operator.hip", "csrc/mx_device.h"],
           "k_spmm_win": ["csrc/k_operator.hip", "csrc/mx_device.h"]}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in SOURCES[kernel]:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _values(path, name_part):
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if name_part in r["Kernel_Name"]:
                out.append(float(r["Counter_Value"]))
    return out


def short_name(name: str) -> str:
    """'void mx::(anonymous namespace)::k_trsm<float, true, 2>(args)' -> 'k_trsm<float, true, 2>'."""
    name = name.replace("(anonymous namespace)::", "")
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    name = name[:cut].strip()
    if name.startswith("void "):
        name = name[5:]
    head = name.split("<", 1)
    head[0] = head[0].split("::")[-1]
    return "<".join(head)


def stats(argv):
    ap = argparse.ArgumentParser(prog="pmc_summary stats")
    ap.add_argument("--csv", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--note", action="append", default=[])
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    rows = []
    with open(a.csv) as f:
        for r in csv.DictReader(f):
            rows.append((short_name(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
                         float(r["AverageNs"]) / 1e6, float(r["Percentage"])))
    rows.sort(key=lambda x: -x[2])
    lines = [f"# {a.title}", "", "Command (repository root on the MI355X box, `cd /tmp && export TMPDIR=/tmp` first):",
             "", "```", *a.command, "```", ""]
    for n in a.note:
        lines += [n, ""]
    lines += ["| kernel | calls | total ms | avg ms | % |", "|---|---:|---:|---:|---:|"]
    for name, calls, tot, avg, pct in rows[:a.top]:
        name = name if len(name) <= 72 else name[:69] + "..."
        lines.append(f"| `{name}` | {calls} | {tot:.1f} | {avg:.4f} | {pct:.2f} |")
    lines.append("")
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def counters(argv):
    ap = argparse.ArgumentParser(prog="pmc_summary counters")
    ap.add_argument("--csv", action="append", required=True, help="counter-collection CSV (repeatable)")
    ap.add_argument("--title", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--note", action="append", default=[])
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    vals: dict = {}
    for path in a.csv:
        with open(path) as f:
            for r in csv.DictReader(f):
                k = short_name(r["Kernel_Name"])
                vals.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    kernels = sorted(vals)
    names = sorted({c for k in kernels for c in vals[k]})
    lines = [f"# {a.title}", "", "Commands (repository root on the MI355X box, `cd /tmp && export TMPDIR=/tmp` "
             "first):", "", "```", *a.command, "```", ""]
    for n in a.note:
        lines += [n, ""]
    lines += ["Per-dispatch averages over all dispatches of each kernel.", "",
              "| counter | " + " | ".join(f"`{k}`" for k in kernels) + " |",
              "|---|" + "---:|" * len(kernels)]
    for c in names:
        cells = []
        for k in kernels:
            v = vals[k].get(c)
            cells.append(f"{sum(v) / len(v):.4g}" if v else "")
        lines.append(f"| {c} | " + " | ".join(cells) + " |")
    lines.append("")
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def main():
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "stats":
        return stats(sys.argv[2:])
    if len(sys.argv) > 1 and sys.argv[1] == "counters":
        return counters(sys.argv[2:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--copy-kernel", default="neg_kernel")
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel", required=True, choices=sorted(SOURCES))
    ap.add_argument("--match", default=None, help="substring of the dispatches' kernel names (default: --kernel)")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    kib = a.copy_mib * 1024.0
    cf, cw = _values(a.copy_fetch, a.copy_kernel), _values(a.copy_write, a.copy_kernel)
    sf, sw = kib / (sum(cf) / len(cf)), kib / (sum(cw) / len(cw))
    kf, kw = _values(a.fetch, a.match or a.kernel), _values(a.write, a.match or a.kernel)
    if not kf or len(kf) != len(kw):
        raise SystemExit("kernel dispatch counts differ or are empty")
    n = len(kf)
    fetch_b = sum(kf) / n * sf * 1024.0
    write_b = sum(kw) / n * sw * 1024.0
    lines = [
        f"# HBM traffic of {a.kernel}, 1.02M-edge chamber (512 subdomains, 32 transmitters)",
        "",
        "Commands (repository root on the MI355X box, `cd /tmp && export TMPDIR=/tmp` first):",
        "",
        "```",
        *a.command,
        "```",
        "",
        f"Copy calibration ({a.copy_mib} MiB read and written per dispatch, {len(cf)} dispatches):",
        f"FETCH_SIZE {sum(cf) / len(cf):.1f} KiB -> factor {sf:.4f}; WRITE_SIZE {sum(cw) / len(cw):.1f} KiB -> factor {sw:.4f}.",
        "",
        f"{a.kernel} (dispatches matching `{a.match or a.kernel}`): {n} dispatches; figures are per-dispatch "
        "averages.",
        "",
        "| per launch | counter (KiB) | scaled bytes |",
        "|---|---:|---:|",
        f"| read | {sum(kf) / n:.1f} | {fetch_b:.4e} |",
        f"| written | {sum(kw) / n:.1f} | {write_b:.4e} |",
        f"| total | | {fetch_b + write_b:.4e} |",
        "",
        f"bytes_per_launch: {fetch_b + write_b:.6e}",
        f"source_sha256: {source_hash(a.kernel)}",
        "",
    ]
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
