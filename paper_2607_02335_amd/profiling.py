"""Turn rocprofv3 output into the short summaries kept under profiles/.

    python -m paper_2607_02335_amd.profiling stats  STATS_CSV  --workload W --command C -o OUT.md
    python -m paper_2607_02335_amd.profiling counters RUN_DIR [RUN_DIR ...] --workload W --command C -o OUT.md
    python -m paper_2607_02335_amd.profiling traffic --workload W --command C \\
        --fetch FETCH_DIR --write WRITE_DIR --calib-fetch DIR --calib-write DIR \\
        --calib-bytes N -o OUT.md

`stats` summarises a `--kernel-trace --stats` run (kernel_stats.csv): calls,
average / min / max duration and share per kernel.  `traffic` reads two
`--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of a workload (per-dispatch
counter_collection.csv, values in KiB) and the same counters of a plain
copy of `calib-bytes` bytes, scales each counter by (known bytes / counter
reading of the copy), averages per kernel and writes a markdown table plus a
JSON sidecar (OUT.json) that bench.py reads: per launch-trace label, the
HBM bytes per launch and a hash of the kernel sources the counters were
taken with, so a figure is dropped once the kernels change.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# rocprofv3 kernel name -> launch-trace label of the library
_LABELS = [
    ("k_apply_", "apply"),
    ("k_assemble", "pi_assemble"),
    ("k_pi_solve", "pi_solve"),
    ("k_pi_combine", "pi_combine"),
    ("k_pi_sweep", "pi_sweep"),
    ("k_dss_axis", "dss_axis"),
    ("k_dot", "dot"),
    ("k_anorm", "assembled_norm"),
    ("k_distribute", "distribute"),
    ("k_cg_ur", "cg_update_ur"),
    ("k_cg_p", "cg_update_p"),
]


def label_of(kernel_name: str):
    for key, lab in _LABELS:
        if key in kernel_name:
            return lab
    return None


def sources_hash() -> str:
    """sha256 over the library's kernel and host sources (sorted by name)."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(CSRC, "*"))):
        if path.endswith((".hip", ".cpp", ".h")):
            h.update(os.path.basename(path).encode())
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("void ", "").replace("fem::", "")


def stats(args) -> None:
    rows = list(csv.DictReader(open(args.csv)))
    lines = [f"# Kernel times: {args.workload}", "",
             f"Command (from the repository root, with `cd /tmp && export TMPDIR=/tmp` first):", "",
             f"    {args.command}", "",
             "| kernel | trace label | calls | avg us | min us | max us | share % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        lab = label_of(r["Name"]) or ""
        lines.append(f"| `{_short(r['Name'])}` | {lab} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def counters(args) -> None:
    """Per-kernel averages of any --pmc counters (one or more runs)."""
    table = collections.defaultdict(dict)
    for d in args.runs:
        paths = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        vals = collections.defaultdict(list)
        for p in paths:
            for r in csv.DictReader(open(p)):
                vals[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
        for (k, c), v in vals.items():
            if args.match and not any(m in k for m in args.match):
                continue
            table[_short(k)][c] = sum(v) / len(v)
    names = sorted({c for row in table.values() for c in row})
    lines = [f"# Counters per dispatch: {args.workload}", "",
             "Commands (from the repository root, with `cd /tmp && export TMPDIR=/tmp` first):", "",
             f"    {args.command}", "",
             "| kernel | " + " | ".join(names) + " |", "|---|" + "---|" * len(names)]
    for k, row in table.items():
        lines.append(f"| `{k}` | " + " | ".join(
            (f"{row[c]:.1f}" if c in row and abs(row[c]) < 1000 else f"{row[c]:.4g}" if c in row else "")
            for c in names) + " |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter_means(run_dir: str):
    paths = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not paths:
        raise SystemExit(f"no counter_collection.csv under {run_dir}")
    vals = collections.defaultdict(list)
    for p in paths:
        for r in csv.DictReader(open(p)):
            vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in vals.items()}, {k: len(v) for k, v in vals.items()}


def traffic(args) -> None:
    fetch, nf = _counter_means(args.fetch)
    write, nw = _counter_means(args.write)
    cf, _ = _counter_means(args.calib_fetch)
    cw, _ = _counter_means(args.calib_write)
    copy = [k for k in cf if "copyBuffer" in k or "copy" in k.lower()]
    if not copy:
        raise SystemExit("no copy kernel in the calibration runs")
    ck = copy[0]
    f_fetch = args.calib_bytes / (cf[ck] * 1024.0)
    f_write = args.calib_bytes / (cw[ck] * 1024.0)
    h = sources_hash()
    out = {"workload": args.workload, "command": args.command, "sources_sha256": h,
           "fetch_scale": f_fetch, "write_scale": f_write, "kernels": {}}
    lines = [f"# HBM traffic per launch: {args.workload}", "",
             "Counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each from its own rocprofv3 `--pmc` run,",
             f"scaled by the ratio of known bytes to counter reading of a plain {args.calib_bytes / 2**30:.0f} GiB copy",
             f"(FETCH x{f_fetch:.3f}, WRITE x{f_write:.3f}).", "",
             "Commands (from the repository root, with `cd /tmp && export TMPDIR=/tmp` first):", "",
             f"    {args.command}", "",
             f"Kernel sources sha256: `{h}`", "",
             "| kernel | trace label | dispatches | read MB | write MB | total MB |", "|---|---|---|---|---|---|"]
    for k in sorted(fetch, key=lambda k: -(fetch[k] + write.get(k, 0.0))):
        lab = label_of(k)
        rd = fetch[k] * 1024.0 * f_fetch
        wr = write.get(k, 0.0) * 1024.0 * f_write
        lines.append(f"| `{_short(k)}` | {lab or ''} | {nf[k]} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | {(rd + wr) / 1e6:.1f} |")
        if lab and lab not in out["kernels"]:
            out["kernels"][lab] = {"kernel": _short(k), "read_bytes": rd, "write_bytes": wr, "bytes": rd + wr}
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(out, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--workload", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("-o", "--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("runs", nargs="+")
    c.add_argument("--workload", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--match", action="append", default=[], help="keep kernels whose name contains this")
    c.add_argument("-o", "--out", required=True)
    t = sub.add_parser("traffic")
    for a in ("--fetch", "--write", "--calib-fetch", "--calib-write", "--workload", "--command"):
        t.add_argument(a, required=True)
    t.add_argument("--calib-bytes", type=float, default=float(1 << 30))
    t.add_argument("-o", "--out", required=True)
    a = ap.parse_args(argv)
    {"stats": stats, "counters": counters, "traffic": traffic}[a.cmd](a)


if __name__ == "__main__":
    main()
