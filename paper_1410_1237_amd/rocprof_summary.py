"""Summaries of rocprofv3 output for the committed profiles.

``stats``: the kernel statistics CSV of ``rocprofv3 --kernel-trace --stats``
as a short text table (with the command that produced it).

``traffic``: HBM bytes per dispatch of one kernel from two counter runs
(``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``, KiB per dispatch), each
scaled by what the same counter reads for a plain copy kernel of known size
in the same run; the result goes into ``profiles/traffic.json`` under
``<record>|<workload>|<heuristics>`` with the digest of the sweep sources, so
the benchmark drops the figure once the kernels change.

    python -m paper_1410_1237_amd.rocprof_summary stats STATS_CSV OUT_TXT --command "..."
    python -m paper_1410_1237_amd.rocprof_summary traffic FETCH_CSV WRITE_CSV --kernel k_sweep_large \\
        --copy copyBuffer --copy-bytes N --key REC|WORKLOAD|HEUR --out profiles/traffic.json --txt OUT_TXT
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def source_digest() -> str:
    h = hashlib.sha256()
    for f in ("sweep.hip", "lv.h"):
        with open(os.path.join(ROOT, "paper_1410_1237_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics", f"# command: {args.command}", "",
             f"{'calls':>7} {'total ms':>10} {'avg us':>10} {'share':>6}  kernel"]
    for r in rows[:args.top]:
        name = r["Name"]
        if len(name) > 110:
            name = name[:107] + "..."
        lines.append(f"{int(r['Calls']):>7} {float(r['TotalDurationNs']) / 1e6:>10.3f} "
                     f"{float(r['AverageNs']) / 1e3:>10.2f} {100 * float(r['TotalDurationNs']) / tot:>5.1f}%  {name}")
    lines.append(f"\n# all kernels: {tot / 1e6:.3f} ms")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _per_dispatch(path, counter):
    """{dispatch id: (kernel name, counter value)} of a counter CSV."""
    out = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        d = int(r.get("Dispatch_Id") or r.get("Correlation_Id"))
        name, val = r["Kernel_Name"], float(r["Counter_Value"])
        prev = out.get(d)
        out[d] = (name, val + (prev[1] if prev else 0.0))
    return out


def traffic(args):
    res = {}
    for counter, path in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        d = _per_dispatch(path, counter)
        kern = [v for n, v in d.values() if args.kernel in n]
        copy = [d[i][1] for i in sorted(d) if args.copy in d[i][0]]
        if not kern or len(copy) < 3:
            raise SystemExit(f"{counter}: no dispatch of {args.kernel!r} or of the probe {args.copy!r}")
        copy_kib = sorted(copy[-3:])[1]  # the probe: the last three copies of the run (median)
        factor = copy_kib * 1024.0 / args.copy_bytes  # counter bytes per real byte moved one way
        res[counter] = {"kib_per_dispatch": sum(kern) / len(kern), "dispatches": len(kern),
                        "copy_kib": copy_kib, "factor": factor}
    fetch = res["FETCH_SIZE"]["kib_per_dispatch"] * 1024.0 / res["FETCH_SIZE"]["factor"]
    write = res["WRITE_SIZE"]["kib_per_dispatch"] * 1024.0 / res["WRITE_SIZE"]["factor"]
    data = {}
    if os.path.exists(args.out):
        data = json.load(open(args.out))
    data[args.key] = {"bytes_per_launch": round(fetch + write), "fetch_bytes": round(fetch),
                      "write_bytes": round(write), "counters": res, "source_digest": source_digest(),
                      "command_fetch": args.command_fetch, "command_write": args.command_write}
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1)
    lines = [f"# HBM traffic of {args.kernel} ({args.key})",
             f"# FETCH_SIZE run: {args.command_fetch}", f"# WRITE_SIZE run: {args.command_write}",
             f"# copy probe: {args.copy_bytes} bytes; counter factor fetch {res['FETCH_SIZE']['factor']:.4f}, "
             f"write {res['WRITE_SIZE']['factor']:.4f}", "",
             f"dispatches: {res['FETCH_SIZE']['dispatches']}",
             f"FETCH_SIZE per dispatch: {res['FETCH_SIZE']['kib_per_dispatch']:.1f} KiB -> {fetch / 1e9:.3f} GB",
             f"WRITE_SIZE per dispatch: {res['WRITE_SIZE']['kib_per_dispatch']:.1f} KiB -> {write / 1e9:.3f} GB",
             f"traffic per launch: {(fetch + write) / 1e9:.3f} GB"]
    with open(args.txt, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("out")
    a.add_argument("--command", required=True)
    a.add_argument("--top", type=int, default=20)
    b = sub.add_parser("traffic")
    b.add_argument("fetch")
    b.add_argument("write")
    b.add_argument("--kernel", required=True)
    b.add_argument("--copy", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--key", required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--txt", required=True)
    b.add_argument("--command-fetch", required=True)
    b.add_argument("--command-write", required=True)
    args = ap.parse_args(argv)
    stats(args) if args.cmd == "stats" else traffic(args)


if __name__ == "__main__":
    sys.exit(main())
