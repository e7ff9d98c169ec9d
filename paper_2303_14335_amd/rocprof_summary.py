"""Short text summaries of rocprofv3 CSV output, and the per-launch HBM
traffic record that bench.py reads for its roofline.

usage:
  python -m paper_2303_14335_amd.rocprof_summary stats <kernel_stats.csv> <command>
  python -m paper_2303_14335_amd.rocprof_summary pmc <out_dir> <command>
  python -m paper_2303_14335_amd.rocprof_summary traffic <fetch_dir> <write_dir> \\
         <kernel substring> <workload name> <copy MiB> <command>

`traffic` takes two --pmc runs of the same program (FETCH_SIZE, then
WRITE_SIZE; KiB per dispatch) and scales each counter by what it reads for
a plain device-to-device copy of known size that the program also makes
(bench.py --copy-probe-mib), so that the result is in bytes.
"""
from __future__ import annotations

import collections
import csv
import json
import os
import sys


def stats(path: str, cmd: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"# rocprofv3 --kernel-trace --stats summary\n# command: {cmd}\n",
           f"{'kernel':70s} {'calls':>7s} {'avg_ns':>12s} {'min_ns':>10s} {'max_ns':>10s} {'pct':>6s}"]
    for r in rows:
        out.append(f"{r['Name'][:70]:70s} {int(r['Calls']):7d} {float(r['AverageNs']):12.1f} "
                   f"{int(float(r['MinNs'])):10d} {int(float(r['MaxNs'])):10d} {float(r['Percentage']):6.2f}")
    return "\n".join(out)


def _counters(d: str):
    rows = list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))
    agg = collections.defaultdict(list)
    for r in rows:
        agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return agg


def pmc(d: str, cmd: str) -> str:
    agg = _counters(d)
    out = [f"# rocprofv3 --pmc summary (per dispatch)\n# command: {cmd}\n",
           f"{'kernel':70s} {'counter':>16s} {'dispatches':>10s} {'mean':>14s} {'min':>14s} {'max':>14s}"]
    for (k, c), v in sorted(agg.items()):
        out.append(f"{k[:70]:70s} {c:>16s} {len(v):10d} {sum(v) / len(v):14.3f} {min(v):14.3f} {max(v):14.3f}")
    return "\n".join(out)


def traffic(fetch_dir: str, write_dir: str, kernel_sub: str, workload: str, copy_mib: int,
            cmd: str) -> dict:
    f = {k: v for (k, c), v in _counters(fetch_dir).items() if c == "FETCH_SIZE"}
    w = {k: v for (k, c), v in _counters(write_dir).items() if c == "WRITE_SIZE"}
    copy_kib = copy_mib * 1024
    copy_f = max(max(v) for k, v in f.items() if "copyBuffer" in k)
    copy_w = max(max(v) for k, v in w.items() if "copyBuffer" in k)
    fetch_scale, write_scale = copy_kib / copy_f, copy_kib / copy_w
    kf = next(k for k in f if kernel_sub in k)
    kw = next(k for k in w if kernel_sub in k)
    fetch = sum(f[kf]) / len(f[kf]) * fetch_scale * 1024
    write = sum(w[kw]) / len(w[kw]) * write_scale * 1024
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    return {"kernel": kf, "workload": workload, "dispatches": len(f[kf]),
            "fetch_kib_raw": round(sum(f[kf]) / len(f[kf]), 3),
            "write_kib_raw": round(sum(w[kw]) / len(w[kw]), 3),
            "copy_probe_kib": copy_kib, "copy_fetch_kib_raw": copy_f, "copy_write_kib_raw": copy_w,
            "fetch_scale": round(fetch_scale, 4), "write_scale": round(write_scale, 4),
            "fetch_bytes_per_launch": round(fetch), "write_bytes_per_launch": round(write),
            "bytes_per_launch": round(fetch + write),
            "kernel_source_hash": bench.kernel_source_hash(), "command": cmd}


def main(argv) -> int:
    if argv[0] == "stats":
        print(stats(argv[1], argv[2]))
    elif argv[0] == "pmc":
        print(pmc(argv[1], argv[2]))
    elif argv[0] == "traffic":
        print(json.dumps(traffic(argv[1], argv[2], argv[3], argv[4], int(argv[5]), argv[6]), indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
