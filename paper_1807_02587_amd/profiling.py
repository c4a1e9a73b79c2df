"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1807_02587_amd.profiling stats <dir>/<name>_kernel_stats.csv
    python -m paper_1807_02587_amd.profiling counters <dir>/<name>_counter_collection.csv

``stats`` prints the per-kernel table (calls, total/average/min/max us,
share) of a ``--kernel-trace --stats`` run; ``counters`` prints, per kernel,
the mean per-dispatch value of every collected counter of a ``--pmc`` run.
"""

from __future__ import annotations

import collections
import csv
import sys


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("hgmm::", "")


def stats(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"{'kernel':40s} {'calls':>6s} {'total_us':>11s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'share%':>7s}"]
    for r in rows:
        out.append(f"{_short(r['Name'])[:40]:40s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e3:11.1f} "
                   f"{float(r['AverageNs']) / 1e3:9.2f} {float(r['MinNs']) / 1e3:9.2f} {float(r['MaxNs']) / 1e3:9.2f} "
                   f"{float(r['Percentage']):7.2f}")
    return "\n".join(out)


def counters(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        k = _short(r.get("Kernel_Name", r.get("Kernel-Name", "?")))
        cname = r.get("Counter_Name", r.get("Counter-Name"))
        val = float(r.get("Counter_Value", r.get("Counter-Value", 0)))
        disp = r.get("Dispatch_Id", r.get("Dispatch-Id"))
        acc[k][cname].append((disp, val))
    out = []
    for k, cs in acc.items():
        for cname, vals in cs.items():
            per = collections.defaultdict(float)
            for d, v in vals:
                per[d] += v
            vs = list(per.values())
            out.append(f"{k[:40]:40s} {cname:14s} dispatches {len(vs):5d} mean {sum(vs) / len(vs):14.1f}")
    return "\n".join(out)


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    print(stats(path) if mode == "stats" else counters(path))
