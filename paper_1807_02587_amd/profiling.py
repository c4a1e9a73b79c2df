"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1807_02587_amd.profiling stats <dir>/<name>_kernel_stats.csv
    python -m paper_1807_02587_amd.profiling steps <dir>/<name>_kernel_trace.csv [first_kernel]
    python -m paper_1807_02587_amd.profiling counters <dir>/<name>_counter_collection.csv

``stats`` prints the per-kernel table (calls, total/average/min/max us,
share) of a ``--kernel-trace --stats`` run; ``steps`` splits the kernel trace
into steps at each launch of ``first_kernel`` (default root_mean_kernel, the
first kernel of a construction) and prints, for the last full step, the span,
the summed kernel time, the summed gaps between kernels and the kernel time
by kernel; ``counters`` prints, per kernel, the mean per-dispatch value of
every collected counter of a ``--pmc`` run.
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


def steps(path: str, first: str = "root_mean_kernel") -> str:
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    name = lambda r: _short(r["Kernel_Name"])
    marks = [i for i, r in enumerate(rows) if name(r) == first]
    if len(marks) < 2:
        return "fewer than two steps in the trace"
    seg = rows[marks[-2]:marks[-1]]
    t0, t1 = int(seg[0]["Start_Timestamp"]), int(seg[-1]["End_Timestamp"])
    dur = lambda r: int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    gaps = sorted(int(seg[i + 1]["Start_Timestamp"]) - int(seg[i]["End_Timestamp"]) for i in range(len(seg) - 1))
    per = collections.defaultdict(lambda: [0, 0.0])
    for r in seg:
        per[name(r)][0] += 1
        per[name(r)][1] += dur(r) / 1e3
    out = [f"one step ({len(marks)} steps in the trace): {len(seg)} kernels, span {(t1 - t0) / 1e3:.1f} us, "
           f"kernel time {sum(dur(r) for r in seg) / 1e3:.1f} us, gaps {sum(gaps) / 1e3:.1f} us "
           f"(median gap {gaps[len(gaps) // 2] / 1e3:.2f} us; overlapping kernels make gaps negative)",
           f"{'kernel':40s} {'calls':>6s} {'us':>9s}"]
    for k, (c, us) in sorted(per.items(), key=lambda x: -x[1][1]):
        out.append(f"{k[:40]:40s} {c:6d} {us:9.1f}")
    return "\n".join(out)


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    if mode == "stats":
        print(stats(path))
    elif mode == "steps":
        print(steps(path, *sys.argv[3:4]))
    else:
        print(counters(path))
