"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1807_02587_amd.profiling stats <dir>/<name>_kernel_stats.csv
    python -m paper_1807_02587_amd.profiling steps <dir>/<name>_kernel_trace.csv [first_kernel]
    python -m paper_1807_02587_amd.profiling counters <dir>/<name>_counter_collection.csv
    python -m paper_1807_02587_amd.profiling traffic <fetch.csv> <write.csv> <copy_bytes> <out.json>
    python -m paper_1807_02587_amd.profiling timeline <dir>/<name>_kernel_trace.csv [first_kernel]
    python -m paper_1807_02587_amd.profiling valu <dir>/<name>_counter_collection.csv <dir>/<name>_kernel_trace.csv <out.json>

``stats`` prints the per-kernel table (calls, total/average/min/max us,
share) of a ``--kernel-trace --stats`` run; ``steps`` splits the kernel trace
into steps at each launch of ``first_kernel`` (default root_mean_kernel, the
first kernel of a construction) and prints, for the last full step, the span,
the summed kernel time, the summed gaps between kernels and the kernel time
by kernel; ``counters`` prints, per kernel, the mean per-dispatch value of
every collected counter of a ``--pmc`` run; ``traffic`` turns a FETCH_SIZE
pass and a WRITE_SIZE pass (KiB per dispatch) into HBM bytes per launch of
each kernel family, scaled by what the same counters read for the largest
plain copy of ``copy_bytes`` bytes in the same runs, and stamps the result
with a hash of the kernel sources (a figure is stale once they change);
``timeline`` lists the kernels of the last full step in start order; ``valu``
turns a pass of VALU_COUNTERS with ``--kernel-trace`` into VALU busy and lane
utilisation and the counted FLOP rate per kernel family.
"""

from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
KERNEL_SOURCES = ("build_kernels.hip", "register_kernels.hip", "soft_kernels.hip", "query_kernels.hip", "hgmm_dev.h")
FAMILIES = {"em_block": "em_block_kernel", "em_tile": "em_tile_kernel", "em_mstep": "em_mstep_kernel",
            "descend": "descend_kernel", "normal": "normal_kernel", "partition": "partition_kernel",
            "flat": "flat_estep_kernel", "soft": "soft_estep_kernel"}


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


def sources_sha1() -> str:
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _per_dispatch(path: str, counter: str) -> dict:
    """kernel name -> list of per-dispatch values of one counter (summed over its instances)."""
    per = collections.defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", r.get("Counter-Name")) != counter:
            continue
        d = r.get("Dispatch_Id", r.get("Dispatch-Id"))
        per[d] += float(r.get("Counter_Value", r.get("Counter-Value", 0)))
        names[d] = r.get("Kernel_Name", r.get("Kernel-Name", "?"))
    out = collections.defaultdict(list)
    for d, v in per.items():
        out[names[d]].append(v)
    return out


def traffic(fetch_csv: str, write_csv: str, copy_bytes: float) -> dict:
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")
    # the calibration copy: the largest single dispatch of a kernel that is not the library's
    cf = max(v for k, vs in fetch.items() if "hgmm::" not in k for v in vs)
    cw = max(v for k, vs in write.items() if "hgmm::" not in k for v in vs)
    sf, sw = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    fam = {}
    for key, prefix in FAMILIES.items():
        fv = [v for k, vs in fetch.items() if _short(k).startswith(prefix) or
              _short(k).startswith("void " + prefix) for v in vs]
        wv = [v for k, vs in write.items() if _short(k).startswith(prefix) or
              _short(k).startswith("void " + prefix) for v in vs]
        if not fv or not wv:
            continue
        f_b = sum(fv) / len(fv) * 1024.0 * sf
        w_b = sum(wv) / len(wv) * 1024.0 * sw
        fam[key] = {"dispatches": len(fv), "fetch_bytes_per_launch": round(f_b), "write_bytes_per_launch": round(w_b),
                    "bytes_per_launch": round(f_b + w_b)}
    return {"copy": {"bytes": copy_bytes, "fetch_kib": cf, "write_kib": cw, "scale_fetch": round(sf, 4),
                     "scale_write": round(sw, 4)},
            "families": fam, "kernel_sources_sha1": sources_sha1()}


VALU_COUNTERS = ("VALUBusy", "VALUUtilization", "SQ_INSTS_VALU_FLOPS_FP32", "SQ_INSTS_VALU_FLOPS_FP32_TRANS",
                 "SQ_INSTS_VALU_FLOPS_FP64")


def valu(counter_csv: str, trace_csv: str, peak_tflops: float = 78.6) -> dict:
    """Per kernel family, from a ``--pmc`` run of VALU_COUNTERS with
    ``--kernel-trace``: mean VALUBusy (percent of the kernel's GPU time with a
    VALU instruction in flight, per CU), mean VALUUtilization (active lanes per
    VALU instruction, percent of 64), the FP32 (with transcendentals) and FP64
    FLOPs the hardware counted per dispatch, the mean kernel duration from the
    trace, and the counted FLOP rate as a fraction of ``peak_tflops``.

    The SQ_INSTS_VALU_FLOPS_* counters count per wave instruction (an FMA as 2),
    not per lane, so they are scaled by the wave size, 64.  Check on the LiDAR
    construction: em_tile_kernel's transcendental count times 64 is exactly its
    8 exp2 and 1 reciprocal per point-iteration."""
    dur = {}
    for r in csv.DictReader(open(trace_csv)):
        dur[r.get("Dispatch_Id", r.get("Dispatch-Id"))] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for r in csv.DictReader(open(counter_csv)):
        c = r.get("Counter_Name", r.get("Counter-Name"))
        if c not in VALU_COUNTERS:
            continue
        d = r.get("Dispatch_Id", r.get("Dispatch-Id"))
        per[d][c] += float(r.get("Counter_Value", r.get("Counter-Value", 0)))
        names[d] = _short(r.get("Kernel_Name", r.get("Kernel-Name", "?")))
    fam = {}
    for key, prefix in FAMILIES.items():
        ds = [d for d, n in names.items() if n.replace("void ", "").startswith(prefix) and d in dur]
        if not ds:
            continue
        mean = lambda c: sum(per[d][c] for d in ds) / len(ds)
        f32 = 64.0 * (mean("SQ_INSTS_VALU_FLOPS_FP32") + mean("SQ_INSTS_VALU_FLOPS_FP32_TRANS"))
        f64 = 64.0 * mean("SQ_INSTS_VALU_FLOPS_FP64")
        t = sum(dur[d] for d in ds) / len(ds)
        rate = (f32 + f64) / t / 1e12 if t > 0 else 0.0
        fam[key] = {"dispatches": len(ds), "valu_busy_pct": round(mean("VALUBusy"), 2),
                    "valu_utilization_pct": round(mean("VALUUtilization"), 2), "fp32_flop_per_launch": round(f32),
                    "fp64_flop_per_launch": round(f64), "mean_us": round(t * 1e6, 2),
                    "counted_tflops": round(rate, 3), "counted_frac": round(rate / peak_tflops, 4)}
    return {"families": fam, "peak_tflops": peak_tflops, "kernel_sources_sha1": sources_sha1()}


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


def timeline(path: str, first: str = "root_mean_kernel") -> str:
    """Kernels of the last complete step of a kernel trace in start order, runs
    of one kernel on one queue merged: start, end, span (us from the step's
    first kernel), queue, count, busy time."""
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    name = lambda r: _short(r["Kernel_Name"])
    marks = [i for i, r in enumerate(rows) if name(r) == first]
    if len(marks) < 2:
        return "fewer than two steps in the trace"
    seg = rows[marks[-2]:marks[-1]]
    t0 = int(seg[0]["Start_Timestamp"])
    runs = []
    for r in seg:
        n, q = name(r).replace("void ", "")[:34], r.get("Queue_Id", "?")
        s, e = (int(r["Start_Timestamp"]) - t0) / 1e3, (int(r["End_Timestamp"]) - t0) / 1e3
        if runs and runs[-1][0] == n and runs[-1][4] == q:
            runs[-1][2] = e
            runs[-1][3] += 1
            runs[-1][5] += e - s
        else:
            runs.append([n, s, e, 1, q, e - s])
    return "\n".join(f"{s:9.1f} {e:9.1f} {e - s:8.1f}  q{q:>3} x{c:<3} busy {busy:8.1f}  {n}"
                     for n, s, e, c, q, busy in runs)


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    if mode == "stats":
        print(stats(path))
    elif mode == "steps":
        print(steps(path, *sys.argv[3:4]))
    elif mode == "timeline":
        print(timeline(path, *sys.argv[3:4]))
    elif mode == "valu":
        res = valu(path, sys.argv[3])
        with open(sys.argv[4], "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res, indent=1))
    elif mode == "traffic":
        res = traffic(path, sys.argv[3], float(sys.argv[4]))
        with open(sys.argv[5], "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res, indent=1))
    else:
        print(counters(path))
