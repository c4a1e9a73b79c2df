"""Throughput of GMM-Tree registration on one MI355X.

One step = the whole hot path for one cloud pair: build the GMM tree of the
source cloud (root statistics, per-level EM, partition) and register the
target cloud against it (adaptive descent, moments, normal equations, solve),
inputs already resident in HBM.  The default workload is the spinning-scanner
pair (64 rings x 1875 azimuths, 4 levels).

Prints one JSON line: pairs/s, ms/step, the dominant kernel's achieved rate
against the MI355X roofline (from HIP events bracketing its launches inside
the timed region), the E-step rate in Mpts/s, the registration error of the
timed runs, and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X peaks.  HBM: published 8 TB/s.  FP32 vector: the published 157.3
# TFLOP/s counts packed (2-wide) FMA; the kernels are built without packed FP32
# instructions, so their ceiling is 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA)
# x 2.4 GHz = 78.6 TFLOP/s, the figure the ALU roofline is quoted against.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_FP32_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# Algorithmic work per unit (every arithmetic step of the method counted once, FMA = 2 FLOP):
#  construction EM, per point-iteration: 8 children x (score 19 + softmax 4 + moments 21) FLOP
EM_FLOP_PER_POINT_ITER = 8 * 44
EM_BYTES_PER_POINT_ITER = 12
#  registration descent, per point: transform 18 + per visited level 8 x 19 + stop level 35 FLOP
DESC_FLOP_FIXED = 18 + 35
DESC_FLOP_PER_LEVEL = 8 * 19
DESC_BYTES_PER_POINT = 12


def progress(msg):
    """One line on stderr per finished section (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def roofline_of(prof, depth, traffic=None):
    """ALU roofline of the kernel family with the largest summed event time.
    prof: hgmm_profile_read per kind; depth: mean levels visited per point by
    the descent (for its FLOP count); traffic: which committed counter summary
    ("lidar" or "batch") gives the HBM bytes per launch, or None."""
    cand = {"em_tile": ("em_tile_kernel (construction EM iteration of large parents)", EM_FLOP_PER_POINT_ITER,
                        EM_BYTES_PER_POINT_ITER),
            "em_block": ("em_block_kernel (all construction EM iterations, one block per parent)",
                         EM_FLOP_PER_POINT_ITER, EM_BYTES_PER_POINT_ITER),
            "descend": ("descend_kernel (registration E-step)", DESC_FLOP_FIXED + DESC_FLOP_PER_LEVEL * depth,
                        DESC_BYTES_PER_POINT)}
    fam_frac = {}
    for k, (_, fu, _) in cand.items():
        if prof[k]["ms"] > 0:
            fam_frac[k] = round(prof[k]["units"] * fu / (prof[k]["ms"] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)
    dom = max(cand, key=lambda k: prof[k]["ms"])
    kname, flop_unit, bytes_unit = cand[dom]
    ms, launches, units = prof[dom]["ms"], prof[dom]["launches"], prof[dom]["units"]
    flop, byts = units * flop_unit, units * bytes_unit
    achieved = flop / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_FP32_TFLOPS, 1), "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": _traffic(dom, traffic) if traffic else None,
            "kernel": kname, "launches": launches, "avg_launch_us": round(ms * 1e3 / max(launches, 1), 2),
            "flop_per_launch": round(flop / max(launches, 1)),
            "frac_of_packed_peak": round(achieved / PEAK_FP32_PACKED_TFLOPS, 4),
            "achieved_hbm_GBs": round(byts / (ms * 1e-3) / 1e9, 1) if ms > 0 else 0.0,
            "frac_by_family": fam_frac, **(_valu(dom, traffic) if traffic else {})}


def mean_depth(stop, level_offsets):
    """Mean number of levels a point visited, from its stop node (index in its tree)."""
    st = stop[stop >= 0]
    return float(np.mean(np.searchsorted(level_offsets, st, side="right"))) if st.size else 0.0


TRAFFIC = {"lidar": os.path.join(ROOT, "profiles", "lidar_hbm_traffic.json"),
           "batch": os.path.join(ROOT, "profiles", "batch_hbm_traffic.json")}


def _traffic(family, which):
    """HBM bytes per launch of a kernel family from the committed FETCH_SIZE /
    WRITE_SIZE summary, or None when there is none or the kernels changed since."""
    from paper_1807_02587_amd import profiling
    try:
        with open(TRAFFIC[which]) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha1") != profiling.sources_sha1() or family not in t.get("families", {}):
        return None
    return t["families"][family]["bytes_per_launch"]


VALU = {"lidar": os.path.join(ROOT, "profiles", "lidar_valu.json"),
        "batch": os.path.join(ROOT, "profiles", "batch_valu.json")}


def _valu(family, which):
    """VALU busy and lane utilisation (percent) and the counted FLOP rate over
    the kernel-trace time of a kernel family, from the committed counter pass,
    or {} when there is none or the kernels changed since."""
    from paper_1807_02587_amd import profiling
    try:
        with open(VALU[which]) as f:
            v = json.load(f)
    except (OSError, ValueError):
        return {}
    if v.get("kernel_sources_sha1") != profiling.sources_sha1() or family not in v.get("families", {}):
        return {}
    f = v["families"][family]
    return {"valu_busy_pct": f["valu_busy_pct"], "valu_utilization_pct": f["valu_utilization_pct"],
            "counted_flop_frac": f["counted_frac"]}


def _workload(name):
    from paper_1807_02587_amd.presets import PRESETS
    from synth import depth_pair, lidar_pair, small_pair
    if name == "lidar":
        p = lidar_pair(1000)
        desc = "lidar 64 rings x 1875 azimuths, ground + 50 boxes + 30 cylinders, 1 m / <=2 deg motion"
    elif name == "small":
        p = small_pair(0)
        desc = "planes+spheres unit cube, 10k points, <=30 deg / 0.1 motion"
    elif name == "depth":
        p = depth_pair(2000)
        desc = "depth camera 640x480 in a furnished room, <=10 deg / 0.2 m motion"
    else:
        raise SystemExit(f"unknown workload {name}")
    return p, PRESETS[name], desc


WEIGHTS = os.path.join(ROOT, "paper_1807_02587_amd", "weights", "warm_mlp.npy")


def batch_section(args, hg):
    """The uneven batch (256 unit-cube pairs, N log-uniform in [2e3, 2e5],
    rotation U(0, 45 deg), depth ceil(log8(N/50))) registered three ways:
    one pair at a time (plain form), batched from identity, batched with the
    learned warm start and its likelihood fallback."""
    import torch
    from paper_1807_02587_amd import warmstart as W
    from synth.torch_scenes import uneven_batch

    src, tgt, off, lv, Rt, tt = uneven_batch(3000, args.batch_pairs)
    B = len(lv)
    ws = hg.Workspace()
    cfg = W.WarmConfig()
    if args.copy_calibration:
        # counter calibration: a plain copy of known size, then the batched
        # plain form twice with the given launch shapes
        a = torch.empty(args.copy_mib << 18, dtype=torch.float32, device=src.device).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        if args.batch_tuning_json:
            with open(args.batch_tuning_json) as f:
                hg.hgmm_set_tuning(**json.load(f))
        for _ in range(2):
            forest = hg.hgmm_build_batch(src, off, lv, ws=ws)
            hg.hgmm_register_batch(forest, tgt, off, ws=ws)
        torch.cuda.synchronize()
        return {"copy_bytes": a.numel() * 4, "steps": 2}

    def plain_sequential(k_list):
        Rs = []
        tree = None
        for k in k_list:
            s_k = src[:, off[k]:off[k + 1]].contiguous()
            t_k = tgt[:, off[k]:off[k + 1]].contiguous()
            tree = hg.hgmm_build(s_k, levels=int(lv[k]), ws=ws, tree=tree)
            Rs.append(hg.hgmm_register(tree, t_k, ws=ws, raise_singular=False)["R"])
        return np.array(Rs)

    last = {}

    def batched_plain():
        # the handle is reused, as a caller registering batch after batch would
        forest = hg.hgmm_build_batch(src, off, lv, ws=ws, forest=last.get("forest"))
        r = hg.hgmm_register_batch(forest, tgt, off, ws=ws)
        last.update(forest=forest, r=r)
        return r["R"]

    net = None
    if os.path.exists(WEIGHTS):
        net = hg.MLP(seed=0)
        net.set_params(np.load(WEIGHTS))

    def batched_warm():
        return W.register_warm(net, src, tgt, off, off, lv, cfg, ws=ws)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    def summary(name, R, sec):
        e = W.rotation_errors_deg(R, Rt)
        ok = int(np.sum(e <= 0.5))
        return {f"{name}_pairs_s": round(B / sec, 2), f"{name}_median_rot_err_deg": round(float(np.median(e)), 4),
                f"{name}_ok_0p5": ok, f"{name}_ok_pairs_s": round(ok / sec, 2)}

    # plain form: one pair at a time, default launch shapes
    defaults = hg.hgmm_get_tuning()
    out = {"workload": f"{B} unit-cube pairs, N log-uniform [2e3, 2e5] (total {int(off[-1])} points per side), "
                       "rotation U(0,45 deg), levels ceil(log8(N/50))"}
    tp = None
    if not args.batch_only:
        plain_sequential(range(min(8, B)))
        Rp, tp = timed(lambda: plain_sequential(range(B)))
        out.update(summary("plain_sequential", Rp, tp))
    # batched forms: launch shapes from the autotuner on this batch (outside the timed runs)
    if args.batch_tuning_json:
        with open(args.batch_tuning_json) as f:
            hg.hgmm_set_tuning(**json.load(f))
        out["autotune"] = {"tuning": hg.hgmm_get_tuning(), "from": args.batch_tuning_json}
    else:
        from paper_1807_02587_amd import autotune
        t_tune = time.perf_counter()
        tun = autotune.tuned(src, off, lv, tgt, off, use_cache=False, reps=1, passes=1, ws=ws)
        out["autotune"] = {"tuning": tun["tuning"], "search_s": round(time.perf_counter() - t_tune, 2),
                           "start_ms": round(tun["start_ms"], 2), "best_ms": round(tun["best_ms"], 2)}
    if args.save_batch_tuning:
        with open(args.save_batch_tuning, "w") as f:
            json.dump(hg.hgmm_get_tuning(), f)
    batched_plain()
    Rb, tb = timed(batched_plain)
    out.update(summary("batched", Rb, tb))
    if tp:
        out["speedup_batched_vs_plain"] = round(tp / tb, 2)
    # the batched plain form once more with HIP events around every launch:
    # per-kernel durations and the roofline of its dominant kernel
    hg.hgmm_profile_reset()
    hg.hgmm_profile(True)
    batched_plain()
    torch.cuda.synchronize()
    hg.hgmm_profile(False)
    prof = {k: hg.hgmm_profile_read(k) for k in hg.PROFILE_KINDS}
    _, stop = hg.hgmm_estep_batch(last["forest"], tgt, off, last["r"]["R"], last["r"]["t"], ws=ws, stop_nodes=True)
    offs_l = np.array([hg.hgmm_level_offset(l) for l in range(8)])
    depth = mean_depth(stop.cpu().numpy(), offs_l)
    ds = prof["descend"]
    out["profiled"] = {"kernels_ms": {k: round(v["ms"], 3) for k, v in prof.items()},
                       "mean_levels_visited": round(depth, 3),
                       "estep_mpts_s": round(ds["units"] / (ds["ms"] * 1e-3) / 1e6, 1) if ds["ms"] > 0 else None,
                       "roofline": roofline_of(prof, depth, traffic="batch")}
    if net is not None:
        batched_warm()
        rw, tw = timed(batched_warm)
        out.update(summary("batched_warm", rw["R"], tw))
        out["warm_fallback_rate"] = round(float(np.mean(rw["fallback"])), 4)
        if tp:
            out["speedup_batched_warm_vs_plain"] = round(tp / tw, 2)
        if tp and out["plain_sequential_ok_0p5"] > 0:
            out["speedup_ok_pairs_s_batched_warm_vs_plain"] = round(
                out["batched_warm_ok_pairs_s"] / out["plain_sequential_ok_pairs_s"], 2)
    hg.hgmm_set_tuning(**defaults)
    return out


def depth_section(args, hg):
    """The depth-camera pair (640x480 camera in a furnished room, about 2.9e5
    points per view, 5 levels, the precision form's workload): build of the
    source tree plus registration from the identity per step, with launch
    shapes from the autotuner on this pair (chosen before the timed steps)."""
    import torch
    from synth import rotation_angle_deg
    p, pr, desc = _workload("depth")
    dev = torch.device("cuda", 0)
    src = torch.from_numpy(p.src).to(dev)
    tgt = torch.from_numpy(p.tgt).to(dev)
    n1, n2 = p.src.shape[1], p.tgt.shape[1]
    ws_b, ws_r = hg.Workspace(dev), hg.Workspace(dev)
    keep = hg.hgmm_get_tuning()
    tree = None

    def step():
        nonlocal tree
        tree = hg.hgmm_build(src, levels=pr["levels"], reg_eps=pr["reg_eps"], min_mass=pr["min_mass"], ws=ws_b,
                             tree=tree)
        return hg.hgmm_register(tree, tgt, lambda_c=pr["lambda_c"], ws=ws_r, raise_singular=False)

    try:
        tun = hg.hgmm_autotune(src, [0, n1], [pr["levels"]], tgt, [0, n2], reg_eps=pr["reg_eps"],
                               min_mass=pr["min_mass"], lambda_c=pr["lambda_c"], reps=1, passes=1)
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        steps = max(3, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(steps):
            r = step()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        shapes = hg.hgmm_get_tuning()
    finally:
        hg.hgmm_set_tuning(**keep)
    return {"workload": f"depth: {desc}", "points_src": n1, "points_tgt": n2, "levels": pr["levels"],
            "reg_eps": pr["reg_eps"], "min_mass": pr["min_mass"], "steps": steps,
            "pairs_s": round(steps / sec, 2), "ms_per_step": round(sec / steps * 1e3, 3),
            "rot_err_deg": round(rotation_angle_deg(r["R"], p.R_true), 4), "iters": int(r["iters"]),
            "autotune_ms": {"start": round(tun["start_ms"], 3), "best": round(tun["best_ms"], 3)},
            "launch_shapes": shapes}


# single-level E-step, per point-component pair: FP64 offset 3, whitening of
# the offset 9, squared norm 5, score 1, rounding bound 5, running maximum /
# denominator / bound update (with one exp2) 9 FLOP
FLAT_FLOP_PER_EVAL = 32


def variants_section(args, hg, tree, tgt, p, pr, steps):
    """The paper's registration variants on one tree of the main workload,
    registration alone from the identity (the tree built once, outside the
    timed region): adaptive descent (lambda_c as configured), the full tree
    descent (lambda_c = 0, "GMM-Tree"), the soft multi-path descent (every
    branch with path expectation >= 0.01, adaptive stop), and the single-level
    mixture of every node of one level ("GMM J=n", n = 8^(level+1)) with its
    linear scan."""
    import torch
    from synth import rotation_angle_deg
    dev = tgt.device
    ws = hg.Workspace(dev)
    n = tgt.shape[1]
    runs = [("adaptive", "tree", pr["lambda_c"])]
    runs.append(("gmm_tree", "tree", 0.0))
    runs.append(("adaptive_soft_tau0.01", "soft", 0.01))
    for lev in range(1, pr["levels"]):
        runs.append((f"gmm_j{8 ** (lev + 1)}", "flat", lev))
    out = {}
    for name, kind, arg in runs:
        if kind == "tree":
            def reg():
                return hg.hgmm_register(tree, tgt, lambda_c=arg, ws=ws, raise_singular=False)
        elif kind == "soft":
            def reg():
                return hg.hgmm_register_soft(tree, tgt, arg, lambda_c=pr["lambda_c"], ws=ws, raise_singular=False)
        else:
            def reg():
                return hg.hgmm_register_flat(tree, tgt, arg, ws=ws, raise_singular=False)
        reg()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = reg()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        hg.hgmm_profile_reset()
        hg.hgmm_profile(True)
        reg()
        torch.cuda.synchronize()
        hg.hgmm_profile(False)
        k = hg.hgmm_profile_read(kind if kind in ("flat", "soft") else "descend")
        row = {"components": (8 ** (arg + 1)) if kind == "flat" else "adaptive" if arg > 0 else "leaves",
               "ms_per_registration": round(sec * 1e3, 3), "iters": int(r["iters"]),
               "rot_err_deg": round(rotation_angle_deg(r["R"], p.R_true), 4),
               "estep_ms_per_iter": round(k["ms"] / max(1, k["launches"]), 4)}
        if kind == "flat" and k["ms"] > 0:
            evals = n * (8 ** (arg + 1)) * k["launches"]
            tf = evals * FLAT_FLOP_PER_EVAL / (k["ms"] * 1e-3) / 1e12
            row.update({"gevals_s": round(evals / (k["ms"] * 1e-3) / 1e9, 1), "estep_tflops": round(tf, 2),
                        "frac_fp32": round(tf / PEAK_FP32_TFLOPS, 4)})
        out[name] = row
    # the per-point density query against the same tree (another consumer of
    # the model): one descent plus one density per point
    hg.hgmm_point_loglik(tree, tgt, lambda_c=pr["lambda_c"], ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ll, _ = hg.hgmm_point_loglik(tree, tgt, lambda_c=pr["lambda_c"], ws=ws)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    query = {"ms_per_query": round(sec * 1e3, 4), "mpts_s": round(n / sec / 1e6, 1),
             "mean_loglik": round(float(ll.mean().item()), 4)}
    return {"workload": "registration alone on the main workload's tree, from the identity", "steps": steps,
            "variants": out, "point_query": query}


def odometry_section(args, hg, frames=16):
    """Frame-to-frame odometry over a sequence of LiDAR sweeps of the main
    workload's street (1 m steps, yaw U(-2, 2 deg) per frame, building fronts
    along the road): the trees of frames 0..F-2 and the registrations of frames
    1..F-1 onto them in one call (batched), against the same work one frame pair
    at a time (build + register per pair); drift of the chained poses against
    the ground truth."""
    import torch
    from synth import lidar_sequence, rotation_angle_deg
    _, pr, _ = _workload("lidar")
    q = lidar_sequence(1000, frames=frames)
    F = frames
    dev = torch.device("cuda", 0)
    xyz = torch.from_numpy(q.clouds).to(dev)
    kw = dict(reg_eps=pr["reg_eps"], min_mass=pr["min_mass"])
    ws = hg.Workspace(dev)
    forest = None

    def batched(prior=False):
        nonlocal forest
        r = hg.hgmm_odometry(xyz, q.offsets, pr["levels"], lambda_c=pr["lambda_c"], prior_restart=prior, ws=ws,
                             forest=forest, **kw)
        forest = r["forest"]
        return r

    frames_t = [xyz[:, int(q.offsets[k]):int(q.offsets[k + 1])].contiguous() for k in range(F)]
    ws_b, ws_r = hg.Workspace(dev), hg.Workspace(dev)
    tree = None

    def sequential():
        nonlocal tree
        out = []
        for k in range(F - 1):
            tree = hg.hgmm_build(frames_t[k], levels=pr["levels"], ws=ws_b, tree=tree, **kw)
            out.append(hg.hgmm_register(tree, frames_t[k + 1], lambda_c=pr["lambda_c"], ws=ws_r,
                                        raise_singular=False))
        return out

    reps = 3
    path = float(np.sum(np.linalg.norm(np.diff(q.t_abs, axis=0), axis=1)))
    out = {"workload": f"{F} LiDAR sweeps of the main workload's street, 1 m apart, "
                       f"{int(np.mean(np.diff(q.offsets)))} points each, {pr['levels']} levels", "path_m": round(path, 2)}
    for name, fn in (("batched", batched), ("batched_prior_restart", lambda: batched(True)),
                     ("one_pair_at_a_time", sequential)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        row = {"ms_per_sequence": round(sec * 1e3, 2), "frame_pairs_s": round((F - 1) / sec, 1)}
        if name != "one_pair_at_a_time":
            err_rel = [rotation_angle_deg(r["R_rel"][k], q.R_abs[k].T @ q.R_abs[k + 1]) for k in range(F - 1)]
            drift_t = float(np.linalg.norm(r["t_abs"][-1] - q.t_abs[-1]))
            row.update({"pair_rot_err_deg_median": round(float(np.median(err_rel)), 4),
                        "pair_rot_err_deg_max": round(float(np.max(err_rel)), 4),
                        "pairs_above_1deg": int(np.sum(np.array(err_rel) > 1.0)),
                        "iters_mean": round(float(np.mean(r["iters"])), 2),
                        "final_drift_deg": round(rotation_angle_deg(r["R_abs"][-1], q.R_abs[-1]), 4),
                        "final_drift_m": round(drift_t, 4),
                        "final_drift_pct_of_path": round(100 * drift_t / path, 3)})
        out[name] = row
    out["speedup_batched"] = round(out["batched"]["frame_pairs_s"] / out["one_pair_at_a_time"]["frame_pairs_s"], 2)
    return out


def warm_section(args, hg):
    """Held-out warm-start pairs (10k points per cloud, rotation U(0, 90 deg),
    translation U(-0.1, 0.1)^3, L = 2; seeds disjoint from training): the plain
    GPU form one pair at a time (hgmm_build + hgmm_register from the identity)
    against the batched form with the learned warm start and the plain-
    likelihood fallback, which includes the target trees, features and network.
    The plain form is timed on the first `plain_pairs` pairs."""
    import torch
    from paper_1807_02587_amd import warmstart as W
    from synth.torch_scenes import cube_pairs

    if not os.path.exists(WEIGHTS):
        return None
    B, n, plain_pairs = args.warm_pairs, 10_000, min(args.warm_pairs, 256)
    S = cube_pairs(5 * 10**6 + 11, B, n=n, max_angle_deg=90)
    off = S.offsets.numpy()
    Rt = S.R_true.cpu().numpy()
    cfg = W.WarmConfig()
    net = hg.MLP(seed=0)
    net.set_params(np.load(WEIGHTS))
    ws = hg.Workspace()

    def plain(k_list):
        Rs, tree = [], None
        for k in k_list:
            s_k = S.src[:, off[k]:off[k + 1]].contiguous()
            t_k = S.tgt[:, off[k]:off[k + 1]].contiguous()
            tree = hg.hgmm_build(s_k, levels=cfg.src_levels, ws=ws, tree=tree)
            Rs.append(hg.hgmm_register(tree, t_k, ws=ws, raise_singular=False)["R"])
        return np.array(Rs)

    def warm():
        return W.register_warm(net, S.src, S.tgt, off, off, [cfg.src_levels] * B, cfg, ws=ws)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    plain(range(8))
    Rp, tp = timed(lambda: plain(range(plain_pairs)))
    warm()
    rw, tw = timed(warm)
    ep = W.rotation_errors_deg(Rp, Rt[:plain_pairs])
    ew = W.rotation_errors_deg(rw["R"], Rt)
    out = {"workload": f"{B} held-out pairs, {n} points per cloud, rotation U(0,90 deg), L = 2 "
                       f"(plain form timed on {plain_pairs})",
           "plain_pairs_s": round(plain_pairs / tp, 2), "plain_median_rot_err_deg": round(float(np.median(ep)), 4),
           "plain_ok_0p5_rate": round(float(np.mean(ep <= 0.5)), 4),
           "batched_warm_pairs_s": round(B / tw, 2), "batched_warm_median_rot_err_deg": round(float(np.median(ew)), 4),
           "batched_warm_ok_0p5_rate": round(float(np.mean(ew <= 0.5)), 4),
           "warm_fallback_rate": round(float(np.mean(rw["fallback"])), 4),
           "speedup_batched_warm_vs_plain": round((B / tw) / (plain_pairs / tp), 2)}
    out["speedup_ok_pairs_s"] = (round(out["batched_warm_pairs_s"] * out["batched_warm_ok_0p5_rate"]
                                       / (out["plain_pairs_s"] * out["plain_ok_0p5_rate"]), 2)
                                 if out["plain_ok_0p5_rate"] > 0 else None)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lidar", choices=["lidar", "small", "depth"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--batch-pairs", type=int, default=256)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched and warm-start sections")
    ap.add_argument("--warm-pairs", type=int, default=1024)
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched forms of the uneven batch (for profiling them)")
    ap.add_argument("--batch-tuning-json", default=None, help="launch shapes of the batched forms from this file")
    ap.add_argument("--save-batch-tuning", default=None, help="write the batched forms' launch shapes to this file")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--tuning-json", default=None, help="launch shapes from this file instead of the autotuner")
    ap.add_argument("--save-tuning", default=None, help="write the launch shapes used to this file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of --copy-mib MiB and a few steps (for counter calibration)")
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--odometry-only", action="store_true", help="run only the odometry section")
    ap.add_argument("--variants-only", action="store_true",
                    help="build the main workload's tree once and run only the registration variants (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); registration of independent "
              "pairs would shard across GPUs by pair, which is not run here.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1807_02587_amd as hg
    from synth import rotation_angle_deg

    if args.batch_only:
        torch.cuda.set_device(0)
        print(json.dumps({"batched": batch_section(args, hg)}), flush=True)
        return

    p, pr, desc = _workload(args.workload)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    src = torch.from_numpy(p.src).to(dev)
    tgt = torch.from_numpy(p.tgt).to(dev)
    n1, n2 = p.src.shape[1], p.tgt.shape[1]
    ws_b, ws_r = hg.Workspace(dev), hg.Workspace(dev)
    tree = None

    def step():
        nonlocal tree
        tree = hg.hgmm_build(src, levels=pr["levels"], reg_eps=pr["reg_eps"], min_mass=pr["min_mass"], ws=ws_b,
                             tree=tree)
        return hg.hgmm_register(tree, tgt, lambda_c=pr["lambda_c"], ws=ws_r, raise_singular=False)

    if args.odometry_only:
        print(json.dumps({"odometry": odometry_section(args, hg)}), flush=True)
        return

    if args.variants_only:
        if args.tuning_json:
            with open(args.tuning_json) as f:
                hg.hgmm_set_tuning(**json.load(f))
        step()
        print(json.dumps({"variants": variants_section(args, hg, tree, tgt, p, pr, max(1, args.steps))}),
              flush=True)
        return

    if args.copy_calibration:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE give the
        # scale from counter units to bytes; then steps with the given shapes
        if args.tuning_json:
            with open(args.tuning_json) as f:
                hg.hgmm_set_tuning(**json.load(f))
        a = torch.empty(args.copy_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        for _ in range(max(1, args.steps)):
            step()
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4, "steps": args.steps}), flush=True)
        return

    tuning = None
    if args.tuning_json:
        with open(args.tuning_json) as f:
            hg.hgmm_set_tuning(**json.load(f))
    elif not args.no_tune:
        # launch shapes for this workload, chosen before the timed region; the
        # search starts from the shapes profiled for the LiDAR workload
        start = os.path.join(ROOT, "profiles", "lidar_launch_shapes.json")
        if args.workload == "lidar" and os.path.exists(start):
            with open(start) as f:
                hg.hgmm_set_tuning(**json.load(f))
        tuning = hg.hgmm_autotune(src, [0, n1], [pr["levels"]], tgt, [0, n2], reg_eps=pr["reg_eps"],
                                  min_mass=pr["min_mass"], lambda_c=pr["lambda_c"], reps=2, passes=2)

    if args.save_tuning:
        with open(args.save_tuning, "w") as f:
            json.dump(hg.hgmm_get_tuning(), f)

    for _ in range(args.warmup):
        step()
    # timed region: K steps with nothing but the library's own launches
    torch.cuda.synchronize()
    errs, iters = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
        errs.append(rotation_angle_deg(r["R"], p.R_true))
        iters.append(r["iters"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = t1 - t0
    # the same K steps again with a HIP event pair around every kernel launch on
    # the library's stream: per-kernel durations for the roofline (the events
    # themselves slow the host side, so this region is not the one timed above)
    hg.hgmm_profile_reset()
    hg.hgmm_profile(True)
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    hg.hgmm_profile(False)
    prof = {k: hg.hgmm_profile_read(k) for k in hg.PROFILE_KINDS}

    # mean number of levels a point visits at the final pose (for the descent FLOP count)
    e = hg.hgmm_estep(tree, tgt, r["R"], r["t"], lambda_c=pr["lambda_c"])
    off = np.array([hg.hgmm_level_offset(l) for l in range(pr["levels"] + 1)])
    stop = e["stop_node"].cpu().numpy()
    depth = mean_depth(stop, off)

    roofline = roofline_of(prof, depth, traffic="lidar")
    ds = prof["descend"]
    estep_mpts = ds["units"] / (ds["ms"] * 1e-3) / 1e6 if ds["ms"] > 0 else 0.0

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t_c = 0.0
        reps = 0
        while t_c < args.cpu_seconds and reps < 8:
            c0 = time.perf_counter()
            ot, _ = oracle.build_tree(p.src, pr["levels"], eps=pr["reg_eps"], min_mass=pr["min_mass"])
            oracle.register(ot, p.tgt, lambda_c=pr["lambda_c"])
            t_c += time.perf_counter() - c0
            reps += 1
        cpu = {"value": round(reps / t_c, 4), "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full pair(s) of the same workload (build {n1} + register {n2} points), "
                         f"single-threaded FP64, {t_c:.1f} s"}

    progress("main workload and CPU baseline done")
    variants = None if args.no_batch else variants_section(args, hg, tree, tgt, p, pr, max(3, args.steps // 2))
    progress("registration variants done")
    batched = None if args.no_batch else batch_section(args, hg)
    progress("batched section done")
    warm_form = None if args.no_batch else warm_section(args, hg)
    progress("warm-start section done")
    depth_form = None if args.no_batch else depth_section(args, hg)
    progress("depth-camera section done")
    odometry = None if args.no_batch else odometry_section(args, hg)

    out = {
        "metric": "cloud pairs registered/s (build + register)",
        "value": round(args.steps / sec, 3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 (E-step, moments) + fp64 (transform, eigen, solves)",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "points_src": n1, "points_tgt": n2,
                   "levels": pr["levels"], "lambda_c": pr["lambda_c"], "reg_eps": pr["reg_eps"],
                   "min_mass": pr["min_mass"], "build_iters": 30, "max_iters": 30, "init": "identity",
                   "launch_shapes": hg.hgmm_get_tuning(),
                   "autotune_ms": None if tuning is None else {"start": round(tuning["start_ms"], 3),
                                                                "best": round(tuning["best_ms"], 3)}},
        "estep_mpts_s": round(estep_mpts, 1),
        "rot_err_deg_median": round(float(np.median(errs)), 4),
        "iters_mean": round(float(np.mean(iters)), 2),
        "mean_levels_visited": round(depth, 3),
        "kernels_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in prof.items()},
        "profiled_region_ms_per_step": round((tp1 - tp0) * 1e3 / args.steps, 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched": batched,
        "warm_start": warm_form,
        "depth_camera": depth_form,
        "variants": variants,
        "odometry": odometry,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
