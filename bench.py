"""Throughput of GMM-Tree registration on one MI355X.

Headline step: the uneven batch of 256 unit-cube cloud pairs (N log-uniform
in [2e3, 2e5] points per cloud, rotation U(0, 45 deg), tree depth
ceil(log8(N / 50))) registered in one batch with the learned warm start and
the plain-likelihood fallback: the source forest, the 2-level target forest,
the level-1 features, the network and its head, the registration capped at
two levels and then over the whole tree, the plain method from the identity
as the arbiter, and the choice per pair.  Inputs are resident in HBM.

Prints one JSON line: pairs/s of that step and, beside it, the plain GPU form
(one pair at a time: build + register from the identity) and the batched
plain form; the median rotation error and the pairs registered within
0.5 deg per second; the E-step rate (device-counted points / descent time);
the dominant kernel's achieved rate against the MI355X roofline, from HIP
events around its launches on the library's stream in a repeat of the timed
steps; the FP64 CPU oracle timed on a bounded sample of the same pairs; and
sections for the other workloads (single small pair, LiDAR pair, depth-camera
pair, 4,096 held-out warm-start pairs, registration variants, odometry,
network training).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cloud pairs registered/s + E-step Mpts/s at rot err<=0.5deg, batched vs plain"

# MI355X peaks.  HBM: published 8 TB/s.  FP32 vector: the published 157.3
# TFLOP/s counts packed (2-wide) FMA; the kernels are built without packed FP32
# instructions, so they can reach at most 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP
# (FMA) x 2.4 GHz = 78.6 TFLOP/s, which is reported beside the published figure.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_BF16_TFLOPS = 2500.0

# Algorithmic work per unit (FMA = 2 FLOP): construction E/M, per
# point-iteration: 8 sibling scores, softmax and 10 moments each, about 380
# FLOP (+ 8 exp), 12 bytes (points sorted by parent); registration E-step, per
# point: transform and stop-level work 40 FLOP plus 215 FLOP per tree level
# the point scores (8 children), 12 bytes.
EM_FLOP_PER_POINT_ITER = 380
EM_BYTES_PER_POINT_ITER = 12
DESC_FLOP_FIXED = 40
DESC_FLOP_PER_LEVEL = 215
DESC_BYTES_PER_POINT = 12
MLP_FLOP_FWD_PER_SAMPLE = 2 * (1280 * 512 + 2 * 512 * 512 + 512 * 9)

WEIGHTS = os.path.join(ROOT, "paper_1807_02587_amd", "weights", "warm_mlp.npy")
BATCH_SHAPES = os.path.join(ROOT, "profiles", "batch_launch_shapes.json")
LIDAR_SHAPES = os.path.join(ROOT, "profiles", "lidar_launch_shapes.json")


def progress(msg):
    """One line on stderr per finished section (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _sync():
    import torch
    torch.cuda.synchronize()


def _timed(fn):
    _sync()
    t0 = time.perf_counter()
    r = fn()
    _sync()
    return r, time.perf_counter() - t0


def _rot_err(R, Rt):
    R = np.asarray(R).reshape(-1, 3, 3)
    Rt = np.asarray(Rt).reshape(-1, 3, 3)
    c = (np.einsum("bij,bij->b", R, Rt) - 1.0) / 2.0
    return np.degrees(np.arccos(np.clip(c, -1.0, 1.0)))


def _profile_kinds(hg):
    return {k: hg.hgmm_profile_read(k) for k in hg.PROFILE_KINDS}


def roofline_of(prof, traffic=None):
    """ALU roofline of the kernel family with the largest summed event time
    (the construction's one-block-per-parent EM and the registration descent
    are within a few percent of each other on the headline step, so either
    can lead; every family's fraction and average launch are reported).
    prof: hgmm_profile_read per kind (event ms, launches, host units, and for
    the descent the device-counted points and levels).  traffic: which
    committed counter summary ("batch" or "lidar") gives HBM bytes per launch."""
    flop = {"em_tile": lambda p: p["units"] * EM_FLOP_PER_POINT_ITER,
            "em_block": lambda p: p["units"] * EM_FLOP_PER_POINT_ITER,
            "descend": lambda p: DESC_FLOP_FIXED * p["points"] + DESC_FLOP_PER_LEVEL * p["levels"]}
    byts = {"em_tile": lambda p: p["units"] * EM_BYTES_PER_POINT_ITER,
            "em_block": lambda p: p["units"] * EM_BYTES_PER_POINT_ITER,
            "descend": lambda p: p["points"] * DESC_BYTES_PER_POINT}
    names = {"em_tile": "em_tile_kernel (construction EM iteration of large parents)",
             "em_block": "em_block_kernel (all construction EM iterations, one block per parent)",
             "descend": "descend_kernel (registration E-step)"}
    fam, fam_us = {}, {}
    for k in flop:
        p = prof[k]
        if p["ms"] > 0 and p["launches"] > 0:
            fam[k] = round(flop[k](p) / (p["ms"] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)
            fam_us[k] = round(p["ms"] * 1e3 / p["launches"], 2)
    dom = max(flop, key=lambda k: prof[k]["ms"])
    p = prof[dom]
    ms, n = p["ms"], max(p["launches"], 1)
    f_launch, b_launch, us = flop[dom](p) / n, byts[dom](p) / n, ms * 1e3 / n
    achieved = f_launch / (us * 1e-6) / 1e12 if us > 0 else 0.0
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
           "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": _traffic(dom, traffic) if traffic else None,
           "kernel": names[dom], "launches": p["launches"], "avg_launch_us": round(us, 2),
           "flop_per_launch": round(f_launch), "algorithmic_bytes_per_launch": round(b_launch),
           "frac_of_nonpacked_peak": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
           "achieved_hbm_GBs": round(b_launch / (us * 1e-6) / 1e9, 1) if us > 0 else 0.0,
           "frac_by_family": fam, "avg_launch_us_by_family": fam_us}
    if traffic:
        out.update(_valu(dom, traffic))
    return out


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
            "counted_tflops": f["counted_tflops"],
            "counted_flop_frac": round(f["counted_tflops"] / PEAK_FP32_TFLOPS, 4)}


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


def _workload(name):
    from paper_1807_02587_amd.presets import PRESETS
    from synth import depth_pair, lidar_pair, small_pair
    if name == "lidar":
        p = lidar_pair(1000)
        desc = "LiDAR pair: 64 rings x 1875 azimuths, ground + 50 boxes + 30 cylinders, 1 m / <=2 deg motion"
    elif name == "small":
        p = small_pair(0)
        desc = "small pair: 4 planes + 2 spheres in the unit cube, 10k points, <=30 deg / 0.1 motion"
    elif name == "depth":
        p = depth_pair(2000)
        desc = "depth-camera pair: 640x480 in a furnished room, <=10 deg / 0.2 m motion"
    else:
        raise SystemExit(f"unknown workload {name}")
    return p, PRESETS[name], desc


def host_info():
    """Host CPU of the box the bench runs on: logical CPUs and model."""
    model = platform.processor() or ""
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


# ---------------------------------------------------------------------------
# headline: the uneven batch, batched + warm start, against the plain form
# ---------------------------------------------------------------------------

class Batch:
    """The uneven batch on the GPU and the three ways of registering it."""

    def __init__(self, hg, pairs):
        from paper_1807_02587_amd import warmstart as W
        from synth.torch_scenes import uneven_batch
        self.hg, self.W = hg, W
        self.src, self.tgt, self.off, self.lv, Rt, tt = uneven_batch(3000, pairs)
        self.Rt = Rt.cpu().numpy() if hasattr(Rt, "cpu") else np.asarray(Rt)
        self.tt = tt.cpu().numpy() if hasattr(tt, "cpu") else np.asarray(tt)
        self.B = len(self.lv)
        self.cfg = W.WarmConfig()
        self.ws = hg.Workspace()
        self.net = hg.MLP(seed=0)
        self.net.set_params(np.load(WEIGHTS))
        self.forest = None
        self.wforest = None

    def release(self):
        """Frees the forest handles (and their streams) kept between steps."""
        import gc
        self.forest = self.wforest = None
        gc.collect()

    def warm(self):
        r = self.W.register_warm(self.net, self.src, self.tgt, self.off, self.off, self.lv, self.cfg, ws=self.ws,
                                 forest=self.wforest)
        self.wforest = r["forest"]
        return r

    def batched_plain(self):
        self.forest = self.hg.hgmm_build_batch(self.src, self.off, self.lv, ws=self.ws, forest=self.forest)
        return self.hg.hgmm_register_batch(self.forest, self.tgt, self.off, ws=self.ws)

    def plain_one_at_a_time(self, ks):
        hg, Rs, tree = self.hg, [], None
        for k in ks:
            s_k = self.src[:, self.off[k]:self.off[k + 1]].contiguous()
            t_k = self.tgt[:, self.off[k]:self.off[k + 1]].contiguous()
            tree = hg.hgmm_build(s_k, levels=int(self.lv[k]), ws=self.ws, tree=tree)
            Rs.append(hg.hgmm_register(tree, t_k, ws=self.ws, raise_singular=False)["R"])
        return np.array(Rs)


def headline(args, hg):
    import torch
    bt = Batch(hg, args.batch_pairs)
    B = bt.B
    if args.copy_calibration:
        # a plain copy of known size beside the steps: its FETCH_SIZE /
        # WRITE_SIZE turn the counters into bytes
        a = torch.empty(args.copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        _sync()
    for _ in range(args.warmup):
        bt.warm()
    # timed region: K steps with nothing but the step's own work
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = bt.warm()
    _sync()
    sec = time.perf_counter() - t0
    err = _rot_err(r["R"], bt.Rt)
    out = {"value": round(args.steps * B / sec, 2), "ms_per_step": round(sec * 1e3 / args.steps, 3),
           "rot_err_deg_median": round(float(np.median(err)), 4), "ok_0p5_rate": round(float(np.mean(err <= 0.5)), 4),
           "fallback_rate": round(float(np.mean(r["fallback"])), 4)}
    out["pairs_s_within_0p5deg"] = round(out["value"] * out["ok_0p5_rate"], 2)
    if args.copy_calibration:
        return out, None, bt
    # the same K steps again with a HIP event pair around every launch on the
    # library's stream (the events slow the host side, so this region is not
    # the timed one): per-kernel durations, device-counted descent work
    hg.hgmm_profile_reset()
    hg.hgmm_profile(True)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        bt.warm()
    _sync()
    t2 = time.perf_counter()
    hg.hgmm_profile(False)
    prof = _profile_kinds(hg)
    d = prof["descend"]
    out["estep_mpts_s"] = round(d["points"] / (d["ms"] * 1e-3) / 1e6, 1) if d["ms"] > 0 else None
    out["estep_levels_per_point"] = round(d["levels"] / d["points"], 3) if d["points"] > 0 else None
    out["kernels_ms_per_step"] = {k: round(v["ms"] / args.steps, 3) for k, v in prof.items()}
    out["profiled_region_ms_per_step"] = round((t2 - t1) * 1e3 / args.steps, 3)
    out["roofline"] = roofline_of(prof, traffic="batch")
    progress("headline (batched + warm) done")
    return out, prof, bt


def plain_forms(args, hg, bt, out):
    """The plain GPU form on the same batch, one pair at a time (build +
    register from the identity per pair), and the batched plain form."""
    B = bt.B
    bt.plain_one_at_a_time(range(min(8, B)))
    Rp, tp = _timed(lambda: bt.plain_one_at_a_time(range(B)))
    ep = _rot_err(Rp, bt.Rt)
    bt.batched_plain()
    rb, tb = _timed(bt.batched_plain)
    eb = _rot_err(rb["R"], bt.Rt)
    plain = {"pairs_s": round(B / tp, 2), "rot_err_deg_median": round(float(np.median(ep)), 4),
             "ok_0p5_rate": round(float(np.mean(ep <= 0.5)), 4)}
    plain["pairs_s_within_0p5deg"] = round(plain["pairs_s"] * plain["ok_0p5_rate"], 2)
    bplain = {"pairs_s": round(B / tb, 2), "rot_err_deg_median": round(float(np.median(eb)), 4),
              "ok_0p5_rate": round(float(np.mean(eb <= 0.5)), 4)}
    # E-step rate of the plain form's registration, one pair at a time
    hg.hgmm_profile_reset()
    hg.hgmm_profile(True)
    bt.plain_one_at_a_time(range(B))
    _sync()
    hg.hgmm_profile(False)
    dp = hg.hgmm_profile_read("descend")
    plain["estep_mpts_s"] = round(dp["points"] / (dp["ms"] * 1e-3) / 1e6, 1) if dp["ms"] > 0 else None
    out["plain_one_pair_at_a_time"] = plain
    out["batched_plain"] = bplain
    out["speedup_vs_plain"] = round(out["value"] / plain["pairs_s"], 2)
    out["speedup_within_0p5deg_vs_plain"] = (round(out["pairs_s_within_0p5deg"] / plain["pairs_s_within_0p5deg"], 1)
                                             if plain["pairs_s_within_0p5deg"] > 0 else None)
    out["estep_speedup_vs_plain"] = (round(out["estep_mpts_s"] / plain["estep_mpts_s"], 2)
                                     if plain["estep_mpts_s"] else None)
    progress("plain forms done")


def cpu_baseline(args, bt):
    """The FP64 oracle's whole warm-start step (source tree, 2-level target
    tree, features, network, head, capped and full registration, plain
    registration from the identity, choice) on a size-stratified sample of the
    same pairs, single-threaded, scaled to the batch by its point count."""
    import oracle
    from oracle import warm as owarm
    params = np.load(WEIGHTS).astype(np.float64)
    off, lv = bt.off, bt.lv
    n = np.diff(off)
    order = np.argsort(n)
    k_all = max(1, bt.B // args.cpu_stride)
    sample = [int(order[min(len(order) - 1, args.cpu_stride // 2 + i * args.cpu_stride)]) for i in range(k_all)]
    # visited in a fixed shuffled order, so that a sample cut short by the
    # time limit still spans the sizes
    sample = [sample[i] for i in np.random.default_rng(0).permutation(len(sample))]
    t_used, pts, done, errs = 0.0, 0, 0, []
    src = bt.src.cpu().numpy()
    tgt = bt.tgt.cpu().numpy()
    for k in sample:
        s_k = np.ascontiguousarray(src[:, off[k]:off[k + 1]])
        t_k = np.ascontiguousarray(tgt[:, off[k]:off[k + 1]])
        c0 = time.perf_counter()
        ts, _ = oracle.build_tree(s_k, int(lv[k]), eps=bt.cfg.reg_eps, min_mass=bt.cfg.min_mass)
        tt, _ = oracle.build_tree(t_k, bt.cfg.tgt_levels, eps=bt.cfg.reg_eps, min_mass=bt.cfg.min_mass)
        r = owarm.register_warm(params, ts, tt, t_k, bt.cfg.reg_eps, lambda_c=bt.cfg.lambda_c,
                                max_iters=bt.cfg.max_iters, coarse_levels=bt.cfg.coarse_levels)
        t_used += time.perf_counter() - c0
        pts += int(n[k])
        done += 1
        errs.append(float(_rot_err(r["R"], bt.Rt[k])[0]))
        if t_used > args.cpu_seconds:
            break
    est = t_used * float(off[-1]) / pts
    return {"value": round(bt.B / est, 4), "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} of the {bt.B} pairs (drawn every {args.cpu_stride} by size; {pts} source points of "
                      f"{int(off[-1])}), the whole warm-start step in FP64 on one thread, {t_used:.1f} s; "
                      f"scaled to the batch by points",
            "sample_rot_err_deg_median": round(float(np.median(errs)), 4), **host_info()}


# ---------------------------------------------------------------------------
# single pairs: small (unit cube), LiDAR, depth camera
# ---------------------------------------------------------------------------

def pair_section(args, hg, name, steps, shapes=None, oracle_reps=0, oracle_seconds=10.0):
    """Build of the source tree plus registration of the target from the
    identity per step, one pair; the FP64 oracle on the same pair."""
    import torch
    p, pr, desc = _workload(name)
    keep = hg.hgmm_get_tuning()
    if shapes and os.path.exists(shapes):
        with open(shapes) as f:
            hg.hgmm_set_tuning(**json.load(f))
    dev = torch.device("cuda", 0)
    src = torch.from_numpy(p.src).to(dev)
    tgt = torch.from_numpy(p.tgt).to(dev)
    ws_b, ws_r = hg.Workspace(dev), hg.Workspace(dev)
    tree = None

    def step():
        nonlocal tree
        tree = hg.hgmm_build(src, levels=pr["levels"], reg_eps=pr["reg_eps"], min_mass=pr["min_mass"], ws=ws_b,
                             tree=tree)
        return hg.hgmm_register(tree, tgt, lambda_c=pr["lambda_c"], ws=ws_r, raise_singular=False)

    try:
        if args.copy_calibration:
            # a plain copy of known size beside the steps (counter scale)
            a = torch.empty(args.copy_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
            b = torch.empty_like(a)
            b.copy_(a)
            _sync()
        for _ in range(3):
            step()
        _sync()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = step()
        _sync()
        sec = time.perf_counter() - t0
        hg.hgmm_profile_reset()
        hg.hgmm_profile(True)
        for _ in range(steps):
            step()
        _sync()
        hg.hgmm_profile(False)
        prof = _profile_kinds(hg)
        shapes_used = hg.hgmm_get_tuning()
    finally:
        hg.hgmm_set_tuning(**keep)
    d = prof["descend"]
    out = {"workload": desc, "points_src": int(p.src.shape[1]), "points_tgt": int(p.tgt.shape[1]),
           "levels": pr["levels"], "reg_eps": pr["reg_eps"], "min_mass": pr["min_mass"], "steps": steps,
           "pairs_s": round(steps / sec, 2), "ms_per_step": round(sec * 1e3 / steps, 3),
           "rot_err_deg": round(float(_rot_err(r["R"], p.R_true)[0]), 4), "iters": int(r["iters"]),
           "estep_mpts_s": round(d["points"] / (d["ms"] * 1e-3) / 1e6, 1) if d["ms"] > 0 else None,
           "kernels_ms_per_step": {k: round(v["ms"] / steps, 4) for k, v in prof.items()},
           "roofline": roofline_of(prof, traffic="lidar" if name == "lidar" else None),
           "launch_shapes": shapes_used, "tree": tree, "tgt": tgt, "pair": p, "preset": pr}
    if oracle_reps:
        import oracle
        t_c, reps = 0.0, 0
        while reps < oracle_reps and (reps == 0 or t_c < oracle_seconds):
            c0 = time.perf_counter()
            ot, _ = oracle.build_tree(p.src, pr["levels"], eps=pr["reg_eps"], min_mass=pr["min_mass"])
            ro = oracle.register(ot, p.tgt, lambda_c=pr["lambda_c"])
            t_c += time.perf_counter() - c0
            reps += 1
        out["oracle"] = {"pairs_s": round(reps / t_c, 4), "cores": 1, "pairs_timed": reps,
                         "rot_err_deg": round(float(_rot_err(ro["R"], p.R_true)[0]), 4)}
    return out


def _public(sec):
    return {k: v for k, v in sec.items() if k not in ("tree", "tgt", "pair", "preset")}


def depth_context_run(hg):
    """The paper-shaped context run of the depth-camera scene: 5000 points
    per view, 3 levels (the Lounge protocol's frame size and depth), GPU and
    oracle from the identity over five generated rooms."""
    import torch
    import oracle
    from paper_1807_02587_amd.presets import PRESETS
    from synth import depth_pair
    pr = PRESETS["depth"]
    rows = []
    for seed in range(2000, 2005):
        p = depth_pair(seed, downsample=5000)
        tree = hg.hgmm_build(torch.from_numpy(p.src).cuda(), levels=3, reg_eps=pr["reg_eps"], min_mass=pr["min_mass"])
        r = hg.hgmm_register(tree, torch.from_numpy(p.tgt).cuda(), lambda_c=pr["lambda_c"], raise_singular=False)
        ot, _ = oracle.build_tree(p.src, 3, eps=pr["reg_eps"], min_mass=pr["min_mass"])
        ro = oracle.register(ot, p.tgt, lambda_c=pr["lambda_c"])
        rows.append((float(_rot_err(r["R"], p.R_true)[0]), float(_rot_err(ro["R"], p.R_true)[0])))
    g, o = np.array(rows).T
    return {"workload": "depth-camera scene, 5000 points per view, 3 levels, 5 rooms, from the identity",
            "gpu_rot_err_deg": [round(x, 4) for x in g], "oracle_rot_err_deg": [round(x, 4) for x in o],
            "gpu_median_deg": round(float(np.median(g)), 4), "oracle_median_deg": round(float(np.median(o)), 4)}


def warm_section(args, hg):
    """Held-out warm-start pairs (10k points per cloud, rotation U(0, 90 deg),
    translation U(-0.1, 0.1)^3, L = 2; seeds disjoint from training): the
    batched warm start with the plain-likelihood fallback against the plain
    GPU form one pair at a time (timed on the first 256 pairs)."""
    from paper_1807_02587_amd import warmstart as W
    from synth.torch_scenes import cube_pairs
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

    plain(range(8))
    Rp, tp = _timed(lambda: plain(range(plain_pairs)))
    warm()
    rw, tw = _timed(warm)
    ep = _rot_err(Rp, Rt[:plain_pairs])
    ew = _rot_err(rw["R"], Rt)
    out = {"workload": f"{B} held-out pairs, {n} points per cloud, rotation U(0,90 deg), L = 2 "
                       f"(plain form timed on the first {plain_pairs})",
           "plain_pairs_s": round(plain_pairs / tp, 2), "plain_median_rot_err_deg": round(float(np.median(ep)), 4),
           "plain_ok_0p5_rate": round(float(np.mean(ep <= 0.5)), 4),
           "batched_warm_pairs_s": round(B / tw, 2), "batched_warm_median_rot_err_deg": round(float(np.median(ew)), 4),
           "batched_warm_p90_rot_err_deg": round(float(np.percentile(ew, 90)), 4),
           "batched_warm_ok_0p5_rate": round(float(np.mean(ew <= 0.5)), 4),
           "batched_warm_ok_5_rate": round(float(np.mean(ew <= 5.0)), 4),
           "batched_warm_iters_mean": round(float(np.mean(rw["iters"])), 2),
           "warm_fallback_rate": round(float(np.mean(rw["fallback"])), 4),
           "speedup_batched_warm_vs_plain": round((B / tw) / (plain_pairs / tp), 2)}
    out["speedup_ok_pairs_s"] = (round(out["batched_warm_pairs_s"] * out["batched_warm_ok_0p5_rate"]
                                       / (out["plain_pairs_s"] * out["plain_ok_0p5_rate"]), 2)
                                 if out["plain_ok_0p5_rate"] > 0 else None)
    return out


def mlp_section(args, hg):
    """The warm-start network on its own: inference and training steps (bf16
    MFMA GEMMs) on random rows, samples/s and the GEMMs' achieved TFLOP/s."""
    import torch
    rows = 4096
    X = torch.randn(rows, 1280, device="cuda")
    T = torch.randn(rows, 9, device="cuda")
    net = hg.MLP(seed=1)
    net.forward(X)
    _, tf = _timed(lambda: [net.forward(X) for _ in range(20)])
    net.train_step(X, T, 1e-4, want_loss=False)
    _, tt = _timed(lambda: [net.train_step(X, T, 1e-4, want_loss=False) for _ in range(20)])
    fwd = MLP_FLOP_FWD_PER_SAMPLE * rows * 20
    return {"rows": rows, "forward_samples_s": round(rows * 20 / tf, 1),
            "forward_tflops": round(fwd / tf / 1e12, 2),
            "train_samples_s": round(rows * 20 / tt, 1),
            "train_tflops": round(3 * fwd / tt / 1e12, 2),
            "frac_of_bf16_peak_train": round(3 * fwd / tt / 1e12 / PEAK_BF16_TFLOPS, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch-pairs", type=int, default=256)
    ap.add_argument("--warm-pairs", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-stride", type=int, default=16, help="oracle sample: every n-th pair by size")
    ap.add_argument("--only", default=None,
                    choices=["headline", "small", "lidar", "depth", "warm", "variants", "odometry", "mlp"],
                    help="run one section only (profiling runs)")
    ap.add_argument("--batch-shapes", default=BATCH_SHAPES, help="launch shapes of the batched forms")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="with --only: a device copy of --copy-mib MiB beside the steps (counter scale)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); independent pairs would shard "
              "across GPUs by pair, which is not run here.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1807_02587_amd as hg
    torch.cuda.set_device(0)
    if not os.path.exists(WEIGHTS):
        raise SystemExit(f"{WEIGHTS} is missing: the warm start's network weights are part of the package")
    with open(args.batch_shapes) as f:
        batch_shapes = json.load(f)
    only = args.only

    def want(name):
        return only is None or only == name

    defaults = hg.hgmm_get_tuning()
    head = prof = bt = cpu = None
    if want("headline"):
        hg.hgmm_set_tuning(**batch_shapes)
        head, prof, bt = headline(args, hg)
        # each forest handle owns streams; with a few hardware queues per
        # process, streams of handles kept alive would share queues with the
        # streams of the handles timed next
        bt.release()
        if only is None:
            plain_forms(args, hg, bt, head)
            bt.release()
        if only is None and not args.no_cpu_baseline:
            cpu = cpu_baseline(args, bt)
            progress("CPU baseline done")
        hg.hgmm_set_tuning(**defaults)
        if only == "headline":
            print(json.dumps({"headline": head}), flush=True)
            return
    sections = {}
    if want("small"):
        sec = pair_section(args, hg, "small", args.steps, oracle_reps=5)
        sections["small_pair"] = _public(sec)
        progress("small pair done")
    lid = None
    if want("lidar") or want("variants"):
        lid = pair_section(args, hg, "lidar", args.steps, shapes=LIDAR_SHAPES, oracle_reps=1 if want("lidar") else 0)
        sections["lidar_pair"] = _public(lid)
        progress("LiDAR pair done")
    if want("variants"):
        hg.hgmm_set_tuning(**json.load(open(LIDAR_SHAPES)))
        sections["variants"] = variants_section(args, hg, lid["tree"], lid["tgt"], lid["pair"], lid["preset"],
                                                max(3, args.steps // 2))
        hg.hgmm_set_tuning(**defaults)
        progress("registration variants done")
    if want("depth"):
        sec = pair_section(args, hg, "depth", max(3, args.steps // 2))
        sections["depth_pair"] = _public(sec)
        sections["depth_pair"]["context_5000_points_3_levels"] = depth_context_run(hg)
        progress("depth pair done")
    if want("warm"):
        hg.hgmm_set_tuning(**batch_shapes)
        sections["warm_start_heldout"] = warm_section(args, hg)
        hg.hgmm_set_tuning(**defaults)
        progress("held-out warm-start pairs done")
    if want("odometry"):
        hg.hgmm_set_tuning(**json.load(open(LIDAR_SHAPES)))
        sections["odometry"] = odometry_section(args, hg)
        hg.hgmm_set_tuning(**defaults)
        progress("odometry done")
    if want("mlp"):
        sections["mlp"] = mlp_section(args, hg)
        progress("network done")
    if only is not None:
        print(json.dumps(sections), flush=True)
        return

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 (E-step, moments) + fp64 (transform, eigen, solves) + bf16 (network)",
        "data": "synthetic",
        "config": {"workload": f"uneven batch: {bt.B} unit-cube pairs, N log-uniform [2e3, 2e5] points per cloud "
                               f"({int(bt.off[-1])} per side), rotation U(0,45 deg), levels ceil(log8(N/50)); "
                               "batched with the learned warm start and the plain-likelihood fallback",
                   "pairs": bt.B, "points_per_side": int(bt.off[-1]), "levels_histogram":
                       {str(L): int(np.sum(np.asarray(bt.lv) == L)) for L in sorted(set(int(v) for v in bt.lv))},
                   "lambda_c": bt.cfg.lambda_c, "reg_eps": bt.cfg.reg_eps, "build_iters": 30,
                   "max_iters": bt.cfg.max_iters, "launch_shapes": batch_shapes,
                   "launch_shapes_file": os.path.relpath(args.batch_shapes, ROOT)},
        **{k: v for k, v in head.items() if k not in ("value", "ms_per_step")},
        "cpu_baseline": cpu,
        "sections": sections,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
