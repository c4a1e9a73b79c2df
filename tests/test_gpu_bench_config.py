"""Parity in the launch configurations that bench.py times, at the benchmark's
full sizes.

* The LiDAR pair (117,816 source and 118,028 target points, 4 levels, 30 EM
  iterations per level, registration from the identity) under the committed
  LiDAR launch shapes: every level of the tree against the oracle's EM from the
  GPU's parent level, and the registered pose against the oracle's
  registration on the exported tree.
* The uneven batch (256 pairs, N log-uniform in [2e3, 2e5], 10.5M points per
  side) under the committed batch launch shapes, built and registered in one
  call each as in bench.py: sampled trees (the smallest, two of median size
  and the largest cloud) level by level against the oracle, the registration
  of the smallest and a median pair against the oracle's, and one E-step of
  the largest pair at its registered pose (stop nodes and log-likelihood).
"""

import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
from synth import lidar_pair, rotation_angle_deg
from gpu_helpers import compare_build_levels, to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EM30_TOL = dict(pi=2e-3, mu=1e-3, cov=1e-2)
EM30_MIN_PARENT = 64
POSE_TOL = 1e-4
FLAG_GAP = 1e-6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hg():
    import paper_1807_02587_amd as hg
    assert torch.cuda.is_available()
    return hg


def _shapes(name):
    with open(os.path.join(ROOT, "profiles", f"{name}_launch_shapes.json")) as f:
        return json.load(f)


def test_lidar_in_bench_launch_shapes(hg):
    from paper_1807_02587_amd.presets import PRESETS
    pr = PRESETS["lidar"]
    p = lidar_pair(1000)
    old = hg.hgmm_set_tuning(**_shapes("lidar"))
    try:
        log(f"[bench lidar] shapes {hg.hgmm_get_tuning()}")
        tree = hg.hgmm_build(torch.from_numpy(p.src).cuda(), levels=pr["levels"], reg_eps=pr["reg_eps"],
                             min_mass=pr["min_mass"])
        host = tree.export()
        glab = tree.labels().cpu().numpy()
        compare_build_levels(oracle, host, glab, p.src, pr["levels"], pr["reg_eps"], pr["min_mass"], 30, EM30_TOL,
                             log, min_parent=EM30_MIN_PARENT)
        r = hg.hgmm_register(tree, torch.from_numpy(p.tgt).cuda(), lambda_c=pr["lambda_c"])
    finally:
        hg.hgmm_set_tuning(**old)
    o = oracle.register(to_oracle(oracle, host), p.tgt, lambda_c=pr["lambda_c"])
    dang = math.radians(rotation_angle_deg(r["R"], o["R"]))
    dt = np.linalg.norm(r["t"] - o["t"]) / host["extent"]
    log(f"[bench lidar] register: iters gpu {r['iters']} oracle {o['iters']}  pose diff {dang:.2e} rad "
        f"{dt:.2e} ext  error vs truth {rotation_angle_deg(r['R'], p.R_true):.4f} deg")
    assert r["status"] == 0 and o["status"] == 0
    assert dang < POSE_TOL and dt < POSE_TOL
    assert abs(r["iters"] - o["iters"]) <= 2


def test_uneven_batch_in_bench_launch_shapes(hg):
    from synth.torch_scenes import uneven_batch
    src, tgt, off, lv, Rt, tt = uneven_batch(3000, 256)
    n = np.diff(off)
    order = np.argsort(n, kind="stable")
    small, large = int(order[0]), int(order[-1])
    med = [int(order[len(order) // 2]), int(order[len(order) // 2 + 1])]
    log(f"[bench batch] {len(n)} pairs, {int(off[-1])} points per side; sampled pairs {small} (n={n[small]}), "
        f"{med} (n={n[med].tolist()}), {large} (n={n[large]})")
    old = hg.hgmm_set_tuning(**_shapes("batch"))
    try:
        ws = hg.Workspace()
        forest = hg.hgmm_build_batch(src, off, lv, ws=ws)
        r = hg.hgmm_register_batch(forest, tgt, off, ws=ws)
        torch.cuda.synchronize()
        for b in [small] + med + [large]:
            host = forest.export(b)
            glab = forest.labels(b).cpu().numpy()
            ps = src[:, off[b]:off[b + 1]].cpu().numpy().astype(np.float32)
            log(f"[bench batch] tree {b}: n={n[b]} levels={lv[b]}")
            compare_build_levels(oracle, host, glab, ps, int(lv[b]), 1e-6, 1.0, 30, EM30_TOL, log,
                                 min_parent=EM30_MIN_PARENT)
        for b in [small, med[0]]:
            host = forest.export(b)
            pt = tgt[:, off[b]:off[b + 1]].cpu().numpy().astype(np.float32)
            o = oracle.register(to_oracle(oracle, host), pt)
            dang = math.radians(rotation_angle_deg(r["R"][b], o["R"]))
            dt = np.linalg.norm(r["t"][b] - o["t"]) / host["extent"]
            log(f"[bench batch] register pair {b}: iters gpu {r['iters'][b]} oracle {o['iters']}  pose diff "
                f"{dang:.2e} rad {dt:.2e} ext")
            assert r["status"][b] == 0 and o["status"] == 0
            assert dang < POSE_TOL and dt < POSE_TOL
            assert abs(int(r["iters"][b]) - o["iters"]) <= 2
        # one E-step of the largest pair at its registered pose
        ll, stop = hg.hgmm_estep_batch(forest, tgt, off, r["R"], r["t"], ws=ws, stop_nodes=True)
        stop = stop.cpu().numpy()
    finally:
        hg.hgmm_set_tuning(**old)
    b = large
    pt = tgt[:, off[b]:off[b + 1]].cpu().numpy().astype(np.float32)
    o = oracle.estep(to_oracle(oracle, forest.export(b)), pt, r["R"][b], r["t"][b])
    g = stop[off[b]:off[b + 1]]
    flagged = o["min_gap"] < FLAG_GAP
    mism = (g != o["stop_node"]) & ~flagged
    log(f"[bench batch] estep pair {b}: loglik gpu {ll[b]:.9f} oracle {o['loglik']:.9f}; stop-node mismatches "
        f"{mism.sum()} (flagged {flagged.sum()} of {len(g)})")
    assert mism.sum() == 0
    assert abs(ll[b] - o["loglik"]) <= 1e-5 * max(1.0, abs(o["loglik"]))
