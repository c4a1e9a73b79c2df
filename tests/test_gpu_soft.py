"""Soft multi-path E-step (Sec. 4.1: a parent's expectation is the sum of its
children's; branches whose expectation falls below tau are pruned) on the GPU
against the FP64 oracle on the same tree and pose.

Posteriors are FP32 on the GPU (exp2 of FP32 score differences), so per-node
moments are compared within 1e-4 relative, leaving out nodes reached by points
whose oracle pruning margin min |E - tau| / tau is below 1e-3 (a pruning
decision that FP32 rounding could flip); poses within 1e-4 rad and 1e-4 *
extent, iterations within 2.
"""

import math
import sys

import numpy as np
import pytest

import oracle
from synth import lidar_pair, rotation_angle_deg, rotation_from_axis_angle, small_pair
from gpu_helpers import gpu_bins_from_oracle, rel_err, to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MARGIN = 1e-3
MOMENT_TOL = 1e-4
POSE_TOL = 1e-4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


_trees = {}


def _case(hg, name):
    if name in _trees:
        return _trees[name]
    from paper_1807_02587_amd.presets import PRESETS
    if name == "small_ragged":
        p, L, eps, mm, lam = small_pair(102, n=7_777, n_tgt=5_013, max_angle_deg=8), 3, 1e-6, 1.0, 0.01
    elif name == "lidar":
        pr = PRESETS["lidar"]
        p, L, eps, mm, lam = lidar_pair(1000), pr["levels"], pr["reg_eps"], pr["min_mass"], pr["lambda_c"]
    tree = hg.hgmm_build(_cuda(p.src), levels=L, reg_eps=eps, min_mass=mm)
    _trees[name] = (p, tree, tree.export(), lam)
    return _trees[name]


@pytest.mark.parametrize("name,tau,lam", [("small_ragged", 0.01, 0.01), ("small_ragged", 0.1, 0.0),
                                          ("small_ragged", 1e-4, 0.0), ("lidar", 0.01, None)])
def test_soft_estep_parity(name, tau, lam):
    import paper_1807_02587_amd as hg
    p, tree, host, lam0 = _case(hg, name)
    lam = lam0 if lam is None else lam
    R = rotation_from_axis_angle([0.3, -1.0, 0.4], math.radians(2.0)) @ p.R_true
    t = p.t_true + 0.002 * p.extent * np.array([1.0, -0.5, 0.25])
    log(f"[soft estep] case={name} tau={tau} lambda_c={lam} n={p.tgt.shape[1]}")
    g = hg.hgmm_estep_soft(tree, _cuda(p.tgt), tau, R, t, lambda_c=lam)
    o = oracle.estep_soft(to_oracle(oracle, host), p.tgt, R, t, lambda_c=lam, tau=tau)
    gs = g["stops"].cpu().numpy()
    near = o["margin"] < MARGIN
    log(f"  points near tau {near.sum()}; stops mean gpu {gs.mean():.3f} oracle {o['stops'].mean():.3f}; "
        f"mismatched stop counts away from tau {(gs != o['stops'])[~near].sum()}")
    assert np.array_equal(gs[~near], o["stops"][~near])
    gb = g["bins"].cpu().numpy()
    ob = gpu_bins_from_oracle(host, o["bins"])
    # nodes that a near-tau point reaches in either run are left out
    sel = (ob[:, 4] > 0) | (gb[:, 4] > 0)
    if near.any():
        on = oracle.estep_soft(to_oracle(oracle, host), np.ascontiguousarray(p.tgt[:, near]), R, t, lambda_c=lam,
                               tau=tau * (1 - 2 * MARGIN))
        sel &= on["bins"][:, 4] == 0
    m0 = rel_err(gb[sel, 0], ob[sel, 0], 1e-30)
    doff = np.abs(gb[sel, 1:4] - ob[sel, 1:4]).max(1) / (np.maximum(ob[sel, 0], 1e-30) * host["extent"])
    d2 = rel_err(gb[sel, 5], ob[sel, 5], 1e-30)
    log(f"  nodes compared {sel.sum()}  M0 rel max {m0.max():.2e}  D/(M0 ext) {doff.max():.2e}  d2 {d2.max():.2e}; "
        f"loglik gpu {g['loglik']:.9f} oracle {o['loglik']:.9f}")
    assert sel.sum() > 0
    assert m0.max() < MOMENT_TOL and doff.max() < MOMENT_TOL and d2.max() < MOMENT_TOL
    if not near.any():
        assert abs(g["loglik"] - o["loglik"]) < MOMENT_TOL * max(1.0, abs(o["loglik"]))


@pytest.mark.parametrize("name", ["small_ragged", "lidar"])
def test_soft_register_parity(name):
    import paper_1807_02587_amd as hg
    p, tree, host, lam = _case(hg, name)
    off = 0.0 if name == "lidar" else 1.0
    R0 = rotation_from_axis_angle([0.2, 0.9, -0.3], math.radians(off)) @ p.R_true
    t0 = p.t_true + off * 0.001 * p.extent * np.array([0.5, -0.2, 0.3])
    tau, tol, iters = 0.01, 1e-5, 60
    r = hg.hgmm_register_soft(tree, _cuda(p.tgt), tau, R0=R0, t0=t0, lambda_c=lam, max_iters=iters, tol_rot=tol,
                              tol_trans_rel=tol)
    o = oracle.register_soft(to_oracle(oracle, host), p.tgt, R0=R0, t0=t0, lambda_c=lam, tau=tau, max_iters=iters,
                             tol_rot=tol, tol_trans=tol * host["extent"])
    dang = math.radians(rotation_angle_deg(r["R"], o["R"]))
    dt = np.linalg.norm(r["t"] - o["t"]) / host["extent"]
    log(f"[soft register] case={name}: iters gpu {r['iters']} oracle {o['iters']}  pose diff {dang:.2e} rad "
        f"{dt:.2e} ext  error vs truth {rotation_angle_deg(r['R'], p.R_true):.4f} deg")
    assert r["status"] == 0 and o["status"] == 0 and o["iters"] < iters
    assert dang < POSE_TOL and dt < POSE_TOL
    assert abs(r["iters"] - o["iters"]) <= 2


def test_soft_edge_cases():
    import paper_1807_02587_amd as hg
    p, tree, host, lam = _case(hg, "small_ragged")
    for bad in (0.0, 1.0, -0.5):
        with pytest.raises(hg.HgmmError):
            hg.hgmm_estep_soft(tree, _cuda(p.tgt), bad)
    for n in (1, 257):
        xyz = np.ascontiguousarray(p.tgt[:, :n])
        g = hg.hgmm_estep_soft(tree, _cuda(xyz), 0.01)
        o = oracle.estep_soft(to_oracle(oracle, host), xyz, lambda_c=0.01, tau=0.01)
        far = o["margin"] >= MARGIN
        assert np.array_equal(g["stops"].cpu().numpy()[far], o["stops"][far])
        assert abs(g["bins"].cpu().numpy()[:, 0].sum() - o["bins"][:, 0].sum()) < 1e-4 * n
