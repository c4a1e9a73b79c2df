"""Single-level variant ("GMM J=n", Sec. 5 list of variants) on the GPU against
the FP64 oracle's single-level E-step and registration on the same tree.

Tolerances as for the tree descent: the chosen component exact except points
whose oracle top-2 gap is below 1e-6 (natural-log units), responsibilities
within 2e-5 relative (the kernel scores in FP64 and forms the posterior from
FP32 exp2 of FP64 differences of at most 8 in log2 units, about 1e-6
relative), per-node moments within 1e-5, poses within 1e-4 rad and
1e-4 * extent.  Levels 0-2 and level 3 (4096 components, several scalar-load
rounds per wave) are both covered.
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

FLAG_GAP = 1e-6
GAMMA_TOL = 2e-5
MOMENT_TOL = 1e-5
POSE_TOL = 1e-4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hg():
    import paper_1807_02587_amd as hg
    assert torch.cuda.is_available()
    hg.library_path()
    return hg


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


_cache = {}


def _case(name):
    if name in _cache:
        return _cache[name]
    from paper_1807_02587_amd.presets import PRESETS
    if name == "small_ragged":
        c = (small_pair(102, n=7_777, n_tgt=5_013, max_angle_deg=8), 3, 1e-6, 1.0)
    elif name == "small_deep":
        c = (small_pair(103, n=40_000, n_tgt=3_001, max_angle_deg=8), 4, 1e-6, 1.0)
    elif name == "lidar":
        pr = PRESETS["lidar"]
        c = (lidar_pair(1000), pr["levels"], pr["reg_eps"], pr["min_mass"])
    else:
        raise KeyError(name)
    _cache[name] = c
    return c


_trees = {}


def _tree(hg, name):
    if name not in _trees:
        p, L, eps, mm = _case(name)
        tree = hg.hgmm_build(_cuda(p.src), levels=L, reg_eps=eps, min_mass=mm)
        _trees[name] = (tree, tree.export())
    return _trees[name]


def _check_estep(hg, name, level, sample=None):
    p, L, _, _ = _case(name)
    tree, host = _tree(hg, name)
    ot = to_oracle(oracle, host)
    R = rotation_from_axis_angle([0.3, -1.0, 0.4], math.radians(2.0)) @ p.R_true
    t = p.t_true + 0.002 * p.extent * np.array([1.0, -0.5, 0.25])
    n = p.tgt.shape[1]
    log(f"[flat estep] case={name} n={n} level={level} J={8 ** (level + 1)}")
    g = hg.hgmm_estep_flat(tree, _cuda(p.tgt), level, R, t)
    stop = g["stop_node"].cpu().numpy()
    gam = g["gamma"].cpu().numpy().astype(np.float64)
    gb = g["bins"].cpu().numpy()
    idx = np.arange(n) if sample is None else sample
    o = oracle.estep_flat(ot, level, np.ascontiguousarray(p.tgt[:, idx]), R, t)
    flagged = o["min_gap"] < FLAG_GAP
    mism = stop[idx] != o["stop_node"]
    log(f"  flagged {flagged.sum()}  mismatches {mism.sum()}  unflagged mismatches {(mism & ~flagged).sum()}")
    assert not np.any(mism & ~flagged)
    ok = ~flagged
    gerr = np.abs(gam[idx][ok] - o["gamma"][ok]) / o["gamma"][ok]
    log(f"  gamma rel err max {gerr.max():.2e} median {np.median(gerr):.2e}")
    assert gerr.max() < GAMMA_TOL
    g0, J = oracle.level_offset(level), oracle.level_nodes(level)
    assert np.all((stop >= g0) & (stop < g0 + J))
    assert gb[:, 4].sum() == n
    assert not np.any(gb[:g0]) and not np.any(gb[g0 + J:])
    if sample is not None:
        return
    ob = gpu_bins_from_oracle(host, o["bins"])
    touched = np.zeros(len(ob), bool)
    touched[o["stop_node"][flagged]] = True
    touched[stop[flagged]] = True
    sel = (ob[:, 4] >= 1) & ~touched
    m0 = rel_err(gb[sel, 0], ob[sel, 0], 1e-30)
    doff = np.abs(gb[sel, 1:4] - ob[sel, 1:4]).max(1) / (ob[sel, 0] * host["extent"])
    l2 = rel_err(gb[sel, 5], ob[sel, 5], 1.0)
    log(f"  bins: active {sel.sum()}  M0 rel max {m0.max():.2e}  D/(M0 ext) max {doff.max():.2e}  "
        f"d2 {l2.max():.2e}; loglik gpu {g['loglik']:.9f} oracle {o['loglik']:.9f}")
    assert np.array_equal(gb[sel, 4], ob[sel, 4])
    assert m0.max() < MOMENT_TOL and doff.max() < MOMENT_TOL and l2.max() < 1e-4
    assert abs(g["loglik"] - o["loglik"]) < 1e-5 * max(1.0, abs(o["loglik"]))


@pytest.mark.parametrize("level", [0, 1, 2])
def test_flat_estep_parity_small(hg, level):
    _check_estep(hg, "small_ragged", level)


def test_flat_estep_parity_chunked_level(hg):
    """Level 3: 4096 components, staged through LDS in chunks of 512."""
    _check_estep(hg, "small_deep", 3)


def test_flat_estep_parity_lidar_full(hg):
    """The LiDAR pair at full size: level 2 (512 components) against the oracle
    on every point, level 3 on a sample of points (each point's result depends
    only on that point)."""
    _check_estep(hg, "lidar", 2)
    n = _case("lidar")[0].tgt.shape[1]
    rng = np.random.default_rng(7)
    _check_estep(hg, "lidar", 3, sample=np.sort(rng.choice(n, 3000, replace=False)))


@pytest.mark.parametrize("name,level", [("small_ragged", 1), ("small_ragged", 2), ("lidar", 1)])
def test_flat_register_parity(hg, name, level):
    p, L, _, _ = _case(name)
    tree, host = _tree(hg, name)
    ot = to_oracle(oracle, host)
    off = 0.0 if name == "lidar" else 1.0
    R0 = rotation_from_axis_angle([0.2, 0.9, -0.3], math.radians(off)) @ p.R_true
    t0 = p.t_true + off * 0.001 * p.extent * np.array([0.5, -0.2, 0.3])
    log(f"[flat register] case={name} level={level}")
    # EM converges linearly; a looser stop (1e-5) and more iterations let every case end by tolerance
    tol, iters = 1e-5, 60
    r = hg.hgmm_register_flat(tree, _cuda(p.tgt), level, R0=R0, t0=t0, max_iters=iters, tol_rot=tol,
                              tol_trans_rel=tol)
    o = oracle.register_flat(ot, level, p.tgt, R0=R0, t0=t0, max_iters=iters, tol_rot=tol,
                             tol_trans=tol * host["extent"])
    dang = math.radians(rotation_angle_deg(r["R"], o["R"]))
    dt = np.linalg.norm(r["t"] - o["t"]) / host["extent"]
    log(f"  iters gpu {r['iters']} oracle {o['iters']}  pose diff {dang:.2e} rad {dt:.2e} ext  "
        f"err vs truth {rotation_angle_deg(r['R'], p.R_true):.4f} deg; loglik {r['loglik']:.6f} {o['loglik']:.6f}")
    assert o["status"] == 0 and r["status"] == 0
    assert o["iters"] < iters, "choose a case that converges"
    assert dang < POSE_TOL and dt < POSE_TOL
    assert abs(r["iters"] - o["iters"]) <= 2
    assert abs(r["loglik"] - o["loglik"]) < 1e-5 * max(1.0, abs(o["loglik"]))


def test_flat_edge_cases(hg):
    p, L, _, _ = _case("small_ragged")
    tree, host = _tree(hg, "small_ragged")
    ot = to_oracle(oracle, host)
    # levels outside the tree are rejected
    for bad in (-1, L):
        with pytest.raises(hg.HgmmError):
            hg.hgmm_estep_flat(tree, _cuda(p.tgt), bad)
        with pytest.raises(hg.HgmmError):
            hg.hgmm_register_flat(tree, _cuda(p.tgt), bad)
    # one point, and a tail of 257 (one full block and one lane)
    for n in (1, 257):
        xyz = np.ascontiguousarray(p.tgt[:, :n])
        g = hg.hgmm_estep_flat(tree, _cuda(xyz), L - 1)
        o = oracle.estep_flat(ot, L - 1, xyz)
        ok = o["min_gap"] >= FLAG_GAP
        assert np.array_equal(g["stop_node"].cpu().numpy()[ok], o["stop_node"][ok])
        assert abs(g["loglik"] - o["loglik"]) < 1e-5 * max(1.0, abs(o["loglik"]))
    # level 0 of the flat variant is the tree's descent stopped at level 0
    a = hg.hgmm_estep_flat(tree, _cuda(p.tgt), 0)
    b = hg.hgmm_estep(tree, _cuda(p.tgt), lambda_c=1.0)
    assert np.array_equal(a["stop_node"].cpu().numpy(), b["stop_node"].cpu().numpy())
    np.testing.assert_allclose(a["gamma"].cpu().numpy(), b["gamma"].cpu().numpy(), rtol=GAMMA_TOL)
