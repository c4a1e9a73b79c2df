"""Batched form (many uneven pairs per call) against the FP64 oracle, tree by
tree and pair by pair, and against itself under a partial activity mask.

The forest's trees are fitted by shared launches whose tiling depends on the
whole batch, so a tree is not bit-identical to a single-cloud build of the same
points; it is held to the same per-level EM tolerances against the oracle.
Registration of pair b depends only on pair b's tree, points and pose, so a
pair's result does not depend on which other pairs are active.
"""

import math
import sys

import numpy as np
import pytest

import oracle
from synth import rotation_angle_deg, rotation_from_axis_angle, small_pair
from gpu_helpers import compare_build_levels, to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EM1_TOL = dict(pi=1e-5, mu=1e-5, cov=1e-5)
EM30_TOL = dict(pi=2e-3, mu=1e-3, cov=1e-2)
POSE_TOL = 1e-4

# (source points, target points, levels, seed): uneven sizes, one tree per depth
# 1..3 and a cloud of 64 points
CASES = [(3000, 2500, 2, 11), (777, 900, 1, 12), (5000, 4100, 3, 13), (10_000, 10_000, 2, 14), (64, 64, 1, 15)]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hg():
    import paper_1807_02587_amd as hg
    assert torch.cuda.is_available()
    return hg


@pytest.fixture(scope="module")
def batch():
    pairs = [small_pair(seed, n=n, n_tgt=m, max_angle_deg=20) for n, m, _, seed in CASES]
    src = np.concatenate([p.src for p in pairs], axis=1)
    tgt = np.concatenate([p.tgt for p in pairs], axis=1)
    soff = np.concatenate([[0], np.cumsum([p.src.shape[1] for p in pairs])]).astype(np.int64)
    toff = np.concatenate([[0], np.cumsum([p.tgt.shape[1] for p in pairs])]).astype(np.int64)
    levels = [L for _, _, L, _ in CASES]
    return pairs, src, tgt, soff, toff, levels


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _starts(pairs):
    """0.5 degree and 0.05 % of the extent away from the truth (the method is local)."""
    R0 = np.stack([rotation_from_axis_angle([0.2, 0.9, -0.3], math.radians(0.5)) @ p.R_true for p in pairs])
    t0 = np.stack([p.t_true + 0.0005 * p.extent * np.array([0.5, -0.2, 0.3]) for p in pairs])
    return R0, t0


MAX_ITERS = 100


@pytest.mark.parametrize("iters", [1, 30])
def test_build_batch_vs_oracle(hg, batch, iters):
    pairs, src, _, soff, _, levels = batch
    forest = hg.hgmm_build_batch(_cuda(src), soff, levels, build_iters=iters)
    tol = EM1_TOL if iters == 1 else EM30_TOL
    for b, p in enumerate(pairs):
        log(f"[batch build] tree {b} n={p.src.shape[1]} levels={levels[b]} iters={iters}")
        host = forest.export(b)
        assert host["levels"] == levels[b] and host["n_points"] == p.src.shape[1]
        glab = forest.labels(b).cpu().numpy()
        assert glab.shape == (levels[b], p.src.shape[1])
        compare_build_levels(oracle, host, glab, p.src, levels[b], 1e-6, 1.0, iters, tol, log,
                             min_parent=0 if iters == 1 else 64)


def test_register_batch_vs_oracle(hg, batch):
    """Every step of every pair's GPU trajectory against the oracle's step from
    the same pose, and whole trajectories of the pairs that converge.

    The update of Algorithm 1 is discontinuous where a point's most likely
    child changes, so while a pair drifts away from the truth (an unstable
    phase in which pose differences grow) rounding differences of 1e-6 rad
    can move one point across a score gap of 1e-4 and the GPU and oracle
    trajectories part, each still the method's own.  Step by step, from the
    GPU's own poses, the two must agree on every iteration; end to end they
    must agree on the pairs that converge."""
    pairs, src, tgt, soff, toff, levels = batch
    forest = hg.hgmm_build_batch(_cuda(src), soff, levels)
    R0, t0 = _starts(pairs)
    tg = _cuda(tgt)
    # the GPU trajectory: registration is bitwise reproducible, so the call
    # with max_iters = k gives the pose after k iterations
    traj = [(R0, t0, np.zeros(len(pairs), np.int32))]
    for k in range(1, MAX_ITERS + 1):
        r = hg.hgmm_register_batch(forest, tg, toff, R0=R0, t0=t0, max_iters=k)
        traj.append((r["R"], r["t"], r["iters"]))
    compared = 0
    for b, p in enumerate(pairs):
        host = forest.export(b)
        ot = to_oracle(oracle, host)
        worst = 0.0
        for k in range(r["iters"][b]):
            Rk, tk = traj[k][0][b], traj[k][1][b]
            o1 = oracle.register(ot, p.tgt, R0=Rk, t0=tk, max_iters=1)
            da = math.radians(rotation_angle_deg(traj[k + 1][0][b], o1["R"]))
            dt = np.linalg.norm(traj[k + 1][1][b] - o1["t"]) / host["extent"]
            worst = max(worst, da, dt)
            assert da < POSE_TOL and dt < POSE_TOL, (b, k, da, dt)
        o = oracle.register(ot, p.tgt, R0=R0[b], t0=t0[b], max_iters=MAX_ITERS)
        dang = math.radians(rotation_angle_deg(r["R"][b], o["R"]))
        dt = np.linalg.norm(r["t"][b] - o["t"]) / host["extent"]
        log(f"[batch register] pair {b}: iters gpu {r['iters'][b]} oracle {o['iters']} status {r['status'][b]} "
            f"{o['status']}  worst step difference {worst:.2e}; end to end {dang:.2e} rad {dt:.2e} ext; err vs "
            f"truth {rotation_angle_deg(r['R'][b], p.R_true):.4f} deg")
        assert r["status"][b] == o["status"] == 0
        if o["iters"] < MAX_ITERS:
            assert dang < POSE_TOL and dt < POSE_TOL
            assert abs(int(r["iters"][b]) - o["iters"]) <= 2
            assert abs(r["loglik"][b] - o["loglik"]) <= 1e-4 * max(1.0, abs(o["loglik"]))
            compared += 1
    log(f"[batch register] {compared} of {len(pairs)} pairs converged within {MAX_ITERS} iterations "
        f"(compared end to end)")


def test_register_batch_active_mask_and_estep(hg, batch):
    pairs, src, tgt, soff, toff, levels = batch
    forest = hg.hgmm_build_batch(_cuda(src), soff, levels)
    R0, t0 = _starts(pairs)
    tg = _cuda(tgt)
    full = hg.hgmm_register_batch(forest, tg, toff, R0=R0, t0=t0)
    act = np.array([1, 0, 1, 0, 1], np.int32)
    part = hg.hgmm_register_batch(forest, tg, toff, R0=R0, t0=t0, active=act)
    for b in range(len(pairs)):
        if act[b]:
            np.testing.assert_array_equal(part["R"][b], full["R"][b])
            np.testing.assert_array_equal(part["t"][b], full["t"][b])
            assert part["iters"][b] == full["iters"][b]
        else:
            np.testing.assert_array_equal(part["R"][b], R0[b])
            np.testing.assert_array_equal(part["t"][b], t0[b])
            assert part["iters"][b] == 0
    # one E-step per pair at the starting poses: mean log-likelihood and every
    # point's stop node against the oracle's (exact outside flagged near ties)
    ll, stop = hg.hgmm_estep_batch(forest, tg, toff, R0, t0, stop_nodes=True)
    stop = stop.cpu().numpy()
    for b, p in enumerate(pairs):
        o = oracle.estep(to_oracle(oracle, forest.export(b)), p.tgt, R0[b], t0[b])
        g = stop[toff[b]:toff[b + 1]]
        flagged = o["min_gap"] < 1e-6
        mism = (g != o["stop_node"]) & ~flagged
        log(f"[batch estep] pair {b}: loglik gpu {ll[b]:.9f} oracle {o['loglik']:.9f}; stop-node mismatches "
            f"{mism.sum()} (flagged {flagged.sum()})")
        assert abs(ll[b] - o["loglik"]) <= 1e-5 * max(1.0, abs(o["loglik"]))
        assert mism.sum() == 0


def test_batch_argument_checks(hg, batch):
    from paper_1807_02587_amd import HgmmError
    pairs, src, tgt, soff, toff, levels = batch
    forest = hg.hgmm_build_batch(_cuda(src), soff, levels)
    more = np.concatenate([toff, [toff[-1] + 100]])
    tgt_more = np.concatenate([tgt, tgt[:, :100]], axis=1)
    with pytest.raises(HgmmError):   # more pairs than the forest has trees
        hg.hgmm_register_batch(forest, _cuda(tgt_more), more)
    bad = soff.copy()
    bad[2] = bad[1] - 1
    with pytest.raises((HgmmError, AssertionError)):
        hg.hgmm_build_batch(_cuda(src), bad, levels)
    with pytest.raises(HgmmError):   # a cloud of fewer than 8 points
        hg.hgmm_build_batch(_cuda(src[:, :12]), np.array([0, 5, 12]), [1, 1])


def test_register_onto_the_first_trees(hg, batch):
    """A batch of B pairs registers onto the first B trees of a larger forest
    (tree b with cloud b): the same results, bit for bit, as in the call with
    every pair (a pair's registration depends only on its tree, points and
    start)."""
    pairs, src, tgt, soff, toff, levels = batch
    forest = hg.hgmm_build_batch(_cuda(src), soff, levels)
    R0, t0 = _starts(pairs)
    full = hg.hgmm_register_batch(forest, _cuda(tgt), toff, R0=R0, t0=t0)
    part = hg.hgmm_register_batch(forest, _cuda(tgt[:, :toff[3]]), toff[:4], R0=R0[:3], t0=t0[:3])
    for k in ("R", "t", "iters", "loglik", "status"):
        np.testing.assert_array_equal(part[k], full[k][:3])
    ll = hg.hgmm_estep_batch(forest, _cuda(tgt[:, :toff[3]]), toff[:4], R0[:3], t0[:3])
    ll_full = hg.hgmm_estep_batch(forest, _cuda(tgt), toff, R0, t0)
    np.testing.assert_array_equal(ll, ll_full[:3])


def test_fold_modes_agree(hg, batch):
    """The previous iteration's fold and M-step inside every tile block
    (fold_tiles large) and once per parent in a launch of its own
    (fold_tiles = 0) sum the same partials in the same order: the trees are
    identical bit for bit."""
    pairs, src, _, soff, _, levels = batch
    old = hg.hgmm_get_tuning()
    out = []
    try:
        for ft in (0, 1 << 30):
            hg.hgmm_set_tuning(block64_max=0, block256_max=0, block512_max=0, fold_tiles=ft)
            f = hg.hgmm_build_batch(_cuda(src), soff, levels)
            out.append([f.export(b) for b in range(len(levels))])
    finally:
        hg.hgmm_set_tuning(**old)
    for a, b in zip(*out):
        for k in ("live", "count", "pi", "mu", "cov", "kappa"):
            np.testing.assert_array_equal(np.asarray(a[k]), np.asarray(b[k]))


def test_tiled_and_block_paths_agree(hg, batch):
    """The same forest built with every parent tiled and with every parent in one
    block: one EM iteration from identical initial children agrees to the FP32
    moment tolerance (only the summation order differs)."""
    pairs, src, _, soff, _, levels = batch
    old = hg.hgmm_get_tuning()
    try:
        hg.hgmm_set_tuning(block64_max=0, block256_max=0, block512_max=0)
        tiled = hg.hgmm_build_batch(_cuda(src), soff, levels, build_iters=1)
        hg.hgmm_set_tuning(block64_max=1 << 20, block256_max=1 << 20, block512_max=1 << 20)
        block = hg.hgmm_build_batch(_cuda(src), soff, levels, build_iters=1)
    finally:
        hg.hgmm_set_tuning(**old)
    for b in range(len(pairs)):
        a, c = tiled.export(b), block.export(b)
        sl = slice(0, 8)   # level 0 starts from identical children in both
        np.testing.assert_array_equal(a["live"][sl], c["live"][sl])
        np.testing.assert_allclose(a["pi"][sl], c["pi"][sl], rtol=1e-5)
        np.testing.assert_allclose(a["mu"][sl], c["mu"][sl], rtol=0, atol=1e-5 * a["extent"])


def test_autotune_small_batch(hg, batch):
    pairs, src, tgt, soff, toff, levels = batch
    old = hg.hgmm_get_tuning()
    try:
        r = hg.hgmm_autotune(_cuda(src), soff, levels, _cuda(tgt), toff, reps=1, passes=1)
        log(f"[autotune] {r}")
        assert r["best_ms"] > 0 and r["best_ms"] <= r["start_ms"] * 1.0001
        assert hg.hgmm_get_tuning() == r["tuning"]
        # the tuned setting still builds a valid forest
        f = hg.hgmm_build_batch(_cuda(src), soff, levels)
        for b in range(len(pairs)):
            h = f.export(b)
            assert abs(h["pi"][:8][h["live"][:8] == 1].sum() - 1.0) < 1e-9
    finally:
        hg.hgmm_set_tuning(**old)


def test_register_graph_matches_stream(hg, batch):
    """reg_graph = 1 (each chunk one hipGraph launch, graph cached in the handle)
    gives bit-identical results to plain launches, on every replay, with eager
    work between the calls; max_iters need not be a multiple of the chunk."""
    pairs, src, tgt, soff, toff, levels = batch
    forest = hg.hgmm_build_batch(_cuda(src), soff, levels)
    R0, t0 = _starts(pairs)
    tg = _cuda(tgt)
    old = hg.hgmm_get_tuning()
    try:
        for max_iters in (25, 7):
            hg.hgmm_set_tuning(reg_graph=0, reg_chunk=2)
            ref = hg.hgmm_register_batch(forest, tg, toff, R0=R0, t0=t0, max_iters=max_iters)
            assert np.all(ref["iters"] <= max_iters)
            hg.hgmm_set_tuning(reg_graph=1, reg_chunk=2)
            for rep in range(3):
                r = hg.hgmm_register_batch(forest, tg, toff, R0=R0, t0=t0, max_iters=max_iters)
                hg.hgmm_estep_batch(forest, tg, toff, R0, t0)   # eager work between replays
                torch.cuda.synchronize()
                for k in ("R", "t", "iters", "loglik", "status"):
                    np.testing.assert_array_equal(r[k], ref[k], err_msg=f"{k} replay {rep} max_iters {max_iters}")
    finally:
        hg.hgmm_set_tuning(**old)


def test_register_graph_follows_reg_tile(hg):
    """The cached registration graph belongs to its launch shapes: changing
    reg_tile between two graph registrations of one tree with the same number
    of tiles (1500 points: two tiles at 768 and at 1024) builds a new graph,
    so the single-level and soft E-steps still cover every point (their FP64
    atomic moments allow only rounding-level differences from plain
    launches)."""
    p = small_pair(31, n=1500, max_angle_deg=5)
    tree = hg.hgmm_build(_cuda(p.src), levels=2)
    tg = _cuda(p.tgt)
    old = hg.hgmm_get_tuning()
    out = {}
    try:
        for graph in (0, 1):
            for rt in (768, 1024):
                hg.hgmm_set_tuning(reg_graph=graph, reg_tile=rt, reg_chunk=2)
                out[graph, rt] = (hg.hgmm_register_flat(tree, tg, 1, max_iters=6),
                                  hg.hgmm_register_soft(tree, tg, tau=0.01, max_iters=6))
    finally:
        hg.hgmm_set_tuning(**old)
    for rt in (768, 1024):
        for a, b in zip(out[1, rt], out[0, rt]):
            np.testing.assert_allclose(a["R"], b["R"], rtol=0, atol=1e-9)
            np.testing.assert_allclose(a["t"], b["t"], rtol=0, atol=1e-9 * p.extent)


def test_morton_sorted_registration_matches(hg, batch):
    """reg_sort = 1 (moving points in Morton order inside each pair) changes only
    how points are grouped into wavefronts: per-point stop nodes and weights of
    the E-step are identical (reported in the caller's point order), while the
    FP32 per-wave partial sums regroup, so bins and the one-step log-likelihood
    agree to FP32 summation rounding.  Four of the five pairs drift away from
    the truth over the iterations (the method is local), which amplifies that
    rounding: their poses after 10 iterations agree to 1e-5 (a tenth of the
    parity tolerance)."""
    pairs, src, tgt, soff, toff, levels = batch
    forest = hg.hgmm_build_batch(_cuda(src), soff, levels)
    R0, t0 = _starts(pairs)
    tg = _cuda(tgt)
    old = hg.hgmm_get_tuning()
    try:
        hg.hgmm_set_tuning(reg_sort=0)
        ref = hg.hgmm_register_batch(forest, tg, toff, R0=R0, t0=t0, max_iters=10)
        ll0 = hg.hgmm_estep_batch(forest, tg, toff, R0, t0)
        hg.hgmm_set_tuning(reg_sort=1)
        r = hg.hgmm_register_batch(forest, tg, toff, R0=R0, t0=t0, max_iters=10)
        ll1 = hg.hgmm_estep_batch(forest, tg, toff, R0, t0)
    finally:
        hg.hgmm_set_tuning(**old)
    np.testing.assert_allclose(ll1, ll0, rtol=1e-6)
    np.testing.assert_allclose(r["R"], ref["R"], atol=1e-5)
    np.testing.assert_allclose(r["t"], ref["t"], atol=1e-5)
    assert np.all(np.abs(r["iters"] - ref["iters"]) <= 1)


def test_morton_sorted_estep_points_match(hg):
    from synth import small_pair
    p = small_pair(102, n=7_777, n_tgt=5_013, max_angle_deg=8)
    tree = hg.hgmm_build(_cuda(p.src), levels=3)
    tg = _cuda(p.tgt)
    old = hg.hgmm_get_tuning()
    try:
        hg.hgmm_set_tuning(reg_sort=0)
        a = hg.hgmm_estep(tree, tg, p.R_true, p.t_true)
        hg.hgmm_set_tuning(reg_sort=1)
        b = hg.hgmm_estep(tree, tg, p.R_true, p.t_true)
    finally:
        hg.hgmm_set_tuning(**old)
    np.testing.assert_array_equal(b["stop_node"].cpu().numpy(), a["stop_node"].cpu().numpy())
    np.testing.assert_array_equal(b["gamma"].cpu().numpy(), a["gamma"].cpu().numpy())
    ba, bb = a["bins"].cpu().numpy(), b["bins"].cpu().numpy()
    act = ba[:, 0] > 0
    ext = tree.info()["extent"]
    # M0 and counts relative; first moments normalised by M0 * extent; sum d^2 relative
    np.testing.assert_array_equal(bb[:, 4], ba[:, 4])
    assert np.all(np.abs(bb[act, 0] - ba[act, 0]) <= 1e-6 * ba[act, 0])
    assert np.all(np.abs(bb[act, 1:4] - ba[act, 1:4]) <= 1e-6 * ba[act, :1] * ext)
    assert np.all(np.abs(bb[act, 5] - ba[act, 5]) <= 1e-6 * ba[act, 5])


def test_level2_lds_staging_matches(hg):
    """reg_lds_levels = 3 (level-2 scoring records staged in LDS) computes the
    same descent: identical stop nodes and weights, bins equal to the rounding
    of FP64 atomic order."""
    from synth import small_pair
    p = small_pair(102, n=7_777, n_tgt=5_013, max_angle_deg=8)
    tree = hg.hgmm_build(_cuda(p.src), levels=4)
    tg = _cuda(p.tgt)
    old = hg.hgmm_get_tuning()
    try:
        hg.hgmm_set_tuning(reg_lds_levels=2)
        a = hg.hgmm_estep(tree, tg, p.R_true, p.t_true, lambda_c=0.0)
        ra = hg.hgmm_register(tree, tg, R0=p.R_true, t0=p.t_true, max_iters=5)
        hg.hgmm_set_tuning(reg_lds_levels=3)
        b = hg.hgmm_estep(tree, tg, p.R_true, p.t_true, lambda_c=0.0)
        rb = hg.hgmm_register(tree, tg, R0=p.R_true, t0=p.t_true, max_iters=5)
    finally:
        hg.hgmm_set_tuning(**old)
    np.testing.assert_array_equal(b["stop_node"].cpu().numpy(), a["stop_node"].cpu().numpy())
    np.testing.assert_array_equal(b["gamma"].cpu().numpy(), a["gamma"].cpu().numpy())
    ba, bb = a["bins"].cpu().numpy(), b["bins"].cpu().numpy()
    np.testing.assert_allclose(bb, ba, rtol=1e-12, atol=1e-12 * np.abs(ba).max())
    np.testing.assert_allclose(rb["R"], ra["R"], atol=1e-9)
