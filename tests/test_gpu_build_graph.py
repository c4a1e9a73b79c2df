"""Construction planned on the device, run as one hipGraph (build_graph = 1) or
as the same launches issued on the stream (build_graph = 2), against the
host-planned construction (build_graph = 0): the same plan and the
same arithmetic, so every exported tree field and every label is
bit-identical.  On a handle, the first construction of a shape is planned on
the host (it records the work counts that size the graph's grids), the next
one captures the graph, later ones replay it.  Covers a batch of uneven clouds
of depths 1-3, replays with new points of the same shape, block-only and
tiles-only plans, a cloud whose plan has work where the captured graph has
none (redone host-planned), and the LiDAR pair."""

import sys

import numpy as np
import pytest

from synth import lidar_pair, small_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("live", "has_children", "count", "pi", "pig", "mu", "cov", "lam", "evec", "kappa")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hg():
    import paper_1807_02587_amd as hg
    assert torch.cuda.is_available()
    return hg


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _same(fa, fb, B):
    for b in range(B):
        ha, hb = fa.export(b), fb.export(b)
        for k in FIELDS + ("origin", "extent"):
            np.testing.assert_array_equal(np.asarray(ha[k]), np.asarray(hb[k]), err_msg=f"tree {b} field {k}")
        np.testing.assert_array_equal(fa.labels(b).cpu().numpy(), fb.labels(b).cpu().numpy(),
                                      err_msg=f"tree {b} labels")


def _batch(seed0, sizes=(3000, 777, 5000, 10_000, 64)):
    levels = (2, 1, 3, 2, 1)
    pairs = [small_pair(seed0 + i, n=n) for i, n in enumerate(sizes)]
    src = np.concatenate([p.src for p in pairs], axis=1)
    off = np.concatenate([[0], np.cumsum([p.src.shape[1] for p in pairs])]).astype(np.int64)
    return src, off, list(levels)


def _host(hg, old, src, off, lv, **shapes):
    hg.hgmm_set_tuning(**dict(old, build_graph=0, **shapes))
    return hg.hgmm_build_batch(_cuda(src), off, lv)


@pytest.mark.parametrize("mode", [1, 2])
def test_batch_graph_equals_host_planned(hg, mode):
    old = hg.hgmm_get_tuning()
    try:
        for shapes in (dict(), dict(block64_max=1 << 20, block256_max=1 << 20, block512_max=1 << 20),
                       dict(block64_max=0, block256_max=0, block512_max=0)):
            forest = None
            ws = hg.Workspace()
            for call, seed0 in enumerate((21, 31, 41, 51)):
                src, off, lv = _batch(seed0)
                ref = _host(hg, old, src, off, lv, **shapes)
                hg.hgmm_set_tuning(**dict(old, build_graph=mode, **shapes))
                forest = hg.hgmm_build_batch(_cuda(src), off, lv, ws=ws, forest=forest)
                _same(forest, ref, len(lv))
            st = forest.graph_stats()
            log(f"[build graph] mode {mode} shapes {shapes}: 4 constructions identical, {st}")
            assert st["replays"] >= 2
            assert st["captures"] >= 1 if mode == 1 else st["captures"] == 0
    finally:
        hg.hgmm_set_tuning(**old)


@pytest.mark.parametrize("mode", [1, 2])
def test_graph_redone_when_plan_differs(hg, mode):
    """A cloud of the same size whose level-1 parents cross a class threshold
    that the hinted plan did not: the graph has no tiled iterations at level 1,
    the call finds tiled parents in the device plan and redoes the construction
    host-planned (results equal either way)."""
    old = hg.hgmm_get_tuning()
    try:
        shapes = dict(block64_max=0, block256_max=0, block512_max=350)
        rng = np.random.default_rng(5)
        n = 2048
        # uniform in the cube: 8 root children of about 256 points (block class)
        uni = rng.uniform(-0.5, 0.5, size=(3, n)).astype(np.float32)
        # a tight cluster of 1800 points beside a sparse one: children of about
        # 450 points (tiled)
        lop = np.concatenate([rng.normal([[0.4], [0.0], [0.0]], 0.02, size=(3, 1800)),
                              rng.uniform(-0.5, 0.5, size=(3, n - 1800))], axis=1).astype(np.float32)
        forest = None
        ws = hg.Workspace()
        off = np.array([0, n], np.int64)
        for call, cloud in enumerate((uni, uni, uni, lop)):
            ref = _host(hg, old, cloud, off, [2], **shapes)
            hg.hgmm_set_tuning(**dict(old, build_graph=mode, **shapes))
            forest = hg.hgmm_build_batch(_cuda(cloud), off, [2], ws=ws, forest=forest)
            _same(forest, ref, 1)
            log(f"[build graph] call {call}: {forest.graph_stats()}; level-1 counts "
                f"{sorted(ref.export(0)['count'][8:72].reshape(8, 8).sum(1).tolist())[-3:]}")
        st = forest.graph_stats()
        assert st["replays"] >= 1 and st["host_builds"] == 2, st
    finally:
        hg.hgmm_set_tuning(**old)


@pytest.mark.parametrize("mode", [1, 2])
def test_lidar_graph_equals_host_planned(hg, mode):
    from paper_1807_02587_amd.presets import PRESETS
    pr = PRESETS["lidar"]
    p = lidar_pair(1000)
    old = hg.hgmm_get_tuning()
    try:
        hg.hgmm_set_tuning(**dict(old, build_graph=0))
        ref = hg.hgmm_build(_cuda(p.src), levels=pr["levels"], reg_eps=pr["reg_eps"], min_mass=pr["min_mass"])
        hg.hgmm_set_tuning(**dict(old, build_graph=mode))
        tree = None
        src = _cuda(p.src)
        ws = hg.Workspace()
        for rep in range(4):   # host-planned, capture, replays into the same handle
            tree = hg.hgmm_build(src, levels=pr["levels"], reg_eps=pr["reg_eps"], min_mass=pr["min_mass"], ws=ws,
                                 tree=tree)
            _same(tree, ref, 1)
        st = tree.graph_stats()
        assert st == (dict(replays=3, captures=1, host_builds=1) if mode == 1 else
                      dict(replays=3, captures=0, host_builds=1)), st
        r0 = hg.hgmm_register(ref, _cuda(p.tgt), lambda_c=pr["lambda_c"])
        r1 = hg.hgmm_register(tree, _cuda(p.tgt), lambda_c=pr["lambda_c"])
        np.testing.assert_array_equal(r0["R"], r1["R"])
        log(f"[build graph] lidar mode {mode}: identical over 4 constructions, {st}")
    finally:
        hg.hgmm_set_tuning(**old)
