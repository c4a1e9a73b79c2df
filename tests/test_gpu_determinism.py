"""Run-to-run reproducibility of registration.

The descent adds its moments in 128-bit fixed point, whose integer sums do
not depend on the order in which waves, blocks and XCDs add, so the moments,
poses, iteration counts and likelihoods of repeated runs are identical bit
for bit, on a 4-level tree and over an odometry sequence.  The FP64-atomics
mode (hgmm_tuning.reg_atomics = 1, the comparison mode) gives the same
results up to FP64 summation order."""

import math
import sys

import numpy as np
import pytest

from synth import lidar_pair, lidar_sequence, rotation_angle_deg, small_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hg():
    import paper_1807_02587_amd as hg
    assert torch.cuda.is_available()
    return hg


@pytest.fixture(scope="module")
def lidar(hg):
    from paper_1807_02587_amd.presets import PRESETS
    pr = PRESETS["lidar"]
    p = lidar_pair(1000)
    tree = hg.hgmm_build(torch.from_numpy(p.src).cuda(), levels=pr["levels"], reg_eps=pr["reg_eps"],
                         min_mass=pr["min_mass"])
    return p, pr, tree, torch.from_numpy(p.tgt).cuda()


def _with_tuning(hg, **knobs):
    class Ctx:
        def __enter__(self):
            self.old = hg.hgmm_set_tuning(**knobs)

        def __exit__(self, *a):
            hg.hgmm_set_tuning(**self.old)
    return Ctx()


@pytest.mark.parametrize("sort", [0, 1])
def test_register_bitwise_reproducible_4_levels(hg, lidar, sort):
    p, pr, tree, tgt = lidar
    with _with_tuning(hg, reg_sort=sort, reg_atomics=0):
        rs = [hg.hgmm_register(tree, tgt, lambda_c=pr["lambda_c"]) for _ in range(3)]
        es = [hg.hgmm_estep(tree, tgt, rs[0]["R"], rs[0]["t"], lambda_c=pr["lambda_c"]) for _ in range(2)]
    for r in rs[1:]:
        np.testing.assert_array_equal(r["R"], rs[0]["R"])
        np.testing.assert_array_equal(r["t"], rs[0]["t"])
        assert r["iters"] == rs[0]["iters"] and r["loglik"] == rs[0]["loglik"]
    np.testing.assert_array_equal(es[1]["bins"].cpu().numpy(), es[0]["bins"].cpu().numpy())
    assert es[1]["loglik"] == es[0]["loglik"]
    log(f"[determinism] sort {sort}: {rs[0]['iters']} iterations, error vs truth "
        f"{rotation_angle_deg(rs[0]['R'], p.R_true):.4f} deg, identical over 3 runs")


def test_fixed_point_against_fp64_atomics(hg, lidar):
    """The comparison mode: the same E-step with FP64 atomic moments gives the
    same stop nodes and moments within FP64 summation error, and the same pose."""
    p, pr, tree, tgt = lidar
    R = p.R_true
    t = p.t_true
    with _with_tuning(hg, reg_atomics=0):
        a = hg.hgmm_estep(tree, tgt, R, t, lambda_c=pr["lambda_c"])
        ra = hg.hgmm_register(tree, tgt, lambda_c=pr["lambda_c"])
    with _with_tuning(hg, reg_atomics=1):
        b = hg.hgmm_estep(tree, tgt, R, t, lambda_c=pr["lambda_c"])
        rb = hg.hgmm_register(tree, tgt, lambda_c=pr["lambda_c"])
    np.testing.assert_array_equal(a["stop_node"].cpu().numpy(), b["stop_node"].cpu().numpy())
    ba, bb = a["bins"].cpu().numpy(), b["bins"].cpu().numpy()
    np.testing.assert_array_equal(ba[:, 4], bb[:, 4])
    m = ba[:, 4] > 0
    e0 = np.abs(ba[m, 0] - bb[m, 0]).max() / np.abs(ba[m, 0]).max()
    e1 = np.abs(ba[m, 1:4] - bb[m, 1:4]).max() / np.abs(ba[m, 1:4]).max()
    e5 = np.abs(ba[m, 5] - bb[m, 5]).max() / np.abs(ba[m, 5]).max()
    # (compare matrix entries: an angle from arccos is only good to ~1e-8 rad near zero)
    dR = float(np.abs(ra["R"] - rb["R"]).max())
    dt = float(np.linalg.norm(ra["t"] - rb["t"]))
    log(f"[fixed vs atomics] M0 {e0:.1e} D {e1:.1e} Q {e5:.1e}; pose max |dR| {dR:.1e}, |dt| {dt:.1e}, iters "
        f"{ra['iters']} {rb['iters']}")
    assert e0 < 1e-12 and e1 < 1e-12 and e5 < 1e-12
    assert dR < 1e-10 and dt < 1e-10 * tree.export()["extent"] and abs(ra["iters"] - rb["iters"]) <= 1


def test_odometry_bitwise_reproducible(hg):
    from paper_1807_02587_amd.presets import PRESETS
    pr = PRESETS["lidar"]
    q = lidar_sequence(1000, frames=5)
    xyz = torch.from_numpy(q.clouds).cuda()
    runs = [hg.hgmm_odometry(xyz, q.offsets, pr["levels"], reg_eps=pr["reg_eps"], min_mass=pr["min_mass"],
                             lambda_c=pr["lambda_c"]) for _ in range(2)]
    for k in ("R_rel", "t_rel", "R_abs", "t_abs", "iters", "status"):
        np.testing.assert_array_equal(runs[1][k], runs[0][k])


def test_batch_bitwise_reproducible(hg):
    pairs = [small_pair(900 + k, n=n, max_angle_deg=10) for k, n in enumerate((3000, 20000, 60000))]
    src = np.ascontiguousarray(np.concatenate([p.src for p in pairs], axis=1))
    tgt = np.ascontiguousarray(np.concatenate([p.tgt for p in pairs], axis=1))
    off = np.concatenate([[0], np.cumsum([p.src.shape[1] for p in pairs])]).astype(np.int64)
    forest = hg.hgmm_build_batch(torch.from_numpy(src).cuda(), off, [2, 3, 4])
    tg = torch.from_numpy(tgt).cuda()
    r1 = hg.hgmm_register_batch(forest, tg, off)
    r2 = hg.hgmm_register_batch(forest, tg, off)
    for k in ("R", "t", "iters", "loglik"):
        np.testing.assert_array_equal(r1[k], r2[k])
