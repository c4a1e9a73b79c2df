"""The allocation-free registration entry point (hgmm_register_noalloc, whose
workspace is the library's static device scratch) against hgmm_register on
the same trees and clouds: two calls in a row, the second on a smaller cloud
and tree, and the size limit."""

import math
import sys

import numpy as np
import pytest

from synth import rotation_angle_deg, rotation_from_axis_angle, small_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

POSE_TOL = 1e-4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hg():
    import paper_1807_02587_amd as hg
    assert torch.cuda.is_available()
    return hg


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_noalloc_matches_register_twice(hg):
    cases = [(small_pair(311, n=30_000, n_tgt=27_011, max_angle_deg=6), 3),
             (small_pair(312, n=9_000, n_tgt=6_001, max_angle_deg=6), 2)]
    for p, L in cases:
        log(f"[noalloc] n_src {p.src.shape[1]} n_tgt {p.tgt.shape[1]} levels {L}")
        tree = hg.hgmm_build(_cuda(p.src), levels=L)
        ext = tree.export()["extent"]
        R0 = rotation_from_axis_angle([0.4, -0.7, 0.2], math.radians(1.5)) @ p.R_true
        t0 = p.t_true + 0.005 * ext * np.array([0.3, 0.5, -0.8])
        tgt = _cuda(p.tgt)
        a = hg.hgmm_register(tree, tgt, R0=R0, t0=t0)
        b = hg.hgmm_register_noalloc(tree, tgt, R0=R0, t0=t0)
        dang = math.radians(rotation_angle_deg(a["R"], b["R"]))
        dt = float(np.linalg.norm(a["t"] - b["t"])) / ext
        log(f"  iters {a['iters']} / {b['iters']}, pose diff {dang:.2e} rad {dt:.2e} ext, "
            f"loglik {a['loglik']:.9f} / {b['loglik']:.9f}")
        assert dang < POSE_TOL and dt < POSE_TOL
        assert abs(a["iters"] - b["iters"]) <= 2
        assert abs(a["loglik"] - b["loglik"]) <= 1e-5 * max(1.0, abs(a["loglik"]))
        if L <= 2:
            # levels 0-1 are binned in a fixed order: the same kernels give the same bits
            np.testing.assert_array_equal(a["R"], b["R"])
            np.testing.assert_array_equal(a["t"], b["t"])
            assert a["iters"] == b["iters"]


def test_noalloc_rejects_clouds_beyond_the_scratch(hg):
    from paper_1807_02587_amd._lib import HgmmError
    p = small_pair(313, n=4_000)
    tree = hg.hgmm_build(_cuda(p.src), levels=2)
    cap = hg.api._lib.load().hgmm_noalloc_scratch_bytes()
    n = 2_000_000
    need = hg.api._lib.load().hgmm_register_workspace_bytes(n, 2)
    assert need > cap
    big = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    with pytest.raises(HgmmError) as e:
        hg.hgmm_register_noalloc(tree, big)
    assert e.value.code == -1
    # the entry point still works after a rejected call
    r = hg.hgmm_register_noalloc(tree, _cuda(p.tgt), R0=p.R_true, t0=p.t_true)
    assert r["status"] == 0
