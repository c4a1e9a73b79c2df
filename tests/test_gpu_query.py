"""Per-point log density under a built tree (the query for other consumers of
the model, e.g. scoring a scan against a map), against the FP64 oracle's stop
nodes and an independent evaluation of the Gaussian density with scipy.

The stop node matches the oracle's except for flagged near-ties; the density
within 1e-5 relative (float32 output of an FP64 evaluation); the mean over the
points equals the E-step's log-likelihood.
"""

import math
import sys

import numpy as np
import pytest
from scipy import stats

import oracle
from synth import lidar_pair, rotation_from_axis_angle, small_pair
from gpu_helpers import to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FLAG_GAP = 1e-6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _unpack(c6):
    a, b, c, d, e, f = c6
    return np.array([[a, b, c], [b, d, e], [c, e, f]])


@pytest.mark.parametrize("name", ["small_ragged", "lidar"])
def test_point_loglik_against_oracle(name):
    import paper_1807_02587_amd as hg
    from paper_1807_02587_amd.presets import PRESETS
    if name == "lidar":
        pr = PRESETS["lidar"]
        p, L, eps, mm, lam = lidar_pair(1000), pr["levels"], pr["reg_eps"], pr["min_mass"], pr["lambda_c"]
    else:
        p, L, eps, mm, lam = small_pair(102, n=7_777, n_tgt=5_013, max_angle_deg=8), 3, 1e-6, 1.0, 0.01
    tree = hg.hgmm_build(torch.from_numpy(p.src).cuda(), levels=L, reg_eps=eps, min_mass=mm)
    host = tree.export()
    R = rotation_from_axis_angle([0.3, -1.0, 0.4], math.radians(1.0)) @ p.R_true
    t = p.t_true + 0.001 * p.extent * np.array([1.0, -0.5, 0.25])
    tgt = torch.from_numpy(p.tgt).cuda()
    ll, node = hg.hgmm_point_loglik(tree, tgt, R, t, lambda_c=lam)
    ll = ll.cpu().numpy().astype(np.float64)
    node = node.cpu().numpy()
    o = oracle.estep(to_oracle(oracle, host), p.tgt, R, t, lambda_c=lam)
    ok = o["min_gap"] >= FLAG_GAP
    assert np.array_equal(node[ok], o["stop_node"][ok])
    # an independent evaluation at a sample of points: log pi^g + log N(T(z); mu, cov)
    Y = p.tgt.T.astype(np.float64) @ R.T + t
    idx = np.nonzero(ok)[0][:: max(1, ok.sum() // 2000)]
    ref = np.array([math.log(host["pig"][g]) + stats.multivariate_normal(host["mu"][g], _unpack(host["cov"][g])).logpdf(Y[i])
                    for i, g in zip(idx, node[idx])])
    err = np.abs(ll[idx] - ref) / np.maximum(1.0, np.abs(ref))
    log(f"[query] {name}: {len(idx)} points checked, max rel err {err.max():.2e}; mean loglik {ll.mean():.6f} "
        f"E-step {o['loglik']:.6f}")
    assert err.max() < 1e-5
    e = hg.hgmm_estep(tree, tgt, R, t, lambda_c=lam)
    assert abs(ll.mean() - e["loglik"]) < 1e-5 * max(1.0, abs(e["loglik"]))
