"""FP64 oracle of the learned warm start's data path (TEST INFRASTRUCTURE ONLY).

The warm start is this project's addition (the paper has no learned part).
Its steps, in the order the GPU path takes them:

* ``canonical_frame``: a cloud's frame from its tree's root statistics: the
  principal axes E (rows: the root eigenvectors under the oracle's sign rule,
  the last row negated if that makes E a proper rotation), the centroid c
  and the RMS radius s = sqrt(trace of the root covariance without its
  regularisation).
* ``features``: the 64 level-1 nodes of the tree in that frame, each as
  (global weight, E (mu - c) / s, upper triangle of E Sigma E^T / s^2); a dead
  node is 10 zeros.
* ``register_warm``: network forward (oracle.mlp), the head's pose, a
  registration of the target capped at two levels of the source tree when it
  is deeper, then the whole tree, and the plain method from the identity as
  the arbiter: the result with the higher final log-likelihood is kept.
"""

from __future__ import annotations

import numpy as np

from . import mlp
from .oracle import OracleTree, level_offset, register


def canonical_frame(tree: OracleTree, reg_eps: float) -> np.ndarray:
    """13 values: E row-major (9), c (3), s."""
    E = np.array(tree.root_evec, dtype=np.float64).reshape(3, 3).copy()
    if np.linalg.det(E) < 0.0:
        E[2] = -E[2]
    tr = float(tree.root_cov[0] + tree.root_cov[3] + tree.root_cov[5]) - 3.0 * reg_eps
    s = np.sqrt(max(tr, 1e-300))
    return np.concatenate([E.ravel(), np.asarray(tree.origin, dtype=np.float64), [s]])


def features(tree: OracleTree, reg_eps: float) -> np.ndarray:
    """640 values: the 64 level-1 nodes in the canonical frame."""
    fr = canonical_frame(tree, reg_eps)
    E, c, s = fr[:9].reshape(3, 3), fr[9:12], fr[12]
    out = np.zeros(640)
    if tree.levels < 2:
        return out
    base = level_offset(1)
    for k in range(64):
        g = base + k
        if not tree.live[g]:
            continue
        m = E @ (tree.mu[g] - c) / s
        S6 = tree.cov[g]
        S = np.array([[S6[0], S6[1], S6[2]], [S6[1], S6[3], S6[4]], [S6[2], S6[4], S6[5]]])
        C = E @ S @ E.T / (s * s)
        out[10 * k:10 * k + 10] = [tree.pig[g], *m, C[0, 0], C[0, 1], C[0, 2], C[1, 1], C[1, 2], C[2, 2]]
    return out


def cut(tree: OracleTree, levels: int) -> OracleTree:
    """The tree's first ``levels`` levels as a tree of its own (the last kept
    level has no children)."""
    t = OracleTree(levels)
    n = level_offset(levels)
    for k in ("live", "has_children", "count", "pi", "pig", "mu", "cov", "lam", "evec", "kappa"):
        getattr(t, k)[...] = getattr(tree, k)[:n]
    t.has_children[level_offset(levels - 1):] = 0
    for k in ("origin", "extent", "n_points", "root_cov", "root_lam", "root_evec"):
        setattr(t, k, getattr(tree, k))
    return t


def initial_pose(params, src_tree: OracleTree, tgt_tree: OracleTree, reg_eps: float):
    """The network's start transform (R0, t0) for a pair: features of both
    trees, forward pass with the device's bf16 rounding points, head."""
    X = np.concatenate([features(src_tree, reg_eps), features(tgt_tree, reg_eps)])[None, :]
    Y, _ = mlp.forward(params, X, bf16=True)
    R0, t0 = mlp.head_pose(Y, canonical_frame(src_tree, reg_eps)[None, :],
                           canonical_frame(tgt_tree, reg_eps)[None, :])
    return R0[0], t0[0]


def register_warm(params, src_tree: OracleTree, tgt_tree: OracleTree, tgt_xyz, reg_eps: float, lambda_c=0.01,
                  max_iters=30, coarse_levels=2):
    """Warm-started registration of tgt_xyz onto src_tree with the plain
    method from the identity as the arbiter.  Returns the registration dict of
    the kept run plus ``fallback`` (True when the identity start won) and the
    network's start (R0, t0)."""
    R0, t0 = initial_pose(params, src_tree, tgt_tree, reg_eps)
    start = (R0, t0)
    if coarse_levels and src_tree.levels > coarse_levels:
        rc = register(cut(src_tree, coarse_levels), tgt_xyz, R0=R0, t0=t0, max_iters=max_iters, lambda_c=lambda_c)
        if rc["status"] == 0:
            R0, t0 = rc["R"], rc["t"]
    warm = register(src_tree, tgt_xyz, R0=R0, t0=t0, max_iters=max_iters, lambda_c=lambda_c)
    plain = register(src_tree, tgt_xyz, max_iters=max_iters, lambda_c=lambda_c)
    use_plain = (warm["status"] != 0) or (plain["status"] == 0 and warm["loglik"] < plain["loglik"])
    out = dict(plain if use_plain else warm)
    out["fallback"] = bool(use_plain)
    out["R0"], out["t0"] = start
    return out
