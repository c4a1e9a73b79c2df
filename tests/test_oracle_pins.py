"""Pins of the FP64 oracle against mathematics and independent library routines.

Nothing here compares the oracle with itself: every expected value comes from
numpy / scipy / sklearn, a closed form, brute force, or an invariant that the
paper's definitions imply.
"""

import json
import math
import os
import warnings

import numpy as np
import pytest
from scipy import optimize, stats
from scipy.spatial.transform import Rotation
from scipy.special import logsumexp

from synth import blob_tree_cloud, rotation_from_axis_angle, small_pair

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _unpack(c6):
    c = np.asarray(c6)
    return np.array([[c[0], c[1], c[2]], [c[1], c[3], c[4]], [c[2], c[4], c[5]]])


def _pack(S):
    return np.array([S[0, 0], S[0, 1], S[0, 2], S[1, 1], S[1, 2], S[2, 2]])


def _rand_spd(rng, scales):
    q = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    return q @ np.diag(scales) @ q.T


# --------------------------------------------------------------------------
# constants the paper fixes
# --------------------------------------------------------------------------

def test_paper_constants(oracle_mod):
    g = json.load(open(GOLDEN))
    assert oracle_mod.level_nodes(0) == g["children_per_node"]["value"]
    # the paper counts recursion levels from 1; level index l here holds 8^(l+1) nodes
    for lev, j in g["components_at_recursion_level"]["value"].items():
        assert oracle_mod.level_nodes(int(lev) - 1) == j
    assert oracle_mod.register.__defaults__[3] == g["lambda_c"]["value"]


# --------------------------------------------------------------------------
# eigen-decomposition (Sec. 4.1 complexity test, Eq. 10-11)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_eigh3_matches_numpy(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    scales = [np.exp(rng.uniform(-12, 2, size=3)), [1.0, 0.5, 1e-4], [3.0, 2.0, 1.0]][seed % 3]
    S = _rand_spd(rng, np.sort(scales)[::-1])
    lam, ev = oracle_mod.eigh3(_pack(S))
    w, V = np.linalg.eigh(S)
    np.testing.assert_allclose(lam, w[::-1], rtol=0, atol=1e-13 * w.max())
    for a in range(3):
        v = V[:, 2 - a]
        big = np.argmax(np.abs(v))
        v = v * np.sign(v[big])
        np.testing.assert_allclose(ev[a], v, atol=1e-10)
        assert ev[a][np.argmax(np.abs(ev[a]))] > 0
    np.testing.assert_allclose(ev @ ev.T, np.eye(3), atol=1e-14)


def test_eigh3_repeated_eigenvalue(oracle_mod):
    """With a repeated eigenvalue only the eigenspace is unique: compare projectors."""
    rng = np.random.default_rng(9)
    S = _rand_spd(rng, [1.0, 1.0, 1e-4])
    lam, ev = oracle_mod.eigh3(_pack(S))
    w, V = np.linalg.eigh(S)
    np.testing.assert_allclose(lam, w[::-1], atol=1e-13)
    np.testing.assert_allclose(ev[:2].T @ ev[:2], V[:, 1:] @ V[:, 1:].T, atol=1e-12)
    np.testing.assert_allclose(np.abs(ev[2]), np.abs(V[:, 0]), atol=1e-12)
    np.testing.assert_allclose(ev.T @ np.diag(lam) @ ev, S, atol=1e-14)


def test_complexity_range(oracle_mod):
    rng = np.random.default_rng(1)
    for _ in range(50):
        S = _rand_spd(rng, np.exp(rng.uniform(-8, 1, size=3)))
        lam, _ = oracle_mod.eigh3(_pack(S))
        kappa = lam[2] / lam.sum()
        assert 0.0 <= kappa <= 1.0 / 3.0 + 1e-15


# --------------------------------------------------------------------------
# PCA-octant child initialisation (construction reading)
# --------------------------------------------------------------------------

def test_octant_init_halfnormal_closed_form(oracle_mod):
    rng = np.random.default_rng(3)
    eps = 1e-6
    S = _rand_spd(rng, [0.5, 0.1, 0.01]) + eps * np.eye(3)
    mu = rng.normal(size=3)
    lam, ev = oracle_mod.eigh3(_pack(S))
    cm, cc = oracle_mod.octant_init(mu, lam, ev, eps)
    hn_mean, hn_var = stats.halfnorm.mean(), stats.halfnorm.var()
    for k in range(8):
        s = np.array([1.0 if ((k >> a) & 1) == 0 else -1.0 for a in range(3)])
        m = mu + sum(s[a] * hn_mean * math.sqrt(lam[a] - eps) * ev[a] for a in range(3))
        C = sum(hn_var * (lam[a] - eps) * np.outer(ev[a], ev[a]) for a in range(3)) + eps * np.eye(3)
        np.testing.assert_allclose(cm[k], m, atol=1e-14)
        np.testing.assert_allclose(_unpack(cc[k]), C, atol=1e-14)


def test_octant_init_monte_carlo(oracle_mod):
    """Children equal the moments of the parent Gaussian restricted to each eigen-octant."""
    rng = np.random.default_rng(4)
    S = _rand_spd(rng, [0.4, 0.09, 0.01])
    mu = np.array([0.3, -0.2, 0.1])
    lam, ev = oracle_mod.eigh3(_pack(S))
    cm, cc = oracle_mod.octant_init(mu, lam, ev, 0.0)
    x = rng.multivariate_normal(mu, S, size=800_000)
    coords = (x - mu) @ ev.T
    octant = ((coords[:, 0] < 0).astype(int) | ((coords[:, 1] < 0).astype(int) << 1) |
              ((coords[:, 2] < 0).astype(int) << 2))
    for k in range(8):
        sel = x[octant == k]
        np.testing.assert_allclose(sel.mean(0), cm[k], atol=4e-3)
        np.testing.assert_allclose(np.cov(sel.T, bias=True), _unpack(cc[k]), atol=3e-3)


# --------------------------------------------------------------------------
# per-parent EM (Eq. 2-3 and the M-step of a Gaussian mixture)
# --------------------------------------------------------------------------

def _sk_em(X, pi, mu, cov, iters, eps):
    from sklearn.mixture import GaussianMixture
    prec = np.array([np.linalg.inv(_unpack(c)) for c in cov])
    gm = GaussianMixture(n_components=8, covariance_type="full", reg_covar=eps, tol=0.0, max_iter=iters,
                         weights_init=np.asarray(pi), means_init=np.asarray(mu), precisions_init=prec,
                         init_params="random", random_state=0)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        gm.fit(X)
    return gm


@pytest.mark.parametrize("seed", [0, 1])
def test_em_matches_sklearn(oracle_mod, seed):
    p = small_pair(seed, n=3000)
    X = p.src.T.astype(np.float64)
    eps = 1e-6
    root = oracle_mod.build_root(p.src, eps)
    cm, cc = oracle_mod.octant_init(root.origin, root.root_lam, root.root_evec, eps)
    pi0 = np.full(8, 0.125)
    out = oracle_mod.em_partition(X, pi0, cm, cc, iters=30, eps=eps, min_mass=1.0)
    assert out["live"].all()
    gm = _sk_em(X, pi0, cm, cc, 30, eps)
    np.testing.assert_allclose(out["pi"], gm.weights_, rtol=1e-9)
    np.testing.assert_allclose(out["mu"], gm.means_, rtol=0, atol=1e-9 * p.extent)
    np.testing.assert_allclose(np.array([_unpack(c) for c in out["cov"]]), gm.covariances_, rtol=1e-7,
                               atol=1e-11)
    np.testing.assert_array_equal(out["label"], gm.predict(X))


def test_em_responsibilities_and_mass(oracle_mod):
    p = small_pair(7, n=2000)
    X = p.src.T.astype(np.float64)
    root = oracle_mod.build_root(p.src)
    cm, cc = oracle_mod.octant_init(root.origin, root.root_lam, root.root_evec, 1e-6)
    out = oracle_mod.em_partition(X, np.full(8, 0.125), cm, cc, iters=5)
    np.testing.assert_allclose(out["resp"].sum(1), 1.0, atol=1e-15)
    np.testing.assert_allclose(out["nk"].sum(), X.shape[0], rtol=1e-12)
    np.testing.assert_allclose(out["pi"].sum(), 1.0, rtol=1e-14)


def test_em_separated_blobs_one_component_each(oracle_mod):
    """A child that owns one blob reproduces its sample mean and covariance."""
    rng = np.random.default_rng(11)
    signs = np.array([[1 if (k >> a) & 1 == 0 else -1 for a in range(3)] for k in range(8)], float)
    centres = signs * np.array([9.0, 5.0, 2.0])
    blobs = [c + rng.normal(size=(50, 3)) @ (np.diag([0.02, 0.01, 0.005]) @ np.linalg.qr(rng.normal(size=(3, 3)))[0])
             for c in centres]
    X = np.concatenate(blobs)
    xyz = np.ascontiguousarray(X.T.astype(np.float32))
    X = xyz.T.astype(np.float64)
    eps = 1e-6
    root = oracle_mod.build_root(xyz, eps)
    cm, cc = oracle_mod.octant_init(root.origin, root.root_lam, root.root_evec, eps)
    out = oracle_mod.em_partition(X, np.full(8, 0.125), cm, cc, iters=30, eps=eps)
    assert set(np.unique(out["resp"])) <= {0.0, 1.0}
    for k in range(8):
        sel = X[out["label"] == k]
        assert sel.shape[0] == 50
        np.testing.assert_allclose(out["mu"][k], sel.mean(0), atol=1e-12)
        np.testing.assert_allclose(_unpack(out["cov"][k]), np.cov(sel.T, bias=True) + eps * np.eye(3), atol=1e-14)
        assert abs(out["pi"][k] - 0.125) < 1e-15


def test_dead_rule(oracle_mod):
    """Children whose soft mass falls below min_mass die and the rest renormalise."""
    rng = np.random.default_rng(2)
    X = rng.normal(size=(5, 3))
    root_mu = X.mean(0)
    lam, ev = oracle_mod.eigh3(_pack(np.cov(X.T, bias=True) + 1e-6 * np.eye(3)))
    cm, cc = oracle_mod.octant_init(root_mu, lam, ev, 1e-6)
    out = oracle_mod.em_partition(X, np.full(8, 0.125), cm, cc, iters=30, min_mass=1.0)
    assert out["live"].sum() <= 5
    assert abs(out["pi"][out["live"] == 1].sum() - 1.0) < 1e-14
    assert np.all(out["pi"][out["live"] == 0] == 0)


# --------------------------------------------------------------------------
# tree construction
# --------------------------------------------------------------------------

def test_root_stats(oracle_mod):
    p = small_pair(5, n=4000)
    X = p.src.T.astype(np.float64)
    t = oracle_mod.build_root(p.src, 1e-6)
    np.testing.assert_allclose(t.origin, X.mean(0), atol=1e-15)
    np.testing.assert_allclose(_unpack(t.root_cov), np.cov(X.T, bias=True) + 1e-6 * np.eye(3), atol=1e-15)
    lo, hi = X.min(0), X.max(0)
    assert abs(t.extent - np.linalg.norm(hi - lo)) < 1e-15


@pytest.mark.parametrize("seed", [0, 3])
def test_two_level_tree_vs_sklearn(oracle_mod, seed):
    """Brute-force EM on a 2-level tree: every level-0 partition re-fit by sklearn."""
    p = small_pair(seed, n=2500)
    X = p.src.T.astype(np.float64)
    eps = 1e-6
    tree, labels = oracle_mod.build_tree(p.src, 2, iters=30, eps=eps)
    checked = 0
    for k in range(8):
        if not tree.live[k] or not tree.has_children[k]:
            continue
        sel = labels[0] == k
        Xp = X[sel]
        if Xp.shape[0] < 60:
            continue
        cm, cc = oracle_mod.octant_init(tree.mu[k], tree.lam[k], tree.evec[k], eps)
        gm = _sk_em(Xp, np.full(8, 0.125), cm, cc, 30, eps)
        ch = slice(8 + 8 * k, 16 + 8 * k)
        if not tree.live[ch].all():
            continue  # sklearn has no dead rule
        np.testing.assert_allclose(tree.pi[ch], gm.weights_, rtol=1e-8)
        np.testing.assert_allclose(tree.mu[ch], gm.means_, atol=1e-9 * p.extent)
        np.testing.assert_allclose(np.array([_unpack(c) for c in tree.cov[ch]]), gm.covariances_, rtol=1e-6,
                                   atol=1e-11)
        np.testing.assert_array_equal(labels[1][sel], 8 * k + gm.predict(Xp))
        checked += 1
    assert checked >= 3


def test_tree_invariants(oracle_mod):
    p = small_pair(9, n=6000)
    tree, labels = oracle_mod.build_tree(p.src, 3)
    n = p.src.shape[1]
    assert tree.count[tree.level_slice(0)].sum() == n
    for l in range(1, 3):
        par = tree.level_slice(l - 1)
        with_children = tree.count[par][tree.has_children[par] == 1].sum()
        assert tree.count[tree.level_slice(l)].sum() == with_children
        # each label at level l is a child of the label at level l-1
        m = labels[l] >= 0
        np.testing.assert_array_equal(labels[l][m] // 8, labels[l - 1][m])
    # sibling weights sum to one, global weights are products along the path
    for l in range(3):
        s = tree.level_slice(l)
        pi = tree.pi[s].reshape(-1, 8)
        live_groups = tree.live[s].reshape(-1, 8).any(1)
        np.testing.assert_allclose(pi[live_groups].sum(1), 1.0, atol=1e-13)
    s1 = tree.level_slice(1)
    idx = np.arange(64)
    live = tree.live[s1] == 1
    np.testing.assert_allclose(tree.pig[s1][live], tree.pi[s1][live] * tree.pi[idx[live] // 8], rtol=1e-14)
    assert np.all(tree.kappa[tree.live == 1] <= 1 / 3 + 1e-15)


# --------------------------------------------------------------------------
# registration E-step (Algorithm 1)
# --------------------------------------------------------------------------

def _logpdf_table(tree, Y, nodes):
    return np.stack([math.log(tree.pi[g]) +
                     np.atleast_1d(stats.multivariate_normal(tree.mu[g], _unpack(tree.cov[g])).logpdf(Y))
                     for g in nodes], axis=1)


def test_descent_one_level_bruteforce(oracle_mod):
    p = small_pair(4, n=3000)
    tree, _ = oracle_mod.build_tree(p.src, 1)
    R = rotation_from_axis_angle([0.2, 1.0, -0.3], 0.05)
    t = np.array([0.01, -0.02, 0.015])
    e = oracle_mod.estep(tree, p.tgt, R, t, lambda_c=0.01)
    Y = p.tgt.T.astype(np.float64) @ R.T + t
    live = [g for g in range(8) if tree.live[g]]
    lp = _logpdf_table(tree, Y, live)
    best = np.array(live)[np.argmax(lp, axis=1)]
    np.testing.assert_array_equal(e["stop_node"], best)
    gam = np.exp(lp.max(1) - logsumexp(lp, axis=1))
    # scores reach |s| ~ 1e4 for far points, so FP64 rounding of s is ~1e-12 absolute
    np.testing.assert_allclose(e["gamma"], gam, rtol=1e-9)
    # moments of Algorithm 1 / Eq. 9
    M0 = np.bincount(best, weights=gam, minlength=8)
    M1 = np.stack([np.bincount(best, weights=gam * Y[:, c], minlength=8) for c in range(3)], 1)
    np.testing.assert_allclose(e["bins"][:8, 0], M0, rtol=1e-12)
    np.testing.assert_allclose(e["bins"][:8, 1:4], M1, rtol=1e-10, atol=1e-12)
    np.testing.assert_array_equal(e["bins"][:8, 4], np.bincount(best, minlength=8))
    # log-likelihood of the selected component (global weight) averaged over points
    ll = np.mean([math.log(tree.pig[g]) + stats.multivariate_normal(tree.mu[g], _unpack(tree.cov[g])).logpdf(y)
                  for g, y in zip(best[:400], Y[:400])])
    e400 = oracle_mod.estep(tree, p.tgt[:, :400].copy(), R, t)
    assert abs(e400["loglik"] - ll) < 1e-11


def test_descent_greedy_path_and_limits(oracle_mod):
    p = small_pair(8, n=4000)
    tree, _ = oracle_mod.build_tree(p.src, 3)
    Y = p.tgt.T[:500].astype(np.float64)
    xyz = np.ascontiguousarray(p.tgt[:, :500])
    e = oracle_mod.estep(tree, xyz, lambda_c=0.01)
    # every choice along the path is the most likely live sibling (checked with scipy densities)
    for i in range(0, 500, 7):
        g = int(e["stop_node"][i])
        lev = int(e["stop_level"][i])
        k = g - oracle_mod.level_offset(lev)
        chain = [(lev, k)]
        while lev > 0:
            lev -= 1
            k //= 8
            chain.append((lev, k))
        for lev, k in chain:
            base = oracle_mod.level_offset(lev) + 8 * (k // 8)
            sib = [base + j for j in range(8) if tree.live[base + j]]
            lp = _logpdf_table(tree, Y[i:i + 1], sib)[0]
            assert sib[int(np.argmax(lp))] == oracle_mod.level_offset(lev) + k
        # stop rule: complex node with children below the last level does not stop
        assert tree.kappa[g] <= 0.01 or e["stop_level"][i] == 2 or not tree.has_children[g]
    # lambda_c = 1 stops every point at level 0; lambda_c = 0 reaches leaves
    e1 = oracle_mod.estep(tree, xyz, lambda_c=1.0)
    assert np.all(e1["stop_level"] == 0)
    live0 = [g for g in range(8) if tree.live[g]]
    np.testing.assert_array_equal(e1["stop_node"], np.array(live0)[np.argmax(_logpdf_table(tree, Y, live0), 1)])
    e0 = oracle_mod.estep(tree, xyz, lambda_c=0.0)
    for g, lev in zip(e0["stop_node"], e0["stop_level"]):
        assert lev == 2 or not tree.has_children[g]
    # conservation and range of the weights
    assert e["bins"][:, 4].sum() == 500
    assert np.all(e["gamma"] <= 1.0) and np.all(e["gamma"] >= 1.0 / 8 - 1e-15)
    assert np.all(tree.live[e["stop_node"]] == 1)


# --------------------------------------------------------------------------
# M-step (Eq. 10-16)
# --------------------------------------------------------------------------

def _random_state(oracle_mod, seed):
    p = small_pair(seed, n=4000)
    tree, _ = oracle_mod.build_tree(p.src, 2)
    R = rotation_from_axis_angle([1, -0.5, 0.2], 0.03)
    t = np.array([0.01, 0.0, -0.02])
    e = oracle_mod.estep(tree, p.tgt, R, t)
    return tree, e, p.tgt.shape[1]


def test_normal_equations_inverse_form(oracle_mod):
    """Eq. 10: the eigen form equals the Sigma^-1 form, H = sum pi* [C;I] S^-1 [C;I]^T."""
    tree, e, n = _random_state(oracle_mod, 2)
    H, g = oracle_mod.normal_equations(tree, e["bins"], n)
    H2 = np.zeros((6, 6))
    g2 = np.zeros(6)
    for j in np.nonzero(e["bins"][:, 0] > 0)[0]:
        b = e["bins"][j]
        pis = b[0] / n
        ms = b[1:4] / b[0]
        c = ms - tree.origin
        Cx = np.array([[0, -c[2], c[1]], [c[2], 0, -c[0]], [-c[1], c[0], 0]])
        A = np.vstack([Cx, np.eye(3)])        # rows: [c x n ; n] = A n
        Si = np.linalg.inv(_unpack(tree.cov[j]))
        H2 += pis * A @ Si @ A.T
        g2 -= pis * A @ Si @ (ms - tree.mu[j])
    np.testing.assert_allclose(H, H2, rtol=1e-9, atol=1e-9 * np.abs(H2).max())
    np.testing.assert_allclose(g, g2, rtol=1e-9, atol=1e-9 * np.abs(g2).max())


def test_stacked_system_lstsq(oracle_mod):
    """Eq. 16: the 3J x 6 weighted system solved by lstsq equals the normal-equation solve."""
    tree, e, n = _random_state(oracle_mod, 3)
    H, g = oracle_mod.normal_equations(tree, e["bins"], n)
    rows, rhs = [], []
    for j in np.nonzero(e["bins"][:, 0] > 0)[0]:
        b = e["bins"][j]
        ms = b[1:4] / b[0]
        for l in range(3):
            nv = tree.evec[j, l]
            w = math.sqrt(b[0] / n / tree.lam[j, l])
            rows.append(w * np.concatenate([np.cross(ms - tree.origin, nv), nv]))
            rhs.append(w * (nv @ (tree.mu[j] - ms)))      # residual sign of Eq. 14 reversed (increment form)
    x_ls = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
    st, R, t, x = oracle_mod.solve_update(H, g, tree.origin, np.eye(3), np.zeros(3))
    assert st == 0
    np.testing.assert_allclose(x, x_ls, rtol=1e-8, atol=1e-12)
    # the update is an exact rotation
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
    assert abs(np.linalg.det(R) - 1) < 1e-14
    np.testing.assert_allclose(Rotation.from_matrix(R).as_rotvec(), x[:3], atol=1e-12)


def test_singular_system(oracle_mod):
    st, *_ = oracle_mod.solve_update(np.zeros((6, 6)), np.zeros(6), np.zeros(3), np.eye(3), np.zeros(3))
    assert st == -6


def _hand_tree(oracle_mod, mus, covs, pis):
    t = oracle_mod.OracleTree(1)
    for k in range(8):
        t.live[k] = 1
        t.pi[k] = pis[k]
        t.pig[k] = pis[k]
        t.mu[k] = mus[k]
        t.cov[k] = _pack(covs[k])
        lam, ev = oracle_mod.eigh3(t.cov[k])
        t.lam[k] = lam
        t.evec[k] = ev
        t.kappa[k] = lam[2] / lam.sum()
        t.count[k] = 1
    t.origin = np.mean(mus, 0)
    t.extent = float(np.linalg.norm(mus.max(0) - mus.min(0)))
    return t


def _fixed_assignment_case(seed, anisotropic):
    rng = np.random.default_rng(seed)
    mus = rng.uniform(-10, 10, size=(8, 3))
    if anisotropic:
        covs = [_rand_spd(rng, [0.5, 0.1, 0.004]) for _ in range(8)]
    else:
        covs = [np.eye(3) * s for s in rng.uniform(0.01, 0.2, size=8)]
    pis = rng.dirichlet(np.ones(8) * 5)
    # target clusters: around a rigid copy of the means, each cluster tight and
    # slightly offset so the optimum is not exact
    Rg = rotation_from_axis_angle(rng.normal(size=3), math.radians(4))
    tg = rng.uniform(-0.2, 0.2, size=3)
    counts = rng.integers(20, 60, size=8)
    pts = []
    for k in range(8):
        c = Rg @ mus[k] + tg + rng.normal(scale=0.05, size=3)
        pts.append(c + rng.normal(scale=0.01, size=(counts[k], 3)))
    tgt = np.ascontiguousarray(np.concatenate(pts).T.astype(np.float32))
    return mus, covs, pis, tgt, counts


def _eq8_optimum(mus, covs, tgt, counts, x0):
    """Minimise Eq. 8 with the hard assignments by scipy least squares."""
    Y = tgt.T.astype(np.float64)
    ends = np.cumsum(counts)
    means = np.array([Y[e - c:e].mean(0) for e, c in zip(ends, counts)])
    N = Y.shape[0]
    Ls = [np.linalg.cholesky(np.linalg.inv(C)) for C in covs]

    def resid(v):
        R = Rotation.from_rotvec(v[:3]).as_matrix()
        out = []
        for k in range(8):
            d = R @ means[k] + v[3:] - mus[k]
            out.append(math.sqrt(counts[k] / N) * (Ls[k].T @ d))
        return np.concatenate(out)

    sol = optimize.least_squares(resid, x0, xtol=1e-15, ftol=1e-15, gtol=1e-15, method="lm")
    return Rotation.from_rotvec(sol.x[:3]).as_matrix(), sol.x[3:], means


def test_fixed_point_isotropic_is_weighted_procrustes(oracle_mod):
    mus, covs, pis, tgt, counts = _fixed_assignment_case(5, anisotropic=False)
    tree = _hand_tree(oracle_mod, mus, covs, pis)
    r = oracle_mod.register(tree, tgt, max_iters=100, tol_rot=1e-14, tol_trans=1e-14)
    assert r["status"] == 0
    Y = tgt.T.astype(np.float64)
    ends = np.cumsum(counts)
    q = np.array([Y[e - c:e].mean(0) for e, c in zip(ends, counts)])
    w = counts / counts.sum() / np.array([C[0, 0] for C in covs])
    cq = (w[:, None] * q).sum(0) / w.sum()
    cm = (w[:, None] * mus).sum(0) / w.sum()
    rot, _ = Rotation.align_vectors(mus - cm, q - cq, weights=w)
    Rp = rot.as_matrix()
    tp = cm - Rp @ cq
    np.testing.assert_allclose(r["R"], Rp, atol=1e-10)
    np.testing.assert_allclose(r["t"], tp, atol=1e-9)


def test_fixed_point_anisotropic_matches_minimiser(oracle_mod):
    mus, covs, pis, tgt, counts = _fixed_assignment_case(6, anisotropic=True)
    tree = _hand_tree(oracle_mod, mus, covs, pis)
    r = oracle_mod.register(tree, tgt, max_iters=200, tol_rot=1e-14, tol_trans=1e-14)
    assert r["status"] == 0
    x0 = np.concatenate([Rotation.from_matrix(r["R"]).as_rotvec(), r["t"]]) + 1e-3
    Rm, tm, _ = _eq8_optimum(mus, covs, tgt, counts, x0)
    np.testing.assert_allclose(r["R"], Rm, atol=1e-8)
    np.testing.assert_allclose(r["t"], tm, atol=1e-7)


def test_exact_recovery_blob_tree(oracle_mod):
    """Noise-free rigid copy of 64 separated blobs: the pose is recovered exactly."""
    xyz, ids, _ = blob_tree_cloud(0)
    tree, labels = oracle_mod.build_tree(xyz, 2)
    for b in range(64):
        assert len(set(labels[1][ids == b])) == 1
    assert len(set(labels[1])) == 64
    Rg = rotation_from_axis_angle([1, 2, 3], math.radians(5))
    tg = 0.02 * tree.extent * np.array([0.6, -0.3, 0.74])
    tgt = (Rg @ xyz.astype(np.float64) + tg[:, None]).astype(np.float32)
    r = oracle_mod.register(tree, tgt, max_iters=60, tol_rot=1e-13, tol_trans=1e-13)
    assert r["status"] == 0 and r["iters"] < 60
    # against the FP32 target, the fixed point is the Eq. 8 optimum with blob assignments
    order = np.argsort(labels[1], kind="stable")
    counts = np.bincount(labels[1], minlength=64)
    covs = [_unpack(tree.cov[8 + k]) for k in range(64)]
    Y = tgt[:, order]
    Yd = Y.T.astype(np.float64)
    ends = np.cumsum(counts)
    means = np.array([Yd[e - c:e].mean(0) for e, c in zip(ends, counts)])
    N = Yd.shape[0]
    Ls = [np.linalg.cholesky(np.linalg.inv(C)) for C in covs]

    def resid(v):
        R = Rotation.from_rotvec(v[:3]).as_matrix()
        return np.concatenate([math.sqrt(counts[k] / N) * (Ls[k].T @ (R @ means[k] + v[3:] - tree.mu[8 + k]))
                               for k in range(64)])

    x0 = np.concatenate([Rotation.from_matrix(r["R"]).as_rotvec(), r["t"]])
    sol = optimize.least_squares(resid, x0, xtol=1e-15, ftol=1e-15, gtol=1e-15, method="lm")
    np.testing.assert_allclose(r["R"], Rotation.from_rotvec(sol.x[:3]).as_matrix(), atol=1e-9)
    np.testing.assert_allclose(r["t"], sol.x[3:], atol=1e-9 * tree.extent)
    # and the pose is the true one up to the FP32 rounding of the target
    np.testing.assert_allclose(r["R"], Rg.T, atol=1e-6)
    np.testing.assert_allclose(r["t"], -Rg.T @ tg, atol=1e-6 * tree.extent)


def test_equivariance_exact_rotation(oracle_mod):
    """register(G Z2, T0 G^-1) follows the same trajectory as register(Z2, T0) for an exact G."""
    p = small_pair(12, n=3000, max_angle_deg=8)
    tree, _ = oracle_mod.build_tree(p.src, 2)
    G = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])     # exact in FP32
    tgtG = np.ascontiguousarray((G @ p.tgt.astype(np.float64)).astype(np.float32))
    assert np.array_equal(tgtG.astype(np.float64), G @ p.tgt.astype(np.float64))
    a = oracle_mod.register(tree, p.tgt, max_iters=8)
    b = oracle_mod.register(tree, tgtG, R0=G.T, max_iters=8)
    assert a["iters"] == b["iters"]
    np.testing.assert_allclose(b["R"] @ G, a["R"], atol=1e-12)
    np.testing.assert_allclose(b["t"], a["t"], atol=1e-12)
    np.testing.assert_allclose(a["trace"][:, 0], b["trace"][:, 0], rtol=1e-12)


# --------------------------------------------------------------------------
# single-level variant ("GMM J=n", Sec. 5): every component of one level
# --------------------------------------------------------------------------

def test_flat_estep_bruteforce(oracle_mod):
    """Level 1 (64 components) scored exhaustively with scipy densities and global weights."""
    p = small_pair(5, n=2500)
    tree, _ = oracle_mod.build_tree(p.src, 2)
    R = rotation_from_axis_angle([0.4, -1.0, 0.1], 0.04)
    t = np.array([-0.01, 0.02, 0.005])
    e = oracle_mod.estep_flat(tree, 1, p.tgt, R, t)
    Y = p.tgt.T.astype(np.float64) @ R.T + t
    live = [g for g in range(8, 72) if tree.live[g]]
    lp = np.stack([math.log(tree.pig[g]) + stats.multivariate_normal(tree.mu[g], _unpack(tree.cov[g])).logpdf(Y)
                   for g in live], axis=1)
    best = np.array(live)[np.argmax(lp, axis=1)]
    np.testing.assert_array_equal(e["stop_node"], best)
    np.testing.assert_allclose(e["gamma"], np.exp(lp.max(1) - logsumexp(lp, axis=1)), rtol=1e-9)
    srt = np.sort(lp, axis=1)
    np.testing.assert_allclose(e["min_gap"], srt[:, -1] - srt[:, -2], rtol=1e-9, atol=1e-9)
    gam = e["gamma"]
    nn = tree.n_nodes
    np.testing.assert_allclose(e["bins"][:, 0], np.bincount(best, weights=gam, minlength=nn), rtol=1e-12)
    for c in range(3):
        np.testing.assert_allclose(e["bins"][:, 1 + c], np.bincount(best, weights=gam * Y[:, c], minlength=nn),
                                   rtol=1e-10, atol=1e-12)
    np.testing.assert_array_equal(e["bins"][:, 4], np.bincount(best, minlength=nn))
    assert np.all(e["bins"][:8, :] == 0) and np.all(e["bins"][72:, :] == 0)
    ll = np.mean(lp.max(1))   # log(pig) + log N of the chosen component, averaged
    assert abs(e["loglik"] - ll) < 1e-10 * max(1.0, abs(ll))


def test_flat_level0_is_tree_descent_stopped_at_level0(oracle_mod):
    """At level 0 the sibling weights are the global ones and lambda_c = 1 stops every
    point there, so the flat E-step and the tree E-step give the same result."""
    p = small_pair(6, n=3000)
    tree, _ = oracle_mod.build_tree(p.src, 3)
    R = rotation_from_axis_angle([1.0, 0.3, -0.2], 0.02)
    t = np.array([0.003, 0.0, -0.004])
    a = oracle_mod.estep_flat(tree, 0, p.tgt, R, t)
    b = oracle_mod.estep(tree, p.tgt, R, t, lambda_c=1.0)
    np.testing.assert_array_equal(a["stop_node"], b["stop_node"])
    np.testing.assert_allclose(a["gamma"], b["gamma"], rtol=1e-13)
    np.testing.assert_allclose(a["bins"], b["bins"], rtol=1e-13, atol=1e-13)
    assert abs(a["loglik"] - b["loglik"]) < 1e-12


def test_flat_deepest_level_range_and_conservation(oracle_mod):
    p = small_pair(7, n=3000)
    tree, _ = oracle_mod.build_tree(p.src, 3)
    e = oracle_mod.estep_flat(tree, 2, p.tgt)
    J = oracle_mod.level_nodes(2)
    g0 = oracle_mod.level_offset(2)
    nlive = int(tree.live[g0:g0 + J].sum())
    assert np.all((e["stop_node"] >= g0) & (e["stop_node"] < g0 + J))
    assert np.all(tree.live[e["stop_node"]] == 1)
    assert e["bins"][:, 4].sum() == p.tgt.shape[1]
    assert np.all(e["gamma"] <= 1.0) and np.all(e["gamma"] >= 1.0 / nlive - 1e-15)
    # the flat search covers the whole level, so its chosen component scores at least as
    # high as the one the tree descent reaches at that level
    d = oracle_mod.estep(tree, p.tgt, lambda_c=0.0)
    idx = np.nonzero(d["stop_level"] == 2)[0][:200]
    assert len(idx) > 50
    Y = p.tgt.T[idx].astype(np.float64)

    def score(g, y):
        return math.log(tree.pig[g]) + stats.multivariate_normal(tree.mu[g], _unpack(tree.cov[g])).logpdf(y)

    worse = 0
    for i, y in zip(idx, Y):
        sf, st = score(e["stop_node"][i], y), score(d["stop_node"][i], y)
        assert sf >= st - 1e-9
        worse += sf > st + 1e-9
    assert worse > 0   # and the greedy descent misses the best component for some points
    with pytest.raises(RuntimeError):
        oracle_mod.estep_flat(tree, 3, p.tgt)


def test_flat_exact_recovery_blob_tree(oracle_mod):
    """Noise-free rigid copy of 64 separated blobs registered against level 1 alone."""
    xyz, ids, _ = blob_tree_cloud(1)
    tree, labels = oracle_mod.build_tree(xyz, 2)
    Rg = rotation_from_axis_angle([-1, 2, 0.5], math.radians(4))
    tg = 0.015 * tree.extent * np.array([-0.3, 0.8, 0.5])
    tgt = (Rg @ xyz.astype(np.float64) + tg[:, None]).astype(np.float32)
    r = oracle_mod.register_flat(tree, 1, tgt, max_iters=60, tol_rot=1e-13, tol_trans=1e-13)
    assert r["status"] == 0 and r["iters"] < 60
    np.testing.assert_allclose(r["R"], Rg.T, atol=1e-6)
    np.testing.assert_allclose(r["t"], -Rg.T @ tg, atol=1e-6 * tree.extent)


# --------------------------------------------------------------------------
# trajectory of frame-to-frame registrations (Sec. 6 LiDAR experiment)
# --------------------------------------------------------------------------

def test_compose_chain_recovers_absolute_poses(oracle_mod):
    """Relative transforms taken from known absolute poses (general, non-commuting
    rotations) chain back to those poses; frame 0 is the identity."""
    rng = np.random.default_rng(3)
    F = 7
    R_abs = np.stack([np.eye(3)] + [Rotation.random(random_state=int(s)).as_matrix()
                                    for s in rng.integers(0, 1 << 30, F - 1)])
    t_abs = np.vstack([np.zeros(3), rng.normal(size=(F - 1, 3))])
    R_rel = np.stack([R_abs[k].T @ R_abs[k + 1] for k in range(F - 1)])
    t_rel = np.stack([R_abs[k].T @ (t_abs[k + 1] - t_abs[k]) for k in range(F - 1)])
    Ra, ta = oracle_mod.compose_chain(R_rel, t_rel)
    np.testing.assert_allclose(Ra, R_abs, atol=1e-12)
    np.testing.assert_allclose(ta, t_abs, atol=1e-12)
    # a point seen from frame F-1 lands where the chain of frame changes puts it
    p = rng.normal(size=3)
    q = p
    for k in range(F - 2, -1, -1):
        q = R_rel[k] @ q + t_rel[k]
    np.testing.assert_allclose(Ra[-1] @ p + ta[-1], q, atol=1e-12)


def test_sequence_ground_truth_is_consistent():
    """The scan sequence's poses put the sweeps of one static scene on top of
    each other: frame-1 points mapped into frame 0 lie close to frame-0 points,
    much closer than with the motion left out."""
    from scipy.spatial import cKDTree
    from synth import lidar_sequence
    q = lidar_sequence(4, frames=2, rings=16, azimuths=600)
    np.testing.assert_allclose(q.R_abs[0], np.eye(3))
    np.testing.assert_allclose(q.t_abs[0], 0.0)
    p0 = q.clouds[:, :q.offsets[1]].T.astype(np.float64)
    p1 = q.clouds[:, q.offsets[1]:].T.astype(np.float64)
    near = p1[np.linalg.norm(p1, axis=1) < 15.0]
    kd = cKDTree(p0)
    d_true = kd.query(near @ q.R_abs[1].T + q.t_abs[1])[0]
    d_none = kd.query(near)[0]
    assert np.median(d_true) < 0.1 and np.median(d_none) > 2 * np.median(d_true)


# --------------------------------------------------------------------------
# soft multi-path E-step (Sec. 4.1: a parent's expectation is the sum of its
# children's; branches below a threshold are pruned)
# --------------------------------------------------------------------------

def _path_expectations(tree, Y, levels):
    """Brute force with scipy densities: every node's path expectation (the
    product of posteriors among siblings with sibling weights pi)."""
    E = np.zeros((Y.shape[0], tree.n_nodes))
    for l in range(levels):
        g0 = oracle_level_offset(l)
        for grp in range(8 ** l):
            base = g0 + 8 * grp
            kids = [base + k for k in range(8) if tree.live[base + k]]
            if not kids:
                continue
            lp = np.stack([math.log(tree.pi[g]) + stats.multivariate_normal(tree.mu[g], _unpack(tree.cov[g])).logpdf(Y)
                           for g in kids], axis=1)
            post = np.exp(lp - logsumexp(lp, axis=1, keepdims=True))
            parent = 1.0 if l == 0 else E[:, oracle_level_offset(l - 1) + grp]
            for j, g in enumerate(kids):
                E[:, g] = parent * post[:, j]
    return E


def oracle_level_offset(l):
    return (8 ** (l + 1) - 8) // 7


def test_soft_estep_unpruned_leaves_bruteforce(oracle_mod):
    """tau -> 0, lambda_c = 0 on a 2-level tree: every point reaches every leaf
    with the product of its two sibling posteriors; the mass is conserved."""
    p = small_pair(21, n=1500)
    tree, _ = oracle_mod.build_tree(p.src, 2)
    R = rotation_from_axis_angle([0.1, 1.0, 0.3], 0.03)
    t = np.array([0.01, 0.0, -0.01])
    e = oracle_mod.estep_soft(tree, p.tgt, R, t, lambda_c=0.0, tau=1e-300)
    Y = p.tgt.T.astype(np.float64) @ R.T + t
    E = _path_expectations(tree, Y, 2)
    leaves = [g for g in range(8, 72) if tree.live[g]]
    np.testing.assert_allclose(e["bins"][leaves, 0], E[:, leaves].sum(0), rtol=1e-9, atol=1e-12)
    for c in range(3):
        np.testing.assert_allclose(e["bins"][leaves, 1 + c], (E[:, leaves] * Y[:, [c]]).sum(0), rtol=1e-8,
                                   atol=1e-10)
    np.testing.assert_allclose(e["bins"][:, 4], e["bins"][:, 0])
    assert abs(e["bins"][:, 0].sum() - Y.shape[0]) < 1e-9
    assert not np.any(e["bins"][:8])


def test_soft_estep_pruning_bruteforce(oracle_mod):
    """tau = 0.05: a leaf receives a point exactly when its own expectation and
    its parent's are at least tau (expectations only shrink down a path)."""
    p = small_pair(22, n=1500)
    tree, _ = oracle_mod.build_tree(p.src, 2)
    tau = 0.05
    e = oracle_mod.estep_soft(tree, p.tgt, lambda_c=0.0, tau=tau)
    Y = p.tgt.T.astype(np.float64)
    E = _path_expectations(tree, Y, 2)
    M0 = np.zeros(tree.n_nodes)
    cnt = np.zeros(Y.shape[0], int)
    for g in range(8, 72):
        if not tree.live[g]:
            continue
        par = (g - 8) // 8
        ok = (E[:, par] >= tau) & (E[:, g] >= tau)
        M0[g] = E[ok, g].sum()
        cnt += ok
    far = e["margin"] > 1e-6
    assert far.mean() > 0.95
    np.testing.assert_allclose(e["bins"][8:72, 0], M0[8:72], rtol=1e-8, atol=1e-8)
    np.testing.assert_array_equal(e["stops"][far], cnt[far])
    assert e["bins"][:, 0].sum() < Y.shape[0]


def test_soft_estep_stops_at_level0_is_soft_posterior(oracle_mod):
    """lambda_c = 1 stops every followed node at level 0: the masses are the
    sums of the level-0 posteriors (the E-step of a soft 8-component EM)."""
    p = small_pair(23, n=1500)
    tree, _ = oracle_mod.build_tree(p.src, 3)
    e = oracle_mod.estep_soft(tree, p.tgt, lambda_c=1.0, tau=1e-300)
    Y = p.tgt.T.astype(np.float64)
    E = _path_expectations(tree, Y, 1)
    np.testing.assert_allclose(e["bins"][:8, 0], E[:, :8].sum(0), rtol=1e-9, atol=1e-12)
    assert not np.any(e["bins"][8:])
    # every level-0 node whose posterior does not underflow is reached
    reach = (E[:, :8] >= 1e-300).sum(1)
    np.testing.assert_array_equal(e["stops"], reach)
    assert reach.max() == int(np.sum(tree.live[:8]))


def test_soft_register_exact_recovery_blob_tree(oracle_mod):
    xyz, ids, _ = blob_tree_cloud(2)
    tree, _ = oracle_mod.build_tree(xyz, 2)
    Rg = rotation_from_axis_angle([2, -1, 0.5], math.radians(4))
    tg = 0.015 * tree.extent * np.array([0.4, 0.2, -0.7])
    tgt = (Rg @ xyz.astype(np.float64) + tg[:, None]).astype(np.float32)
    r = oracle_mod.register_soft(tree, tgt, lambda_c=0.01, tau=0.01, max_iters=60, tol_rot=1e-13, tol_trans=1e-13)
    assert r["status"] == 0 and r["iters"] < 60
    np.testing.assert_allclose(r["R"], Rg.T, atol=1e-6)
    np.testing.assert_allclose(r["t"], -Rg.T @ tg, atol=1e-6 * tree.extent)


# --------------------------------------------------------------------------
# learned warm start: canonical frame, features, start pose (oracle.warm)
# --------------------------------------------------------------------------

def _warm_hand_tree(oracle_mod, R=np.eye(3), t=np.zeros(3)):
    """A 2-level tree set by hand: root covariance R diag(4, 1, 0.25) R^T + eps,
    origin R (1, 2, 3) + t, one live level-1 node (index 5) with weight 0.1,
    mean R (origin offset (0.5, -0.25, 2)) + origin, covariance
    R diag(0.04, 0.01, 0.09) R^T."""
    eps = 1e-6
    tr = oracle_mod.OracleTree(2)
    C = R @ np.diag([4.0, 1.0, 0.25]) @ R.T + eps * np.eye(3)
    tr.root_cov = np.array([C[0, 0], C[0, 1], C[0, 2], C[1, 1], C[1, 2], C[2, 2]])
    lam, ev = oracle_mod.eigh3(tr.root_cov)
    tr.root_lam, tr.root_evec = lam, ev
    tr.origin = R @ np.array([1.0, 2.0, 3.0]) + t
    g = oracle_mod.level_offset(1) + 5
    tr.live[g] = 1
    tr.pig[g] = 0.1
    tr.mu[g] = tr.origin + R @ np.array([0.5, -0.25, 2.0])
    S = R @ np.diag([0.04, 0.01, 0.09]) @ R.T
    tr.cov[g] = [S[0, 0], S[0, 1], S[0, 2], S[1, 1], S[1, 2], S[2, 2]]
    return tr, eps


def test_warm_features_of_a_hand_built_tree(oracle_mod):
    """In the tree's own principal axes the node's feature row is, by hand,
    (0.1, (0.5, -0.25, 2) / s, 0.04 / s^2, 0, 0, 0.01 / s^2, 0, 0.09 / s^2)
    with s = sqrt(4 + 1 + 0.25); every dead node is zeros; the same tree
    rotated and moved gives the same features."""
    from oracle import warm
    tr, eps = _warm_hand_tree(oracle_mod)
    f = warm.features(tr, eps)
    s = np.sqrt(5.25)
    ref = np.zeros(640)
    ref[50:60] = [0.1, 0.5 / s, -0.25 / s, 2.0 / s, 0.04 / s ** 2, 0.0, 0.0, 0.01 / s ** 2, 0.0, 0.09 / s ** 2]
    np.testing.assert_allclose(f, ref, atol=1e-12)
    fr = warm.canonical_frame(tr, eps)
    np.testing.assert_allclose(fr[:9].reshape(3, 3), np.eye(3), atol=1e-12)
    np.testing.assert_allclose(fr[9:], [1.0, 2.0, 3.0, s], atol=1e-12)
    R = rotation_from_axis_angle([1.0, 1.0, 1.0], np.radians(10.0))
    tr2, _ = _warm_hand_tree(oracle_mod, R, np.array([0.3, -2.0, 5.0]))
    np.testing.assert_allclose(warm.features(tr2, eps), ref, atol=1e-12)


def test_warm_frame_of_a_built_tree(oracle_mod):
    """On a built tree the frame is a proper rotation that diagonalises the
    root covariance, c is the centroid and s the RMS distance to it."""
    from oracle import warm
    p = small_pair(71, n=3000)
    tr, _ = oracle_mod.build_tree(p.src, 2, eps=1e-6)
    fr = warm.canonical_frame(tr, 1e-6)
    E = fr[:9].reshape(3, 3)
    assert abs(np.linalg.det(E) - 1.0) < 1e-12
    np.testing.assert_allclose(E @ E.T, np.eye(3), atol=1e-12)
    x = p.src.astype(np.float64)
    c = x.mean(1)
    S = np.cov(x, bias=True)
    D = E @ S @ E.T
    assert np.abs(D - np.diag(np.diag(D))).max() < 1e-12 * np.abs(D).max()
    np.testing.assert_allclose(fr[9:12], c, atol=1e-12)
    assert abs(fr[12] - np.sqrt(np.mean(np.sum((x - c[:, None]) ** 2, 0)))) < 1e-12


def test_warm_identity_head_maps_a_rotated_copy_back(oracle_mod):
    """A network whose output is the identity in canonical coordinates (zero
    weights, last bias (1,0,0, 0,1,0, 0,0,0)) starts a pair from the
    transform between the two clouds' frames.  For an exact rigid copy,
    target = R_g source + t_g, with a rotation small enough to keep the
    eigenvector signs, that start is exactly the inverse motion."""
    from oracle import mlp, warm
    p = small_pair(72, n=4000)
    src = p.src.astype(np.float64)
    Rg = rotation_from_axis_angle([0.3, -0.5, 0.8], np.radians(6.0))
    tg = np.array([0.05, -0.02, 0.03])
    tgt = (Rg @ src + tg[:, None])
    ts, _ = oracle_mod.build_tree(p.src, 2, eps=1e-6)
    tt, _ = oracle_mod.build_tree(tgt.astype(np.float32), 2, eps=1e-6)
    params = np.zeros(mlp.param_count())
    params[-9:] = [1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0]
    R0, t0 = warm.initial_pose(params, ts, tt, 1e-6)
    # tgt was rounded to FP32 before its tree was built: 1e-7 relative
    np.testing.assert_allclose(R0, Rg.T, atol=1e-6)
    np.testing.assert_allclose(t0, -Rg.T @ tg, atol=1e-6)
