"""Shared helpers of the GPU tests (conversion between the library's export
and the oracle's tree layout; seeded inputs)."""

import numpy as np

FIELDS = ("live", "has_children", "count", "pi", "pig", "mu", "cov", "lam", "evec", "kappa")


def to_oracle(oracle_mod, host):
    ot = oracle_mod.OracleTree(host["levels"])
    for k in FIELDS:
        getattr(ot, k)[...] = host[k]
    ot.origin = np.array(host["origin"], dtype=np.float64)
    ot.extent = float(host["extent"])
    ot.n_points = int(host["n_points"])
    return ot


def gpu_bins_from_oracle(tree_host, obins):
    """Oracle bins (M0, M1 absolute, cnt, sum d2) -> library layout (M0, D about mu, cnt, sum d2)."""
    b = np.zeros_like(obins)
    b[:, 0] = obins[:, 0]
    b[:, 1:4] = obins[:, 1:4] - obins[:, :1] * tree_host["mu"]
    b[:, 4:6] = obins[:, 4:6]
    return b


def rel_err(a, b, floor):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def compare_build_levels(oracle_mod, host, glab, src, L, eps, mm, iters, tol, log, min_parent=0):
    """Each level of a GPU tree against the oracle's EM run from the GPU's parent level.

    A sibling group whose set of live children differs between the two (a
    child's soft mass crossed min_mass at a different iteration in FP32 and
    FP64) is a discrete divergence, like a near tie: it is counted, required to
    be rare, and excluded from the parameter comparison.  Sibling groups whose
    parent holds fewer than ``min_parent`` points are only checked for being a
    valid mixture, and nodes of fewer than min_parent / 4 points are left out
    of the parameter comparison (after many EM iterations such groups amplify
    rounding without bound).  Returns the largest errors seen (pi, mu / extent,
    cov / trace)."""
    root = oracle_mod.build_root(src, eps, levels=L)
    np.testing.assert_allclose(host["origin"], root.origin, rtol=0, atol=1e-12 * host["extent"])
    assert abs(host["extent"] - root.extent) <= 1e-12 * root.extent
    worst = dict(pi=0.0, mu=0.0, cov=0.0)
    for l in range(L):
        ot = to_oracle(oracle_mod, host)
        ot.root_cov, ot.root_lam, ot.root_evec = root.root_cov, root.root_lam, root.root_evec
        lab = glab.copy()
        if l + 1 < L:
            lab[l + 1:] = -1
        oracle_mod.build_level(ot, src, lab, l, iters=iters, eps=eps, min_mass=mm)
        sl = ot.level_slice(l)
        live_g = host["live"][sl].reshape(-1, 8)
        live_o = ot.live[sl].reshape(-1, 8)
        populated = (live_g.any(1) | live_o.any(1))
        pcount = host["count"][ot.level_slice(l - 1)] if l > 0 else np.array([src.shape[1]])
        small = pcount < min_parent
        if small.any():
            # validity of the small groups: live weights sum to one, SPD covariances, finite means
            for gi in np.flatnonzero(small & live_g.any(1)):
                idx = sl.start + 8 * gi + np.flatnonzero(live_g[gi])
                assert abs(host["pi"][idx].sum() - 1.0) < 1e-9
                assert np.all(host["lam"][idx] > 0) and np.all(np.isfinite(host["mu"][idx]))
            log(f"    {small.sum()} sibling groups with parents of < {min_parent} points: validity only")
        diverged = np.any(live_g != live_o, axis=1) & populated & ~small
        # nodes of fewer than min_parent / 4 points are as ill-conditioned as small groups
        keep = np.repeat(~diverged & ~small, 8) & (host["live"][sl] == 1) & (host["count"][sl] >= min_parent // 4)
        e_pi = np.abs(host["pi"][sl][keep] - ot.pi[sl][keep]) / ot.pi[sl][keep]
        e_mu = np.abs(host["mu"][sl][keep] - ot.mu[sl][keep]).max(1) / host["extent"]
        tr = ot.cov[sl][keep][:, [0, 3, 5]].sum(1)
        e_cov = np.abs(host["cov"][sl][keep] - ot.cov[sl][keep]).max(1) / tr
        e_k = np.abs(host["kappa"][sl][keep] - ot.kappa[sl][keep])
        m = glab[l] >= 0
        grp = np.where(m, glab[l] // 8, 0)
        in_div = m & (diverged[grp] | small[grp])
        mis = (glab[l] != lab[l]) & ~in_div
        if diverged.any():
            pc = host["count"][ot.level_slice(l - 1)][diverged] if l > 0 else [src.shape[1]]
            log(f"    diverged groups {diverged.sum()}/{populated.sum()} (parent sizes {list(pc)[:8]})")
        mx = lambda a: float(a.max()) if a.size else 0.0
        log(f"  level {l}: live {host['live'][sl].sum()}/{ot.live[sl].sum()}  pi {mx(e_pi):.1e} mu {mx(e_mu):.1e} "
            f"cov {mx(e_cov):.1e} kappa {mx(e_k):.1e}  label mismatches {mis.sum()} ({mis.mean():.1e})")
        if e_pi.size:
            i = int(np.argmax(e_pi))
            log(f"    worst pi node {np.flatnonzero(keep)[i] + sl.start}: gpu {host['pi'][sl][keep][i]:.9e} "
                f"oracle {ot.pi[sl][keep][i]:.9e} count {host['count'][sl][keep][i]}")
        worst = dict(pi=max(worst["pi"], mx(e_pi)), mu=max(worst["mu"], mx(e_mu)), cov=max(worst["cov"], mx(e_cov)))
        assert diverged.sum() <= max(2, 0.01 * populated.sum())
        assert mx(e_pi) < tol["pi"] and mx(e_mu) < tol["mu"] and mx(e_cov) < tol["cov"], (l, mx(e_pi), mx(e_mu),
                                                                                          mx(e_cov))
        assert mis.mean() < 1e-3
    return worst
