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


# a point's label may differ from the oracle's after one EM iteration only
# where the oracle's two best sibling scores (natural log units) are this close
LABEL_FLAG_GAP = 1e-4


def _node_score(ot, g, pts):
    """FP64 score log pi - log det(Sigma) / 2 - d^T Sigma^-1 d / 2 of points
    pts (m, 3) under node g of an oracle tree (-inf for a dead node)."""
    if not ot.live[g]:
        return np.full(len(pts), -np.inf)
    c = ot.cov[g]
    C = np.array([[c[0], c[1], c[2]], [c[1], c[3], c[4]], [c[2], c[4], c[5]]])
    d = pts - ot.mu[g]
    return (np.log(ot.pi[g]) - 0.5 * np.linalg.slogdet(C)[1]
            - 0.5 * np.einsum("ij,ij->i", d, np.linalg.solve(C, d.T).T))


def _sibling_gap(ot, sl, src, lab_o, lab_g, rows_mask):
    """|score(oracle label) - score(GPU label)| under the oracle's parameters,
    for the points of rows_mask (labels are indices inside the level)."""
    rows = np.flatnonzero(rows_mask)
    pts = src[:, rows].astype(np.float64).T
    out = np.zeros(len(rows))
    for i in range(len(rows)):
        a = _node_score(ot, sl.start + lab_o[rows[i]], pts[i:i + 1])[0]
        b = _node_score(ot, sl.start + lab_g[rows[i]], pts[i:i + 1])[0]
        out[i] = abs(a - b)
    return out


def compare_finalize(host, ot, sl, keep, tol, log):
    """Node finalize outputs of the kept nodes of one level against the oracle
    run from the same parents: eigenvalues (relative to the trace), eigenvectors
    under the same sign rule (each axis where its eigenvalue is separated from
    the others well beyond the covariance difference), global weights."""
    lam_g, lam_o = host["lam"][sl][keep], ot.lam[sl][keep]
    out = dict(lam=0.0, evec=0.0, pig=0.0)
    if not keep.any():
        return out
    assert np.all(lam_g[:, 0] >= lam_g[:, 1]) and np.all(lam_g[:, 1] >= lam_g[:, 2]) and np.all(lam_g[:, 2] > 0)
    tr = lam_o.sum(1)
    e_lam = np.abs(lam_g - lam_o).max(1) / tr
    out["lam"] = float(e_lam.max())
    # an eigenvalue moves by at most the spectral norm of the covariance
    # difference, at most 3x its largest entry
    assert out["lam"] < 3 * tol["cov"], out["lam"]
    e_pig = np.abs(host["pig"][sl][keep] - ot.pig[sl][keep]) / ot.pig[sl][keep]
    out["pig"] = float(e_pig.max())
    assert out["pig"] < tol["pi"] * 1.01 + 1e-12, out["pig"]
    ev_g, ev_o = host["evec"][sl][keep], ot.evec[sl][keep]
    dcov = np.abs(host["cov"][sl][keep] - ot.cov[sl][keep]).max(1) + 1e-15 * tr
    # GPU sign rule: the largest-magnitude component of each eigenvector is positive
    big = np.take_along_axis(ev_g, np.abs(ev_g).argmax(2)[..., None], 2)[..., 0]
    assert np.all(big > 0)
    for a in range(3):
        others = [b for b in range(3) if b != a]
        gap = np.min(np.abs(lam_o[:, [a]] - lam_o[:, others]), axis=1)
        sep = gap > 1e3 * dcov
        if not sep.any():
            continue
        # where the oracle's two largest components nearly tie in magnitude the
        # sign rule may pick either sign: compare up to sign there
        mag = np.sort(np.abs(ev_o[:, a, :]), axis=1)
        loose = (mag[:, 2] - mag[:, 1]) < 1e3 * dcov / np.maximum(gap, 1e-300)
        d_same = np.linalg.norm(ev_g[:, a, :] - ev_o[:, a, :], axis=1)
        d_flip = np.linalg.norm(ev_g[:, a, :] + ev_o[:, a, :], axis=1)
        d = np.where(loose, np.minimum(d_same, d_flip), d_same)
        bound = 10.0 * dcov / np.maximum(gap, 1e-300)
        assert np.all(d[sep] <= bound[sep] + 1e-12), (a, float((d[sep] / (bound[sep] + 1e-12)).max()))
        out["evec"] = max(out["evec"], float(d[sep].max()))
    return out


def check_finalize_against_eigh3(oracle_mod, host, log):
    """Unit parity of node finalize: the oracle's Jacobi eigen-decomposition of
    the GPU's own exported (regularised) covariances reproduces the GPU's
    eigenvalues, eigenvectors and complexity kappa = lam3 / sum(lam) to ~1e-12
    (both are FP64).  Global weights are the product of the weights down the
    path."""
    live = np.flatnonzero(host["live"] == 1)
    worst = dict(lam=0.0, evec=0.0, kappa=0.0, pig=0.0)
    for g in live:
        lam, ev = oracle_mod.eigh3(host["cov"][g])
        tr = lam.sum()
        e_l = float(np.abs(host["lam"][g] - lam).max() / tr)
        e_k = abs(host["kappa"][g] - lam[2] / tr)
        worst["lam"] = max(worst["lam"], e_l)
        worst["kappa"] = max(worst["kappa"], e_k)
        assert e_l < 1e-12 and e_k < 1e-12, (g, e_l, e_k)
        for a in range(3):
            gap = min(abs(lam[a] - lam[b]) for b in range(3) if b != a) / tr
            if gap < 1e-6:
                continue
            mag = np.sort(np.abs(ev[a]))
            d = np.linalg.norm(host["evec"][g][a] - ev[a])
            if mag[2] - mag[1] < 1e-9:
                d = min(d, np.linalg.norm(host["evec"][g][a] + ev[a]))
            worst["evec"] = max(worst["evec"], d)
            assert d < 1e-12 / gap + 1e-13, (g, a, d, gap)
    # global weight = own weight times the parent's global weight
    for l in range(host["levels"]):
        lo = (8 ** (l + 1) - 8) // 7
        n = 8 ** (l + 1)
        idx = np.arange(lo, lo + n)
        idx = idx[host["live"][idx] == 1]
        par = 1.0 if l == 0 else host["pig"][(8 ** l - 8) // 7 + (idx - lo) // 8]
        e = np.abs(host["pig"][idx] - host["pi"][idx] * par) / host["pig"][idx]
        worst["pig"] = max(worst["pig"], float(e.max()) if e.size else 0.0)
        assert np.all(e < 1e-14)
    log(f"  finalize vs oracle eigh3 on {len(live)} nodes: lam {worst['lam']:.1e} evec {worst['evec']:.1e} "
        f"kappa {worst['kappa']:.1e} pig {worst['pig']:.1e}")
    return worst


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
        fin = compare_finalize(host, ot, sl, keep, tol, log)
        m = glab[l] >= 0
        mo = lab[l] >= 0
        grp = np.where(m, glab[l] // 8, 0)
        grp_o = np.where(mo, lab[l] // 8, 0)
        in_div = (m & (diverged[grp] | small[grp])) | (mo & (diverged[grp_o] | small[grp_o]))
        mis = (glab[l] != lab[l]) & ~in_div
        assert np.all(m[mis] & mo[mis])
        # counts: the exported count of every node is the number of points the
        # GPU labels with it; against the oracle's partition a count can only
        # move by the points whose label differs
        cnt_g = np.bincount(glab[l][m], minlength=sl.stop - sl.start)
        np.testing.assert_array_equal(host["count"][sl], cnt_g)
        cnt_o = np.bincount(lab[l][mo], minlength=sl.stop - sl.start)
        assert np.abs(cnt_g - cnt_o).sum() <= 2 * int((glab[l] != lab[l]).sum())
        if l == L - 1:
            assert not host["has_children"][sl].any()
        if l > 0:
            # has_children of the parent level follows from this level's live
            # children (groups whose live set differs are discrete divergences)
            psl = ot.level_slice(l - 1)
            okp = ~diverged & ~small
            np.testing.assert_array_equal(host["has_children"][psl][okp], ot.has_children[psl][okp])
        if iters == 1 and mis.any():
            # after one iteration from identical parents every label must match
            # the oracle's except where the oracle's own top-2 scores nearly tie
            gap = _sibling_gap(ot, sl, src, lab[l], glab[l], mis)
            log(f"    label mismatches {mis.sum()}, largest oracle score gap among them {gap.max():.2e}")
            assert np.all(gap < LABEL_FLAG_GAP), gap.max()
        if diverged.any():
            pc = host["count"][ot.level_slice(l - 1)][diverged] if l > 0 else [src.shape[1]]
            log(f"    diverged groups {diverged.sum()}/{populated.sum()} (parent sizes {list(pc)[:8]})")
        mx = lambda a: float(a.max()) if a.size else 0.0
        log(f"  level {l}: live {host['live'][sl].sum()}/{ot.live[sl].sum()}  pi {mx(e_pi):.1e} mu {mx(e_mu):.1e} "
            f"cov {mx(e_cov):.1e} kappa {mx(e_k):.1e} lam {fin['lam']:.1e} evec {fin['evec']:.1e} "
            f"pig {fin['pig']:.1e}  label mismatches {mis.sum()} ({mis.mean():.1e})")
        if e_pi.size:
            i = int(np.argmax(e_pi))
            log(f"    worst pi node {np.flatnonzero(keep)[i] + sl.start}: gpu {host['pi'][sl][keep][i]:.9e} "
                f"oracle {ot.pi[sl][keep][i]:.9e} count {host['count'][sl][keep][i]}")
        worst = dict(pi=max(worst["pi"], mx(e_pi)), mu=max(worst["mu"], mx(e_mu)), cov=max(worst["cov"], mx(e_cov)),
                     kappa=max(worst.get("kappa", 0.0), mx(e_k)), lam=max(worst.get("lam", 0.0), fin["lam"]),
                     evec=max(worst.get("evec", 0.0), fin["evec"]), pig=max(worst.get("pig", 0.0), fin["pig"]))
        assert diverged.sum() <= max(2, 0.01 * populated.sum())
        assert mx(e_pi) < tol["pi"] and mx(e_mu) < tol["mu"] and mx(e_cov) < tol["cov"], (l, mx(e_pi), mx(e_mu),
                                                                                          mx(e_cov))
        # kappa = lam3 / sum(lam) moves by at most twice the trace-relative
        # eigenvalue error
        assert mx(e_k) < 2 * tol["cov"], (l, mx(e_k))
        assert mis.mean() < 1e-3
    return worst
