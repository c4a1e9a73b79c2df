"""Learned warm start on the GPU against the FP64 NumPy network oracle.

Tolerances: the GEMM sees exactly representable bf16 operands, so its FP32
accumulation matches FP64 to ~1e-6 relative.  The network keeps activations in
bf16; the oracle rounds at the same places, so the two differ only where an
FP32 accumulation lands on the other side of a bf16 rounding boundary, a
relative difference of ~1e-2 at most.
"""

import math
import sys

import numpy as np
import pytest

import oracle.mlp as omlp
from synth import rotation_from_axis_angle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hg():
    import paper_1807_02587_amd as hg
    assert torch.cuda.is_available()
    return hg


def _bf16_bits(x):
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return torch.from_numpy(r.view(np.int16).copy()).cuda()


@pytest.mark.parametrize("M,N,K", [(16, 16, 32), (37, 70, 45), (130, 9, 512), (64, 512, 96)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_bf16_mfma(hg, M, N, K, ta, tb):
    rng = np.random.default_rng(M * 7 + N + K)
    A = omlp.bf16_round(rng.normal(size=(M, K)))
    Bm = omlp.bf16_round(rng.normal(size=(K, N)))
    Ast = A.T.copy() if ta else A
    Bst = Bm.T.copy() if tb else Bm
    C = hg.hgmm_gemm_bf16(_bf16_bits(Ast), _bf16_bits(Bst), M, N, K, ta=ta, tb=tb).cpu().numpy()
    ref = A @ Bm
    err = np.abs(C - ref).max() / np.abs(ref).max()
    assert err < 2e-6, err


def _params(seed):
    rng = np.random.default_rng(seed)
    p = []
    for i in range(4):
        k, n = omlp.DIMS[i], omlp.DIMS[i + 1]
        p.append(rng.normal(scale=math.sqrt(2.0 / k), size=k * n))
        p.append(rng.normal(scale=0.05, size=n))
    return np.concatenate(p).astype(np.float32)


@pytest.mark.parametrize("P", [33, 1100, 4100])
def test_mlp_forward_and_gradients_vs_oracle(hg, P):
    """Forward and every gradient element against the FP64 oracle.  From 1024
    rows the weight gradients' reduction over the rows is split into slices of
    at least 512 rows (2 slices at 1100 rows, 8 at 4100, both with a shorter
    last slice) whose partial products are added in slice order."""
    rng = np.random.default_rng(3)
    params = _params(4)
    net = hg.MLP(seed=1)
    net.set_params(params)
    np.testing.assert_array_equal(net.get_params(), params)
    X = rng.normal(size=(P, 1280)).astype(np.float32)
    T = rng.normal(size=(P, 9)).astype(np.float32)
    Xg, Tg = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    Y = net.forward(Xg).cpu().numpy()
    Yo, _ = omlp.forward(params.astype(np.float64), X.astype(np.float64), bf16=True)
    ey = np.abs(Y - Yo).max() / np.abs(Yo).max()
    log(f"[mlp] P={P} forward rel err {ey:.2e}")
    assert ey < 1e-2
    g, loss = net.backward(Xg, Tg, trans_weight=0.5)
    lo, go = omlp.loss_and_grad(params.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                                trans_weight=0.5, bf16=True)
    assert abs(loss - lo) < 1e-2 * abs(lo)
    # element by element, per weight matrix and per bias vector: the largest
    # difference against the largest reference entry of that block
    o = 0
    for i in range(4):
        for part, n in (("W", omlp.DIMS[i] * omlp.DIMS[i + 1]), ("b", omlp.DIMS[i + 1])):
            e = np.abs(g[o:o + n] - go[o:o + n]).max() / np.abs(go[o:o + n]).max()
            log(f"[mlp] layer {i + 1} {part} grad max |diff| / max |ref| {e:.2e}")
            assert e < 1e-2, (i, part, e)
            o += n


def test_adam_step_vs_oracle(hg):
    """Three training steps on the device against the oracle's Adam step fed
    with the device's own gradients at each step's parameters: every FP32
    master weight agrees element by element, and the forward after the steps
    (which reads the refreshed bf16 copy) agrees with the oracle network."""
    rng = np.random.default_rng(21)
    P = 17
    lr = 2e-3
    params = _params(8)
    net = hg.MLP(seed=5)
    net.set_params(params)
    X = rng.normal(size=(P, 1280)).astype(np.float32)
    T = rng.normal(size=(P, 9)).astype(np.float32)
    Xg, Tg = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    m = np.zeros(net.n_params)
    v = np.zeros(net.n_params)
    for step in (1, 2, 3):
        before = net.get_params()
        g, _ = net.backward(Xg, Tg, trans_weight=0.5)
        net.train_step(Xg, Tg, lr, trans_weight=0.5, want_loss=False)
        after = net.get_params()
        ref, m, v = omlp.adam_step(before, m, v, g, step, lr)
        # FP32 update of an FP32 weight: a few ulps of the weight, plus the
        # FP32 moment arithmetic's ~1e-6 relative error on a step of size ~lr
        tol = 4.0 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64) + 1e-5 * lr
        err = np.abs(after - ref)
        log(f"[adam] step {step}: max |diff| {err.max():.2e}, max diff / tol {np.max(err / tol):.2f}, "
            f"mean |move| {np.mean(np.abs(after - before)):.2e}")
        assert np.all(err <= tol), (step, int(np.argmax(err / tol)))
    Y = net.forward(Xg).cpu().numpy()
    Yo, _ = omlp.forward(after.astype(np.float64), X.astype(np.float64), bf16=True)
    assert np.abs(Y - Yo).max() / np.abs(Yo).max() < 1e-2


def test_mlp_training_reduces_loss(hg):
    rng = np.random.default_rng(5)
    X = torch.from_numpy(rng.normal(size=(64, 1280)).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.normal(scale=0.5, size=(64, 9)).astype(np.float32)).cuda()
    net = hg.MLP(seed=2)
    first = net.train_step(X, T, 1e-3)
    for _ in range(150):
        last = net.train_step(X, T, 1e-3)
    log(f"[mlp] overfit loss {first:.4f} -> {last:.4f}")
    assert last < 0.2 * first


def test_features_and_head_vs_numpy(hg):
    from synth import small_pair
    pairs = [small_pair(40 + k, n=3000) for k in range(3)]
    src = np.concatenate([p.src for p in pairs], axis=1)
    off = np.array([0, 3000, 6000, 9000])
    forest = hg.hgmm_build_batch(torch.from_numpy(src).cuda(), off, [2, 2, 2])
    feat, fr = hg.hgmm_warm_features(forest, [0, 1, 2])
    feat, fr = feat.cpu().numpy(), fr.cpu().numpy()
    for b in range(3):
        h = forest.export(b)
        E = fr[b, :9].reshape(3, 3)
        c, s = fr[b, 9:12], fr[b, 12]
        np.testing.assert_allclose(E @ E.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(E) - 1) < 1e-12
        np.testing.assert_allclose(c, h["origin"], atol=1e-12)
        X = pairs[b].src.T.astype(np.float64)
        assert abs(s - np.sqrt(np.mean(np.sum((X - X.mean(0)) ** 2, 1)))) < 1e-9
        for k in range(64):
            g = 8 + k
            f = feat[b, 10 * k:10 * k + 10]
            if not h["live"][g]:
                assert np.all(f == 0)
                continue
            mu = E @ (h["mu"][g] - c) / s
            S6 = h["cov"][g]
            S = np.array([[S6[0], S6[1], S6[2]], [S6[1], S6[3], S6[4]], [S6[2], S6[4], S6[5]]])
            Cn = E @ S @ E.T / s ** 2
            ref = np.array([h["pig"][g], *mu, Cn[0, 0], Cn[0, 1], Cn[0, 2], Cn[1, 1], Cn[1, 2], Cn[2, 2]])
            np.testing.assert_allclose(f, ref, rtol=1e-5, atol=1e-6)
    # head: GPU composition against the oracle's, and target -> pose round trip
    rng = np.random.default_rng(9)
    Y = rng.normal(size=(3, 9)).astype(np.float32)
    frg = torch.from_numpy(fr).cuda()
    R0, t0 = hg.hgmm_warm_head_pose(torch.from_numpy(Y).cuda(), frg, frg.flip(0).contiguous())
    Ro, to = omlp.head_pose(Y, fr, fr[::-1].copy())
    np.testing.assert_allclose(R0.cpu().numpy().reshape(3, 3, 3), Ro, atol=1e-6)
    np.testing.assert_allclose(t0.cpu().numpy(), to, atol=1e-6)
    Rt = np.stack([rotation_from_axis_angle(rng.normal(size=3), 0.7) for _ in range(3)])
    tt = rng.normal(size=(3, 3))
    Tg = hg.hgmm_warm_head_target(torch.from_numpy(Rt.reshape(3, 9)).cuda(), torch.from_numpy(tt).cuda(), frg,
                                  frg.flip(0).contiguous()).cpu().numpy()
    np.testing.assert_allclose(Tg, omlp.head_target(Rt, tt, fr, fr[::-1].copy()), atol=1e-6)


def test_warm_pipeline_smoke(hg):
    """Short training on generated pairs, then both fallback rules on held-out
    pairs.  Rule "plain": every pair ends with the higher final log-likelihood
    of the warm run and the plain method from the identity, so never below the
    plain method.  Rule "identity": a pair keeps its warm result only if that
    ends at or above the identity pose's log-likelihood; every other pair ends
    exactly where the plain method from the identity does."""
    from paper_1807_02587_amd import warmstart as W
    from synth.torch_scenes import cube_pairs
    cfg = W.WarmConfig()
    X, T = W.training_set(2048, seed=7, cfg=cfg, chunk=1024, n=4000, log=log)
    assert torch.isfinite(X).all() and torch.isfinite(T).all()
    net = hg.MLP(seed=3)
    hist = W.train(net, X, T, epochs=3, batch=256, lr=1e-3, cfg=cfg, log=log)
    assert hist[-1] < hist[0]
    B = 64
    S = cube_pairs(10**6 + 1, B, n=4000, max_angle_deg=90)
    off = S.offsets.numpy()
    forest = hg.hgmm_build_batch(S.src, off, [2] * B)
    Ri = np.broadcast_to(np.eye(3), (B, 3, 3)).copy()
    plain = hg.hgmm_register_batch(forest, S.tgt, off, max_iters=cfg.max_iters, lambda_c=cfg.lambda_c, R0=Ri,
                                   t0=np.zeros((B, 3)))
    ll_id = hg.hgmm_estep_batch(forest, S.tgt, off, Ri, np.zeros((B, 3)), lambda_c=cfg.lambda_c)
    assert np.isfinite(ll_id).all()
    ok = plain["status"] == 0

    r = W.register_warm(net, S.src, S.tgt, off, off, [2] * B, cfg, src_forest=forest, fallback="plain")
    err = W.rotation_errors_deg(r["R"], S.R_true.cpu().numpy())
    log(f"[warm] rule plain: median err {np.median(err):.3f} deg, fallback {r['fallback'].mean():.2f}")
    assert np.all(r["loglik"][ok] >= plain["loglik"][ok])
    fb = r["fallback"]
    np.testing.assert_array_equal(r["R"][fb], plain["R"][fb])
    np.testing.assert_array_equal(r["loglik"][fb], plain["loglik"][fb])

    r = W.register_warm(net, S.src, S.tgt, off, off, [2] * B, cfg, src_forest=forest, fallback="identity")
    fb = r["fallback"]
    log(f"[warm] rule identity: fallback {fb.mean():.2f}")
    assert np.all(r["loglik"][~fb] >= ll_id[~fb])
    np.testing.assert_array_equal(r["R"][fb], plain["R"][fb])
    np.testing.assert_array_equal(r["t"][fb], plain["t"][fb])
    np.testing.assert_array_equal(r["loglik"][fb], plain["loglik"][fb])


def test_trained_network_gain(hg):
    """The committed network against the method without it, on held-out pairs
    (rotation U(0, 90 deg), 10k points, L = 2): the warm start with the plain-
    likelihood fallback reaches a median rotation error <= 0.5 deg where the
    plain method from the identity does not, and never ends at a lower final
    likelihood than the plain method."""
    import os
    from paper_1807_02587_amd import warmstart as W
    from synth.torch_scenes import cube_pairs
    wpath = os.path.join(os.path.dirname(hg.__file__), "weights", "warm_mlp.npy")
    assert os.path.exists(wpath), "trained weights are part of the package"
    net = hg.MLP(seed=0)
    net.set_params(np.load(wpath))
    cfg = W.WarmConfig()
    B = 256
    S = cube_pairs(2 * 10**6 + 17, B, n=10_000, max_angle_deg=90)
    off = S.offsets.numpy()
    Rt = S.R_true.cpu().numpy()
    forest = hg.hgmm_build_batch(S.src, off, [cfg.src_levels] * B)
    plain = hg.hgmm_register_batch(forest, S.tgt, off, max_iters=cfg.max_iters, lambda_c=cfg.lambda_c)
    warm = W.register_warm(net, S.src, S.tgt, off, off, [cfg.src_levels] * B, cfg, src_forest=forest)
    ep = W.rotation_errors_deg(plain["R"], Rt)
    ew = W.rotation_errors_deg(warm["R"], Rt)
    log(f"[gain] plain median {np.median(ep):.3f} deg, <=0.5 deg {np.mean(ep <= 0.5):.3f}; "
        f"warm median {np.median(ew):.3f} deg, <=0.5 deg {np.mean(ew <= 0.5):.3f}, fallback {warm['fallback'].mean():.3f}")
    assert np.median(ew) <= 0.5 < np.median(ep)
    assert np.mean(ew <= 0.5) >= np.mean(ep <= 0.5) + 0.3
    ok = plain["status"] == 0
    assert np.all(warm["loglik"][ok] >= plain["loglik"][ok] - 1e-12)


def test_warm_start_on_one_forest(hg):
    """The warm start builds the source and target trees as one forest (target
    b is tree B + b): its network inputs and initial poses agree with those
    from separately built forests (the trees differ only in FP64 summation
    order), the result never has a lower likelihood than the plain method on
    the same trees, and the success rate matches the separate build's."""
    import os
    from paper_1807_02587_amd import warmstart as W
    from synth.torch_scenes import cube_pairs
    net = hg.MLP(seed=0)
    net.set_params(np.load(os.path.join(os.path.dirname(hg.__file__), "weights", "warm_mlp.npy")))
    cfg = W.WarmConfig()
    B = 64
    S = cube_pairs(3 * 10**6 + 5, B, n=10_000, max_angle_deg=90)
    off = S.offsets.numpy()
    Rt = S.R_true.cpu().numpy()
    sep_forest = hg.hgmm_build_batch(S.src, off, [cfg.src_levels] * B)
    sep = W.register_warm(net, S.src, S.tgt, off, off, [cfg.src_levels] * B, cfg, src_forest=sep_forest)
    one = W.register_warm(net, S.src, S.tgt, off, off, [cfg.src_levels] * B, cfg)
    assert one["forest"].ntrees == 2 * B
    dR0 = float(np.abs(one["R0"] - sep["R0"]).max())
    log(f"[one forest] initial poses differ by {dR0:.2e} at most")
    assert dR0 < 1e-3
    Ri = np.broadcast_to(np.eye(3), (B, 3, 3)).copy()
    plain = hg.hgmm_register_batch(one["forest"], S.tgt, off, max_iters=cfg.max_iters, lambda_c=cfg.lambda_c, R0=Ri,
                                   t0=np.zeros((B, 3)))
    ok = plain["status"] == 0
    assert np.all(one["loglik"][ok] >= plain["loglik"][ok])
    e1 = W.rotation_errors_deg(one["R"], Rt)
    e0 = W.rotation_errors_deg(sep["R"], Rt)
    log(f"[one forest] within 0.5 deg: one forest {np.mean(e1 <= 0.5):.3f}, separate {np.mean(e0 <= 0.5):.3f}")
    assert abs(np.mean(e1 <= 0.5) - np.mean(e0 <= 0.5)) <= 0.1


@pytest.mark.parametrize("rule", ["plain", "identity"])
def test_warm_entry_point_matches_the_call_sequence(hg, rule):
    """hgmm_register_warm_batch (capped registration, full registration, the
    fallback rule) gives the results of the same steps made as separate
    batched calls, bit for bit."""
    from synth.torch_scenes import cube_pairs
    B = 32
    S = cube_pairs(4 * 10**6 + 3, B, n=4000, max_angle_deg=60)
    off = S.offsets.numpy()
    forest = hg.hgmm_build_batch(S.src, off, [3] * B)
    rng = np.random.default_rng(5)
    Rt, tt = S.R_true.cpu().numpy(), S.t_true.cpu().numpy()
    R0 = np.stack([rotation_from_axis_angle(rng.normal(size=3), math.radians(rng.uniform(0, 20))) @ Rt[b]
                   for b in range(B)])
    t0 = tt + rng.normal(scale=0.02, size=tt.shape)
    kw = dict(max_iters=30, lambda_c=0.01)
    rc = hg.hgmm_register_batch(forest, S.tgt, off, R0=R0, t0=t0, max_levels=2, **kw)
    ok = rc["status"] == 0
    Rs = np.where(ok[:, None, None], rc["R"], R0)
    ts = np.where(ok[:, None], rc["t"], t0)
    r = hg.hgmm_register_batch(forest, S.tgt, off, R0=Rs, t0=ts, **kw)
    Ri, ti = np.broadcast_to(np.eye(3), (B, 3, 3)).copy(), np.zeros((B, 3))
    if rule == "plain":
        r2 = hg.hgmm_register_batch(forest, S.tgt, off, R0=Ri, t0=ti, **kw)
        fb = ((r["loglik"] < r2["loglik"]) & (r2["status"] == 0)) | (r["status"] != 0)
    else:
        ll_id = hg.hgmm_estep_batch(forest, S.tgt, off, Ri, ti, lambda_c=0.01)
        fb = (r["loglik"] < ll_id) | (r["status"] != 0)
        r2 = hg.hgmm_register_batch(forest, S.tgt, off, R0=Ri, t0=ti, active=fb.astype(np.int32), **kw)
    got = hg.hgmm_register_warm_batch(forest, S.tgt, off, R0, t0, coarse_levels=2, rule=rule, **kw)
    log(f"[warm entry] rule {rule}: fallback {fb.mean():.2f}")
    np.testing.assert_array_equal(got["fallback"], fb)
    for k in ("R", "t", "iters", "loglik", "status"):
        want = np.where(fb.reshape((B,) + (1,) * (r[k].ndim - 1)), r2[k], r[k])
        np.testing.assert_array_equal(got[k], want)
