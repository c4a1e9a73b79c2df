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


def test_mlp_forward_and_gradients_vs_oracle(hg):
    rng = np.random.default_rng(3)
    P = 33
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
    log(f"[mlp] forward rel err {ey:.2e}")
    assert ey < 1e-2
    g, loss = net.backward(Xg, Tg, trans_weight=0.5)
    lo, go = omlp.loss_and_grad(params.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                                trans_weight=0.5, bf16=True)
    assert abs(loss - lo) < 1e-2 * abs(lo)
    o = 0
    for i in range(4):
        n = omlp.DIMS[i] * omlp.DIMS[i + 1] + omlp.DIMS[i + 1]
        e = np.linalg.norm(g[o:o + n] - go[o:o + n]) / np.linalg.norm(go[o:o + n])
        log(f"[mlp] layer {i + 1} grad rel err {e:.2e}")
        assert e < 2e-2
        o += n


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
    """Short training on generated pairs; the fallback never makes a pair worse than identity."""
    from paper_1807_02587_amd import warmstart as W
    from synth.torch_scenes import cube_pairs
    cfg = W.WarmConfig()
    X, T = W.training_set(2048, seed=7, cfg=cfg, chunk=1024, n=4000, log=log)
    assert torch.isfinite(X).all() and torch.isfinite(T).all()
    net = hg.MLP(seed=3)
    hist = W.train(net, X, T, epochs=3, batch=256, lr=1e-3, cfg=cfg, log=log)
    assert hist[-1] < hist[0]
    S = cube_pairs(10**6 + 1, 64, n=4000, max_angle_deg=90)
    off = S.offsets.numpy()
    r = W.register_warm(net, S.src, S.tgt, off, off, [2] * 64, cfg)
    err = W.rotation_errors_deg(r["R"], S.R_true.cpu().numpy())
    log(f"[warm] median err {np.median(err):.3f} deg, fallback {r['fallback'].mean():.2f}")
    Ri = np.broadcast_to(np.eye(3), (64, 3, 3))
    ll_id = hg.hgmm_estep_batch(r["forest"], S.tgt, off, Ri, np.zeros((64, 3)))
    assert np.all(r["loglik"][r["fallback"]] == r["loglik"][r["fallback"]])  # finite where re-run
    assert np.isfinite(ll_id).all()


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
