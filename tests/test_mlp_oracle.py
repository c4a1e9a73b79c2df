"""Pins of the warm-start network oracle: finite differences, rotation head
identities and bf16 rounding."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import mlp


def _net(seed):
    rng = np.random.default_rng(seed)
    p = []
    for i in range(4):
        k, n = mlp.DIMS[i], mlp.DIMS[i + 1]
        p.append(rng.normal(scale=np.sqrt(2.0 / k), size=k * n))
        p.append(rng.normal(scale=0.1, size=n))
    return np.concatenate(p)


def test_param_count():
    assert mlp.param_count() == 1_185_801


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    params = _net(1)
    X = rng.normal(size=(3, 1280))
    T = rng.normal(size=(3, 9))
    loss, g = mlp.loss_and_grad(params, X, T, trans_weight=0.7)
    offs = np.cumsum([0] + [mlp.DIMS[i] * mlp.DIMS[i + 1] + mlp.DIMS[i + 1] for i in range(4)])
    idx = np.concatenate([rng.integers(offs[i], offs[i + 1], size=8) for i in range(4)])
    h = 1e-6
    for j in idx:
        pp, pm = params.copy(), params.copy()
        pp[j] += h
        pm[j] -= h
        lp, _ = mlp.loss_and_grad(pp, X, T, trans_weight=0.7)
        lm, _ = mlp.loss_and_grad(pm, X, T, trans_weight=0.7)
        fd = (lp - lm) / (2 * h)
        # central differences carry ~eps*loss/h ~ 1e-9 of rounding noise
        assert abs(fd - g[j]) <= 1e-6 * abs(fd) + 2e-8 * max(1.0, loss), (j, fd, g[j])


def test_six_d_head():
    rng = np.random.default_rng(2)
    R = Rotation.random(50, random_state=3).as_matrix()
    v = np.concatenate([R[:, :, 0], R[:, :, 1]], axis=1)
    np.testing.assert_allclose(mlp.six_d_to_rotation(v), R, atol=1e-14)
    Q = mlp.six_d_to_rotation(rng.normal(size=(50, 6)))
    np.testing.assert_allclose(np.einsum("pji,pjk->pik", Q, Q), np.broadcast_to(np.eye(3), (50, 3, 3)), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(Q), 1.0, atol=1e-14)


def test_head_pose_target_round_trip():
    rng = np.random.default_rng(4)
    P = 20

    def frames():
        E = Rotation.random(P, random_state=int(rng.integers(1 << 30))).as_matrix()
        return np.concatenate([E.reshape(P, 9), rng.normal(size=(P, 3)), rng.uniform(0.5, 2, size=(P, 1))], 1)

    fs, ft = frames(), frames()
    R = Rotation.random(P, random_state=7).as_matrix()
    t = rng.normal(size=(P, 3))
    T = mlp.head_target(R, t, fs, ft)
    R2, t2 = mlp.head_pose(T, fs, ft)
    np.testing.assert_allclose(R2, R, atol=1e-13)
    np.testing.assert_allclose(t2, t, atol=1e-12)
    # the canonical transform maps canonical target coordinates onto canonical source ones
    z = rng.normal(size=(P, 3))
    x = np.einsum("pij,pj->pi", R, z) + t
    v = np.einsum("pij,pj->pi", ft[:, :9].reshape(P, 3, 3), z - ft[:, 9:12]) / ft[:, 12:13]
    u = np.einsum("pij,pj->pi", fs[:, :9].reshape(P, 3, 3), x - fs[:, 9:12]) / fs[:, 12:13]
    Rc = mlp.six_d_to_rotation(T[:, :6])
    scale = ft[:, 12] / fs[:, 12]
    np.testing.assert_allclose(u, scale[:, None] * np.einsum("pij,pj->pi", Rc, v) + T[:, 6:9], atol=1e-12)


@pytest.mark.parametrize("x,expect", [(1.0, 1.0), (1.00390625, 1.0), (1.01171875, 1.015625), (-3.0, -3.0),
                                      (1.0 + 2 ** -7 + 2 ** -12, 1.0078125 + 0.0)])
def test_bf16_rounding(x, expect):
    assert mlp.bf16_round(np.array([x]))[0] == expect


def test_adam_two_steps_by_hand():
    """Two Adam steps on one weight, worked out by hand (beta 0.9 / 0.999, eps 1e-8,
    lr 0.1, w0 = 1, gradients +2 then -1):
    step 1: m = 0.2, v = 0.004, corrections 0.1 and 0.001 give m_hat = 2, v_hat = 4,
            w = 1 - 0.1 * 2 / (2 + 1e-8) = 0.9000000005;
    step 2: m = 0.18 - 0.1 = 0.08, v = 0.003996 + 0.001 = 0.004996, corrections
            0.19 and 0.001999 give m_hat = 8/19, v_hat = 4996/1999 (sqrt 1.5809015228...),
            w = 0.9000000005 - 0.1 * (8/19) / (1.5809015228... + 1e-8) = 0.87336629670..."""
    w, m, v = mlp.adam_step(np.array([1.0]), np.zeros(1), np.zeros(1), np.array([2.0]), 1, 0.1)
    assert m[0] == pytest.approx(0.2, rel=1e-15) and v[0] == pytest.approx(0.004, rel=1e-13)
    assert w[0] == pytest.approx(0.9000000005, abs=1e-15)
    w, m, v = mlp.adam_step(w, m, v, np.array([-1.0]), 2, 0.1)
    assert m[0] == pytest.approx(0.08, rel=1e-13) and v[0] == pytest.approx(0.004996, rel=1e-13)
    assert w[0] == pytest.approx(0.8733662967024313, abs=1e-14)


def test_adam_invariants():
    """The first step moves every weight by lr in the direction against its
    gradient whatever the gradient's size (the bias corrections make m_hat = g
    and v_hat = g^2); a constant gradient keeps that true at every step; the
    step is invariant to a positive rescaling of the gradient (up to eps)."""
    rng = np.random.default_rng(11)
    w0 = rng.normal(size=200)
    g = rng.choice([-1.0, 1.0], size=200) * 10.0 ** rng.uniform(-2, 3, size=200)
    w, m, v = mlp.adam_step(w0, np.zeros(200), np.zeros(200), g, 1, 1e-3)
    np.testing.assert_allclose(w0 - w, 1e-3 * np.sign(g), rtol=1e-5)
    for step in range(2, 40):
        w_prev = w
        w, m, v = mlp.adam_step(w, m, v, g, step, 1e-3)
        np.testing.assert_allclose(w_prev - w, 1e-3 * np.sign(g), rtol=1e-5)
    a1, _, _ = mlp.adam_step(w0, 0.3 * g, 0.01 * g * g, g, 5, 1e-3)
    a2, _, _ = mlp.adam_step(w0, 0.3 * 7.0 * g, 0.01 * 49.0 * g * g, 7.0 * g, 5, 1e-3)
    np.testing.assert_allclose(a1, a2, rtol=1e-12, atol=1e-9)
