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
