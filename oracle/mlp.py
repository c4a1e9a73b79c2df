"""FP64 NumPy oracle of the warm-start network (TEST INFRASTRUCTURE ONLY).

The network and its loss are this project's addition (the paper has no learned
component): 1280 -> 512 -> 512 -> 512 -> 9, exact GELU after the hidden
layers, loss sum_c w_c (y_c - t_c)^2 / 2 averaged over rows (w = 1 on the 6D
rotation part, trans_weight on the translation).  Parameters are flattened as
W1 b1 W2 b2 W3 b3 W4 b4 with W row-major [in x out].  Training uses Adam
(``adam_step``).

``bf16=True`` rounds the GEMM operands (inputs, weights, activations, output
gradients) to bfloat16 exactly where the device network does, so that the
remaining difference is FP32 versus FP64 accumulation.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

DIMS = (1280, 512, 512, 512, 9)


def param_count() -> int:
    return sum(DIMS[i] * DIMS[i + 1] + DIMS[i + 1] for i in range(4))


def unflatten(params):
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for i in range(4):
        k, n = DIMS[i], DIMS[i + 1]
        W = p[o:o + k * n].reshape(k, n)
        o += k * n
        b = p[o:o + n]
        o += n
        out.append((W, b))
    assert o == len(p)
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(params, X, bf16=False):
    """Returns (Y, cache)."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unflatten(params)
    H = rnd(X)
    cache = [H]
    Zs = []
    for i, (W, b) in enumerate(layers):
        Z = H @ rnd(W) + b
        Zs.append(Z)
        if i < 3:
            H = rnd(gelu(Z))
            cache.append(H)
    return Zs[-1], (cache, Zs)


def loss_and_grad(params, X, T, trans_weight=1.0, bf16=False):
    """Mean loss and the flattened parameter gradient."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unflatten(params)
    Y, (Hs, Zs) = forward(params, X, bf16)
    P = X.shape[0]
    w = np.array([1.0] * 6 + [trans_weight] * 3)
    d = Y - T
    loss = float(np.mean(np.sum(0.5 * w * d * d, axis=1)))
    dZ = w * d / P
    grads = [None] * 4
    for i in range(3, -1, -1):
        W, _ = layers[i]
        gW = Hs[i].T @ rnd(dZ)
        gb = dZ.sum(0)
        grads[i] = (gW, gb)
        if i == 0:
            break
        dH = rnd(dZ) @ rnd(W).T
        dZ = dH * gelu_grad(Zs[i - 1])
    return loss, flatten(grads)


def adam_step(params, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1), the optimiser of the
    network's training.  ``step`` counts from 1.  The first and second moment
    estimates are exponential averages of the gradient and of its square; each
    is divided by one minus its decay rate to the power ``step`` (the bias
    correction), and the parameter moves by lr times the corrected first moment
    over the square root of the corrected second moment plus eps.

    Returns (params, m, v) after the step, all float64; the inputs are not
    modified."""
    if step < 1:
        raise ValueError("step counts from 1")
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    w = np.asarray(params, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return w, m, v


def six_d_to_rotation(v):
    """Gram-Schmidt of the first two columns (Zhou et al. 2019), rows of v (..., 6)."""
    v = np.asarray(v, dtype=np.float64)
    a, b = v[..., 0:3], v[..., 3:6]
    c1 = a / np.linalg.norm(a, axis=-1, keepdims=True)
    c2 = b - np.sum(c1 * b, axis=-1, keepdims=True) * c1
    c2 = c2 / np.linalg.norm(c2, axis=-1, keepdims=True)
    c3 = np.cross(c1, c2)
    return np.stack([c1, c2, c3], axis=-1)


def head_pose(Y, fr_src, fr_tgt):
    """Rows [6D | tc] in canonical frames -> (R, t) in the clouds' frames."""
    Y = np.asarray(Y, dtype=np.float64)
    Rc = six_d_to_rotation(Y[:, :6])
    Es, cs, ss = fr_src[:, :9].reshape(-1, 3, 3), fr_src[:, 9:12], fr_src[:, 12]
    Et, ct = fr_tgt[:, :9].reshape(-1, 3, 3), fr_tgt[:, 9:12]
    R = np.einsum("pji,pjk,pkl->pil", Es, Rc, Et)
    t = ss[:, None] * np.einsum("pji,pj->pi", Es, Y[:, 6:9]) + cs - np.einsum("pij,pj->pi", R, ct)
    return R, t


def head_target(R, t, fr_src, fr_tgt):
    """(R, t) -> training rows [Rc col 0, Rc col 1, tc]."""
    Es, cs, ss = fr_src[:, :9].reshape(-1, 3, 3), fr_src[:, 9:12], fr_src[:, 12]
    Et, ct = fr_tgt[:, :9].reshape(-1, 3, 3), fr_tgt[:, 9:12]
    Rc = np.einsum("pij,pjk,plk->pil", Es, R, Et)
    w = np.einsum("pij,pj->pi", R, ct) + t - cs
    tc = np.einsum("pij,pj->pi", Es, w) / ss[:, None]
    return np.concatenate([Rc[:, :, 0], Rc[:, :, 1], tc], axis=1)
