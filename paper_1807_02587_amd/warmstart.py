"""Learned warm start for batched registration (orchestration of library calls).

Pipeline per batch of pairs (every arithmetic step runs in the library's HIP
kernels; this module only sequences calls and moves handles around):

1. build the source trees (levels per pair) and the 2-level target trees,
   as one forest (sources first) so that both share every launch;
2. level-1 features of both trees in canonical frames (hgmm_warm_features);
3. network forward (hgmm_mlp_forward) -> 6D rotation + translation;
4. head -> initial transforms (hgmm_warm_head_pose);
5. batched registration from those transforms, coarse to fine: first with
   the descent capped at cfg.coarse_levels levels, then with the whole tree;
6. fallback: the plain method from the identity is the reference.  Rule "plain"
   (default): every pair is also registered from the identity and keeps
   whichever result has the higher final log-likelihood.  Rule "identity"
   (cheaper): a pair whose final log-likelihood is below the log-likelihood of
   the identity transform (one E-step) is registered again from the identity.
   Steps 5 and 6 are one library call (hgmm_register_warm_batch).

Training data come from the batched GPU scene generator; the label of a pair
is the plain method's converged pose when started at the ground truth.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import api as hg


@dataclass
class WarmConfig:
    src_levels: int = 2
    tgt_levels: int = 2
    reg_eps: float = 1e-6
    min_mass: float = 1.0
    lambda_c: float = 0.01
    max_iters: int = 30
    trans_weight: float = 1.0
    # coarse-to-fine: from the network's pose, first register with the descent
    # capped at this many levels (wider basin), then with the whole tree; 0 off
    coarse_levels: int = 2


def features_for(src_forest, tgt_forest, B, cfg: WarmConfig, tgt_first: int = 0):
    """Features of source trees 0..B-1 and target trees tgt_first..tgt_first+B-1
    (one library call when both are in one forest)."""
    if src_forest is tgt_forest:
        ids = np.concatenate([np.arange(B), np.arange(tgt_first, tgt_first + B)])
        f, fr = hg.hgmm_warm_features(src_forest, ids, cfg.reg_eps)
        return torch.cat([f[:B], f[B:]], dim=1).contiguous(), fr[:B], fr[B:]
    fs, frs = hg.hgmm_warm_features(src_forest, np.arange(B), cfg.reg_eps)
    ft, frt = hg.hgmm_warm_features(tgt_forest, np.arange(tgt_first, tgt_first + B), cfg.reg_eps)
    return torch.cat([fs, ft], dim=1).contiguous(), frs, frt


def training_set(n_pairs: int, seed: int, cfg: WarmConfig = WarmConfig(), chunk: int = 1024, n: int = 10_000,
                 max_angle_deg: float = 90.0, log=None, time_budget_s: float | None = None):
    """(X (m, 1280) float32, T (m, 9) float32) on the GPU, m = n_pairs, or fewer
    (whole chunks) when generation would exceed ``time_budget_s``."""
    from synth.torch_scenes import cube_pairs
    Xs, Ts = [], []
    ws = hg.Workspace()
    done = 0
    c = 0
    t0 = time.time()
    while done < n_pairs:
        B = min(chunk, n_pairs - done)
        S = cube_pairs(seed * 100_003 + c, B, n=n, max_angle_deg=max_angle_deg)
        off = S.offsets.numpy()
        src_f = hg.hgmm_build_batch(S.src, off, [cfg.src_levels] * B, reg_eps=cfg.reg_eps, min_mass=cfg.min_mass,
                                    ws=ws)
        tgt_f = hg.hgmm_build_batch(S.tgt, off, [cfg.tgt_levels] * B, reg_eps=cfg.reg_eps, min_mass=cfg.min_mass,
                                    ws=ws)
        X, frs, frt = features_for(src_f, tgt_f, B, cfg)
        lab = hg.hgmm_register_batch(src_f, S.tgt, off, max_iters=cfg.max_iters, lambda_c=cfg.lambda_c,
                                     R0=S.R_true.cpu().numpy(), t0=S.t_true.cpu().numpy(), ws=ws)
        R = torch.from_numpy(lab["R"].reshape(B, 9)).cuda()
        t = torch.from_numpy(lab["t"]).cuda()
        T = hg.hgmm_warm_head_target(R, t, frs, frt)
        Xs.append(X)
        Ts.append(T)
        done += B
        c += 1
        el = time.time() - t0
        if log:
            log(f"training pairs {done}/{n_pairs} ({el:.1f} s)")
        if time_budget_s is not None and done < n_pairs and el * (done + chunk) / done > time_budget_s:
            if log:
                log(f"stopping generation at {done} pairs (time budget {time_budget_s:.0f} s)")
            break
    return torch.cat(Xs).contiguous(), torch.cat(Ts).contiguous()


def train(mlp, X, T, epochs: int = 20, batch: int = 512, lr: float = 1e-3, lr_min: float = 1e-5, seed: int = 0,
          cfg: WarmConfig = WarmConfig(), log=None):
    """Adam with cosine learning-rate decay; returns the per-epoch mean losses."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    N = X.shape[0]
    steps_per_epoch = N // batch
    total = max(1, epochs * steps_per_epoch)
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g, device="cuda")
        acc, cnt = 0.0, 0
        for i in range(steps_per_epoch):
            idx = perm[i * batch:(i + 1) * batch]
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            rate = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / total))
            want = (i % 50 == 0) or i == steps_per_epoch - 1
            loss = mlp.train_step(xb, tb, rate, cfg.trans_weight, want_loss=want)
            if want:
                acc += loss
                cnt += 1
            step += 1
        hist.append(acc / max(cnt, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.5f}")
    return hist


def register_warm(mlp, src, tgt, src_off, tgt_off, src_levels, cfg: WarmConfig = WarmConfig(), ws=None,
                  src_forest=None, fallback: str = "plain", forest=None):
    """Warm-started batched registration with the likelihood fallback
    (``fallback`` = "plain" or "identity", see the module docstring).

    Without ``src_forest`` the source and target trees are built as one
    forest of 2B trees (source b is tree b, target b is tree B + b);
    ``forest`` (optional) is a handle of an earlier call to rebuild in place.
    With ``src_forest`` (B source trees) only the target forest is built.

    Returns dict(R (B,3,3), t, iters, loglik, fallback (B,) bool, R0, t0,
    forest) where forest holds the source trees 0..B-1."""
    ws = ws or hg.Workspace()
    B = len(src_levels)
    if src_forest is None:
        both = torch.cat([src, tgt], dim=1).contiguous()
        src_off = np.asarray(src_off, dtype=np.int64)
        off = np.concatenate([src_off, np.asarray(tgt_off, dtype=np.int64)[1:] + src_off[-1]])
        levels = [int(v) for v in np.atleast_1d(src_levels)] + [cfg.tgt_levels] * B
        src_forest = hg.hgmm_build_batch(both, off, levels, reg_eps=cfg.reg_eps, min_mass=cfg.min_mass, ws=ws,
                                         forest=forest)
        tgt_forest, tgt_first = src_forest, B
    else:
        tgt_forest = hg.hgmm_build_batch(tgt, tgt_off, [cfg.tgt_levels] * B, reg_eps=cfg.reg_eps,
                                         min_mass=cfg.min_mass, ws=ws)
        tgt_first = 0
    X, frs, frt = features_for(src_forest, tgt_forest, B, cfg, tgt_first)
    Y = mlp.forward(X)
    R0, t0 = hg.hgmm_warm_head_pose(Y, frs, frt)
    R0 = R0.cpu().numpy().reshape(B, 3, 3)
    t0 = t0.cpu().numpy()
    # coarse to fine from the head's transforms, then the fallback rule (one
    # library call)
    r = hg.hgmm_register_warm_batch(src_forest, tgt, tgt_off, R0, t0, coarse_levels=cfg.coarse_levels, rule=fallback,
                                    max_iters=cfg.max_iters, lambda_c=cfg.lambda_c, ws=ws)
    r.update(R0=R0, t0=t0, forest=src_forest)
    return r


def rotation_errors_deg(R, R_true):
    R = np.asarray(R).reshape(-1, 3, 3)
    Rt = np.asarray(R_true).reshape(-1, 3, 3)
    c = (np.einsum("bij,bij->b", R, Rt) - 1.0) / 2.0
    return np.degrees(np.arccos(np.clip(c, -1.0, 1.0)))
