"""Train and evaluate the warm-start network on generated pairs.

    python -m paper_1807_02587_amd.train_warm --pairs 200000 --epochs 20 \
        --out weights.npy --report report.json

Training pairs: unit-cube plane+sphere scenes, 10k points per cloud, rotation
angle U(0, 90 deg), translation U(-0.1, 0.1)^3; label = the plain method's
converged pose started at the ground truth.  Evaluation: held-out pairs
(seeds >= 1e6) registered by the plain method from the identity and by the
warm start under both fallback rules (plain-method likelihood, the default;
identity-pose likelihood).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import api as hg
from . import warmstart as W


def log(msg):
    print(msg, flush=True)


def evaluate(net, n_pairs=4096, chunk=512, n=10_000, max_angle_deg=90.0, cfg=W.WarmConfig(), seed=10**6,
             fallback="plain"):
    from synth.torch_scenes import cube_pairs
    err_plain, err_warm, fb, it_plain, it_warm, t_plain, t_warm = [], [], [], [], [], 0.0, 0.0
    ws = hg.Workspace()
    done = 0
    c = 0
    while done < n_pairs:
        B = min(chunk, n_pairs - done)
        S = cube_pairs(seed + c, B, n=n, max_angle_deg=max_angle_deg)
        off = S.offsets.numpy()
        Rt = S.R_true.cpu().numpy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        forest = hg.hgmm_build_batch(S.src, off, [cfg.src_levels] * B, reg_eps=cfg.reg_eps, min_mass=cfg.min_mass,
                                     ws=ws)
        rp = hg.hgmm_register_batch(forest, S.tgt, off, max_iters=cfg.max_iters, lambda_c=cfg.lambda_c, ws=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rw = W.register_warm(net, S.src, S.tgt, off, off, [cfg.src_levels] * B, cfg, ws=ws, fallback=fallback)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_plain += t1 - t0
        t_warm += t2 - t1
        err_plain.append(W.rotation_errors_deg(rp["R"], Rt))
        err_warm.append(W.rotation_errors_deg(rw["R"], Rt))
        fb.append(rw["fallback"])
        it_plain.append(rp["iters"])
        it_warm.append(rw["iters"])
        done += B
        c += 1
        log(f"evaluated {done}/{n_pairs} pairs: plain median {np.median(np.concatenate(err_plain)):.3f} deg, "
            f"warm median {np.median(np.concatenate(err_warm)):.3f} deg")
    ep, ew, fb = np.concatenate(err_plain), np.concatenate(err_warm), np.concatenate(fb)
    stats = lambda e: dict(median_deg=float(np.median(e)), p90_deg=float(np.percentile(e, 90)),
                           success_0p5=float(np.mean(e <= 0.5)), success_5=float(np.mean(e <= 5.0)))
    return dict(pairs=n_pairs, points_per_cloud=n, max_angle_deg=max_angle_deg, fallback_rule=fallback,
                plain=dict(**stats(ep), mean_iters=float(np.mean(np.concatenate(it_plain))),
                           pairs_per_s=n_pairs / t_plain),
                warm=dict(**stats(ew), mean_iters=float(np.mean(np.concatenate(it_warm))),
                          pairs_per_s=n_pairs / t_warm, fallback_rate=float(np.mean(fb)),
                          worse_than_plain=float(np.mean(ew > ep + 1e-6))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=200_000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-pairs", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--out", default=None)
    ap.add_argument("--report", default=None)
    ap.add_argument("--gen-budget-s", type=float, default=None, help="stop generating pairs after about this long")
    ap.add_argument("--init", default=None, help="start from these weights (.npy) instead of a fresh network")
    args = ap.parse_args()
    cfg = W.WarmConfig()
    t0 = time.time()
    X, T = W.training_set(args.pairs, seed=args.seed, cfg=cfg, log=log, time_budget_s=args.gen_budget_s)
    log(f"training set: {X.shape[0]} pairs in {time.time() - t0:.1f} s")
    net = hg.MLP(seed=args.seed)
    if args.init:
        net.set_params(np.load(args.init))
    t1 = time.time()
    hist = W.train(net, X, T, epochs=args.epochs, batch=args.batch, lr=args.lr, cfg=cfg, log=log)
    log(f"training: {time.time() - t1:.1f} s")
    if args.out:
        np.save(args.out, net.get_params())
    rep = evaluate(net, n_pairs=args.eval_pairs, cfg=cfg, fallback="plain")
    rep["identity_rule"] = evaluate(net, n_pairs=args.eval_pairs, cfg=cfg, fallback="identity")["warm"]
    rep.update(train_pairs=int(X.shape[0]), epochs=args.epochs, loss_history=hist, train_seconds=time.time() - t1,
               generation_seconds=t1 - t0)
    log(json.dumps(rep))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
