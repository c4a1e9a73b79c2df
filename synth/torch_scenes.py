"""Batched GPU generator of unit-cube plane+sphere pairs (training inputs).

Same scene distribution as ``scenes.small_pair``: 4 planes (normal on S2,
anchor in [-0.25, 0.25]^3, sqrt(3)-side patch clipped to the cube) and 2
spheres (r in [0.1, 0.3], inside the cube), area-proportional counts (largest
remainder), independent source and target resampling, isotropic noise, target
moved by a random axis/angle/translation.  It draws from torch's CUDA
generator, so its pairs differ from the NumPy generator's for the same seed;
it exists to synthesise the hundreds of thousands of pairs the learned warm
start trains on.  Inputs only: no registration arithmetic.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import torch


@dataclass
class TorchPairs:
    src: torch.Tensor      # (3, B*n) float32, CSR by offsets
    tgt: torch.Tensor      # (3, B*n) float32
    offsets: torch.Tensor  # (B+1,) int64 (host)
    R_true: torch.Tensor   # (B, 3, 3) float64: src ~= R_true @ tgt + t_true
    t_true: torch.Tensor   # (B, 3) float64
    angle_deg: torch.Tensor


def _unit(x):
    return x / x.norm(dim=-1, keepdim=True).clamp_min(1e-12)


def _rodrigues(axis, ang):
    a = _unit(axis)
    K = torch.zeros(a.shape[0], 3, 3, dtype=a.dtype, device=a.device)
    K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -a[:, 2], a[:, 1], -a[:, 0]
    K = K - K.transpose(1, 2)
    s, c = torch.sin(ang)[:, None, None], torch.cos(ang)[:, None, None]
    eye = torch.eye(3, dtype=a.dtype, device=a.device).expand_as(K)
    return eye + s * K + (1 - c) * (K @ K)


def _largest_remainder(w, total):
    q = w / w.sum(1, keepdim=True) * total
    base = q.floor()
    rem = (total - base.sum(1)).long()
    order = torch.argsort(-(q - base), dim=1)
    ranks = torch.empty_like(order)
    ranks.scatter_(1, order, torch.arange(w.shape[1], device=w.device).expand_as(order))
    return (base + (ranks < rem[:, None]).double()).long()


def cube_pairs(seed: int, B: int, n: int = 10_000, max_angle_deg: float = 90.0, max_trans: float = 0.1,
               noise: float = 0.005, device="cuda") -> TorchPairs:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = dict(dtype=torch.float64, device=device)

    def rnd(*shape):
        return torch.rand(*shape, generator=g, **f64)

    def nrm(*shape):
        return torch.randn(*shape, generator=g, **f64)

    normals = _unit(nrm(B, 4, 3))
    anchors = rnd(B, 4, 3) * 0.5 - 0.25
    helper = torch.where((normals[..., :1].abs() < 0.9), torch.tensor([1.0, 0.0, 0.0], **f64),
                         torch.tensor([0.0, 1.0, 0.0], **f64))
    u = _unit(torch.cross(normals, helper, dim=-1))
    v = torch.cross(normals, u, dim=-1)
    side = math.sqrt(3.0)
    st = (rnd(B, 4, 4096, 2) - 0.5) * side
    mc = anchors[:, :, None] + st[..., :1] * u[:, :, None] + st[..., 1:] * v[:, :, None]
    frac = (mc.abs() <= 0.5).all(-1).double().mean(-1).clamp_min(1e-3)
    r = 0.1 + 0.2 * rnd(B, 2)
    centres = (rnd(B, 2, 3) * 2 - 1) * (0.5 - r[..., None])
    areas = torch.cat([3.0 * frac, 4 * math.pi * r * r], dim=1)  # (B, 6)
    counts = _largest_remainder(areas, n)                        # (B, 6)

    def sample():
        ends = counts.cumsum(1)
        idx = torch.arange(n, device=device)[None].expand(B, n)
        surf = torch.searchsorted(ends, idx.contiguous(), right=True).clamp_max(5)  # (B, n)
        pts = torch.empty(B, n, 3, **f64)
        is_plane = surf < 4
        # planes: rejection sampling inside the cube
        ps = surf.clamp_max(3)
        a = torch.gather(anchors, 1, ps[..., None].expand(B, n, 3))
        uu = torch.gather(u, 1, ps[..., None].expand(B, n, 3))
        vv = torch.gather(v, 1, ps[..., None].expand(B, n, 3))
        todo = is_plane.clone()
        while bool(todo.any()):
            s2 = (rnd(B, n, 2) - 0.5) * side
            cand = a + s2[..., :1] * uu + s2[..., 1:] * vv
            ok = todo & (cand.abs() <= 0.5).all(-1)
            pts[ok] = cand[ok]
            todo = todo & ~ok
        # spheres: uniform on the surface
        ss = (surf - 4).clamp(0, 1)
        c = torch.gather(centres, 1, ss[..., None].expand(B, n, 3))
        rr = torch.gather(r, 1, ss)
        sph = c + rr[..., None] * _unit(nrm(B, n, 3))
        pts = torch.where(is_plane[..., None], pts, sph)
        return pts

    src = sample()
    tgt = sample()
    src = src + noise * nrm(B, n, 3)
    tgt = tgt + noise * nrm(B, n, 3)
    axis = nrm(B, 3)
    ang = torch.deg2rad(rnd(B) * max_angle_deg)
    Rg = _rodrigues(axis, ang)
    tg = (rnd(B, 3) * 2 - 1) * max_trans
    tgt = torch.einsum("bij,bnj->bni", Rg, tgt) + tg[:, None]
    soa = lambda p: p.reshape(B * n, 3).T.contiguous().float()
    offsets = torch.arange(B + 1, dtype=torch.int64) * n
    R_true = Rg.transpose(1, 2).contiguous()
    t_true = -torch.einsum("bij,bj->bi", R_true, tg)
    return TorchPairs(src=soa(src), tgt=soa(tgt), offsets=offsets, R_true=R_true, t_true=t_true,
                      angle_deg=torch.rad2deg(ang))


def uneven_batch(seed_base: int = 3000, count: int = 256, n_min: int = 2_000, n_max: int = 200_000,
                 max_angle_deg: float = 45.0, leaf_points: float = 50.0, device="cuda"):
    """``count`` pairs with N log-uniform in [n_min, n_max] (same N draw as the
    NumPy ``scenes.uneven_batch``), concatenated CSR; tree depth per pair is
    ceil(log8(N / leaf_points)).  Returns (src, tgt, offsets (B+1,), levels (B,),
    R_true (B,3,3), t_true (B,3)) with the clouds on ``device``."""
    import numpy as np
    srcs, tgts, Rs, ts, lv, ns = [], [], [], [], [], []
    for k in range(count):
        g = np.random.Generator(np.random.PCG64(np.random.SeedSequence((seed_base + k, 7))))
        nk = int(round(math.exp(g.uniform(math.log(n_min), math.log(n_max)))))
        P = cube_pairs(seed_base + k, 1, n=nk, max_angle_deg=max_angle_deg, device=device)
        srcs.append(P.src)
        tgts.append(P.tgt)
        Rs.append(P.R_true[0])
        ts.append(P.t_true[0])
        lv.append(max(1, int(math.ceil(math.log(nk / leaf_points, 8)))))
        ns.append(nk)
    off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    return (torch.cat(srcs, 1).contiguous(), torch.cat(tgts, 1).contiguous(), off, np.array(lv, np.int32),
            torch.stack(Rs).cpu().numpy(), torch.stack(ts).cpu().numpy())
