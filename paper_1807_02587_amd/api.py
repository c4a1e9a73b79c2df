"""Python names for the C ABI (argument marshalling; no arithmetic of the method)."""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import BuildParams, RegParams, TreeHost, check


def library_path() -> str:
    _lib.load()
    return _lib.LIB_PATH


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _cloud(xyz: torch.Tensor) -> torch.Tensor:
    if not (isinstance(xyz, torch.Tensor) and xyz.is_cuda and xyz.dtype == torch.float32 and xyz.dim() == 2
            and xyz.shape[0] == 3 and xyz.is_contiguous()):
        raise ValueError("points must be a contiguous float32 CUDA tensor of shape (3, N) (SoA)")
    return xyz


class Workspace:
    """Grow-only device scratch buffer handed to the library."""

    def __init__(self, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        return self.buf

    def ptr(self, nbytes: int):
        b = self.get(nbytes)
        return C.c_void_p(b.data_ptr()), C.c_size_t(b.numel())


def hgmm_tree_nodes(levels: int) -> int:
    return int(_lib.load().hgmm_tree_nodes(levels))


def hgmm_level_offset(level: int) -> int:
    return int(_lib.load().hgmm_level_offset(level))


def hgmm_set_tuning(fused_max=-1, min_tile=-1, target_tiles=-1, max_tile=-1, reg_tile=-1):
    check(_lib.load().hgmm_set_tuning(fused_max, min_tile, target_tiles, max_tile, reg_tile), "hgmm_set_tuning")


class Tree:
    """Owning wrapper of an hgmm_tree handle."""

    def __init__(self, handle: C.c_void_p, n_points: int, levels: int, ntrees: int = 1):
        self.handle = handle
        self.n_points = n_points
        self.levels = levels
        self.ntrees = ntrees

    def __del__(self):
        try:
            if self.handle is not None and self.handle.value:
                _lib.load().hgmm_tree_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def info(self, index: int = 0):
        lv = C.c_int(0)
        nn = C.c_int64(0)
        org = (C.c_double * 3)()
        ext = C.c_double(0)
        check(_lib.load().hgmm_tree_info(self.handle, index, C.byref(lv), C.byref(nn), org, C.byref(ext)),
              "hgmm_tree_info")
        return dict(levels=lv.value, n_nodes=nn.value, origin=np.array(org[:]), extent=ext.value)

    def export(self, index: int = 0) -> dict:
        inf = self.info(index)
        n = inf["n_nodes"]
        out = dict(live=np.zeros(n, np.int32), has_children=np.zeros(n, np.int32), count=np.zeros(n, np.int64),
                   pi=np.zeros(n), pig=np.zeros(n), mu=np.zeros((n, 3)), cov=np.zeros((n, 6)),
                   lam=np.zeros((n, 3)), evec=np.zeros((n, 3, 3)), kappa=np.zeros(n))
        th = TreeHost()
        for k, v in out.items():
            setattr(th, k, v.ctypes.data)
        check(_lib.load().hgmm_tree_export(self.handle, index, C.byref(th)), "hgmm_tree_export")
        out.update(levels=th.levels, n_points=th.n_points, origin=np.array(th.origin[:]), extent=th.extent)
        return out

    def labels(self, index: int = 0, n_points: int | None = None, stream=None) -> torch.Tensor:
        n = self.n_points if n_points is None else n_points
        lab = torch.empty((self.levels, n), dtype=torch.int32, device="cuda")
        check(_lib.load().hgmm_tree_labels(self.handle, index, C.c_void_p(lab.data_ptr()), _stream(stream)),
              "hgmm_tree_labels")
        torch.cuda.current_stream().synchronize()
        return lab


def hgmm_build(xyz: torch.Tensor, levels: int = 2, build_iters: int = 30, reg_eps: float = 1e-6,
               min_mass: float = 1.0, ws: Workspace | None = None, tree: Tree | None = None, stream=None) -> Tree:
    xyz = _cloud(xyz)
    lib = _lib.load()
    n = xyz.shape[1]
    p = BuildParams(levels, build_iters, reg_eps, min_mass)
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_build_workspace_bytes(n, levels))
    h = C.c_void_p(tree.handle.value if tree is not None else None)
    check(lib.hgmm_build(C.c_void_p(xyz.data_ptr()), n, C.byref(p), wptr, wlen, _stream(stream), C.byref(h)),
          "hgmm_build")
    if tree is not None:
        tree.handle, tree.n_points, tree.levels = h, n, levels
        return tree
    return Tree(h, n, levels)


def _pose_args(R0, t0):
    R = None if R0 is None else np.ascontiguousarray(np.asarray(R0, dtype=np.float64).reshape(9))
    t = None if t0 is None else np.ascontiguousarray(np.asarray(t0, dtype=np.float64).reshape(3))
    return R, t


def hgmm_register(tree: Tree, xyz: torch.Tensor, max_iters: int = 30, lambda_c: float = 0.01,
                  tol_rot: float = 1e-6, tol_trans_rel: float = 1e-6, R0=None, t0=None,
                  ws: Workspace | None = None, stream=None, raise_singular: bool = True) -> dict:
    xyz = _cloud(xyz)
    lib = _lib.load()
    n = xyz.shape[1]
    p = RegParams(max_iters, 0, lambda_c, tol_rot, tol_trans_rel)
    R0a, t0a = _pose_args(R0, t0)
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_register_workspace_bytes(n, tree.levels))
    R = np.zeros(9)
    t = np.zeros(3)
    iters = C.c_int(0)
    ll = C.c_double(0)
    rc = lib.hgmm_register(tree.handle, C.c_void_p(xyz.data_ptr()), n, C.byref(p),
                           None if R0a is None else R0a.ctypes.data_as(C.c_void_p),
                           None if t0a is None else t0a.ctypes.data_as(C.c_void_p), wptr, wlen, _stream(stream),
                           R.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p), C.byref(iters), C.byref(ll))
    if rc != 0 and (raise_singular or rc != -6):
        check(rc, "hgmm_register")
    return dict(R=R.reshape(3, 3), t=t, iters=iters.value, loglik=ll.value, status=rc)


def hgmm_estep(tree: Tree, xyz: torch.Tensor, R=None, t=None, lambda_c: float = 0.01, ws: Workspace | None = None,
               points: bool = True, loglik: bool = True, stream=None) -> dict:
    xyz = _cloud(xyz)
    lib = _lib.load()
    n = xyz.shape[1]
    R = np.eye(3) if R is None else R
    t = np.zeros(3) if t is None else t
    Ra, ta = _pose_args(R, t)
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_register_workspace_bytes(n, tree.levels))
    nn = hgmm_tree_nodes(tree.levels)
    bins = torch.empty((nn, 6), dtype=torch.float64, device=xyz.device)
    stop = torch.empty(n, dtype=torch.int32, device=xyz.device) if points else None
    gam = torch.empty(n, dtype=torch.float32, device=xyz.device) if points else None
    ll = C.c_double(0)
    check(lib.hgmm_estep(tree.handle, C.c_void_p(xyz.data_ptr()), n, Ra.ctypes.data_as(C.c_void_p),
                         ta.ctypes.data_as(C.c_void_p), lambda_c, wptr, wlen, _stream(stream),
                         None if stop is None else C.c_void_p(stop.data_ptr()),
                         None if gam is None else C.c_void_p(gam.data_ptr()), C.c_void_p(bins.data_ptr()),
                         C.byref(ll) if loglik else None), "hgmm_estep")
    torch.cuda.current_stream().synchronize()
    return dict(stop_node=stop, gamma=gam, bins=bins, loglik=ll.value if loglik else None)


def hgmm_normal_equations(tree: Tree, bins: torch.Tensor, n: int, ws: Workspace | None = None, stream=None):
    lib = _lib.load()
    if not (bins.is_cuda and bins.dtype == torch.float64 and bins.is_contiguous()):
        raise ValueError("bins must be a contiguous float64 CUDA tensor")
    ws = ws or Workspace(bins.device)
    wptr, wlen = ws.ptr(lib.hgmm_register_workspace_bytes(n, tree.levels))
    H = np.zeros(36)
    g = np.zeros(6)
    check(lib.hgmm_normal_equations(tree.handle, C.c_void_p(bins.data_ptr()), n, wptr, wlen, _stream(stream),
                                    H.ctypes.data_as(C.c_void_p), g.ctypes.data_as(C.c_void_p)),
          "hgmm_normal_equations")
    return H.reshape(6, 6), g


def hgmm_tree_import(src, stream=None) -> Tree:
    """Device tree from a host tree (an object or dict with the hgmm_tree_host fields)."""
    get = (lambda k: src[k]) if isinstance(src, dict) else (lambda k: getattr(src, k))
    levels = int(get("levels"))
    keep = {}
    th = TreeHost()
    th.levels = levels
    th.n_points = int(get("n_points"))
    th.origin[:] = [float(v) for v in np.asarray(get("origin"))]
    th.extent = float(get("extent"))
    for k, dt in (("live", np.int32), ("has_children", np.int32), ("count", np.int64), ("pi", np.float64),
                  ("pig", np.float64), ("mu", np.float64), ("cov", np.float64), ("lam", np.float64),
                  ("evec", np.float64), ("kappa", np.float64)):
        a = np.ascontiguousarray(np.asarray(get(k), dtype=dt))
        keep[k] = a
        setattr(th, k, a.ctypes.data)
    h = C.c_void_p(None)
    check(_lib.load().hgmm_tree_import(C.byref(th), _stream(stream), C.byref(h)), "hgmm_tree_import")
    return Tree(h, int(get("n_points")), levels)


PROFILE_KINDS = {"em_tile": 0, "em_fused": 1, "partition": 2, "scatter": 3, "descend": 4, "normal": 5, "root": 6}


def hgmm_profile(enable: bool = True) -> None:
    check(_lib.load().hgmm_profile(1 if enable else 0), "hgmm_profile")


def hgmm_profile_reset() -> None:
    _lib.load().hgmm_profile_reset()


def hgmm_profile_read(kind) -> dict:
    k = PROFILE_KINDS[kind] if isinstance(kind, str) else int(kind)
    ms = C.c_double(0)
    n = C.c_int64(0)
    u = C.c_double(0)
    check(_lib.load().hgmm_profile_read(k, C.byref(ms), C.byref(n), C.byref(u)), "hgmm_profile_read")
    return dict(ms=ms.value, launches=n.value, units=u.value)
