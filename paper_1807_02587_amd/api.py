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


def _dev(t, shape, dtype, name):
    """Require a contiguous CUDA tensor of exactly this shape and dtype (None = any size)."""
    ok = (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
          and t.dim() == len(shape) and all(s is None or s == d for s, d in zip(shape, t.shape)))
    if not ok:
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of shape {shape}, "
                         f"got {getattr(t, 'dtype', type(t))} {tuple(getattr(t, 'shape', ()))}")
    return t


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


TUNING_KEYS = ("block64_max", "block256_max", "block512_max", "min_tile", "target_tiles", "max_tile", "reg_tile",
               "reg_chunk", "reg_graph", "reg_sort", "tile_threads", "reg_lds_levels", "build_graph", "reg_atomics",
               "fold_tiles")


def hgmm_get_tuning() -> dict:
    t = _lib.Tuning()
    check(_lib.load().hgmm_get_tuning(C.byref(t)), "hgmm_get_tuning")
    return {k: int(getattr(t, k)) for k in TUNING_KEYS}


def hgmm_autotune(src: torch.Tensor, src_offsets, levels, tgt: torch.Tensor | None = None, tgt_offsets=None,
                  build_iters: int = 30, reg_eps: float = 1e-6, min_mass: float = 1.0, max_iters: int = 30,
                  lambda_c: float = 0.01, tol_rot: float = 1e-6, tol_trans_rel: float = 1e-6, reps: int = 2,
                  passes: int = 2, ws: "Workspace | None" = None, stream=None) -> dict:
    """Time candidate launch shapes on this batch (construction, plus registration
    from the identity when ``tgt`` is given) and keep the fastest in effect."""
    src = _cloud(src)
    lib = _lib.load()
    soff = np.ascontiguousarray(np.asarray(src_offsets, dtype=np.int64))
    lev = np.ascontiguousarray(np.asarray(levels, dtype=np.int32))
    B = len(lev)
    assert soff.shape == (B + 1,) and soff[-1] == src.shape[1]
    bp = BuildParams(int(lev.max()), build_iters, reg_eps, min_mass)
    rp = RegParams(max_iters, 0, lambda_c, tol_rot, tol_trans_rel)
    toff = None
    if tgt is not None:
        tgt = _cloud(tgt)
        toff = np.ascontiguousarray(np.asarray(tgt_offsets, dtype=np.int64))
        assert toff.shape == (B + 1,) and toff[-1] == tgt.shape[1]
    need = lib.hgmm_autotune_workspace_bytes(soff.ctypes.data_as(C.c_void_p), lev.ctypes.data_as(C.c_void_p),
                                             None if toff is None else toff.ctypes.data_as(C.c_void_p), B)
    if need == 0:
        raise ValueError("invalid offsets or levels")
    ws = ws or Workspace(src.device)
    wptr, wlen = ws.ptr(need)
    best = _lib.Tuning()
    bms, sms = C.c_double(0), C.c_double(0)
    check(lib.hgmm_autotune(C.c_void_p(src.data_ptr()), soff.ctypes.data_as(C.c_void_p), lev.ctypes.data_as(C.c_void_p),
                            B, None if tgt is None else C.c_void_p(tgt.data_ptr()),
                            None if toff is None else toff.ctypes.data_as(C.c_void_p), C.byref(bp), C.byref(rp), wptr,
                            wlen, _stream(stream), reps, passes, C.byref(best), C.byref(bms), C.byref(sms)),
          "hgmm_autotune")
    return dict(tuning={k: int(getattr(best, k)) for k in TUNING_KEYS}, best_ms=bms.value, start_ms=sms.value)


def hgmm_set_tuning(**knobs) -> dict:
    """Change some launch shapes (names as in TUNING_KEYS); returns the previous setting."""
    old = hgmm_get_tuning()
    unknown = set(knobs) - set(TUNING_KEYS)
    if unknown:
        raise KeyError(f"unknown tuning knobs {sorted(unknown)}")
    new = dict(old, **{k: int(v) for k, v in knobs.items()})
    t = _lib.Tuning(*[new[k] for k in TUNING_KEYS])
    check(_lib.load().hgmm_set_tuning(C.byref(t)), "hgmm_set_tuning")
    return old


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

    def graph_stats(self) -> dict:
        """Constructions of this handle so far: graph replays, graphs captured,
        host-planned constructions (see build_graph in hgmm_tuning)."""
        r, c, h = C.c_int64(0), C.c_int64(0), C.c_int64(0)
        check(_lib.load().hgmm_build_graph_stats(self.handle, C.byref(r), C.byref(c), C.byref(h)),
              "hgmm_build_graph_stats")
        return dict(replays=r.value, captures=c.value, host_builds=h.value)

    def labels(self, index: int = 0, n_points: int | None = None, stream=None) -> torch.Tensor:
        """(levels, n) int32 most-likely-child labels of tree ``index`` (local node index at each level)."""
        if getattr(self, "offsets", None) is not None:
            n, L = int(self.offsets[index + 1] - self.offsets[index]), int(self.tree_levels[index])
        else:
            n, L = self.n_points, self.levels
        n = n if n_points is None else n_points
        lab = torch.empty((L, n), dtype=torch.int32, device="cuda")
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
                  ws: Workspace | None = None, stream=None, raise_singular: bool = True, max_levels: int = 0) -> dict:
    xyz = _cloud(xyz)
    lib = _lib.load()
    n = xyz.shape[1]
    p = RegParams(max_iters, max_levels, lambda_c, tol_rot, tol_trans_rel)
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


def hgmm_register_noalloc(tree: Tree, xyz: torch.Tensor, max_iters: int = 30, lambda_c: float = 0.01,
                          tol_rot: float = 1e-6, tol_trans_rel: float = 1e-6, R0=None, t0=None, stream=None,
                          raise_singular: bool = True, max_levels: int = 0) -> dict:
    """hgmm_register with the library's static scratch instead of a workspace
    (the call allocates nothing; calls that overlap on one device race)."""
    xyz = _cloud(xyz)
    lib = _lib.load()
    n = xyz.shape[1]
    p = RegParams(max_iters, max_levels, lambda_c, tol_rot, tol_trans_rel)
    R0a, t0a = _pose_args(R0, t0)
    R = np.zeros(9)
    t = np.zeros(3)
    iters = C.c_int(0)
    ll = C.c_double(0)
    rc = lib.hgmm_register_noalloc(tree.handle, C.c_void_p(xyz.data_ptr()), n, C.byref(p),
                                   None if R0a is None else R0a.ctypes.data_as(C.c_void_p),
                                   None if t0a is None else t0a.ctypes.data_as(C.c_void_p), _stream(stream),
                                   R.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p), C.byref(iters),
                                   C.byref(ll))
    if rc != 0 and (raise_singular or rc != -6):
        check(rc, "hgmm_register_noalloc")
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


def hgmm_register_flat(tree: Tree, xyz: torch.Tensor, level: int, max_iters: int = 30, tol_rot: float = 1e-6,
                       tol_trans_rel: float = 1e-6, R0=None, t0=None, ws: Workspace | None = None, stream=None,
                       raise_singular: bool = True) -> dict:
    """Registration with the single-level variant: the live nodes of tree level
    ``level`` as one mixture, every component scored for every point."""
    xyz = _cloud(xyz)
    lib = _lib.load()
    n = xyz.shape[1]
    p = RegParams(max_iters, 0, 0.0, tol_rot, tol_trans_rel)
    R0a, t0a = _pose_args(R0, t0)
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_register_workspace_bytes(n, tree.levels))
    R = np.zeros(9)
    t = np.zeros(3)
    iters = C.c_int(0)
    ll = C.c_double(0)
    rc = lib.hgmm_register_flat(tree.handle, C.c_void_p(xyz.data_ptr()), n, int(level), C.byref(p),
                                None if R0a is None else R0a.ctypes.data_as(C.c_void_p),
                                None if t0a is None else t0a.ctypes.data_as(C.c_void_p), wptr, wlen, _stream(stream),
                                R.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p), C.byref(iters),
                                C.byref(ll))
    if rc != 0 and (raise_singular or rc != -6):
        check(rc, "hgmm_register_flat")
    return dict(R=R.reshape(3, 3), t=t, iters=iters.value, loglik=ll.value, status=rc)


def hgmm_estep_flat(tree: Tree, xyz: torch.Tensor, level: int, R=None, t=None, ws: Workspace | None = None,
                    points: bool = True, loglik: bool = True, stream=None) -> dict:
    """One single-level E-step over tree level ``level`` at a fixed transform."""
    xyz = _cloud(xyz)
    lib = _lib.load()
    n = xyz.shape[1]
    Ra, ta = _pose_args(np.eye(3) if R is None else R, np.zeros(3) if t is None else t)
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_register_workspace_bytes(n, tree.levels))
    bins = torch.empty((hgmm_tree_nodes(tree.levels), 6), dtype=torch.float64, device=xyz.device)
    stop = torch.empty(n, dtype=torch.int32, device=xyz.device) if points else None
    gam = torch.empty(n, dtype=torch.float32, device=xyz.device) if points else None
    ll = C.c_double(0)
    check(lib.hgmm_estep_flat(tree.handle, C.c_void_p(xyz.data_ptr()), n, int(level), Ra.ctypes.data_as(C.c_void_p),
                              ta.ctypes.data_as(C.c_void_p), wptr, wlen, _stream(stream),
                              None if stop is None else C.c_void_p(stop.data_ptr()),
                              None if gam is None else C.c_void_p(gam.data_ptr()), C.c_void_p(bins.data_ptr()),
                              C.byref(ll) if loglik else None), "hgmm_estep_flat")
    torch.cuda.current_stream().synchronize()
    return dict(stop_node=stop, gamma=gam, bins=bins, loglik=ll.value if loglik else None)


def hgmm_register_soft(tree: Tree, xyz: torch.Tensor, tau: float = 0.01, max_iters: int = 30,
                       lambda_c: float = 0.01, tol_rot: float = 1e-6, tol_trans_rel: float = 1e-6, R0=None, t0=None,
                       ws: Workspace | None = None, stream=None, raise_singular: bool = True) -> dict:
    """Registration with the soft multi-path E-step (branches with path expectation >= tau)."""
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
    rc = lib.hgmm_register_soft(tree.handle, C.c_void_p(xyz.data_ptr()), n, float(tau), C.byref(p),
                                None if R0a is None else R0a.ctypes.data_as(C.c_void_p),
                                None if t0a is None else t0a.ctypes.data_as(C.c_void_p), wptr, wlen, _stream(stream),
                                R.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p), C.byref(iters),
                                C.byref(ll))
    if rc != 0 and (raise_singular or rc != -6):
        check(rc, "hgmm_register_soft")
    return dict(R=R.reshape(3, 3), t=t, iters=iters.value, loglik=ll.value, status=rc)


def hgmm_estep_soft(tree: Tree, xyz: torch.Tensor, tau: float = 0.01, R=None, t=None, lambda_c: float = 0.01,
                    ws: Workspace | None = None, points: bool = True, loglik: bool = True, stream=None) -> dict:
    """One soft multi-path E-step at a fixed transform: per-node bins and, per
    point, the number of nodes reached."""
    xyz = _cloud(xyz)
    lib = _lib.load()
    n = xyz.shape[1]
    Ra, ta = _pose_args(np.eye(3) if R is None else R, np.zeros(3) if t is None else t)
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_register_workspace_bytes(n, tree.levels))
    bins = torch.empty((hgmm_tree_nodes(tree.levels), 6), dtype=torch.float64, device=xyz.device)
    stops = torch.empty(n, dtype=torch.int32, device=xyz.device) if points else None
    ll = C.c_double(0)
    check(lib.hgmm_estep_soft(tree.handle, C.c_void_p(xyz.data_ptr()), n, float(tau), Ra.ctypes.data_as(C.c_void_p),
                              ta.ctypes.data_as(C.c_void_p), float(lambda_c), wptr, wlen, _stream(stream),
                              None if stops is None else C.c_void_p(stops.data_ptr()), C.c_void_p(bins.data_ptr()),
                              C.byref(ll) if loglik else None), "hgmm_estep_soft")
    torch.cuda.current_stream().synchronize()
    return dict(stops=stops, bins=bins, loglik=ll.value if loglik else None)


def hgmm_point_loglik(tree: Tree, xyz: torch.Tensor, R=None, t=None, lambda_c: float = 0.01,
                      ws: Workspace | None = None, stream=None):
    """Per-point log density under the tree at the adaptive stop node (float32
    CUDA tensor) and the stop nodes (int32)."""
    xyz = _cloud(xyz)
    lib = _lib.load()
    n = xyz.shape[1]
    Ra, ta = _pose_args(np.eye(3) if R is None else R, np.zeros(3) if t is None else t)
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_register_workspace_bytes(n, tree.levels))
    ll = torch.empty(n, dtype=torch.float32, device=xyz.device)
    node = torch.empty(n, dtype=torch.int32, device=xyz.device)
    check(lib.hgmm_point_loglik(tree.handle, C.c_void_p(xyz.data_ptr()), n, Ra.ctypes.data_as(C.c_void_p),
                                ta.ctypes.data_as(C.c_void_p), float(lambda_c), wptr, wlen, _stream(stream),
                                C.c_void_p(node.data_ptr()), C.c_void_p(ll.data_ptr())), "hgmm_point_loglik")
    return ll, node


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


PROFILE_KINDS = {"em_tile": 0, "em_block": 1, "partition": 2, "scatter": 3, "descend": 4, "normal": 5, "root": 6,
                 "em_mstep": 7, "flat": 8, "soft": 9}


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
    pts = C.c_double(0)
    lev = C.c_double(0)
    check(_lib.load().hgmm_profile_work(k, C.byref(pts), C.byref(lev)), "hgmm_profile_work")
    return dict(ms=ms.value, launches=n.value, units=u.value, points=pts.value, levels=lev.value)


def hgmm_build_batch(xyz: torch.Tensor, offsets, levels, build_iters: int = 30, reg_eps: float = 1e-6,
                     min_mass: float = 1.0, ws: Workspace | None = None, forest: Tree | None = None,
                     stream=None) -> Tree:
    """Forest of len(levels) trees from CSR-concatenated clouds (SoA (3, total))."""
    xyz = _cloud(xyz)
    lib = _lib.load()
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    lev = np.ascontiguousarray(np.asarray(levels, dtype=np.int32))
    B = len(lev)
    assert off.shape == (B + 1,) and off[-1] == xyz.shape[1]
    p = BuildParams(int(lev.max()), build_iters, reg_eps, min_mass)
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_build_batch_workspace_bytes(off.ctypes.data_as(C.c_void_p),
                                                             lev.ctypes.data_as(C.c_void_p), B))
    h = C.c_void_p(forest.handle.value if forest is not None else None)
    check(lib.hgmm_build_batch(C.c_void_p(xyz.data_ptr()), off.ctypes.data_as(C.c_void_p),
                               lev.ctypes.data_as(C.c_void_p), B, C.byref(p), wptr, wlen, _stream(stream),
                               C.byref(h)), "hgmm_build_batch")
    if forest is not None:
        forest.handle, forest.n_points, forest.levels, forest.ntrees = h, int(off[-1]), int(lev.max()), B
        forest.offsets, forest.tree_levels = off, lev
        return forest
    t = Tree(h, int(off[-1]), int(lev.max()), B)
    t.offsets, t.tree_levels = off, lev
    return t


def hgmm_register_batch(forest: Tree, xyz: torch.Tensor, offsets, max_iters: int = 30, lambda_c: float = 0.01,
                        tol_rot: float = 1e-6, tol_trans_rel: float = 1e-6, R0=None, t0=None, active=None,
                        ws: Workspace | None = None, stream=None, max_levels: int = 0) -> dict:
    xyz = _cloud(xyz)
    lib = _lib.load()
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    B = len(off) - 1
    p = RegParams(max_iters, max_levels, lambda_c, tol_rot, tol_trans_rel)
    R0a = None if R0 is None else np.ascontiguousarray(np.asarray(R0, dtype=np.float64).reshape(B, 9))
    t0a = None if t0 is None else np.ascontiguousarray(np.asarray(t0, dtype=np.float64).reshape(B, 3))
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_register_batch_workspace_bytes(forest.handle, off.ctypes.data_as(C.c_void_p), B))
    R = np.zeros((B, 9))
    t = np.zeros((B, 3))
    iters = np.zeros(B, np.int32)
    ll = np.zeros(B)
    st = np.zeros(B, np.int32)
    act = None if active is None else np.ascontiguousarray(np.asarray(active, dtype=np.int32))
    check(lib.hgmm_register_batch(forest.handle, C.c_void_p(xyz.data_ptr()), off.ctypes.data_as(C.c_void_p), B,
                                  C.byref(p), None if R0a is None else R0a.ctypes.data_as(C.c_void_p),
                                  None if t0a is None else t0a.ctypes.data_as(C.c_void_p),
                                  None if act is None else act.ctypes.data_as(C.c_void_p), wptr, wlen,
                                  _stream(stream), R.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p),
                                  iters.ctypes.data_as(C.c_void_p), ll.ctypes.data_as(C.c_void_p),
                                  st.ctypes.data_as(C.c_void_p)), "hgmm_register_batch")
    return dict(R=R.reshape(B, 3, 3), t=t, iters=iters, loglik=ll, status=st)


def hgmm_register_warm_batch(forest: Tree, xyz: torch.Tensor, offsets, R0, t0, coarse_levels: int = 2,
                             rule: str = "plain", max_iters: int = 30, lambda_c: float = 0.01, tol_rot: float = 1e-6,
                             tol_trans_rel: float = 1e-6, ws: Workspace | None = None, stream=None) -> dict:
    """Warm-started registration of B pairs (cloud b onto tree b) from R0, t0
    with the plain method from the identity as fallback and arbiter (rule
    "plain" or "identity"; see include/hgmm.h).  Returns dict(R (B,3,3), t,
    iters, loglik, status, fallback (B,) bool)."""
    xyz = _cloud(xyz)
    lib = _lib.load()
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    B = len(off) - 1
    if rule not in ("plain", "identity"):
        raise ValueError(f"unknown fallback rule {rule!r}")
    p = RegParams(max_iters, 0, lambda_c, tol_rot, tol_trans_rel)
    R0a = np.ascontiguousarray(np.asarray(R0, dtype=np.float64).reshape(B, 9))
    t0a = np.ascontiguousarray(np.asarray(t0, dtype=np.float64).reshape(B, 3))
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_register_batch_workspace_bytes(forest.handle, off.ctypes.data_as(C.c_void_p), B))
    R, t, ll = np.zeros((B, 9)), np.zeros((B, 3)), np.zeros(B)
    iters, st, fb = np.zeros(B, np.int32), np.zeros(B, np.int32), np.zeros(B, np.int32)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    check(lib.hgmm_register_warm_batch(forest.handle, C.c_void_p(xyz.data_ptr()), ptr(off), B, C.byref(p),
                                       int(coarse_levels), 0 if rule == "plain" else 1, ptr(R0a), ptr(t0a), wptr, wlen,
                                       _stream(stream), ptr(R), ptr(t), ptr(iters), ptr(ll), ptr(st), ptr(fb)),
          "hgmm_register_warm_batch")
    return dict(R=R.reshape(B, 3, 3), t=t, iters=iters, loglik=ll, status=st, fallback=fb.astype(bool))


def hgmm_odometry(xyz: torch.Tensor, offsets, levels: int, build_iters: int = 30, reg_eps: float = 1e-6,
                  min_mass: float = 1.0, max_iters: int = 30, lambda_c: float = 0.01, tol_rot: float = 1e-6,
                  tol_trans_rel: float = 1e-6, R0=None, t0=None, prior_restart: bool = False,
                  ws: Workspace | None = None, forest: Tree | None = None, stream=None) -> dict:
    """Frame-to-frame odometry over F frames concatenated CSR-style (SoA (3, total)):
    the trees of frames 0..F-2 built as one forest, frame k+1 registered onto
    tree k for every k in one call, the transforms chained into each frame's
    pose in frame 0.  Returns R_rel (F-1,3,3), t_rel (F-1,3), R_abs (F,3,3),
    t_abs (F,3), iters, status and the forest (tree k = frame k's model).
    prior_restart: a second start of every pair from the neighbouring pair's
    motion, keeping the run with the higher log-likelihood."""
    xyz = _cloud(xyz)
    lib = _lib.load()
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    F = len(off) - 1
    assert off[-1] == xyz.shape[1]
    bp = BuildParams(int(levels), build_iters, reg_eps, min_mass)
    rp = RegParams(max_iters, 0, lambda_c, tol_rot, tol_trans_rel)
    R0a = None if R0 is None else np.ascontiguousarray(np.asarray(R0, dtype=np.float64).reshape(F - 1, 9))
    t0a = None if t0 is None else np.ascontiguousarray(np.asarray(t0, dtype=np.float64).reshape(F - 1, 3))
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_odometry_workspace_bytes(off.ctypes.data_as(C.c_void_p), F, int(levels)))
    h = C.c_void_p(forest.handle.value if forest is not None else None)
    m = max(F - 1, 1)
    Rr, tr = np.zeros((m, 9)), np.zeros((m, 3))
    Ra, ta = np.zeros((m + 1, 9)), np.zeros((m + 1, 3))
    iters, st = np.zeros(m, np.int32), np.zeros(m, np.int32)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    check(lib.hgmm_odometry(C.c_void_p(xyz.data_ptr()), ptr(off), F, C.byref(bp), C.byref(rp),
                            None if R0a is None else ptr(R0a), None if t0a is None else ptr(t0a),
                            1 if prior_restart else 0, wptr, wlen,
                            _stream(stream), C.byref(h), ptr(Rr), ptr(tr), ptr(Ra), ptr(ta), ptr(iters), ptr(st)),
          "hgmm_odometry")
    lev = np.full(F - 1, int(levels), np.int32)
    if forest is None:
        forest = Tree(h, int(off[F - 1]), int(levels), F - 1)
    else:
        forest.handle, forest.n_points, forest.levels, forest.ntrees = h, int(off[F - 1]), int(levels), F - 1
    forest.offsets, forest.tree_levels = off[:F].copy(), lev
    return dict(R_rel=Rr.reshape(F - 1, 3, 3), t_rel=tr, R_abs=Ra.reshape(F, 3, 3), t_abs=ta, iters=iters, status=st,
                forest=forest)


def hgmm_estep_batch(forest: Tree, xyz: torch.Tensor, offsets, R, t, lambda_c: float = 0.01,
                     ws: Workspace | None = None, stream=None, stop_nodes: bool = False):
    """Mean log-likelihood per pair at fixed transforms R (B,3,3), t (B,3); with
    stop_nodes=True also each point's stop node (int32 CUDA tensor, index inside
    its pair's tree, -1 if unassigned)."""
    xyz = _cloud(xyz)
    lib = _lib.load()
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    B = len(off) - 1
    Ra = np.ascontiguousarray(np.asarray(R, dtype=np.float64).reshape(B, 9))
    ta = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(B, 3))
    ws = ws or Workspace(xyz.device)
    wptr, wlen = ws.ptr(lib.hgmm_register_batch_workspace_bytes(forest.handle, off.ctypes.data_as(C.c_void_p), B))
    ll = np.zeros(B)
    stop = torch.empty(int(off[-1]), dtype=torch.int32, device=xyz.device) if stop_nodes else None
    check(lib.hgmm_estep_batch(forest.handle, C.c_void_p(xyz.data_ptr()), off.ctypes.data_as(C.c_void_p), B,
                               Ra.ctypes.data_as(C.c_void_p), ta.ctypes.data_as(C.c_void_p), lambda_c, wptr, wlen,
                               _stream(stream), ll.ctypes.data_as(C.c_void_p),
                               None if stop is None else C.c_void_p(stop.data_ptr())), "hgmm_estep_batch")
    if stop_nodes:
        torch.cuda.current_stream().synchronize()
        return ll, stop
    return ll


class MLP:
    """Owning wrapper of an hgmm_mlp handle (the warm-start network)."""

    def __init__(self, seed: int = 0):
        self.lib = _lib.load()
        self.handle = C.c_void_p(None)
        check(self.lib.hgmm_mlp_create(C.c_uint64(seed), C.byref(self.handle)), "hgmm_mlp_create")
        self.n_params = int(self.lib.hgmm_mlp_param_count())

    def __del__(self):
        try:
            if self.handle is not None and self.handle.value:
                self.lib.hgmm_mlp_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        check(self.lib.hgmm_mlp_get_params(self.handle, out.ctypes.data_as(C.c_void_p)), "hgmm_mlp_get_params")
        return out

    def set_params(self, params) -> None:
        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        assert a.shape == (self.n_params,)
        check(self.lib.hgmm_mlp_set_params(self.handle, a.ctypes.data_as(C.c_void_p)), "hgmm_mlp_set_params")

    def forward(self, X: torch.Tensor, stream=None) -> torch.Tensor:
        _dev(X, (None, 1280), torch.float32, "X")
        if X.shape[0] < 1:
            raise ValueError("X needs at least one row")
        Y = torch.empty((X.shape[0], 9), dtype=torch.float32, device=X.device)
        check(self.lib.hgmm_mlp_forward(self.handle, C.c_void_p(X.data_ptr()), X.shape[0], C.c_void_p(Y.data_ptr()),
                                        _stream(stream)), "hgmm_mlp_forward")
        return Y

    def train_step(self, X: torch.Tensor, T: torch.Tensor, lr: float, trans_weight: float = 1.0,
                   want_loss: bool = True, stream=None):
        _dev(X, (None, 1280), torch.float32, "X")
        _dev(T, (X.shape[0], 9), torch.float32, "T")
        loss = C.c_double(0)
        check(self.lib.hgmm_mlp_train_step(self.handle, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                           X.shape[0], C.c_float(lr), C.c_float(trans_weight), _stream(stream),
                                           C.byref(loss) if want_loss else None), "hgmm_mlp_train_step")
        return loss.value if want_loss else None

    def backward(self, X: torch.Tensor, T: torch.Tensor, trans_weight: float = 1.0, stream=None):
        _dev(X, (None, 1280), torch.float32, "X")
        _dev(T, (X.shape[0], 9), torch.float32, "T")
        g = np.zeros(self.n_params, np.float32)
        loss = C.c_double(0)
        check(self.lib.hgmm_mlp_backward(self.handle, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                         X.shape[0], C.c_float(trans_weight), _stream(stream),
                                         g.ctypes.data_as(C.c_void_p), C.byref(loss)), "hgmm_mlp_backward")
        return g, loss.value


def hgmm_warm_features(forest: Tree, tree_ids, reg_eps: float = 1e-6, stream=None):
    """(features (n, 640) float32 CUDA, frames (n, 13) float64 CUDA) of the listed trees."""
    ids = np.ascontiguousarray(np.asarray(tree_ids, dtype=np.int32))
    n = len(ids)
    feat = torch.empty((n, 640), dtype=torch.float32, device="cuda")
    fr = torch.empty((n, 13), dtype=torch.float64, device="cuda")
    check(_lib.load().hgmm_warm_features(forest.handle, ids.ctypes.data_as(C.c_void_p), n, reg_eps,
                                         C.c_void_p(feat.data_ptr()), C.c_void_p(fr.data_ptr()), _stream(stream)),
          "hgmm_warm_features")
    return feat, fr


def hgmm_warm_head_pose(Y: torch.Tensor, fr_src: torch.Tensor, fr_tgt: torch.Tensor, stream=None):
    P = _dev(Y, (None, 9), torch.float32, "Y").shape[0]
    _dev(fr_src, (P, 13), torch.float64, "fr_src")
    _dev(fr_tgt, (P, 13), torch.float64, "fr_tgt")
    R0 = torch.empty((P, 9), dtype=torch.float64, device="cuda")
    t0 = torch.empty((P, 3), dtype=torch.float64, device="cuda")
    check(_lib.load().hgmm_warm_head_pose(C.c_void_p(Y.data_ptr()), C.c_void_p(fr_src.data_ptr()),
                                          C.c_void_p(fr_tgt.data_ptr()), P, C.c_void_p(R0.data_ptr()),
                                          C.c_void_p(t0.data_ptr()), _stream(stream)), "hgmm_warm_head_pose")
    return R0, t0


def hgmm_warm_head_target(R: torch.Tensor, t: torch.Tensor, fr_src: torch.Tensor, fr_tgt: torch.Tensor, stream=None):
    P = _dev(R, (None, 9), torch.float64, "R").shape[0]
    _dev(t, (P, 3), torch.float64, "t")
    _dev(fr_src, (P, 13), torch.float64, "fr_src")
    _dev(fr_tgt, (P, 13), torch.float64, "fr_tgt")
    T = torch.empty((P, 9), dtype=torch.float32, device="cuda")
    check(_lib.load().hgmm_warm_head_target(C.c_void_p(R.data_ptr()), C.c_void_p(t.data_ptr()),
                                            C.c_void_p(fr_src.data_ptr()), C.c_void_p(fr_tgt.data_ptr()), P,
                                            C.c_void_p(T.data_ptr()), _stream(stream)), "hgmm_warm_head_target")
    return T


def hgmm_gemm_bf16(A_bits: torch.Tensor, B_bits: torch.Tensor, M, N, K, ta=False, tb=False, lda=None, ldb=None,
                   stream=None) -> torch.Tensor:
    """C = op(A) op(B) with raw bf16 operands (int16 tensors holding bf16 bit patterns)."""
    lda = lda if lda is not None else (M if ta else K)
    ldb = ldb if ldb is not None else (K if tb else N)
    for X, rows, ld, cols, nm in ((A_bits, K if ta else M, lda, M if ta else K, "A"),
                                  (B_bits, N if tb else K, ldb, K if tb else N, "B")):
        if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype in (torch.int16, torch.bfloat16)
                and X.is_contiguous() and ld >= cols and X.numel() >= (rows - 1) * ld + cols):
            raise ValueError(f"{nm} must be a contiguous 16-bit CUDA tensor holding a {rows} x {cols} matrix "
                             f"with leading dimension {ld}")
    Cm = torch.empty((M, N), dtype=torch.float32, device="cuda")
    check(_lib.load().hgmm_gemm_bf16(int(ta), int(tb), M, N, K, C.c_void_p(A_bits.data_ptr()), lda,
                                     C.c_void_p(B_bits.data_ptr()), ldb, C.c_void_p(Cm.data_ptr()), N,
                                     _stream(stream)), "hgmm_gemm_bf16")
    return Cm
