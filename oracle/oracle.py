"""ctypes wrapper of the FP64 C oracle (TEST INFRASTRUCTURE ONLY).

The shared object is compiled from ``hgmm_oracle.c`` with gcc (no fast-math)
on first use, or by ``build_library()``.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hgmm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_library(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE semantics)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Tree(C.Structure):
    _fields_ = [
        ("levels", C.c_int32), ("pad_", C.c_int32), ("n_nodes", C.c_int64), ("n_points", C.c_int64),
        ("origin", C.c_double * 3), ("extent", C.c_double), ("root_cov", C.c_double * 6),
        ("root_lam", C.c_double * 3), ("root_evec", C.c_double * 9),
        ("live", C.c_void_p), ("has_children", C.c_void_p), ("count", C.c_void_p),
        ("pi", C.c_void_p), ("pig", C.c_void_p), ("mu", C.c_void_p), ("cov", C.c_void_p),
        ("lam", C.c_void_p), ("evec", C.c_void_p), ("kappa", C.c_void_p),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build_library(force=True)
        lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        lib.oracle_level_offset.restype = C.c_int64
        lib.oracle_level_offset.argtypes = [C.c_int]
        lib.oracle_eigh3.argtypes = [P, P, P]
        lib.oracle_octant_init.argtypes = [P, P, P, C.c_double, P, P]
        lib.oracle_octant_init.restype = None
        lib.oracle_em_partition.argtypes = [P, C.c_int64, C.c_int, C.c_double, C.c_double, P, P, P, P, P, P, P]
        lib.oracle_build_root.argtypes = [P, C.c_int64, C.c_double, P]
        lib.oracle_build_level.argtypes = [P, C.c_int64, C.c_int, C.c_int, C.c_double, C.c_double, P, P]
        lib.oracle_build.argtypes = [P, C.c_int64, C.c_int, C.c_int, C.c_double, C.c_double, P, P]
        lib.oracle_estep.argtypes = [P, P, C.c_int64, P, P, C.c_double, P, P, P, P, P, P]
        lib.oracle_normal_equations.argtypes = [P, P, C.c_int64, P, P]
        lib.oracle_solve_update.argtypes = [P, P, P, P, P, P]
        lib.oracle_register.argtypes = [P, P, C.c_int64, C.c_int, C.c_double, C.c_double, C.c_double,
                                        P, P, P, P, P]
        lib.oracle_estep_flat.argtypes = [P, C.c_int, P, C.c_int64, P, P, P, P, P, P, P]
        lib.oracle_register_flat.argtypes = [P, C.c_int, P, C.c_int64, C.c_int, C.c_double, C.c_double,
                                             P, P, P, P]
        lib.oracle_estep_soft.argtypes = [P, P, C.c_int64, P, P, C.c_double, C.c_double, P, P, P, P]
        lib.oracle_register_soft.argtypes = [P, P, C.c_int64, C.c_double, C.c_double, C.c_int, C.c_double,
                                             C.c_double, P, P, P, P]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def level_offset(level: int) -> int:
    return (8 ** (level + 1) - 8) // 7


def level_nodes(level: int) -> int:
    return 8 ** (level + 1)


class OracleTree:
    """FP64 tree in host memory, laid out as the C oracle expects."""

    def __init__(self, levels: int):
        self.levels = int(levels)
        n = level_offset(levels)
        self.n_nodes = n
        self.live = np.zeros(n, np.int32)
        self.has_children = np.zeros(n, np.int32)
        self.count = np.zeros(n, np.int64)
        self.pi = np.zeros(n)
        self.pig = np.zeros(n)
        self.mu = np.zeros((n, 3))
        self.cov = np.zeros((n, 6))
        self.lam = np.zeros((n, 3))
        self.evec = np.zeros((n, 3, 3))
        self.kappa = np.zeros(n)
        self.origin = np.zeros(3)
        self.extent = 0.0
        self.n_points = 0
        self.root_cov = np.zeros(6)
        self.root_lam = np.zeros(3)
        self.root_evec = np.zeros((3, 3))

    def _struct(self) -> _Tree:
        t = _Tree()
        t.levels = self.levels
        t.n_nodes = self.n_nodes
        t.n_points = int(self.n_points)
        t.origin[:] = [float(v) for v in self.origin]
        t.extent = float(self.extent)
        t.root_cov[:] = [float(v) for v in self.root_cov]
        t.root_lam[:] = [float(v) for v in self.root_lam]
        t.root_evec[:] = [float(v) for v in self.root_evec.ravel()]
        for name in ("live", "has_children", "count", "pi", "pig", "mu", "cov", "lam", "evec", "kappa"):
            arr = getattr(self, name)
            assert arr.flags.c_contiguous
            setattr(t, name, arr.ctypes.data)
        return t

    def _absorb(self, t: _Tree):
        self.origin = np.array(t.origin[:])
        self.extent = t.extent
        self.n_points = t.n_points
        self.root_cov = np.array(t.root_cov[:])
        self.root_lam = np.array(t.root_lam[:])
        self.root_evec = np.array(t.root_evec[:]).reshape(3, 3)

    def level_slice(self, level: int) -> slice:
        return slice(level_offset(level), level_offset(level) + level_nodes(level))


def _soa(xyz) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32))
    assert a.ndim == 2 and a.shape[0] == 3
    return a


def _check(st, what):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def eigh3(cov6):
    lib = _load()
    c = np.ascontiguousarray(np.asarray(cov6, dtype=np.float64))
    lam = np.zeros(3)
    ev = np.zeros((3, 3))
    lib.oracle_eigh3(_p(c), _p(lam), _p(ev))
    return lam, ev


def octant_init(mu, lam, evec, eps):
    lib = _load()
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    evec = np.ascontiguousarray(evec, dtype=np.float64)
    cm = np.zeros((8, 3))
    cc = np.zeros((8, 6))
    lib.oracle_octant_init(_p(mu), _p(lam), _p(evec), C.c_double(eps), _p(cm), _p(cc))
    return cm, cc


def em_partition(pts_n3, pi, mu, cov, live=None, iters=30, eps=1e-6, min_mass=1.0):
    """One parent's EM (AoS FP64 points).  Returns dict of final parameters."""
    lib = _load()
    pts = np.ascontiguousarray(pts_n3, dtype=np.float64)
    n = pts.shape[0]
    pi = np.array(pi, dtype=np.float64)
    mu = np.array(mu, dtype=np.float64).reshape(8, 3).copy()
    cov = np.array(cov, dtype=np.float64).reshape(8, 6).copy()
    live = np.ones(8, np.int32) if live is None else np.array(live, dtype=np.int32)
    resp = np.zeros((n, 8))
    label = np.zeros(n, np.int32)
    nk = np.zeros(8)
    st = lib.oracle_em_partition(_p(pts), n, iters, C.c_double(eps), C.c_double(min_mass), _p(pi), _p(mu),
                                 _p(cov), _p(live), _p(resp), _p(label), _p(nk))
    _check(st, "em_partition")
    return dict(pi=pi, mu=mu, cov=cov, live=live, resp=resp, label=label, nk=nk)


def build_root(xyz, eps=1e-6, levels=1) -> OracleTree:
    lib = _load()
    a = _soa(xyz)
    t = OracleTree(levels)
    s = t._struct()
    _check(lib.oracle_build_root(_p(a), a.shape[1], C.c_double(eps), C.byref(s)), "build_root")
    t._absorb(s)
    return t


def build_level(tree: OracleTree, xyz, labels, level, iters=30, eps=1e-6, min_mass=1.0):
    """Recompute one level from the parents stored in ``tree`` (labels row level-1 read)."""
    lib = _load()
    a = _soa(xyz)
    assert labels.dtype == np.int32 and labels.flags.c_contiguous and labels.shape == (tree.levels, a.shape[1])
    s = tree._struct()
    _check(lib.oracle_build_level(_p(a), a.shape[1], level, iters, C.c_double(eps), C.c_double(min_mass),
                                  C.byref(s), _p(labels)), "build_level")
    tree._absorb(s)


def build_tree(xyz, levels, iters=30, eps=1e-6, min_mass=1.0):
    """Full top-down construction; returns (tree, labels[levels, n])."""
    lib = _load()
    a = _soa(xyz)
    n = a.shape[1]
    t = OracleTree(levels)
    labels = np.full((levels, n), -1, np.int32)
    s = t._struct()
    _check(lib.oracle_build(_p(a), n, levels, iters, C.c_double(eps), C.c_double(min_mass), C.byref(s),
                            _p(labels)), "build")
    t._absorb(s)
    return t, labels


def estep(tree: OracleTree, xyz, R=None, t=None, lambda_c=0.01):
    lib = _load()
    a = _soa(xyz)
    n = a.shape[1]
    R = np.eye(3) if R is None else np.ascontiguousarray(R, dtype=np.float64)
    t = np.zeros(3) if t is None else np.ascontiguousarray(t, dtype=np.float64)
    out = dict(stop_node=np.zeros(n, np.int32), stop_level=np.zeros(n, np.int32), gamma=np.zeros(n),
               min_gap=np.zeros(n), bins=np.zeros((tree.n_nodes, 6)))
    ll = C.c_double(0.0)
    s = tree._struct()
    _check(lib.oracle_estep(C.byref(s), _p(a), n, _p(R), _p(t), C.c_double(lambda_c), _p(out["stop_node"]),
                            _p(out["stop_level"]), _p(out["gamma"]), _p(out["min_gap"]), _p(out["bins"]),
                            C.byref(ll)), "estep")
    out["loglik"] = ll.value
    return out


def estep_flat(tree: OracleTree, level, xyz, R=None, t=None):
    """Single-level variant ("GMM J=n"): the live nodes of tree level ``level``
    as one mixture with their global weights, every component scored for every
    point; stop_node is the chosen component (-1 when the level has none)."""
    lib = _load()
    a = _soa(xyz)
    n = a.shape[1]
    R = np.eye(3) if R is None else np.ascontiguousarray(R, dtype=np.float64)
    t = np.zeros(3) if t is None else np.ascontiguousarray(t, dtype=np.float64)
    out = dict(stop_node=np.zeros(n, np.int32), gamma=np.zeros(n), min_gap=np.zeros(n),
               bins=np.zeros((tree.n_nodes, 6)))
    ll = C.c_double(0.0)
    s = tree._struct()
    _check(lib.oracle_estep_flat(C.byref(s), int(level), _p(a), n, _p(R), _p(t), _p(out["stop_node"]),
                                 _p(out["gamma"]), _p(out["min_gap"]), _p(out["bins"]), C.byref(ll)), "estep_flat")
    out["loglik"] = ll.value
    return out


def register_flat(tree: OracleTree, level, xyz, R0=None, t0=None, max_iters=30, tol_rot=1e-6, tol_trans=None):
    """EM registration of ``xyz`` with the single-level variant of ``tree``."""
    lib = _load()
    a = _soa(xyz)
    n = a.shape[1]
    R = np.eye(3) if R0 is None else np.array(R0, dtype=np.float64, order="C")
    t = np.zeros(3) if t0 is None else np.array(t0, dtype=np.float64, order="C")
    if tol_trans is None:
        tol_trans = 1e-6 * tree.extent
    iters = C.c_int(0)
    ll = C.c_double(0.0)
    s = tree._struct()
    st = lib.oracle_register_flat(C.byref(s), int(level), _p(a), n, max_iters, C.c_double(tol_rot),
                                  C.c_double(tol_trans), _p(R), _p(t), C.byref(iters), C.byref(ll))
    return dict(status=st, R=R, t=t, iters=iters.value, loglik=ll.value)


def estep_soft(tree: OracleTree, xyz, R=None, t=None, lambda_c=0.01, tau=0.01):
    """Soft multi-path E-step: every branch whose path expectation is >= tau,
    stop nodes weighted by it (bins {E, E q, E, E d^2})."""
    lib = _load()
    a = _soa(xyz)
    n = a.shape[1]
    R = np.eye(3) if R is None else np.ascontiguousarray(R, dtype=np.float64)
    t = np.zeros(3) if t is None else np.ascontiguousarray(t, dtype=np.float64)
    out = dict(bins=np.zeros((tree.n_nodes, 6)), margin=np.zeros(n), stops=np.zeros(n, np.int32))
    ll = C.c_double(0.0)
    s = tree._struct()
    _check(lib.oracle_estep_soft(C.byref(s), _p(a), n, _p(R), _p(t), C.c_double(lambda_c), C.c_double(tau),
                                 _p(out["bins"]), C.byref(ll), _p(out["margin"]), _p(out["stops"])), "estep_soft")
    out["loglik"] = ll.value
    return out


def register_soft(tree: OracleTree, xyz, R0=None, t0=None, lambda_c=0.01, tau=0.01, max_iters=30, tol_rot=1e-6,
                  tol_trans=None):
    """EM registration with the soft multi-path E-step."""
    lib = _load()
    a = _soa(xyz)
    n = a.shape[1]
    R = np.eye(3) if R0 is None else np.array(R0, dtype=np.float64, order="C")
    t = np.zeros(3) if t0 is None else np.array(t0, dtype=np.float64, order="C")
    if tol_trans is None:
        tol_trans = 1e-6 * tree.extent
    iters = C.c_int(0)
    ll = C.c_double(0.0)
    s = tree._struct()
    st = lib.oracle_register_soft(C.byref(s), _p(a), n, C.c_double(lambda_c), C.c_double(tau), max_iters,
                                  C.c_double(tol_rot), C.c_double(tol_trans), _p(R), _p(t), C.byref(iters),
                                  C.byref(ll))
    return dict(status=st, R=R, t=t, iters=iters.value, loglik=ll.value)


def normal_equations(tree: OracleTree, bins, n):
    lib = _load()
    b = np.ascontiguousarray(bins, dtype=np.float64)
    H = np.zeros((6, 6))
    g = np.zeros(6)
    s = tree._struct()
    lib.oracle_normal_equations(C.byref(s), _p(b), int(n), _p(H), _p(g))
    return H, g


def solve_update(H, g, origin, R, t):
    lib = _load()
    H = np.ascontiguousarray(H, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    R = np.array(R, dtype=np.float64, order="C")
    t = np.array(t, dtype=np.float64)
    x = np.zeros(6)
    st = lib.oracle_solve_update(_p(H), _p(g), _p(o), _p(R), _p(t), _p(x))
    return st, R, t, x


def register(tree: OracleTree, xyz, R0=None, t0=None, max_iters=30, lambda_c=0.01, tol_rot=1e-6,
             tol_trans=None):
    """Full EM registration of ``xyz`` (SoA) onto ``tree``.  Returns dict."""
    lib = _load()
    a = _soa(xyz)
    n = a.shape[1]
    R = np.eye(3) if R0 is None else np.array(R0, dtype=np.float64, order="C")
    t = np.zeros(3) if t0 is None else np.array(t0, dtype=np.float64, order="C")
    if tol_trans is None:
        tol_trans = 1e-6 * tree.extent
    iters = C.c_int(0)
    ll = C.c_double(0.0)
    trace = np.zeros((max_iters, 20))
    s = tree._struct()
    st = lib.oracle_register(C.byref(s), _p(a), n, max_iters, C.c_double(lambda_c), C.c_double(tol_rot),
                             C.c_double(tol_trans), _p(R), _p(t), C.byref(iters), C.byref(ll), _p(trace))
    return dict(status=st, R=R, t=t, iters=iters.value, loglik=ll.value, trace=trace[: iters.value])


def compose_chain(R_rel, t_rel):
    """Poses of a chain of frame-to-frame transforms (the trajectory of the LiDAR
    experiment, Sec. 6): with frame k coordinates = R_rel[k] @ (frame k+1
    coordinates) + t_rel[k], frame 0 coordinates = R_abs[k] @ (frame k
    coordinates) + t_abs[k], where R_abs[0] = I, t_abs[0] = 0 and
    R_abs[k] = R_abs[k-1] R_rel[k-1], t_abs[k] = R_abs[k-1] t_rel[k-1] + t_abs[k-1]."""
    R_rel = np.asarray(R_rel, dtype=np.float64)
    t_rel = np.asarray(t_rel, dtype=np.float64)
    F = len(R_rel) + 1
    R_abs = np.zeros((F, 3, 3))
    t_abs = np.zeros((F, 3))
    R_abs[0] = np.eye(3)
    for k in range(1, F):
        R_abs[k] = R_abs[k - 1] @ R_rel[k - 1]
        t_abs[k] = R_abs[k - 1] @ t_rel[k - 1] + t_abs[k - 1]
    return R_abs, t_abs
