"""Shared helpers of the GPU tests (conversion between the library's export
and the oracle's tree layout; seeded inputs)."""

import numpy as np

FIELDS = ("live", "has_children", "count", "pi", "pig", "mu", "cov", "lam", "evec", "kappa")


def to_oracle(oracle_mod, host):
    ot = oracle_mod.OracleTree(host["levels"])
    for k in FIELDS:
        getattr(ot, k)[...] = host[k]
    ot.origin = np.array(host["origin"], dtype=np.float64)
    ot.extent = float(host["extent"])
    ot.n_points = int(host["n_points"])
    return ot


def gpu_bins_from_oracle(tree_host, obins):
    """Oracle bins (M0, M1 absolute, cnt, sum d2) -> library layout (M0, D about mu, cnt, sum d2)."""
    b = np.zeros_like(obins)
    b[:, 0] = obins[:, 0]
    b[:, 1:4] = obins[:, 1:4] - obins[:, :1] * tree_host["mu"]
    b[:, 4:6] = obins[:, 4:6]
    return b


def rel_err(a, b, floor):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)
