"""Cached autotuning of launch shapes (hgmm_autotune) per workload signature.

The signature is the batch size, the log2 histogram of cloud sizes, the tree
depths and the device name, so batches of the same shape reuse a setting.
The cache is a JSON file (``HGMM_TUNING_CACHE``, default
``~/.cache/hgmm/tuning.json``).
"""

from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import torch

from . import api as hg


def cache_path() -> str:
    return os.environ.get("HGMM_TUNING_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "hgmm", "tuning.json"))


def signature(src_offsets, levels, tgt_offsets=None) -> str:
    so = np.diff(np.asarray(src_offsets, dtype=np.int64))
    lv = np.asarray(levels, dtype=np.int64)
    parts = [len(so), np.bincount(np.log2(np.maximum(so, 1)).astype(int), minlength=32).tolist(),
             np.bincount(lv, minlength=8).tolist(), torch.cuda.get_device_name()]
    if tgt_offsets is not None:
        to = np.diff(np.asarray(tgt_offsets, dtype=np.int64))
        parts.append(np.bincount(np.log2(np.maximum(to, 1)).astype(int), minlength=32).tolist())
    return hashlib.sha1(json.dumps(parts).encode()).hexdigest()[:16]


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned(src, src_offsets, levels, tgt=None, tgt_offsets=None, use_cache: bool = True, **kw) -> dict:
    """Set the launch shapes for this workload: from the cache when present,
    otherwise by running the autotuner (and storing its choice).  Returns
    dict(tuning, source, best_ms, start_ms)."""
    key = signature(src_offsets, levels, tgt_offsets)
    cache = _load() if use_cache else {}
    if key in cache:
        hg.hgmm_set_tuning(**cache[key]["tuning"])
        return dict(cache[key], source="cache")
    r = hg.hgmm_autotune(src, src_offsets, levels, tgt, tgt_offsets, **kw)
    if use_cache:
        cache[key] = r
        os.makedirs(os.path.dirname(cache_path()), exist_ok=True)
        tmp = cache_path() + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path())
    return dict(r, source="search")
