"""Kernel-variant autotuning with an on-disk cache.

The library times its compiled configurations of each size-class kernel on a batch
(open_autotune) and keeps the fastest per context; this module stores the choice as JSON,
keyed by device name, library build and rank, so later processes load it instead of
re-timing.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import native


def _lib_id():
    st = os.stat(native.LIB_PATH)
    return hashlib.sha1(("%s:%d:%d" % (native.LIB_PATH, st.st_size, int(st.st_mtime))).encode()).hexdigest()[:16]


def cache_key(ctx, k):
    name = torch.cuda.get_device_properties(ctx.device).name
    return "%s|%s|k%d" % (name, _lib_id(), k)


def load(ctx, k, path):
    """Apply a cached choice for rank k if one exists; returns it or None."""
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    choice = data.get(cache_key(ctx, k))
    if choice is None:
        return None
    ctx.tune_set(k, choice["choice"])
    return choice["choice"]


def tune(ctx, F, row_ptr, col, val, lam, weighted=True, reps=5, path=None, force=False):
    """Autotune rank F.shape[1] on this batch unless a cached choice applies; store the result.
    Returns (choice, timing table or None when loaded from the cache)."""
    k = F.shape[1]
    if not force:
        got = load(ctx, k, path)
        if got is not None:
            return got, None
    _, table = native.open_autotune(ctx, F, row_ptr, col, val, lam, weighted, reps)
    choice = ctx.tune_get(k)
    if path:
        data = {}
        if os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
        data[cache_key(ctx, k)] = {"choice": choice, "ms": table}
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return choice, table
