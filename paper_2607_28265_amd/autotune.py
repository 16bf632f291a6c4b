"""Launch-shape autotuning with a JSON cache.

The timing and the choice happen in the library (gw_autotune); this module
only keys the result by workload and device and stores it in the file named by
GW_AUTOTUNE_CACHE (default ~/.cache/gwswig_autotune.json), so that later
processes reuse a shape without re-timing.
"""
from __future__ import annotations

import json
import os

from . import _lib


def _cache_path() -> str:
    return os.environ.get("GW_AUTOTUNE_CACHE", os.path.expanduser("~/.cache/gwswig_autotune.json"))


def _key(ctx, like, n, marg, prec, extra) -> str:
    import torch
    dev = torch.cuda.get_device_name(ctx.device) if torch.cuda.is_available() else "none"
    return json.dumps([dev, like, int(n), int(ctx.n_freq), int(ctx.n_det), marg, prec, extra])


def _load() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass


def tune(ctx, theta, like: int, marg: int, prec: int, reps: int = 3, use_cache: bool = True, extra=None):
    """Apply the best launch shape for this workload (cached, or timed now).

    Returns (shape, ms_per_call or None when taken from the cache).
    """
    key = _key(ctx, like, theta.shape[0], marg, prec, extra)
    cache = _load() if use_cache else {}
    if key in cache and len(cache[key].get("shape", ())) == 3:
        a, b, c = cache[key]["shape"]
        if like == _lib.GW_FULL:
            ctx.set_full_shape(a, b)
        else:
            ctx.set_het_shape(a, b, c)
        return (a, b, c), None
    shape, ms = _lib.gw_autotune(ctx.handle, theta, like, marg, prec, reps)
    if use_cache:
        cache[key] = {"shape": list(shape), "ms": ms}
        _store(cache)
    return shape, ms
