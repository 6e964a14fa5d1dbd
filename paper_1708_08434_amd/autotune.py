"""Cache of autotuned Gauss-Seidel launch schedules.

The search itself runs in the library (mg_autotune: every launch variant of
the half-sweep kernel timed per level with HIP events).  This module keys the
result by the device name, the precision and the tree's boxes per level, and
stores it in a JSON file ($MG_TUNE_CACHE, default
~/.cache/paper_1708_08434_amd/tune.json) so later runs on the same tree shape
skip the search.
"""
import json
import os

from . import mg as M


def cache_path():
    return os.environ.get("MG_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1708_08434_amd",
                                       "tune.json"))


def _key(tree, precision):
    import torch
    dev = torch.cuda.get_device_name(tree.device)
    ls = list(tree.info.level_start[:tree.nlev + 1])
    counts = [int(ls[i + 1] - ls[i]) for i in range(tree.nlev)]
    return f"{dev}|{M.MG_GSRB_VARIANTS} variants|{'mixed' if precision == M.MG_MIXED else 'fp64'}|{counts}"


def tune(tree, precision=M.MG_FP64, reps=16, use_cache=True):
    """Apply the cached schedule for this tree shape, or search and cache one.
    Returns (schedule per level, from_cache)."""
    path = cache_path()
    key = _key(tree, precision)
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        M.mg_set_schedule(tree.h, precision, cache[key])
        return list(cache[key]), True
    sched = [int(v) for v in M.mg_autotune(tree.h, precision, reps, tree.nlev)]
    if use_cache:
        cache[key] = sched
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return sched, False
