"""Autotuner for the batched hashing kernel.

The kernel has two launch choices per output width (hth_set_tuning): how
many single-wave workgroups the persistent grid keeps per compute unit, and
the range of task sizes (128 * 8^j executions) the device planner may pick
from.  This module times candidates on the caller's own batch with HIP
events around the whole call (planner and kernels: the task level also sets
how many tasks the planner writes), applies the fastest, and remembers it per
width and batch shape (number of strings and total bytes, in powers of two)
in a JSON cache file.  Every candidate computes the same values; only speed differs.
"""
import json
import math
import os

import numpy as np

from . import hth

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hth_autotune.json")

# (waves_per_cu, min_task_level, max_task_level)
CANDIDATES = [
    (8, 0, 5), (4, 0, 5), (12, 0, 5), (16, 0, 5),
    (8, 0, 0), (8, 1, 1), (8, 2, 2), (12, 0, 0), (16, 0, 0),
]


def shape_key(width, count, total_bytes):
    """Cache key: width and the powers of two of the string count and bytes."""
    return f"w{width}-n{int(math.log2(max(count, 1)))}-b{int(math.log2(max(total_bytes, 1)))}"


def _time(seed, data, offsets, lengths, width, out, reps):
    timers = [hth.Timer() for _ in range(reps)]
    hth.hash_batch(seed, data, offsets, lengths, width, out=out)  # plan once, warm the caches
    for t in timers:
        t.record_start()
        hth.hash_batch(seed, data, offsets, lengths, width, out=out)
        t.record_stop()
    return float(np.median([t.elapsed_ms() for t in timers]))


def tune(seed, data, offsets, lengths, width, total_bytes=None, reps=3, candidates=CANDIDATES,
         cache_file=DEFAULT_CACHE, use_cache=True):
    """Pick and apply the fastest launch choice for this batch; returns
    (choice, {choice: ms}) where choice = (waves_per_cu, min_level, max_level)."""
    import torch
    count = offsets.numel()
    if total_bytes is None:
        total_bytes = int(lengths.sum().item())
    key = shape_key(width, count, total_bytes)
    cache = {}
    if use_cache and cache_file and os.path.exists(cache_file):
        try:
            cache = json.load(open(cache_file))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        choice = tuple(cache[key]["choice"])
        hth.set_tuning(width, *choice)
        return choice, {}
    out = torch.empty((count, width), dtype=torch.uint8, device=data.device)
    times = {}
    for c in candidates:
        hth.set_tuning(width, *c)
        times[c] = _time(seed, data, offsets, lengths, width, out, reps)
    choice = min(times, key=times.get)
    hth.set_tuning(width, *choice)
    if cache_file:
        cache[key] = {"choice": list(choice), "ms": times[choice]}
        try:
            os.makedirs(os.path.dirname(cache_file), exist_ok=True)
            with open(cache_file, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return choice, times
