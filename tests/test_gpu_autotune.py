"""The autotuner (autotune.py): every launch choice computes the same
values, the tuned launch equals the default one bit for bit, and a cached
choice is reused without timing again."""
import os

import numpy as np
import pytest

from paper_2104_08865_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_autotune_choice_and_cache(tmp_path):
    import torch
    from paper_2104_08865_amd import autotune, hth
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    width = 24
    lens = wl.uneven_lengths(3, n=20_000)
    offs, total = wl.pack(lens)
    data = wl.random_bytes_torch(3, total, "cuda")
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    n = torch.from_numpy(lens.view(np.int64)).cuda()
    seed = hth.expand_seed(71)
    print(f"[autotune] strings={lens.size} bytes={total}", flush=True)
    try:
        hth.set_tuning(width)
        ref = hth.hash_batch(seed, data, o, n, width).cpu().numpy()
        cache = str(tmp_path / "tune.json")
        choice, times = autotune.tune(seed, data, o, n, width, total_bytes=total, reps=2, cache_file=cache)
        assert choice in autotune.CANDIDATES and set(times) == set(autotune.CANDIDATES)
        assert all(t > 0 for t in times.values())
        assert (hth.hash_batch(seed, data, o, n, width).cpu().numpy() == ref).all()
        # every candidate gives the same values
        for c in autotune.CANDIDATES:
            hth.set_tuning(width, *c)
            assert (hth.hash_batch(seed, data, o, n, width).cpu().numpy() == ref).all(), c
        # a second call finds the choice in the cache and times nothing
        choice2, times2 = autotune.tune(seed, data, o, n, width, total_bytes=total, cache_file=cache)
        assert choice2 == choice and times2 == {} and os.path.exists(cache)
    finally:
        hth.set_tuning(width)
