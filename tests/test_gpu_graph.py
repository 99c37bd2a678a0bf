"""Captured batches (hth_batch_graph_*): every replay is bit-exact with the
eager call and the oracle, with eager work between replays, and a replay
re-plans when the contents of the captured buffers change."""
import os

import numpy as np
import pytest

from paper_2104_08865_amd import workloads as wl

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.mark.parametrize("width", [24, 40])
def test_graph_replays_match_eager_and_oracle(oracle_lib, width):
    import torch
    from paper_2104_08865_amd import hth
    seed = hth.expand_seed(7)
    ent = oracle_lib.expand_seed(7)
    lens = wl.uneven_lengths(seed=9, n=3000, hi=300_000, extra_upto=40)
    offs, total = wl.pack(lens)
    data_np = wl.random_bytes(9, total)
    data = torch.from_numpy(data_np).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    n = torch.from_numpy(lens.view(np.int64)).cuda()
    print(f"[graph] width={width} strings={lens.size} bytes={total}", flush=True)
    eager = hth.hash_batch(seed, data, o, n, width).cpu().numpy()
    ref = oracle_lib.hash_batch(ent, data_np, offs, lens, width, nthreads=NTHREADS)
    assert (eager == ref).all()
    g = hth.BatchGraph(seed, data, o, n, width)
    for rep in range(4):
        g.out.fill_(0xAB)
        g.launch()
        g.check()
        got = g.out.cpu().numpy()
        assert (got == eager).all(), f"replay {rep}"
        # eager work between replays: another batch on the same stream, a torch op
        hth.hash_batch(seed, data, o, n, 16)
        torch.cuda.synchronize()
        data.add_(0)
    # new contents and new lengths in the same buffers: the replay re-plans
    data_np2 = wl.random_bytes(10, total)
    lens2 = lens.copy()
    lens2[::3] = lens2[::3] // 2
    data.copy_(torch.from_numpy(data_np2))
    n.copy_(torch.from_numpy(lens2.view(np.int64)))
    g.launch()
    g.check()
    got = g.out.cpu().numpy()
    ref2 = oracle_lib.hash_batch(ent, data_np2, offs, lens2, width, nthreads=NTHREADS)
    assert (got == ref2).all()
    g.free()
