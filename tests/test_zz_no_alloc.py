"""hth_hash_batch_noalloc (static scratch, no allocation) against hth_hash_batch
and the oracle, on two calls in a row (the second smaller), through the C ABI."""
import os

import numpy as np
import pytest

from paper_2104_08865_amd import workloads as wl

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def env(oracle_lib):
    import torch
    from paper_2104_08865_amd import hth
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.init()
    seed = hth.expand_seed(11)
    torch.cuda.synchronize()
    return {"torch": torch, "hth": hth, "seed": seed, "ent": oracle_lib.expand_seed(11), "oracle": oracle_lib}


def _batch(byte_seed, lens):
    lens = np.asarray(lens, dtype=np.uint64)
    offs, total = wl.pack(lens)
    return wl.random_bytes(byte_seed, total), offs, lens


def _both(env, data, offs, lens, width):
    torch, hth = env["torch"], env["hth"]
    d = torch.from_numpy(data).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    n = torch.from_numpy(lens.view(np.int64)).cuda()
    out = torch.full((lens.size, width), 0xA5, dtype=torch.uint8, device="cuda")
    hth.hash_batch_noalloc(env["seed"], d, o, n, width, out)
    hth.batch_check()
    ref = hth.hash_batch(env["seed"], d, o, n, width)
    hth.batch_check()
    return out.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("width", (16, 24, 32, 40))
def test_noalloc_two_calls_match_hash_batch(env, width):
    # call 1: uneven lengths (tail-only to multi-task strings, cross-task sums)
    lens1 = np.concatenate([wl.uneven_lengths(seed=21, n=3000, hi=1 << 18), np.arange(0, 300),
                            [5 << 20, 9 << 20, (3 << 20) + 77]]).astype(np.uint64)
    # call 2: smaller, other bytes and lengths
    lens2 = np.concatenate([np.arange(0, 521), wl.uneven_lengths(seed=22, n=400, hi=1 << 16),
                            [(2 << 20) + 5]]).astype(np.uint64)
    for call, (bseed, lens) in enumerate(((31, lens1), (32, lens2)), 1):
        data, offs, lens = _batch(bseed, lens)
        print(f"[noalloc] call {call} width={width} strings={lens.size} bytes={int(lens.sum())}", flush=True)
        g, ref = _both(env, data, offs, lens, width)
        bad = np.nonzero((g != ref).any(axis=1))[0]
        assert bad.size == 0, f"call {call}: {bad.size} rows differ from hth_hash_batch, first {bad[0]}"
        c = env["oracle"].hash_batch(env["ent"], data, offs, lens, width, nthreads=NTHREADS)
        bad = np.nonzero((g != c).any(axis=1))[0]
        assert bad.size == 0, f"call {call}: {bad.size} rows differ from the oracle, first {bad[0]}"


def test_noalloc_rejects_count_above_limit(env):
    torch, hth = env["torch"], env["hth"]
    n = 65536 + 1
    o = torch.zeros(n, dtype=torch.int64, device="cuda")
    d = torch.zeros(16, dtype=torch.uint8, device="cuda")
    out = torch.zeros((n, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(hth.HthError) as ei:
        hth.hash_batch_noalloc(env["seed"], d, o, o, 16, out)
    assert ei.value.status == hth.HTH_E_TOO_LARGE
    # and a batch at the limit is accepted and right
    lens = np.full(65536, 40, dtype=np.uint64)
    data, offs, lens = _batch(33, lens)
    g, ref = _both(env, data, offs, lens, 16)
    assert (g == ref).all()
