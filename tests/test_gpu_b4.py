"""The 256-bit block family (b = 4, §6.3) on the GPU: bit-exact with the
oracle's b = 4 family through every path (batches at every task size, the
tail-only kernel, captured batches, the serving loop)."""
import os

import numpy as np
import pytest

from paper_2104_08865_amd import workloads as wl

pytestmark = pytest.mark.gpu

WIDTHS = (16, 24, 32, 40)
NTHREADS = min(16, os.cpu_count() or 1)


def xb4(width):
    """Bytes of one b = 4 execution."""
    return wl.execution_bytes(width) // 2


@pytest.fixture(scope="module")
def env(oracle_lib):
    import torch
    from paper_2104_08865_amd import hth
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    seed = hth.expand_seed(21, block_words=4)
    torch.cuda.synchronize()
    return {"torch": torch, "hth": hth, "seed": seed, "ent": oracle_lib.expand_seed(21, b=4), "oracle": oracle_lib}


def _check(env, data_np, offs, lens, width, label):
    torch, hth = env["torch"], env["hth"]
    print(f"[b4] {label} width={width} strings={len(lens)} bytes={int(np.sum(lens))}", flush=True)
    d = torch.from_numpy(np.ascontiguousarray(data_np)).cuda() if data_np.size else torch.zeros(1, dtype=torch.uint8, device="cuda")
    o = torch.from_numpy(np.asarray(offs, dtype=np.uint64).view(np.int64)).cuda()
    n = torch.from_numpy(np.asarray(lens, dtype=np.uint64).view(np.int64)).cuda()
    g = hth.hash_batch(env["seed"], d, o, n, width)
    hth.batch_check()
    g = g.cpu().numpy()
    c = env["oracle"].hash_batch(env["ent"], data_np, offs, lens, width, nthreads=NTHREADS, b=4)
    bad = np.nonzero((g != c).any(axis=1))[0]
    assert bad.size == 0, f"{label} width {width}: {bad.size} mismatches, first string {bad[0]} (len {int(lens[bad[0]])})"


def test_b4_seed(env):
    hth = env["hth"]
    assert env["seed"].block_words == 4
    assert hth.entropy_words(4) == env["ent"].size == 10229
    assert (env["seed"].entropy() == env["ent"]).all()
    with pytest.raises(hth.HthError):
        hth.expand_seed(1, block_words=5)


@pytest.mark.parametrize("width", WIDTHS)
def test_b4_every_length_to_1400(env, width):
    lens = np.arange(0, 1401, dtype=np.uint64)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(31, total + 64)
    _check(env, data, offs + np.uint64(5), lens, width, "lengths 0..1400 at offset 5")


@pytest.mark.parametrize("width", WIDTHS)
def test_b4_unaligned_strings_with_short_tails(env, width):
    """Strings of 9 .. 257 executions plus T < 16 bytes starting 1, 2, 3
    bytes past a 4-byte boundary, the last one ending at the end of the
    buffer (the staged path's last word of each execution loaded on its own)."""
    xb = xb4(width)
    offs, lens, at = [], [], 0
    for n in (9, 32, 33, 257):
        for t in range(16):
            for sh in (1, 2, 3):
                at = (at + 3) // 4 * 4 + sh
                offs.append(at)
                lens.append(n * xb + t)
                at += n * xb + t
    data = wl.random_bytes(32, at)
    _check(env, data, np.asarray(offs, dtype=np.uint64), np.asarray(lens, dtype=np.uint64), width,
           "unaligned strings with short tails")


@pytest.mark.parametrize("width", WIDTHS)
def test_b4_tree_boundaries(env, width):
    """Execution counts around the 256-execution pass, the level-3 (512) and
    level-4 (4096) boundaries, and with many base-8 digits set."""
    xb = xb4(width)
    lens = []
    for n in (63, 64, 65, 127, 128, 129, 191, 192, 255, 256, 257, 511, 512, 513, 1023, 1024, 2047, 2048, 2049,
              4095, 4096, 4097, 4096 + 512 + 64 + 8 + 1, 2 * 4096 + 7 * 512 + 7 * 64 + 7 * 8 + 7):
        for extra in (0, 1, xb - 1):
            lens.append(n * xb + extra)
    lens = np.array(lens, dtype=np.uint64)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(32, total)
    _check(env, data, offs, lens, width, "tree boundaries")


@pytest.mark.parametrize("width", WIDTHS)
def test_b4_small_strings_around_one_node(env, width):
    """Strings of 1 .. 17 executions of the b = 4 family (the small-string
    kernel's, the one-node case of 8, the first task strings), tails of 0, 1,
    7 and almost an execution, at offsets 0 .. 7 mod 8."""
    xb = xb4(width)
    lens = np.array([n * xb + extra for n in range(1, 18) for extra in (0, 1, 7, xb - 1)], dtype=np.uint64)
    offs, total = wl.pack(lens)
    offs = offs + np.arange(lens.size, dtype=np.uint64) % np.uint64(8)
    data = wl.random_bytes(36, total + 8)
    _check(env, data, offs, lens, width, "1-17 executions")


@pytest.mark.parametrize("level", [0, 1, 2])
def test_b4_forced_task_levels(env, level):
    """Tasks of 256 * 8^level executions: level 0 merges levels 3 and up
    across tasks with device atomics."""
    hth = env["hth"]
    width = 32
    xb = xb4(width)
    lens = np.array([n * xb + 9 for n in (100, 255, 256, 4097, 70000)] + [10, 0], dtype=np.uint64)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(33, total)
    try:
        hth.set_tuning(width, 0, level, level)
        _check(env, data, offs, lens, width, f"task level {level}")
    finally:
        hth.set_tuning(width)


def test_b4_uneven_subset(env):
    """30,000 log-uniform lengths in [16 B, 256 KiB) plus 0..520, width 24."""
    lens = wl.uneven_lengths(3, n=30_000)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(34, total)
    _check(env, data, offs, lens, 24, "uneven subset")


@pytest.mark.parametrize("width", WIDTHS)
def test_b4_throughput_batch_sampled(env, width):
    """1024 x 1 MiB in one launch; 32 sampled strings against the oracle."""
    torch, hth = env["torch"], env["hth"]
    n, sz = 1024, 1 << 20
    print(f"[b4] 1024 x 1 MiB width={width}", flush=True)
    data = wl.random_bytes_torch(35, n * sz, "cuda")
    offs = torch.arange(n, dtype=torch.int64, device="cuda") * sz
    lens = torch.full((n,), sz, dtype=torch.int64, device="cuda")
    out = hth.hash_batch(env["seed"], data, offs, lens, width).cpu().numpy()
    hth.batch_check()
    rng = np.random.default_rng(width)
    sample = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 30)]))
    strs = np.stack([wl.random_bytes(35, sz, start_byte=int(i) * sz) for i in sample])
    ref = env["oracle"].hash_batch(env["ent"], strs.ravel(), np.arange(sample.size, dtype=np.uint64) * np.uint64(sz),
                                   np.full(sample.size, sz, dtype=np.uint64), width, nthreads=NTHREADS, b=4)
    assert (out[sample] == ref).all()
    del data
    torch.cuda.empty_cache()


def test_b4_graph_and_server(env):
    """A captured b = 4 batch and a b = 4 server give the oracle's values."""
    torch, hth = env["torch"], env["hth"]
    lens = wl.lognormal_lengths(seed=36, n=400, cap=1 << 20)
    offs, total = wl.pack(lens)
    data_np = wl.random_bytes(36, total)
    ref = env["oracle"].hash_batch(env["ent"], data_np, offs, lens, 40, nthreads=NTHREADS, b=4)
    d = torch.from_numpy(data_np).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    n = torch.from_numpy(lens.view(np.int64)).cuda()
    g = hth.BatchGraph(env["seed"], d, o, n, 40)
    for _ in range(2):
        g.launch()
        g.check()
        assert (g.out.cpu().numpy() == ref).all()
    g.free()
    with hth.Server(env["seed"]) as srv:
        got = srv.wait_many([srv.submit(data_np[int(a):int(a) + int(b)], 40) for a, b in zip(offs, lens)])
    assert (got == ref).all()
