"""The composed 64-bit hash (hth_hash_batch64) on the GPU: bit-exact with
the oracle's composition (simple tabulation of short strings, tabulation of
the HalftimeHash value of longer ones) at every length around the direct /
hashed boundary, both block sizes, the uneven batch, the short-key workload
at full size (sampled), and the degenerate batches."""
import os

import numpy as np
import pytest

from paper_2104_08865_amd import workloads as wl

pytestmark = pytest.mark.gpu

WIDTHS = (16, 24, 32, 40)
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def env(oracle_lib):
    import torch
    from paper_2104_08865_amd import hth
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    seeds = {b: hth.expand_seed(41, block_words=b) for b in (8, 4)}
    ents = {b: oracle_lib.expand_seed(41, b=b) for b in (8, 4)}
    torch.cuda.synchronize()
    return {"torch": torch, "hth": hth, "seeds": seeds, "ents": ents, "oracle": oracle_lib}


def _dev(env, data_np, offs, lens):
    torch = env["torch"]
    d = torch.from_numpy(np.ascontiguousarray(data_np)).cuda() if data_np.size else torch.zeros(1, dtype=torch.uint8, device="cuda")
    o = torch.from_numpy(np.asarray(offs, dtype=np.uint64).view(np.int64)).cuda()
    n = torch.from_numpy(np.asarray(lens, dtype=np.uint64).view(np.int64)).cuda()
    return d, o, n


def _gpu64(env, b, data_np, offs, lens, width, tab_seed):
    hth = env["hth"]
    d, o, n = _dev(env, data_np, offs, lens)
    t = hth.tab_tables(tab_seed, width)
    z = hth.hash_batch64(env["seeds"][b], t, d, o, n, width)
    hth.batch_check()
    return z.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("b", [8, 4])
@pytest.mark.parametrize("width", WIDTHS)
def test_every_length_to_1400(env, width, b):
    lens = np.arange(0, 1401, dtype=np.uint64)
    offs, total = wl.pack(lens)
    offs = offs + np.uint64(3)
    data = wl.random_bytes(51, total + 16)
    print(f"[compose] lengths 0..1400 width={width} b={b}", flush=True)
    g = _gpu64(env, b, data, offs, lens, width, 52)
    c = env["oracle"].hash64_batch(env["ents"][b], env["oracle"].tab_expand(52, width), data, offs, lens, width,
                                   nthreads=NTHREADS, b=b)
    bad = np.nonzero(g != c)[0]
    assert bad.size == 0, f"{bad.size} mismatches, first length {int(lens[bad[0]])}"


@pytest.mark.parametrize("width", [16, 40])
def test_uneven_subset(env, width):
    """30,000 log-uniform lengths in [16 B, 256 KiB) plus 0..520."""
    lens = wl.uneven_lengths(3, n=30_000)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(53, total)
    print(f"[compose] uneven subset width={width}", flush=True)
    g = _gpu64(env, 8, data, offs, lens, width, 54)
    c = env["oracle"].hash64_batch(env["ents"][8], env["oracle"].tab_expand(54, width), data, offs, lens, width,
                                   nthreads=NTHREADS)
    assert (g == c).all()


@pytest.mark.parametrize("width", WIDTHS)
def test_identity_tables_reproduce_batch_values(env, width):
    """Identity tables on key window m: for strings longer than the inner
    width the result is word m of hth_hash_batch's value; for shorter ones,
    word m of the zero-padded string."""
    torch, hth = env["torch"], env["hth"]
    lens = np.array([0, 1, 5, 8, width - 1, width, width + 1, 300, 5000, 70_000], dtype=np.uint64)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(55, total)
    d, o, n = _dev(env, data, offs, lens)
    ref = hth.hash_batch(env["seeds"][8], d, o, n, width).cpu().numpy()
    for m in range(width // 8):
        t = np.zeros((width + 1, 256), dtype=np.uint64)
        for i in range(8 * m, 8 * m + 8):
            t[i] = np.arange(256, dtype=np.uint64) << np.uint64(8 * (i - 8 * m))
        tt = torch.from_numpy(t.ravel().view(np.int64)).cuda()
        z = hth.hash_batch64(env["seeds"][8], tt, d, o, n, width).cpu().numpy().view(np.uint64)
        for i, L in enumerate(lens):
            if L > width:
                want = ref[i, 8 * m:8 * m + 8].view("<u8")[0]
            else:
                key = np.zeros(width, dtype=np.uint8)
                key[:int(L)] = data[int(offs[i]):int(offs[i] + L)]
                want = key[8 * m:8 * m + 8].view("<u8")[0]
            assert int(z[i]) == int(want), (int(L), m)


def test_degenerate_batches(env):
    torch, hth = env["torch"], env["hth"]
    t = hth.tab_tables(1, 16)
    e = torch.zeros(0, dtype=torch.int64, device="cuda")
    z = hth.hash_batch64(env["seeds"][8], t, torch.zeros(1, dtype=torch.uint8, device="cuda"), e, e, 16)
    assert z.numel() == 0
    for L in (0, 16, 17):
        data = wl.random_bytes(56, L)
        g = _gpu64(env, 8, data, [0], [L], 16, 1)
        assert int(g[0]) == env["oracle"].hash64(env["ents"][8], env["oracle"].tab_expand(1, 16), data, 16)
    with pytest.raises(ValueError):
        hth.hash_batch64(env["seeds"][8], t, torch.zeros(1, dtype=torch.uint8, device="cuda"), e, e, 24)


def _sampled(env, data_t, offs, lens, width, tab_seed, sample, label):
    """Full-size batch on the GPU; the sampled strings recomputed by the oracle."""
    torch, hth = env["torch"], env["hth"]
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    n = torch.from_numpy(lens.view(np.int64)).cuda()
    t = hth.tab_tables(tab_seed, width)
    print(f"[compose] {label} strings={lens.size} width={width}", flush=True)
    z = hth.hash_batch64(env["seeds"][8], t, data_t, o, n, width)
    hth.batch_check()
    z = z.cpu().numpy().view(np.uint64)
    tab = env["oracle"].tab_expand(tab_seed, width)
    pieces = [data_t[int(offs[i]):int(offs[i] + lens[i])].cpu().numpy() for i in sample]
    buf = np.concatenate(pieces) if pieces else np.zeros(0, np.uint8)
    so, _ = wl.pack(lens[sample])
    ref = env["oracle"].hash64_batch(env["ents"][8], tab, buf, so, lens[sample], width, nthreads=NTHREADS)
    assert (z[sample] == ref).all()
    return z, pieces


def test_full_uneven_batch_sampled(env):
    """The uneven batch (200,521 strings, 5.4 GB) at inner width 16, as the
    benchmark runs it: 600 sampled strings against the oracle."""
    torch = env["torch"]
    lens = wl.uneven_lengths(3)
    offs, total = wl.pack(lens)
    data = wl.random_bytes_torch(3, total, "cuda")
    rng = np.random.default_rng(1)
    sample = np.unique(np.concatenate([rng.integers(0, lens.size, 590), np.arange(lens.size - 10, lens.size)]))
    _sampled(env, data, offs, lens, 16, 2, sample, "uneven batch")
    del data
    torch.cuda.empty_cache()


def test_full_short_keys_sampled(env):
    """16,777,216 keys of 0..64 bytes at inner width 16, as the benchmark runs
    them: 4,000 sampled keys against the oracle, and the sample's distinct
    keys have distinct values."""
    torch = env["torch"]
    lens = wl.short_key_lengths()
    offs, total = wl.pack(lens)
    data = wl.random_bytes_torch(7, total, "cuda")
    rng = np.random.default_rng(2)
    sample = np.unique(np.concatenate([rng.integers(0, lens.size, 3990), np.arange(lens.size - 10, lens.size)]))
    z, pieces = _sampled(env, data, offs, lens, 16, 2, sample, "short keys")
    by_key = {}
    for i, p in zip(sample, pieces):
        by_key.setdefault(p.tobytes(), set()).add(int(z[i]))
    assert all(len(v) == 1 for v in by_key.values())
    assert len({next(iter(v)) for v in by_key.values()}) == len(by_key)
    del data
    torch.cuda.empty_cache()
