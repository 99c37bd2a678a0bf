"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Integer hashing leaves no room for tolerance: every output byte must match.
Inputs come from the seeded generators in paper_2104_08865_amd.workloads.
"""
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
    torch.cuda.init()
    seed = hth.expand_seed(1)
    torch.cuda.synchronize()
    return {"torch": torch, "hth": hth, "seed": seed, "ent": oracle_lib.expand_seed(1), "oracle": oracle_lib}


def _gpu_hash(env, data_np, offs, lens, width, seed=None):
    torch = env["torch"]
    d = torch.from_numpy(np.ascontiguousarray(data_np)).cuda() if data_np.size else torch.zeros(1, dtype=torch.uint8, device="cuda")
    o = torch.from_numpy(np.asarray(offs, dtype=np.uint64).view(np.int64)).cuda()
    n = torch.from_numpy(np.asarray(lens, dtype=np.uint64).view(np.int64)).cuda()
    out = env["hth"].hash_batch(seed or env["seed"], d, o, n, width)
    env["hth"].batch_check()
    return out.cpu().numpy()


def _check(env, data_np, offs, lens, width, label):
    print(f"[parity] {label} width={width} strings={len(lens)} bytes={int(np.sum(lens))}", flush=True)
    g = _gpu_hash(env, data_np, offs, lens, width)
    c = env["oracle"].hash_batch(env["ent"], data_np, offs, lens, width, nthreads=NTHREADS)
    bad = np.nonzero((g != c).any(axis=1))[0]
    assert bad.size == 0, f"{label} width {width}: {bad.size} mismatches, first at string {bad[0]} (len {int(lens[bad[0]])})"


def test_seed_expansion_matches_oracle(env):
    assert (env["seed"].entropy() == env["ent"]).all()


@pytest.mark.parametrize("width", WIDTHS)
def test_small_batch(env, width):
    """1024 x 1 KiB plus the edge lengths 0, 1, 7, 8, 63, 64 and 1, 8, 64 and
    512 executions +-1, packed back to back (unaligned starts)."""
    lens = wl.small_batch_lengths(width)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(1, total)
    _check(env, data, offs, lens, width, "small batch")


@pytest.mark.parametrize("width", WIDTHS)
def test_unaligned_strings_with_short_tails(env, width):
    """Strings of N executions plus T < 16 bytes starting sh = 1, 2, 3 bytes
    past a 4-byte boundary (hashed by the hashing kernel: N >= 9), the last
    one ending at the end of the buffer: the staged copies of such strings
    stop at each execution's end and the word holding its last bytes comes
    from a separate load, which these values pin."""
    xb = wl.execution_bytes(width)
    offs, lens, at = [], [], 0
    for n in (9, 16, 17, 64, 129):
        for t in range(16):
            for sh in (1, 2, 3):
                at = (at + 3) // 4 * 4 + sh
                offs.append(at)
                lens.append(n * xb + t)
                at += n * xb + t
    data = wl.random_bytes(12, at)  # (exactly as long as the strings need)
    _check(env, data, np.asarray(offs, dtype=np.uint64), np.asarray(lens, dtype=np.uint64), width,
           "unaligned strings with short tails")


@pytest.mark.parametrize("width", WIDTHS)
def test_every_length_to_1400_and_odd_offsets(env, width):
    lens = np.arange(0, 1401, dtype=np.uint64)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(11, total + 64)
    _check(env, data, offs + np.uint64(3), lens, width, "lengths 0..1400 at offset 3")


@pytest.mark.parametrize("width", WIDTHS)
def test_tree_boundaries(env, width):
    """Execution counts around pass (128), level-3 (512), task-spanning level-4
    (4096) boundaries and with every base-8 digit set."""
    xb = wl.execution_bytes(width)
    lens = []
    for n in (63, 64, 65, 127, 128, 129, 511, 512, 513, 1023, 1024, 4095, 4096, 4097, 4096 + 512 + 64 + 8 + 1,
              2 * 4096 + 7 * 512 + 7 * 64 + 7 * 8 + 7):
        for extra in (0, 1, xb - 1):
            lens.append(n * xb + extra)
    lens = np.array(lens, dtype=np.uint64)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(12, total)
    _check(env, data, offs, lens, width, "tree boundaries")


@pytest.mark.parametrize("width", WIDTHS)
def test_small_strings_around_one_node(env, width):
    """Strings of 1 .. 17 executions (the small-string kernel's strings,
    among them the one-node case of exactly 8, and the first ones hashed as
    tasks), each with no tail, a one-byte tail and an almost full one, at
    unaligned addresses (offsets 0 .. 7 mod 8)."""
    xb = wl.execution_bytes(width)
    lens = np.array([n * xb + extra for n in range(1, 18) for extra in (0, 1, 7, xb - 1)], dtype=np.uint64)
    offs, total = wl.pack(lens)
    offs = offs + np.arange(lens.size, dtype=np.uint64) % np.uint64(8)
    data = wl.random_bytes(16, total + 8)
    _check(env, data, offs, lens, width, "1-17 executions")


@pytest.mark.parametrize("level", [0, 1, 2])
def test_forced_task_levels_same_result(env, level):
    """Every task size gives the oracle's values: level 0 merges every level
    from 3 up across tasks with device atomics, coarser levels fold the lower
    ones inside one wave."""
    hth = env["hth"]
    width = 24
    xb = wl.execution_bytes(width)
    lens = np.array([n * xb + 5 for n in (100, 511, 512, 4097, 70000)] + [10, 0], dtype=np.uint64)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(13, total)
    try:
        hth.set_tuning(width, 0, level, level)
        _check(env, data, offs, lens, width, f"task level {level}")
    finally:
        hth.set_tuning(width)


def test_batch_invariance_and_overlap(env):
    """A string hashes the same alone, in a mix, and when strings overlap."""
    width = 40
    data = wl.random_bytes(14, 3_000_000)
    offs = np.array([0, 5, 1_000_003, 17, 0, 2_999_999], dtype=np.uint64)
    lens = np.array([2_000_000, 1_000_000, 1_999_997, 123_456, 0, 1], dtype=np.uint64)
    mix = _gpu_hash(env, data, offs, lens, width)
    for i in range(lens.size):
        alone = _gpu_hash(env, data, offs[i:i + 1], lens[i:i + 1], width)
        assert (alone[0] == mix[i]).all()
    _check(env, data, offs, lens, width, "overlap")


def test_raw_entropy_seed(env):
    """A seed built from caller entropy (here: all words distinct small
    integers) gives the oracle's values for that entropy."""
    hth = env["hth"]
    words = np.arange(1, hth.entropy_words() + 1, dtype=np.uint64) * np.uint64(0x9E3779B1)
    seed = hth.seed_from_entropy(words)
    lens = np.array([0, 9, 5000, 200_000], dtype=np.uint64)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(15, total)
    for width in WIDTHS:
        g = _gpu_hash(env, data, offs, lens, width, seed=seed)
        c = env["oracle"].hash_batch(words, data, offs, lens, width)
        assert (g == c).all()


@pytest.fixture(scope="module")
def throughput_batch(env):
    """The 4096 x 1 MiB batch (splitmix64 seed 2) on the GPU and a host copy."""
    torch = env["torch"]
    n, sz = 4096, 1 << 20
    data = wl.random_bytes_torch(2, n * sz, "cuda")
    host = data.cpu().numpy()
    yield n, sz, data, host
    del data
    torch.cuda.empty_cache()


@pytest.mark.parametrize("width", WIDTHS)
def test_throughput_batch_full(env, throughput_batch, width):
    """The 4096 x 1 MiB batch hashed in one launch, in the benchmark's
    configuration and with the finest tasks (which merge every string across
    tasks): all 4096 strings checked against the oracle (threads over
    strings)."""
    torch, hth = env["torch"], env["hth"]
    n, sz, data, host = throughput_batch
    print(f"[parity] 4096 x 1 MiB width={width}", flush=True)
    offs = torch.arange(n, dtype=torch.int64, device="cuda") * sz
    lens = torch.full((n,), sz, dtype=torch.int64, device="cuda")
    seed2 = hth.expand_seed(2)
    outs = {}
    for level in (None, 0):
        try:
            if level is not None:
                hth.set_tuning(width, 0, level, level)
            outs[level] = hth.hash_batch(seed2, data, offs, lens, width).cpu().numpy()
            hth.batch_check()
        finally:
            hth.set_tuning(width)
    ref = env["oracle"].hash_batch(env["oracle"].expand_seed(2), host, np.arange(n, dtype=np.uint64) * np.uint64(sz),
                                   np.full(n, sz, dtype=np.uint64), width, nthreads=NTHREADS)
    for level, out in outs.items():
        bad = np.nonzero((out != ref).any(axis=1))[0]
        assert bad.size == 0, f"task level {level}: {bad.size} mismatches, first string {bad[0]}"


def test_offsets_and_lengths_with_bit_31_set(env):
    """Regression: 64-bit offsets and lengths whose low 32-bit half has bit 31
    set (a sign-extended half once turned such offsets into wild addresses)."""
    torch, hth = env["torch"], env["hth"]
    big = (1 << 31) + (3 << 20)
    print(f"[parity] offsets/lengths with bit 31 set, buffer {big} bytes", flush=True)
    data = wl.random_bytes_torch(21, big, "cuda")
    offs = np.array([(1 << 31) + 3, (1 << 31) - 7, 0, (1 << 31) + (1 << 20)], dtype=np.uint64)
    lens = np.array([(1 << 20) + 5, 300_000, (1 << 31) + 1000, 77], dtype=np.uint64)
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    n = torch.from_numpy(lens.view(np.int64)).cuda()
    seed = env["seed"]
    for width in (16, 40):
        g = hth.hash_batch(seed, data, o, n, width).cpu().numpy()
        hth.batch_check()
        for i in range(lens.size):
            s = wl.random_bytes(21, int(lens[i]), start_byte=int(offs[i]))
            ref = env["oracle"].hash_bytes(env["ent"], s, width)
            assert (g[i] == ref).all(), (width, i)
    del data
    torch.cuda.empty_cache()


def test_uneven_batch_full(env):
    """The uneven batch (200,000 log-uniform lengths 16 B - 256 KiB plus every
    length 0..520, packed back to back), every string checked."""
    torch, hth = env["torch"], env["hth"]
    lens = wl.uneven_lengths(3)
    offs, total = wl.pack(lens)
    print(f"[parity] uneven batch strings={lens.size} bytes={total}", flush=True)
    data = wl.random_bytes(3, total)
    d = torch.from_numpy(data).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    n = torch.from_numpy(lens.view(np.int64)).cuda()
    seed3 = hth.expand_seed(3)
    out = hth.hash_batch(seed3, d, o, n, 24).cpu().numpy()
    hth.batch_check()
    ref = env["oracle"].hash_batch(env["oracle"].expand_seed(3), data, offs, lens, 24, nthreads=NTHREADS)
    bad = np.nonzero((out != ref).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} mismatches, first string {bad[0]} len {int(lens[bad[0]])}"


def test_long_string_oracle_1gib(env):
    """One 1 GiB string (798,915 HH32 executions: seven base-8 digits, task
    accumulators up to level 6) against the oracle."""
    torch, hth = env["torch"], env["hth"]
    sz = 1 << 30
    print("[parity] one 1 GiB string, width 32", flush=True)
    data = wl.random_bytes(4, sz)
    d = torch.from_numpy(data).cuda()
    o = torch.zeros(1, dtype=torch.int64, device="cuda")
    n = torch.full((1,), sz, dtype=torch.int64, device="cuda")
    seed4 = hth.expand_seed(4)
    g = hth.hash_batch(seed4, d, o, n, 32).cpu().numpy()
    ref = env["oracle"].hash_bytes(env["oracle"].expand_seed(4), data, 32)
    assert (g[0] == ref).all()


@pytest.mark.timeout(600)
def test_long_string_8gib_oracle(env):
    """The 8 GiB string at full size (6,391,320 HH32 executions: eight base-8
    digits, so tree level 7 and its keys) against the oracle, for the
    benchmark's launch, the cross-task atomic cascade (tasks of 128
    executions) and in-wave folding of levels 3 and 4 (tasks of 128 * 8^2
    executions).  The oracle hashes the whole string on one host core
    (tens of seconds)."""
    torch, hth = env["torch"], env["hth"]
    sz = 8 << 30
    print("[parity] one 8 GiB string, width 32, three decompositions", flush=True)
    data = wl.random_bytes_torch(4, sz, "cuda")
    o = torch.zeros(1, dtype=torch.int64, device="cuda")
    n = torch.full((1,), sz, dtype=torch.int64, device="cuda")
    seed4 = hth.expand_seed(4)
    got = {}
    try:
        for name, tune in (("default", None), ("level 0", (0, 0, 0)), ("level 2", (0, 2, 2))):
            if tune is not None:
                hth.set_tuning(32, *tune)
            got[name] = hth.hash_batch(seed4, data, o, n, 32).cpu().numpy()[0]
            hth.batch_check()
    finally:
        hth.set_tuning(32)
    host = data.cpu().numpy()
    del data
    torch.cuda.empty_cache()
    print("[parity] 8 GiB string: oracle on one core ...", flush=True)
    ref = env["oracle"].hash_bytes(env["oracle"].expand_seed(4), host, 32)
    for name, g in got.items():
        assert (g == ref).all(), name


@pytest.mark.parametrize("n,level", [(300_000, None), (300_000, 0), (262_145, None), (1_100_000, None)])
def test_large_plan_scan_path(env, n, level):
    """Plans of more than 256 planner blocks (262,144 strings), which get the
    planner's scan kernel: 293 blocks (300,000 strings), 257 (262,145) and
    1,075 (1.1M; the 16M-key tests of the composed hash give each wave of the
    scan several 256-block rounds).
    Tail-only strings of 0..999 bytes, every 100th string of 15-21
    executions, every 5,000th of 600 KB (several tasks at level 0, so
    cross-task merges).  Every string with executions and 3,000 sampled
    others are checked against the oracle; the tail-only kernel and the
    hashing kernel must cover every string exactly once."""
    torch, hth = env["torch"], env["hth"]
    width = 24
    i = np.arange(n, dtype=np.uint64)
    lens = (i * np.uint64(2654435761)) % np.uint64(1000)
    lens[::100] = 20_000 + (i[::100] % np.uint64(7)) * np.uint64(1000)
    lens[::5000] = 600_000
    offs, total = wl.pack(lens)
    data = wl.random_bytes(61, total)
    print(f"[parity] large plan strings={n} bytes={total} level={level}", flush=True)
    try:
        if level is not None:
            hth.set_tuning(width, 0, level, level)
        got = _gpu_hash(env, data, offs, lens, width)
    finally:
        hth.set_tuning(width)
    rng = np.random.default_rng(7)
    sel = np.unique(np.concatenate([np.nonzero(lens >= 1344)[0], rng.integers(0, n, 3000)]))
    pieces = [data[int(offs[k]):int(offs[k] + lens[k])] for k in sel]
    so, _ = wl.pack(lens[sel])
    ref = env["oracle"].hash_batch(env["ent"], np.concatenate(pieces), so, lens[sel], width, nthreads=NTHREADS)
    bad = np.nonzero((got[sel] != ref).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} mismatches, first string {sel[bad[0]]} (len {int(lens[sel[bad[0]]])})"
