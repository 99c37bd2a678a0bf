"""Streaming (hth_stream_*): a string appended in pieces of any size hashes
to the batch value of the whole string (and the oracle's), in both
families, across save/load; pieces are device tensors."""
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
    return {"torch": torch, "hth": hth, "oracle": oracle_lib}


def _pieces(rng, total, xb):
    """Piece lengths: empty, tiny, around one execution, large; summing to total."""
    out, at = [], 0
    while at < total:
        kind = rng.integers(0, 5)
        cap = [0, 60, xb + 3, 9 * xb, 700 * xb][kind]
        n = int(min(total - at, rng.integers(0, cap + 1)))
        out.append(n)
        at += n
    return out


@pytest.mark.parametrize("block", [8, 4])
@pytest.mark.parametrize("width", [16, 24, 32, 40])
def test_stream_equals_batch_and_oracle(env, width, block):
    torch, hth, o = env["torch"], env["hth"], env["oracle"]
    seed = hth.expand_seed(41, block_words=block)
    ent = o.expand_seed(41, b=block)
    xb = wl.execution_bytes(width) * block // 8
    total = 3_000_000 + width
    data_np = wl.random_bytes(42, total)
    data = torch.from_numpy(data_np).cuda()
    rng = np.random.default_rng(width + block)
    pieces = _pieces(rng, total, xb)
    print(f"[stream] width={width} b={block} bytes={total} pieces={len(pieces)}", flush=True)
    st = hth.Stream(seed, width)
    at = 0
    mids = []
    for i, n in enumerate(pieces):
        st.update(data[at:at + n])
        at += n
        if i % 7 == 3:  # intermediate values: the hash of the prefix so far
            mids.append((at, st.final().clone()))
    got = st.final().cpu().numpy()
    assert len(st) == total
    torch.cuda.synchronize()
    whole = hth.hash_batch(seed, data, torch.zeros(1, dtype=torch.int64, device="cuda"),
                           torch.full((1,), total, dtype=torch.int64, device="cuda"), width).cpu().numpy()[0]
    assert (got == whole).all()
    assert (got == o.hash_bytes(ent, data_np, width, b=block)).all()
    for at, h in mids[:4]:
        assert (h.cpu().numpy() == o.hash_bytes(ent, data_np[:at], width, b=block)).all(), at
    st.free()


def test_stream_save_load_reset(env):
    """A checkpoint taken mid-string resumes in another stream object; reset
    returns to the empty string; a state refuses a stream of another width."""
    torch, hth, o = env["torch"], env["hth"], env["oracle"]
    seed = hth.expand_seed(43)
    ent = o.expand_seed(43)
    data_np = wl.random_bytes(44, 900_001)
    data = torch.from_numpy(data_np).cuda()
    a = hth.Stream(seed, 32)
    a.update(data[:123_457])
    state = a.save()
    b = hth.Stream(seed, 32)
    b.load(state)
    for s in (a, b):
        s.update(data[123_457:])
    ref = o.hash_bytes(ent, data_np, 32)
    assert (a.final().cpu().numpy() == ref).all()
    assert (b.final().cpu().numpy() == ref).all()
    a.reset()
    a.update(data[:5])
    assert (a.final().cpu().numpy() == o.hash_bytes(ent, data_np[:5], 32)).all()
    empty = hth.Stream(seed, 32)
    assert (empty.final().cpu().numpy() == o.hash_bytes(ent, b"", 32)).all()
    other = hth.Stream(seed, 24)
    with pytest.raises(hth.HthError):
        other.load(state)
    for s in (a, b, empty, other):
        s.free()


def test_stream_load_rejects_tampered_states(env):
    """A saved state that appending cannot produce is refused on the host
    before anything is copied: a stack level holding more than 7 items, a
    level count that is not the matching base-8 digit of the execution
    count, an execution count or byte count that disagrees with the rest.
    The untouched state still loads and resumes to the oracle's value."""
    import struct
    torch, hth, o = env["torch"], env["hth"], env["oracle"]
    seed = hth.expand_seed(47)
    ent = o.expand_seed(47)
    data_np = wl.random_bytes(48, 400_000)
    data = torch.from_numpy(data_np).cuda()
    a = hth.Stream(seed, 16)
    a.update(data[:250_001])  # 217 executions of 1152 bytes: digits (1, 3, 3), 8 bytes carried
    state = bytearray(a.save())
    hdr = "<4I2Q2I"
    magic, version, width, block, execs, total, carry, _ = struct.unpack_from(hdr, state, 0)
    assert (width, block, execs, total, carry) == (16, 8, 217, 250_001, 250_001 - 217 * 1152)
    cnt_at = struct.calcsize(hdr)
    assert list(struct.unpack_from("<20I", state, cnt_at))[:4] == [1, 3, 3, 0]
    tampered = []
    for lvl, val in ((0, 9), (1, 4), (3, 1), (19, 7)):
        t = bytearray(state)
        struct.pack_into("<I", t, cnt_at + 4 * lvl, val)
        tampered.append(t)
    for field, val in ((4, execs + 1), (5, total + 1), (5, total - carry)):
        t = bytearray(state)
        vals = list(struct.unpack_from(hdr, t, 0))
        vals[field] = val
        struct.pack_into(hdr, t, 0, *vals)
        tampered.append(t)
    b = hth.Stream(seed, 16)
    for t in tampered:
        with pytest.raises(hth.HthError):
            b.load(bytes(t))
    b.load(bytes(state))
    b.update(data[250_001:])
    assert (b.final().cpu().numpy() == o.hash_bytes(ent, data_np, 16)).all()
    for s in (a, b):
        s.free()


def test_stream_long_string_pieces(env):
    """A 1 GiB string appended in 37 uneven pieces (blocks up to level 6)."""
    torch, hth, o = env["torch"], env["hth"], env["oracle"]
    seed = hth.expand_seed(45)
    sz = 1 << 30
    data = wl.random_bytes_torch(46, sz, "cuda")
    rng = np.random.default_rng(46)
    cuts = np.sort(rng.integers(1, sz, 36))
    st = hth.Stream(seed, 24)
    prev = 0
    for c in list(cuts) + [sz]:
        st.update(data[prev:int(c)])
        prev = int(c)
    got = st.final().cpu().numpy()
    whole = hth.hash_batch(seed, data, torch.zeros(1, dtype=torch.int64, device="cuda"),
                           torch.full((1,), sz, dtype=torch.int64, device="cuda"), 24).cpu().numpy()[0]
    assert (got == whole).all()
    st.free()
    del data
    torch.cuda.empty_cache()


def _views(torch, data, lens, own_every=3):
    """The pieces as tensors: views into `data`, except every own_every-th,
    copied into an allocation of its own (so pieces lie below and above
    each other in memory)."""
    out, at = [], 0
    for i, n in enumerate(lens):
        v = data[at:at + n]
        out.append(v.clone() if i % own_every == 1 else v)
        at += n
    return out


@pytest.mark.parametrize("block", [8, 4])
@pytest.mark.parametrize("width", [16, 24, 32, 40])
def test_stream_gather_equals_batch_and_oracle(env, width, block):
    """Gathered updates (hth_stream_update_gather) of 1 .. 80 pieces,
    mixed with plain updates, give the batch value of the whole string and
    the oracle's value of every prefix taken between calls."""
    torch, hth, o = env["torch"], env["hth"], env["oracle"]
    seed = hth.expand_seed(51, block_words=block)
    ent = o.expand_seed(51, b=block)
    xb = wl.execution_bytes(width) * block // 8
    total = 2_500_000 + 3 * width
    data_np = wl.random_bytes(52, total)
    data = torch.from_numpy(data_np).cuda()
    rng = np.random.default_rng(100 + width + block)
    lens = _pieces(rng, total, xb)
    views = _views(torch, data, lens)
    print(f"[gather] width={width} b={block} bytes={total} pieces={len(lens)}", flush=True)
    st = hth.Stream(seed, width)
    i, mids = 0, []
    while i < len(views):
        if rng.integers(0, 4) == 0:
            st.update(views[i])
            i += 1
        else:
            k = int(rng.integers(1, 81))
            st.update_gather(views[i:i + k])
            i += k
        if len(mids) < 4 and i < len(views) and rng.integers(0, 2) == 0:
            mids.append((sum(lens[:i]), st.final().clone()))
    got = st.final().cpu().numpy()
    assert len(st) == total
    whole = hth.hash_batch(seed, data, torch.zeros(1, dtype=torch.int64, device="cuda"),
                           torch.full((1,), total, dtype=torch.int64, device="cuda"), width).cpu().numpy()[0]
    assert (got == whole).all()
    assert (got == o.hash_bytes(ent, data_np, width, b=block)).all()
    for at, h in mids:
        assert (h.cpu().numpy() == o.hash_bytes(ent, data_np[:at], width, b=block)).all(), at
    st.free()


def _gather_groups(lens, carry, e0, xb, gmax=64, table=1024):
    """Sizes of the groups a gathered call forms: pieces are taken while a
    group holds at most gmax pieces and its aligned blocks of 8^L
    executions plus the executions that straddle pieces number at most
    `table`.  (Only to check that a test's pieces need several groups.)"""
    def blocks(x, end):
        c = 0
        while x < end:
            L = 0
            while x % 8 ** (L + 1) == 0 and x + 8 ** (L + 1) <= end:
                L += 1
            x += 8 ** L
            c += 1
        return c
    groups, i = [], 0
    while i < len(lens):
        at, nxt, n, taken = carry, 0, 0, 0
        while i < len(lens) and taken < gmax:
            m = lens[i]
            if m == 0:
                i += 1
                continue
            a, b = -(-at // xb), (at + m) // xb
            tn, tnxt = n, nxt
            if b > a:
                tn += (a - nxt) + blocks(e0 + a, e0 + b)
                tnxt = b
            if tn + ((at + m) // xb - tnxt) > table:
                break
            n, nxt, at, taken, i = tn, tnxt, at + m, taken + 1, i + 1
        groups.append(taken)
        e0, carry = e0 + at // xb, at % xb
    return groups


def test_stream_gather_splits_groups_and_resumes(env):
    """Some 400 pieces in two gathered calls: the library splits them into
    groups by piece count and by table size (pieces of 2 (8^3 - 1)
    executions starting one past a multiple of 8^3 cut into 42 aligned
    blocks each; two-execution pieces between them restore that start); the
    value is the batch's and the oracle's, and a state saved between the
    calls resumes in another stream object."""
    torch, hth, o = env["torch"], env["hth"], env["oracle"]
    width, xb = 24, wl.execution_bytes(24)
    seed = hth.expand_seed(53)
    ent = o.expand_seed(53)
    rng = np.random.default_rng(54)
    lens = [xb] + [1022 * xb, 2 * xb] * 150
    kinds = rng.integers(0, 4, 99)
    lens += [int(rng.integers(0, [1, 200, 3 * xb, 700 * xb][k] + 1)) for k in kinds]
    total = sum(lens)
    groups = _gather_groups(lens[:301], 0, 0, xb)
    assert len(groups) >= 3 and max(groups[:-1]) < 64, groups  # split by table size
    data_np = wl.random_bytes(55, total)
    data = torch.from_numpy(data_np).cuda()
    views = _views(torch, data, lens, own_every=5)
    print(f"[gather] {len(lens)} pieces, {total} bytes; groups of the first 301: {groups}", flush=True)
    a = hth.Stream(seed, width)
    a.update_gather(views[:301])
    state = a.save()
    b = hth.Stream(seed, width)
    b.load(state)
    for s in (a, b):
        s.update_gather(views[301:])
    ref = o.hash_bytes(ent, data_np, width)
    whole = hth.hash_batch(seed, data, torch.zeros(1, dtype=torch.int64, device="cuda"),
                           torch.full((1,), total, dtype=torch.int64, device="cuda"), width).cpu().numpy()[0]
    assert (whole == ref).all()
    for s in (a, b):
        assert len(s) == total
        assert (s.final().cpu().numpy() == ref).all()
        s.free()


def test_stream_gather_argument_errors(env):
    """Null arrays with pieces, or a null piece of non-zero length, are
    refused before anything is enqueued; count 0 and empty pieces are
    no-ops."""
    import ctypes
    torch, hth, o = env["torch"], env["hth"], env["oracle"]
    seed = hth.expand_seed(56)
    st = hth.Stream(seed, 16)
    L = hth.lib()
    lens = (ctypes.c_uint64 * 2)(5, 7)
    ptrs = (ctypes.c_void_p * 2)(None, None)
    assert L.hth_stream_update_gather(st._h, ptrs, lens, 2, None) != 0
    assert L.hth_stream_update_gather(st._h, None, lens, 2, None) != 0
    assert L.hth_stream_update_gather(st._h, None, None, 0, None) == 0
    st.update_gather([])
    st.update_gather([torch.empty(0, dtype=torch.uint8, device="cuda")] * 3)
    assert len(st) == 0
    assert (st.final().cpu().numpy() == o.hash_bytes(o.expand_seed(56), b"", 16)).all()
    st.free()


def test_stream_gather_back_to_back_calls(env):
    """Twelve gathered calls in a row with nothing between them (each call's
    push runs beside the next call's hashing, the two root buffers taking
    turns), then the value; reset and free right after a gathered call."""
    torch, hth, o = env["torch"], env["hth"], env["oracle"]
    width, xb = 40, wl.execution_bytes(40)
    seed = hth.expand_seed(57)
    ent = o.expand_seed(57)
    rng = np.random.default_rng(58)
    lens = [int(rng.integers(0, 900 * xb)) for _ in range(36)]
    total = sum(lens)
    data_np = wl.random_bytes(59, total)
    data = torch.from_numpy(data_np).cuda()
    views = _views(torch, data, lens, own_every=4)
    st = hth.Stream(seed, width)
    for c in range(0, 36, 3):
        st.update_gather(views[c:c + 3])
    assert (st.final().cpu().numpy() == o.hash_bytes(ent, data_np, width)).all()
    st.update_gather(views[:5])
    st.reset()
    st.update_gather(views[:2])
    st.update(views[2])
    at = lens[0] + lens[1] + lens[2]
    assert (st.final().cpu().numpy() == o.hash_bytes(ent, data_np[:at], width)).all()
    st.update_gather(views[3:9])
    st.free()  # (its last push may still be running)
    torch.cuda.synchronize()
