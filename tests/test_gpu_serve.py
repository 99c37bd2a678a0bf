"""The serving loop (hth_serve_*): served results equal the oracle's and the
batched path's, whatever they were batched with; admission by device memory
defers requests instead of failing them; limits answer TOO_LARGE and BUSY."""
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
    seed = hth.expand_seed(5)
    torch.cuda.synchronize()
    return {"torch": torch, "hth": hth, "seed": seed, "ent": oracle_lib.expand_seed(5), "oracle": oracle_lib}


def _oracle(env, data, offs, lens, widths):
    out = np.zeros((lens.size, 40), dtype=np.uint8)
    for w in (16, 24, 32, 40):
        sel = np.nonzero(widths == w)[0]
        if sel.size:
            out[sel, :w] = env["oracle"].hash_batch(env["ent"], data, offs[sel], lens[sel], w, nthreads=NTHREADS)
    return out


def test_served_mix_matches_oracle(env):
    """3000 lognormal requests (median 4 KiB, sigma 2, capped at 4 MiB here)
    at all four widths, plus empty and one-byte requests, submitted as fast
    as possible; every result checked."""
    hth = env["hth"]
    lens = np.concatenate([wl.lognormal_lengths(seed=5, n=3000, cap=4 << 20), np.array([0, 1, 0], dtype=np.uint64)])
    widths = np.concatenate([wl.coin_widths(5, 3000, choices=(16, 24, 32, 40)), np.array([16, 40, 24], np.uint32)])
    offs, total = wl.pack(lens)
    data = wl.random_bytes(5, total)
    print(f"[serve] mix requests={lens.size} bytes={total}", flush=True)
    with hth.Server(env["seed"], max_batch_requests=512) as srv:
        tickets = [srv.submit(data[int(o):int(o) + int(n)], int(w)) for o, n, w in zip(offs, lens, widths)]
        assert None not in tickets
        got = srv.wait_many(np.array(tickets, dtype=np.uint64))
        st = srv.stats()
    assert st["completed"] == lens.size and st["bytes"] == total and st["batches"] >= 1
    ref = _oracle(env, data, offs, lens, widths)
    bad = np.nonzero((got != ref).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} mismatches, first request {bad[0]} len {int(lens[bad[0]])} width {widths[bad[0]]}"


def test_alone_equals_mixed_and_batched(env):
    """A request's value does not depend on its batch: served alone, served
    in a mix and hashed by hth_hash_batch give the same bytes."""
    torch, hth = env["torch"], env["hth"]
    lens = wl.lognormal_lengths(seed=6, n=200, cap=1 << 20)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(6, total)
    with hth.Server(env["seed"]) as srv:
        mixed = srv.wait_many([srv.submit(data[int(o):int(o) + int(n)], 24) for o, n in zip(offs, lens)])
        for i in (0, 17, 199):
            t = srv.submit(data[int(offs[i]):int(offs[i] + lens[i])], 24)
            assert srv.wait(t, 24) == bytes(mixed[i, :24])
    d = torch.from_numpy(data).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    n = torch.from_numpy(lens.view(np.int64)).cuda()
    batched = hth.hash_batch(env["seed"], d, o, n, 24).cpu().numpy()
    assert (mixed[:, :24] == batched).all()
    assert (mixed[:, 24:] == 0).all()


def test_admission_defers_when_device_budget_is_full(env):
    """A 1 MiB device budget and 120 requests of 300-500 KB queued while
    batching is held, then released: at most three fit on the device at
    once, the others wait (deferred) and still hash correctly."""
    hth = env["hth"]
    rng = np.random.default_rng(8)
    n = 120
    lens = rng.integers(300_000, 500_000, n).astype(np.uint64)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(8, total)
    widths = np.where(np.arange(n) % 2 == 0, 16, 40).astype(np.uint32)
    with hth.Server(env["seed"], max_device_bytes=1 << 20, max_request_bytes=512 << 10,
                    host_stage_bytes=256 << 20) as srv:
        srv.pause()
        tickets = srv.replay(data, offs, lens, widths, np.zeros(n, dtype=np.uint64))
        assert srv.stats()["completed"] == 0
        srv.pause(False)
        got = srv.wait_many(tickets)
        st = srv.stats()
    assert st["deferred"] > 0 and st["completed"] == n and st["batches"] >= n // 3
    assert (got == _oracle(env, data, offs, lens, widths)).all()


def test_requests_as_large_as_both_rings(env):
    """max_request_bytes equal to the device budget and the staging size:
    after a small request leaves both rings' heads mid-lap, two requests of
    exactly that size are still admitted once the rings drain (an empty ring
    starts its next allocation at the beginning of a lap)."""
    import time
    hth = env["hth"]
    cap = 1 << 20
    lens = np.array([1000, cap, cap, 3000], dtype=np.uint64)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(9, total)
    widths = np.array([16, 40, 24, 32], dtype=np.uint32)
    got = np.zeros((lens.size, 40), dtype=np.uint8)
    with hth.Server(env["seed"], max_device_bytes=cap, max_request_bytes=cap, host_stage_bytes=cap) as srv:
        for i in range(lens.size):
            t0 = time.monotonic()
            ticket = None
            while ticket is None:  # BUSY while the host ring holds the previous request
                ticket = srv.submit(data[int(offs[i]):int(offs[i] + lens[i])], int(widths[i]))
                assert time.monotonic() - t0 < 10, f"request {i} of {int(lens[i])} bytes never admitted"
            got[i, :widths[i]] = np.frombuffer(srv.wait(ticket, int(widths[i])), dtype=np.uint8)
    assert (got == _oracle(env, data, offs, lens, widths)).all()


def test_limits_too_large_and_busy(env):
    hth = env["hth"]
    with hth.Server(env["seed"], max_request_bytes=1 << 20, max_outstanding=4) as srv:
        with pytest.raises(hth.HthError) as e:
            srv.submit(np.zeros((1 << 20) + 1, dtype=np.uint8), 16)
        assert e.value.status == hth.HTH_E_TOO_LARGE
        with pytest.raises(hth.HthError) as e:
            srv.submit(b"abc", 20)
        assert e.value.status == hth.HTH_E_INVALID
        data = wl.random_bytes(9, 4000)
        tickets = [srv.submit(data[:1000 * (i + 1)], 32) for i in range(4)]
        assert None not in tickets
        assert srv.submit(data, 32) is None  # four results uncollected
        assert srv.stats()["busy"] == 1
        first = srv.wait(tickets[0], 32)
        t = srv.submit(data, 32)
        assert t is not None
        with pytest.raises(hth.HthError) as e:
            srv.poll(tickets[0])  # already collected
        assert e.value.status == hth.HTH_E_INVALID
        rest = [srv.wait(x, 32) for x in tickets[1:] + [t]]
    ref = env["oracle"].hash_batch(env["ent"], data, np.zeros(5, np.uint64),
                                   np.array([1000, 2000, 3000, 4000, 4000], np.uint64), 32)
    assert [first] + rest == [bytes(r) for r in ref]


@pytest.fixture(scope="module")
def requests20k():
    n = 20_000
    lens = wl.lognormal_lengths(seed=5, n=n)
    widths = wl.coin_widths(5, n)
    offs, total = wl.pack(lens)
    return {"n": n, "lens": lens, "widths": widths, "offs": offs, "total": total, "data": wl.random_bytes(5, total),
            "arrive": np.cumsum(wl.poisson_gaps(5, n, 20_000.0))}


@pytest.mark.parametrize("threads", [1, 4])
def test_replay_poisson_and_spot_check(env, requests20k, threads):
    """A Poisson replay of the serving workload (20,000 requests at 20,000
    requests/s, from 1 and from 4 client threads): every result equals
    hth_hash_batch's, 2% of them are checked against the oracle, and the
    report carries latencies."""
    torch, hth = env["torch"], env["hth"]
    rq = requests20k
    n, lens, widths, offs, data = rq["n"], rq["lens"], rq["widths"], rq["offs"], rq["data"]
    print(f"[serve] replay requests={n} bytes={rq['total']} threads={threads}", flush=True)
    with hth.Server(env["seed"]) as srv:
        tickets = srv.replay(data, offs, lens, widths, (rq["arrive"] * 1e9).astype(np.uint64), threads=threads)
        got = srv.wait_many(tickets)
        st = srv.stats()
    assert st["completed"] == n and st["latency_p99_us"] >= st["latency_p50_us"] > 0
    d = torch.from_numpy(data).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    ln = torch.from_numpy(lens.view(np.int64)).cuda()
    for w in (16, 40):
        sel = np.nonzero(widths == w)[0]
        ref = hth.hash_batch(env["seed"], d, o[torch.from_numpy(sel).cuda()], ln[torch.from_numpy(sel).cuda()], w)
        assert (got[sel, :w] == ref.cpu().numpy()).all()
    spot = np.arange(threads, n, 50)
    assert (got[spot] == _oracle(env, data, offs[spot], lens[spot], widths[spot])).all()


def test_burst_from_many_threads(env, requests20k):
    """Every request due at once from 8 client threads with a small staging
    area (submits are refused BUSY and retried): all results still match."""
    torch, hth = env["torch"], env["hth"]
    rq = requests20k
    n = 5000
    lens, widths, offs, data = rq["lens"][:n], rq["widths"][:n], rq["offs"][:n], rq["data"]
    with hth.Server(env["seed"], host_stage_bytes=32 << 20, max_device_bytes=32 << 20) as srv:
        tickets = srv.replay(data, offs, lens, widths, np.zeros(n, dtype=np.uint64), threads=8)
        got = srv.wait_many(tickets)
        st = srv.stats()
    assert st["completed"] == n
    d = torch.from_numpy(data).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    ln = torch.from_numpy(lens.view(np.int64)).cuda()
    for w in (16, 40):
        sel = np.nonzero(widths == w)[0]
        ref = hth.hash_batch(env["seed"], d, o[torch.from_numpy(sel).cuda()], ln[torch.from_numpy(sel).cuda()], w)
        assert (got[sel, :w] == ref.cpu().numpy()).all()


def test_pinned_requests_mixed_with_staged(env, requests20k):
    """Requests left in the caller's pinned memory (hth_serve_submit_pinned,
    including empty and one-byte ones at odd addresses) interleaved with
    staged ones, then a pinned replay of 5,000 requests from 4 threads with
    every request due at once under a 32 MiB device budget: every result
    equals the oracle's."""
    hth = env["hth"]
    rq = requests20k
    n = 600
    lens = np.concatenate([rq["lens"][:n - 3] % (256 << 10), np.array([0, 1, 3], np.uint64)])
    widths = np.concatenate([rq["widths"][:n - 3], np.array([24, 32, 40], np.uint32)])
    offs, total = wl.pack(lens)
    offs = offs + 1  # every request at an odd address of the pinned buffer
    data = wl.random_bytes(11, total + 1)
    pinned = hth.pinned_bytes(data)
    print(f"[serve] pinned mix requests={n} bytes={total}", flush=True)
    with hth.Server(env["seed"]) as srv:
        tickets = []
        for i in range(n):
            o, ln, w = int(offs[i]), int(lens[i]), int(widths[i])
            t = srv.submit_pinned(pinned[o:o + ln], w) if i % 3 else srv.submit(data[o:o + ln], w)
            assert t is not None
            tickets.append(t)
        got = srv.wait_many(np.array(tickets, dtype=np.uint64))
    assert (got == _oracle(env, data, offs, lens, widths)).all()

    m = 5000
    lens, widths, offs = rq["lens"][:m], rq["widths"][:m], rq["offs"][:m]
    pinned = hth.pinned_bytes(rq["data"])
    with hth.Server(env["seed"], max_device_bytes=32 << 20) as srv:
        tickets = srv.replay(pinned, offs, lens, widths, np.zeros(m, dtype=np.uint64), threads=4, pinned=True)
        got = srv.wait_many(tickets)
        st = srv.stats()
    assert st["completed"] == m
    assert (got == _oracle(env, rq["data"], offs, lens, widths)).all()
