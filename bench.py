"""Throughput benchmark of the HalftimeHash hot path on one MI355X.

One step hashes the throughput batch -- 4096 strings of 1 MiB (4 GiB of
uniformly random bytes from splitmix64 seed 2, already resident in HBM) --
once at each output width 16, 24, 32 and 40 bytes: four launches of the
batched kernel (each preceded by its short planning step), i.e. the whole
hot path over one batch.  `value` is hashed bytes per second over the timed
steps (decimal GB/s).

Extra objects on the JSON line:
  roofline      the dominant kernel (the slowest width's hashing kernel)
                against the 8 TB/s HBM peak: algorithmic bytes per launch over
                its average duration, timed with HIP events on the launch
                stream; `traffic` is the counter-measured HBM traffic per
                launch from profiles/ when it was taken on the current kernel
                source, else null.
  per_width     the same figures for every width.
  cpu_baseline  the CPU oracle on this host, single-threaded, on a bounded
                sample of the same batch; the sample is also checked
                bit-for-bit against the GPU output.
  uneven        the uneven batch (200,521 strings of 0 B - 256 KiB, width 24):
                one persistent launch per step, the same launch replayed from
                a HIP graph, and one launch per string on a stated sample of
                strings; its own roofline, traffic and CPU baseline.
  latency       the serving loop: capacity, then p50/p99 at three offered
                loads; 1.6 % of the served results recomputed by the oracle.

  python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
  python bench.py --workload uneven   # 200,521 strings of 16 B - 256 KiB, width 24:
                                      # one persistent launch vs a captured graph vs
                                      # one launch per string (autotuned launch choice)
  python bench.py --workload long     # one 8 GiB string, width 32
Each workload prints one JSON line of the same shape.
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WIDTHS = (16, 24, 32, 40)
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2104_08865_amd", "csrc", "hth_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hash_main_throughput_traffic.json")
UNEVEN_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hash_main_uneven_traffic.json")
DEFAULT_CHOICES = ((0, 0, 5), (8, 0, 5))  # the launch choice the uneven counters were taken with


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256[:16] of the kernel source with comments and blank lines removed:
    an edit of a comment leaves the committed counters valid, any code change
    does not."""
    with open(KERNEL_SRC) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    code = [re.sub(r"//.*$", "", line).rstrip() for line in text.splitlines()]
    return hashlib.sha256("\n".join(line for line in code if line.strip()).encode()).hexdigest()[:16]


def measured_traffic(width, path=None):
    """HBM bytes per launch from a committed counter summary, if it was
    taken on the current kernel source."""
    try:
        doc = json.load(open(path or TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if doc.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    row = doc.get("per_width", {}).get(str(width))
    return None if row is None else row.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def pinned_oracle(fn):
    """Run fn() pinned to one host core (restored afterwards); returns
    (result, seconds, core)."""
    prev = os.sched_getaffinity(0)
    core = min(prev)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        r = fn()
        return r, time.perf_counter() - t0, core
    finally:
        os.sched_setaffinity(0, prev)


def cpu_baseline(gpu_out, n_strings, string_bytes, sample_per_width, b=8):
    import oracle
    from paper_2104_08865_amd import workloads as wl
    ent = oracle.expand_seed(2, b=b)
    total_bytes, total_s, exact = 0, 0.0, True
    idx = np.linspace(0, n_strings - 1, sample_per_width).astype(np.int64)
    data = np.concatenate([wl.random_bytes(2, string_bytes, start_byte=int(i) * string_bytes) for i in idx])
    offs = (np.arange(idx.size, dtype=np.uint64) * np.uint64(string_bytes))
    lens = np.full(idx.size, string_bytes, dtype=np.uint64)
    for width in WIDTHS:
        ref, dt, core = pinned_oracle(lambda: oracle.hash_batch(ent, data, offs, lens, width, nthreads=1, b=b))
        total_s += dt
        total_bytes += data.size
        exact &= bool((gpu_out[width][idx] == ref).all())
        log(f"[bench] cpu oracle width {width}: {idx.size} strings checked in {dt:.1f} s, exact={exact}")
    return {
        "value": total_bytes / total_s / 1e9,
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{sample_per_width} of the 4096 1 MiB strings at each width 16/24/32/40 "
                  f"({total_bytes / 2**20:.0f} MiB hashed), single thread pinned to core {core}",
        "seconds": total_s,
        "cpu_model": cpu_model(),
        "host_cpus": len(os.sched_getaffinity(0)),
        "bit_exact_vs_gpu": exact,
    }


def run_main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1024, help="oracle strings per width")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration for profiles)")
    ap.add_argument("--workload", choices=("throughput", "uneven", "long", "serve", "compose"), default="throughput")
    ap.add_argument("--serve-requests", type=int, default=100_000, help="requests per offered load (serve)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg of the default line")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch leg of the default line")
    ap.add_argument("--no-autotune", action="store_true", help="uneven workload: default launch choice")
    ap.add_argument("--uneven-subsets", action="store_true",
                    help="uneven workload: also hash subsets of the batch by execution count, each alone")
    ap.add_argument("--block-words", type=int, default=8, choices=(4, 8),
                    help="throughput workload: the family's block size b (8, or 4 for the 256-bit family)")
    ap.add_argument("--no-per-string", action="store_true",
                    help="uneven workload: skip the per-string launch comparison (for profiling runs)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library hashes on a single MI355X and has no multi-GPU path "
              "(batches would shard by string with no exchange; see the design notes). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "uneven":
        line = run_uneven(args)
    elif args.workload == "long":
        line = run_long(args)
    elif args.workload == "serve":
        line = run_serve(args)
    elif args.workload == "compose":
        line = run_compose(args)
    else:
        line = run_throughput(args)
    print(json.dumps(line), flush=True)


def run_throughput(args):
    import torch
    from paper_2104_08865_amd import hth
    from paper_2104_08865_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, sz = 4096, 1 << 20
    log("[bench] generating 4096 x 1 MiB (splitmix64 seed 2) on the GPU")
    data = wl.random_bytes_torch(2, n * sz, dev)
    offs = torch.arange(n, dtype=torch.int64, device=dev) * sz
    lens = torch.full((n,), sz, dtype=torch.int64, device=dev)
    b = args.block_words
    seed = hth.expand_seed(2, block_words=b)
    outs = {w: torch.empty((n, w), dtype=torch.uint8, device=dev) for w in WIDTHS}
    hth.reserve(n)
    torch.cuda.synchronize()

    if args.calibration_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        for w in WIDTHS:
            hth.hash_batch(seed, data, offs, lens, w, out=outs[w])
    hth.batch_check()
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")

    timers = {w: [hth.Timer() for _ in range(args.steps)] for w in WIDTHS}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for w in WIDTHS:
            hth.hash_batch(seed, data, offs, lens, w, out=outs[w], timer=timers[w][k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hth.batch_check()
    log(f"[bench] timed {args.steps} steps in {t1 - t0:.3f} s")

    step_bytes = len(WIDTHS) * n * sz
    wall = t1 - t0
    value = step_bytes * args.steps / wall / 1e9
    per_width = {}
    for w in WIDTHS:
        samples = [t.elapsed_ms() for t in timers[w]]
        ms = float(np.mean(samples))
        algo = n * sz + 16 * n + w * n  # input bytes + offsets/lengths + output
        achieved = algo / (ms * 1e-3) / 1e9
        per_width[str(w)] = {
            "kernel": f"hth::hash_main_kernel<{w}, {b}, false>",
            "avg_ms": ms,
            "median_ms": float(np.median(samples)),
            "median_GBps": algo / (float(np.median(samples)) * 1e-3) / 1e9,
            "algorithmic_bytes": algo,
            "achieved_GBps": achieved,
            "frac_of_hbm_peak": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(w) if b == 8 else None,
        }
    # the device's plain streaming-read rate over the same 4 GiB buffer
    probe = [hth.Timer() for _ in range(5)]
    hth.read_probe(data)
    for t in probe:
        hth.read_probe(data, timer=t)
    read_ms = float(np.median([t.elapsed_ms() for t in probe]))
    read_ceiling = data.numel() / (read_ms * 1e-3) / 1e9
    log(f"[bench] read-stream ceiling {read_ceiling:.0f} GB/s")
    dom = max(WIDTHS, key=lambda w: per_width[str(w)]["avg_ms"])
    d = per_width[str(dom)]
    roofline = {
        "bound": "hbm",
        "achieved": d["achieved_GBps"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": d["achieved_GBps"] / HBM_PEAK_GBS,
        "traffic": d["traffic"],
        "kernel": d["kernel"],
        "algorithmic_bytes_per_launch": d["algorithmic_bytes"],
        "avg_launch_ms": d["avg_ms"],
        "read_stream_ceiling_GBps": read_ceiling,
        "frac_of_read_stream_ceiling": d["achieved_GBps"] / read_ceiling,
    }

    cpu = None
    if not args.no_cpu_baseline:
        host_out = {w: outs[w].cpu().numpy() for w in WIDTHS}
        cpu = cpu_baseline(host_out, n, sz, args.cpu_sample, b)

    line = {
        "metric": "hashed GB/s vs HBM peak (bit-exact to oracle); p50/p99 latency at fixed rate",
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "throughput batch: 4096 strings x 1 MiB, uniform random bytes (splitmix64 seed 2), "
                        "hashed at widths 16/24/32/40 (one launch per width)"
                        + ("" if b == 8 else f", {64 * b}-bit block family (b = {b})"),
            "strings": n,
            "string_bytes": sz,
            "widths": list(WIDTHS),
            "seed": 2,
            "block_words": b,
        },
        "roofline": roofline,
        "per_width": per_width,
        "cpu_baseline": cpu,
    }
    del data, outs
    torch.cuda.empty_cache()
    if not args.no_uneven:
        line["uneven"] = uneven_leg(args)
    if not args.no_serve:
        line["latency"] = serve_legs(args.serve_requests)
    return line


SERVE_LOADS = (0.25, 0.5, 0.8)
SERVE_CLIENTS = 4  # replay threads of the staged submits (their copies into the staging overlap)
SERVE_PINNED_CLIENTS = 4  # replay threads of the pinned submits (no copy)


def serve_legs(n_req, verify=False):
    """The serving workload: lognormal request lengths (median 4 KiB,
    sigma 2, capped at 16 MiB), widths 16/40 at 50/50, bytes from splitmix64
    seed 5, replayed from pinned host memory into one server
    (hth_serve_replay_pinned: the requests' bytes are copied to the device by
    the server's batches, with no staging copy).  First at no pacing (every
    request due at once) to measure the server's capacity, then with Poisson
    arrivals at 0.25, 0.5 and 0.8 of that capacity; the capacity of the
    staged submit path (bytes copied into the server's pinned staging by the
    client threads) is reported beside it."""
    import torch
    from paper_2104_08865_amd import hth
    from paper_2104_08865_amd import workloads as wl

    lens = wl.lognormal_lengths(seed=5, n=n_req)
    widths = wl.coin_widths(5, n_req)
    unit_gaps = wl.poisson_gaps(5, n_req, 1.0)
    offs, total = wl.pack(lens)
    log(f"[bench] serving: {n_req} requests, {total} bytes, mean {total / n_req:.0f} B")
    data = wl.random_bytes(5, total)
    pinned = hth.pinned_bytes(data)
    seed = hth.expand_seed(5)
    torch.cuda.synchronize()
    res = {"workload": "serving: lognormal lengths (median 4 KiB, sigma 2, cap 16 MiB), widths 16/40 50/50, "
                       "bytes splitmix64 seed 5, submitted from pinned host memory; Poisson arrivals",
           "requests_per_load": n_req, "mean_request_bytes": total / n_req, "client_threads": SERVE_PINNED_CLIENTS,
           "client_threads_staged": SERVE_CLIENTS,
           "loads": []}
    with hth.Server(seed, max_device_bytes=2 << 30, host_stage_bytes=2 << 30) as srv:
        # the staged submit path's capacity (client threads copy into staging)
        tickets = srv.replay(data, offs, lens, widths, np.zeros(n_req, dtype=np.uint64), threads=SERVE_CLIENTS)
        staged = srv.wait_many(tickets)
        st = srv.stats()
        res["capacity_staged_submit"] = {"requests_per_s": st["completed"] / st["elapsed_s"], "GBps": st["gbps"],
                                         "p50_us": st["latency_p50_us"], "p99_us": st["latency_p99_us"],
                                         "mean_batch_requests": st["mean_batch_requests"]}
        log(f"[bench] serving capacity, staged submits: {st['gbps']:.1f} GB/s")
        srv.reset_stats()
        # capacity: every request due at once
        tickets = srv.replay(pinned, offs, lens, widths, np.zeros(n_req, dtype=np.uint64),
                             threads=SERVE_PINNED_CLIENTS, pinned=True)
        got = srv.wait_many(tickets)
        res["staged_equals_pinned"] = bool((staged == got).all())
        res["oracle_spot_check"] = _serve_spot_check(data, offs, lens, widths, got)
        st = srv.stats()
        cap_rps = st["completed"] / st["elapsed_s"]
        res["capacity"] = {"requests_per_s": cap_rps, "GBps": st["gbps"], "p50_us": st["latency_p50_us"],
                           "p99_us": st["latency_p99_us"], "mean_batch_requests": st["mean_batch_requests"]}
        log(f"[bench] serving capacity {cap_rps:.0f} req/s, {st['gbps']:.1f} GB/s")
        for load in SERVE_LOADS:
            rate = load * cap_rps
            arrive = (np.cumsum(unit_gaps) / rate * 1e9).astype(np.uint64)
            srv.reset_stats()
            tickets = srv.replay(pinned, offs, lens, widths, arrive, threads=SERVE_PINNED_CLIENTS, pinned=True)
            out = srv.wait_many(tickets)
            st = srv.stats()
            same = bool((out == got).all())
            res["loads"].append({"offered_fraction_of_capacity": load, "offered_requests_per_s": rate,
                                 "achieved_requests_per_s": st["completed"] / st["elapsed_s"],
                                 "GBps": st["gbps"], "p50_us": st["latency_p50_us"], "p99_us": st["latency_p99_us"],
                                 "max_us": st["latency_max_us"], "mean_batch_requests": st["mean_batch_requests"],
                                 "deferred": st["deferred"], "busy": st["busy"], "same_as_capacity_run": same})
            log(f"[bench] load {load}: p50 {st['latency_p50_us']:.0f} us, p99 {st['latency_p99_us']:.0f} us, "
                f"{st['gbps']:.1f} GB/s, identical={same}")
    if verify:
        # every served result equals the batched path's
        dev = torch.device("cuda:0")
        d = torch.from_numpy(data).to(dev)
        o = torch.from_numpy(offs.view(np.int64)).to(dev)
        n = torch.from_numpy(lens.view(np.int64)).to(dev)
        ok = True
        for w in (16, 40):
            sel = torch.from_numpy(np.nonzero(widths == w)[0]).to(dev)
            ref = hth.hash_batch(seed, d, o[sel], n[sel], w).cpu().numpy()
            ok &= bool((got[sel.cpu().numpy(), :w] == ref).all())
        res["served_equals_batched"] = ok
        del d
    return res


SERVE_SPOT_STRIDE = 64  # every 64th request (1.6 %) is recomputed by the oracle


def _serve_spot_check(data, offs, lens, widths, got):
    """Every SERVE_SPOT_STRIDE-th served result against the CPU oracle (all
    host cores; a verification aid, not a timing)."""
    import oracle
    from paper_2104_08865_amd import workloads as wl
    ent = oracle.expand_seed(5)
    idx = np.arange(0, lens.size, SERVE_SPOT_STRIDE)
    exact = True
    t0 = time.perf_counter()
    for w in (16, 40):
        sel = idx[widths[idx] == w]
        sub_lens = lens[sel]
        sub_offs, _ = wl.pack(sub_lens)
        sub = np.concatenate([data[int(offs[i]):int(offs[i]) + int(lens[i])] for i in sel])
        ref = oracle.hash_batch(ent, sub, sub_offs, sub_lens, w, nthreads=min(16, os.cpu_count() or 1))
        exact &= bool((got[sel, :w] == ref).all())
    dt = time.perf_counter() - t0
    log(f"[bench] serving oracle spot check: {idx.size} requests, exact={exact} ({dt:.1f} s)")
    return {"requests": int(idx.size), "fraction": idx.size / lens.size,
            "sample": f"every {SERVE_SPOT_STRIDE}th request of the capacity run, recomputed by the CPU oracle",
            "bit_exact": exact}


def run_serve(args):
    """Serving workload line: value = served GB/s at capacity."""
    import torch
    torch.cuda.set_device(torch.device("cuda:0"))
    res = serve_legs(args.serve_requests, verify=True)
    cap = res["capacity"]
    return {
        "metric": "hashed GB/s vs HBM peak (bit-exact to oracle); p50/p99 latency at fixed rate",
        "value": cap["GBps"], "unit": "GB/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": args.serve_requests / cap["requests_per_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": res["workload"], "requests_per_load": res["requests_per_load"]},
        "latency": res, "cpu_baseline": None,
    }


def _roofline(kernel, algo_bytes, avg_ms, traffic=None):
    achieved = algo_bytes / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
            "algorithmic_bytes_per_launch": algo_bytes, "avg_launch_ms": avg_ms}


def _timed_launches(hth, torch, launch, steps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        launch()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


UNEVEN_PER_STRING_SAMPLE = 4096  # strings launched one by one in the default line's uneven leg


def run_uneven(args):
    """200,000 log-uniform lengths in [16 B, 256 KiB) plus every length 0..520
    (bytes from splitmix64 seed 3, packed back to back, so most strings start
    unaligned), width 24."""
    leg = uneven_leg(args, autotune=not args.no_autotune, per_string=None if not args.no_per_string else 0)
    return _uneven_line(args, leg)


def uneven_leg(args, autotune=False, per_string=UNEVEN_PER_STRING_SAMPLE):
    """The uneven batch: one persistent launch per step (timed over args.steps),
    the same launch replayed from a HIP graph, and one launch per string --
    for every string (per_string None), a stated sample of strings spread over
    the batch (per_string > 0) or none (0).  Returns the leg's figures."""
    import torch
    from paper_2104_08865_amd import autotune as at, hth
    from paper_2104_08865_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    width = 24
    lens = wl.uneven_lengths(3)
    offs, total = wl.pack(lens)
    count = lens.size
    log(f"[bench] uneven batch: {count} strings, {total} bytes")
    data = wl.random_bytes_torch(3, total, dev)
    o = torch.from_numpy(offs.view(np.int64)).to(dev)
    n = torch.from_numpy(lens.view(np.int64)).to(dev)
    seed = hth.expand_seed(3)
    hth.reserve(count)
    if args.calibration_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not autotune:
        choice, times = (0, 0, 5), {}
        hth.set_tuning(width)
    else:
        choice, times = at.tune(seed, data, o, n, width, total_bytes=total, use_cache=False)
    log(f"[bench] uneven launch choice (waves/CU, min level, max level) = {choice}")
    out = torch.empty((count, width), dtype=torch.uint8, device=dev)

    # one persistent launch per step
    for _ in range(args.warmup):
        hth.hash_batch(seed, data, o, n, width, out=out)
    timers = [hth.Timer() for _ in range(args.steps)]
    it = iter(timers)
    wall = _timed_launches(hth, torch, lambda: hth.hash_batch(seed, data, o, n, width, out=out, timer=next(it)),
                           args.steps)
    hth.batch_check()
    kernel_ms = float(np.mean([t.elapsed_ms() for t in timers]))
    persistent = out.cpu().numpy()

    # the same launch captured in a graph
    g = hth.BatchGraph(seed, data, o, n, width)
    for _ in range(args.warmup):
        g.launch()
    gwall = _timed_launches(hth, torch, g.launch, args.steps)
    g.check()
    graph_out = g.out.cpu().numpy()

    # one launch per string
    if per_string == 0:
        sidx, swall, sbytes, per_out = None, None, None, None
    else:
        sidx = np.arange(count) if per_string is None else np.linspace(0, count - 1, per_string).astype(np.int64)
        swall, per_out = _per_string(hth, torch, seed, data, o, n, width, sidx, dev)
        sbytes = int(lens[sidx].sum())
    agree = bool((persistent == graph_out).all() and (per_out is None or (persistent[sidx] == per_out).all()))
    pstr = f"{sbytes / swall / 1e9:.2f}" if swall else "skipped"
    log(f"[bench] persistent {total / wall * args.steps / 1e9:.0f} GB/s, graph {total / gwall * args.steps / 1e9:.0f} "
        f"GB/s, per-string {pstr} GB/s, identical={agree}")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        idx = np.arange(0, count, 20)
        sub_lens = lens[idx]
        sub_offs, sub_total = wl.pack(sub_lens)
        sub = np.concatenate([wl.random_bytes(3, int(lens[i]), start_byte=int(offs[i])) for i in idx])
        ent = oracle.expand_seed(3)
        ref, dt, core = pinned_oracle(lambda: oracle.hash_batch(ent, sub, sub_offs, sub_lens, width, nthreads=1))
        cpu = {"value": sub_total / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"every 20th string of the batch ({idx.size} strings, {sub_total} bytes), "
                         f"single thread pinned to core {core}",
               "seconds": dt, "bit_exact_vs_gpu": bool((ref == persistent[idx]).all())}
        log(f"[bench] uneven cpu oracle: {idx.size} strings in {dt:.1f} s, exact={cpu['bit_exact_vs_gpu']}")
    subsets = _uneven_subsets(hth, torch, seed, data, o, n, lens, width) if getattr(args, "uneven_subsets", False) \
        else None
    del data, out, g
    torch.cuda.empty_cache()

    algo = total + 16 * count + width * count
    persistent_gbps = total * args.steps / wall / 1e9
    per_gbps = sbytes / swall / 1e9 if swall else None
    return {
        "workload": "uneven batch: 200,000 log-uniform lengths in [16 B, 256 KiB) plus every length 0..520, "
                    "packed back to back (splitmix64 seed 3), width 24",
        "strings": int(count), "bytes": int(total), "width": width, "seed": 3,
        "launch_choice": {"waves_per_cu": choice[0], "task_levels": [choice[1], choice[2]]},
        "steps": args.steps, "ms_per_step": wall / args.steps * 1e3,
        "persistent_GBps": persistent_gbps,
        "roofline": _roofline(f"hth::hash_main_kernel<{width}, 8, false>", algo, kernel_ms,
                              measured_traffic(width, UNEVEN_TRAFFIC_FILE) if choice in DEFAULT_CHOICES else None),
        "graph_replay_GBps": total * args.steps / gwall / 1e9,
        "per_string_launches_GBps": per_gbps,
        "per_string_sample": None if sidx is None else
            (f"all {count} strings" if per_string is None else
             f"{sidx.size} strings spread evenly over the batch ({sbytes} bytes), one hth_hash_batch call each"),
        "persistent_over_per_string": persistent_gbps / per_gbps if per_gbps else None,
        "all_identical": agree,
        "autotune_ms": {f"{c[0]}/{c[1]}-{c[2]}": round(t, 4) for c, t in times.items()},
        "subsets": subsets,
        "cpu_baseline": cpu,
    }


UNEVEN_SUBSETS = (("shorter than one execution (tail only)", 0, 0), ("1-8 executions", 1, 8),
                  ("9-16 executions", 9, 16), ("17-63 executions", 17, 63), ("1-63 executions", 1, 63),
                  ("64-127 executions", 64, 127), (">= 128 executions", 128, None), ("all", 0, None))


def _uneven_subsets(hth, torch, seed, data, o, n, lens, width):
    """The uneven batch's strings grouped by execution count, each group
    hashed alone (its offsets and lengths in one call): median of 8 calls of
    HIP events around the hashing, tail-only and small-string kernels."""
    from paper_2104_08865_amd import workloads as wl
    N = lens // wl.execution_bytes(width)
    timer = hth.Timer()
    rows = []
    for label, lo, hi in UNEVEN_SUBSETS:
        sel = (N >= lo) & (N <= hi if hi is not None else True)
        idx = torch.from_numpy(np.nonzero(sel)[0]).to(o.device)
        so, sn = o[idx].contiguous(), n[idx].contiguous()
        ms = []
        for _ in range(10):
            hth.hash_batch(seed, data, so, sn, width, timer=timer)
            ms.append(timer.elapsed_ms())
        m = float(np.median(ms[2:]))
        b = int(lens[sel].sum())
        rows.append({"subset": label, "strings": int(sel.sum()), "bytes": b, "ms": m, "GBps": b / m / 1e6})
        log(f"[bench] uneven subset {label}: {int(sel.sum())} strings, {m:.4f} ms, {b / m / 1e6:.0f} GB/s")
    return rows


def _per_string(hth, torch, seed, data, o, n, width, idx, dev):
    """The same library call once per string of the index sample idx (one
    launch each); returns the wall time and their outputs."""
    import ctypes
    L = hth.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    per = torch.empty((idx.size, width), dtype=torch.uint8, device=dev)
    sp, dp, op, np_, pp = seed.handle, ctypes.c_void_p(data.data_ptr()), o.data_ptr(), n.data_ptr(), per.data_ptr()
    log(f"[bench] per-string launches ({idx.size} strings) ...")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, i in enumerate(idx.tolist()):
        rc = L.hth_hash_batch(sp, dp, ctypes.c_void_p(op + 8 * i), ctypes.c_void_p(np_ + 8 * i), 1,
                              ctypes.c_void_p(pp + width * k), width, stream)
        if rc:
            raise RuntimeError(L.hth_last_error())
    torch.cuda.synchronize()
    swall = time.perf_counter() - t0
    return swall, per.cpu().numpy()


def _uneven_line(args, leg):
    return {
        "metric": "hashed GB/s vs HBM peak (bit-exact to oracle); p50/p99 latency at fixed rate",
        "value": leg["persistent_GBps"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": leg["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": leg["workload"] + ", one persistent launch", "strings": leg["strings"],
                   "bytes": leg["bytes"], "width": leg["width"], "seed": leg["seed"],
                   "launch_choice": leg["launch_choice"]},
        "roofline": leg["roofline"],
        "graph_replay_GBps": leg["graph_replay_GBps"],
        "per_string_launches_GBps": leg["per_string_launches_GBps"],
        "per_string_sample": leg["per_string_sample"],
        "persistent_over_per_string": leg["persistent_over_per_string"],
        "all_three_identical": leg["all_identical"],
        "autotune_ms": leg["autotune_ms"],
        **({"subsets": leg["subsets"]} if leg.get("subsets") else {}),
        "cpu_baseline": leg["cpu_baseline"],
    }


def run_long(args):
    """One 8 GiB string of uniformly random bytes (splitmix64 seed 4), width 32."""
    import torch
    import oracle
    from paper_2104_08865_amd import autotune, hth
    from paper_2104_08865_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    width, sz = 32, 8 << 30
    log("[bench] one 8 GiB string")
    data = wl.random_bytes_torch(4, sz, dev)
    o = torch.zeros(1, dtype=torch.int64, device=dev)
    n = torch.full((1,), sz, dtype=torch.int64, device=dev)
    seed = hth.expand_seed(4)
    choice, times = autotune.tune(seed, data, o, n, width, total_bytes=sz, use_cache=False)
    log(f"[bench] autotuned launch choice = {choice}")
    out = torch.empty((1, width), dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        hth.hash_batch(seed, data, o, n, width, out=out)
    timers = [hth.Timer() for _ in range(args.steps)]
    it = iter(timers)
    wall = _timed_launches(hth, torch, lambda: hth.hash_batch(seed, data, o, n, width, out=out, timer=next(it)),
                           args.steps)
    hth.batch_check()
    kernel_ms = float(np.mean([t.elapsed_ms() for t in timers]))
    whole = out.cpu().numpy()[0]

    # the same string through the streaming API, appended in pieces
    hth.set_tuning(width)
    st = hth.Stream(seed, width)
    streaming = {}
    for piece in (128 << 20, 1 << 30):
        rates, same = [], True
        for rep in range(3):
            st.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for at in range(0, sz, piece):
                st.update(data[at:at + piece])
            h = st.final()
            torch.cuda.synchronize()
            rates.append(sz / (time.perf_counter() - t0) / 1e9)
            same &= bool((h.cpu().numpy() == whole).all())
        streaming[f"{piece >> 20} MiB pieces"] = {"GBps": max(rates), "same_value_as_batch": same}
        log(f"[bench] streaming in {piece >> 20} MiB pieces: {max(rates):.0f} GB/s, same value={same}")
    # the same 128 MiB pieces through gathered updates: `per` pieces a call
    # (the library hashes the blocks of a call's pieces in one launch per
    # group of up to 64 pieces and 1024 blocks)
    piece = 128 << 20
    views = [data[at:at + piece] for at in range(0, sz, piece)]
    for per in (8, len(views)):
        rates, same = [], True
        for rep in range(3):
            st.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c in range(0, len(views), per):
                st.update_gather(views[c:c + per])
            h = st.final()
            torch.cuda.synchronize()
            rates.append(sz / (time.perf_counter() - t0) / 1e9)
            same &= bool((h.cpu().numpy() == whole).all())
        key = f"{piece >> 20} MiB pieces, {per} per gathered call"
        streaming[key] = {"GBps": max(rates), "same_value_as_batch": same}
        log(f"[bench] streaming in {key}: {max(rates):.0f} GB/s, same value={same}")
    st.free()
    cpu = None
    if not args.no_cpu_baseline:
        # the whole string through the oracle on one pinned core (tens of
        # seconds), compared with the GPU's value
        host = data.cpu().numpy()
        log("[bench] cpu oracle on the whole 8 GiB string ...")
        ref, dt, core = pinned_oracle(lambda: oracle.hash_bytes(oracle.expand_seed(4), host, width))
        cpu = {"value": sz / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole 8 GiB string, single thread pinned to core {core}", "seconds": dt,
               "cpu_model": cpu_model(), "host_cpus": len(os.sched_getaffinity(0)),
               "bit_exact_vs_gpu": bool((ref == whole).all())}
        log(f"[bench] cpu oracle: {cpu['value']:.2f} GB/s, exact={cpu['bit_exact_vs_gpu']}")
        del host
    algo = sz + 16 + width
    return {
        "metric": "hashed GB/s vs HBM peak (bit-exact to oracle); p50/p99 latency at fixed rate",
        "value": sz * args.steps / wall / 1e9, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "one 8 GiB string of uniform random bytes (splitmix64 seed 4), width 32",
                   "bytes": sz, "width": width, "seed": 4,
                   "launch_choice": {"waves_per_cu": choice[0], "task_levels": [choice[1], choice[2]]}},
        "roofline": _roofline(f"hth::hash_main_kernel<{width}, 8, false>", algo, kernel_ms),
        "autotune_ms": {f"{c[0]}/{c[1]}-{c[2]}": round(t, 4) for c, t in times.items()},
        "streaming": streaming,
        "cpu_baseline": cpu,
    }


def _event_ms(torch, launch, steps):
    """Average ms of `launch` over `steps` calls, by events on the current stream."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        launch()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def run_compose(args):
    """The composed 64-bit hash (HalftimeHash + simple tabulation), inner
    width 16: 16,777,216 hash-table keys of 0..64 bytes (lengths uniform,
    bytes from splitmix64 seed 7, packed back to back), then the uneven batch."""
    import torch
    from paper_2104_08865_amd import hth
    from paper_2104_08865_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    width = 16
    seed = hth.expand_seed(7)
    tables = hth.tab_tables(8, width)

    # short keys
    lens = wl.short_key_lengths()
    offs, total = wl.pack(lens)
    count = lens.size
    log(f"[bench] compose: {count} keys, {total} bytes")
    data = wl.random_bytes_torch(7, total, dev)
    o = torch.from_numpy(offs.view(np.int64)).to(dev)
    n = torch.from_numpy(lens.view(np.int64)).to(dev)
    hth.reserve(count)
    z = torch.empty(count, dtype=torch.int64, device=dev)
    h = torch.empty((count, width), dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        hth.hash_batch64(seed, tables, data, o, n, width, out=z)
        hth.hash_batch(seed, data, o, n, width, out=h)
    wall = _timed_launches(hth, torch, lambda: hth.hash_batch64(seed, tables, data, o, n, width, out=z), args.steps)
    ms64 = _event_ms(torch, lambda: hth.hash_batch64(seed, tables, data, o, n, width, out=z), args.steps)
    ms16 = _event_ms(torch, lambda: hth.hash_batch(seed, data, o, n, width, out=h), args.steps)
    hth.batch_check()
    keys_per_s = count * args.steps / wall
    # algorithmic bytes of one call: offset, length and result of every key,
    # the bytes of the short keys, the HalftimeHash input of the longer ones
    # plus their 16-byte values written and read back
    long_ = lens > width
    algo = int(count * 24 + total + int(long_.sum()) * 2 * width)
    log(f"[bench] composed: {keys_per_s / 1e6:.0f} M keys/s ({ms64:.3f} ms per call); "
        f"HalftimeHash alone (16-byte values): {ms16:.3f} ms per call")
    zs = z.cpu().numpy().view(np.uint64)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ent = oracle.expand_seed(7)
        tab = oracle.tab_expand(8, width)
        m = 1 << 20
        sub = data[:int(offs[m - 1] + lens[m - 1])].cpu().numpy()
        ref, dt, core = pinned_oracle(lambda: oracle.hash64_batch(ent, tab, sub, offs[:m], lens[:m], width))
        cpu = {"value": m / dt, "unit": "keys/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {m} of the {count} keys, single thread pinned to core {core}",
               "seconds": dt, "cpu_model": cpu_model(), "host_cpus": len(os.sched_getaffinity(0)),
               "bit_exact_vs_gpu": bool((zs[:m] == ref).all())}
        log(f"[bench] cpu oracle: {m / dt / 1e6:.2f} M keys/s, exact={cpu['bit_exact_vs_gpu']}")
    del data, o, n, z, h
    torch.cuda.empty_cache()

    # the uneven batch, composed and as plain 16-byte values
    ulens = wl.uneven_lengths(3)
    uoffs, utotal = wl.pack(ulens)
    udata = wl.random_bytes_torch(3, utotal, dev)
    uo = torch.from_numpy(uoffs.view(np.int64)).to(dev)
    un = torch.from_numpy(ulens.view(np.int64)).to(dev)
    uz = torch.empty(ulens.size, dtype=torch.int64, device=dev)
    uh = torch.empty((ulens.size, width), dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        hth.hash_batch64(seed, tables, udata, uo, un, width, out=uz)
        hth.hash_batch(seed, udata, uo, un, width, out=uh)
    ums64 = _event_ms(torch, lambda: hth.hash_batch64(seed, tables, udata, uo, un, width, out=uz), args.steps)
    ums16 = _event_ms(torch, lambda: hth.hash_batch(seed, udata, uo, un, width, out=uh), args.steps)
    hth.batch_check()
    log(f"[bench] uneven batch composed: {utotal / ums64 / 1e6:.0f} GB/s; 16-byte values: {utotal / ums16 / 1e6:.0f} GB/s")
    del udata

    return {
        "metric": "composed 64-bit hash (HalftimeHash + simple tabulation) keys/s",
        "value": keys_per_s, "unit": "keys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "16,777,216 keys of 0..64 bytes (uniform lengths, splitmix64 seed 7), "
                               "inner width 16, tables from splitmix64 seed 8",
                   "keys": count, "key_bytes": total, "inner_width": width},
        "roofline": _roofline("whole hth_hash_batch64 call (planner, hashing, tail-only and tabulation kernels)",
                              algo, ms64),
        "plain_hash_batch_width16_ms": ms16,
        "uneven_batch": {"strings": int(ulens.size), "bytes": utotal, "composed_GBps": utotal / ums64 / 1e6,
                         "values16_GBps": utotal / ums16 / 1e6, "composed_ms": ums64, "values16_ms": ums16},
        "cpu_baseline": cpu,
    }


if __name__ == "__main__":
    run_main()
