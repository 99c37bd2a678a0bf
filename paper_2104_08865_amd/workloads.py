"""Seeded synthetic inputs for the hash workloads.

This module holds input generators only and none of the hash arithmetic: the
tests, the benchmark and the oracle-side checks all draw their bytes, string
lengths and arrival times from here, so both sides of every comparison see the
same inputs.

Randomness is splitmix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): output i of a stream started at
state s is mix(s + (i + 1) * GAMMA).  It is counter based, so any slice of a
stream can be generated independently, on the CPU (numpy) or on the GPU
(torch), with identical results.

Byte buffers: byte i of a buffer made from seed s is byte (i mod 8), little
endian, of output floor(i / 8) of the stream started at s.  Lengths, arrival
gaps and output widths come from separate streams seeded s + 1000, s + 2000
and s + 3000.  A uniform variate is the top 53 bits of an output over 2^53.

The workloads mirror the paper's setting: long uniformly random strings (the
paper measures on 250 KB to 256 KiB random strings and on long strings), plus
uneven batches and request streams for the batched and served forms.
"""
import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
_M64 = (1 << 64) - 1


def _mix_np(z):
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= np.uint64(MIX1)
    z ^= z >> np.uint64(27)
    z *= np.uint64(MIX2)
    z ^= z >> np.uint64(31)
    return z


def splitmix64(seed, n, start=0):
    """Outputs start .. start+n-1 of the stream started at `seed` (numpy uint64)."""
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & _M64) + idx * np.uint64(GAMMA)
        return _mix_np(state)


def random_bytes(seed, nbytes, start_byte=0):
    """Bytes [start_byte, start_byte + nbytes) of the buffer made from `seed`
    (numpy uint8, CPU)."""
    if nbytes == 0:
        return np.zeros(0, dtype=np.uint8)
    w0 = start_byte // 8
    w1 = (start_byte + nbytes + 7) // 8
    raw = np.empty((w1 - w0) * 8, dtype=np.uint8)
    step = 1 << 22
    for a in range(w0, w1, step):
        n = min(step, w1 - a)
        raw[(a - w0) * 8:(a - w0 + n) * 8] = splitmix64(seed, n, start=a).astype("<u8").view(np.uint8)
    off = start_byte - 8 * w0
    return raw[off:off + nbytes]


def _signed(c):
    return c - (1 << 64) if c >= (1 << 63) else c


def random_bytes_torch(seed, nbytes, device, chunk_words=1 << 26):
    """The same buffer as random_bytes(seed, nbytes), built with torch int64
    arithmetic on `device` (wrapping 64-bit products; logical right shifts are
    done as arithmetic shifts followed by a mask)."""
    import torch

    nwords = (nbytes + 7) // 8
    out = torch.empty(nwords * 8, dtype=torch.uint8, device=device)
    out64 = out.view(torch.int64)
    g = _signed(GAMMA)
    m1 = _signed(MIX1)
    m2 = _signed(MIX2)
    s = _signed(seed & _M64)

    def lsr(z, r):
        return (z >> r) & ((1 << (64 - r)) - 1)

    for w0 in range(0, nwords, chunk_words):
        n = min(chunk_words, nwords - w0)
        z = torch.arange(w0 + 1, w0 + n + 1, dtype=torch.int64, device=device)
        z.mul_(g).add_(s)
        z.bitwise_xor_(lsr(z, 30)).mul_(m1)
        z.bitwise_xor_(lsr(z, 27)).mul_(m2)
        z.bitwise_xor_(lsr(z, 31))
        out64[w0:w0 + n] = z
        del z
    return out[:nbytes]


def uniform01(seed, n, start=0):
    """n uniform variates in [0, 1): top 53 bits over 2^53."""
    return (splitmix64(seed, n, start) >> np.uint64(11)).astype(np.float64) / float(1 << 53)


# ---------------------------------------------------------------------------
# Workload shapes.
# ---------------------------------------------------------------------------

def execution_bytes(width):
    """Bytes of one full EHC execution of a width (b = 8 blocks of 8 bytes,
    d items of w = 3 blocks each).  Used only to place boundary lengths."""
    d = {16: 6, 24: 7, 32: 7, 40: 5}[width]
    return 64 * d * 3


def small_batch_lengths(width=16):
    """The small parity case: 1024 strings of 1 KiB, then the lengths
    0, 1, 7, 8, 63, 64, then 1, 8, 64 and 512 executions of `width`, each
    minus one, exact and plus one byte."""
    xb = execution_bytes(width)
    lens = [1024] * 1024 + [0, 1, 7, 8, 63, 64]
    for n in (1, 8, 64, 512):
        lens += [n * xb - 1, n * xb, n * xb + 1]
    return np.array(lens, dtype=np.uint64)


def uneven_lengths(seed=3, n=200_000, lo=16, hi=262_144, extra_upto=520):
    """Log-uniform lengths in [lo, hi) (floor of exp(ln lo + u ln(hi/lo))),
    followed by every length 0 .. extra_upto once."""
    u = uniform01(seed + 1000, n)
    lens = np.floor(np.exp(math.log(lo) + u * math.log(hi / lo))).astype(np.uint64)
    lens = np.minimum(lens, np.uint64(hi - 1))
    return np.concatenate([lens, np.arange(extra_upto + 1, dtype=np.uint64)])


def lognormal_lengths(seed=5, n=100_000, median=4096, sigma=2.0, cap=16 << 20):
    """Lognormal lengths (Box-Muller normal from two uniforms), median
    `median`, log-sd `sigma`, clamped to [1, cap]."""
    u1 = uniform01(seed + 1000, n, start=0)
    u2 = uniform01(seed + 1000, n, start=n)
    z = np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * math.pi * u2)
    lens = np.floor(np.exp(math.log(median) + sigma * z))
    return np.clip(lens, 1, cap).astype(np.uint64)


def short_key_lengths(seed=7, n=1 << 24, hi=64):
    """Hash-table keys: lengths uniform over 0 .. hi bytes."""
    u = uniform01(seed + 4000, n)
    return np.minimum((u * (hi + 1)).astype(np.uint64), np.uint64(hi))


def poisson_gaps(seed, n, rate):
    """Exponential inter-arrival gaps (seconds) for `rate` arrivals per second."""
    u = uniform01(seed + 2000, n)
    return -np.log(1.0 - u) / rate


def coin_widths(seed, n, choices=(16, 40)):
    """Output widths drawn uniformly from `choices`."""
    u = uniform01(seed + 3000, n)
    idx = np.minimum((u * len(choices)).astype(np.int64), len(choices) - 1)
    return np.array(choices, dtype=np.uint32)[idx]


def pack(lengths):
    """Back-to-back offsets of strings with these lengths, and the total."""
    lengths = np.asarray(lengths, dtype=np.uint64)
    offsets = np.zeros(lengths.size, dtype=np.uint64)
    if lengths.size > 1:
        offsets[1:] = np.cumsum(lengths[:-1], dtype=np.uint64)
    total = int(lengths.sum()) if lengths.size else 0
    return offsets, total
