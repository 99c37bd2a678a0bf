"""HalftimeHash CPU oracle (ctypes loader).

TEST INFRASTRUCTURE ONLY.  A plain, slow, single-threaded C reference of the
hash family, written from the paper's definitions (see hth_oracle.c for the
steps and the sections each follows).  It shares no code with the GPU library
in paper_2104_08865_amd/.  Only tests/, __graft_entry__.smoke() and the
benchmark's cpu_baseline leg may import it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hth_oracle.c")
LIB_PATH = os.path.join(_HERE, "libhth_ref.so")

_lib = None

WIDTHS = (16, 24, 32, 40)


def build():
    """Compile the oracle with the host C compiler (plain -O2, no SIMD flags)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", LIB_PATH + ".tmp", _SRC, "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.hth_ref_shape.argtypes = [ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
        L.hth_ref_tables.argtypes = [ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]
        L.hth_ref_layout.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, u64p]
        L.hth_ref_entropy_words.restype = ctypes.c_uint64
        L.hth_ref_entropy_offset.restype = ctypes.c_int64
        L.hth_ref_entropy_offset.argtypes = [ctypes.c_uint32]
        L.hth_ref_expand_seed.argtypes = [ctypes.c_uint64, u64p]
        L.hth_ref_nh.restype = ctypes.c_uint64
        L.hth_ref_nh.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64]
        L.hth_ref_nh_batch.argtypes = [ctypes.c_uint32, u64p, u64p, u64p, ctypes.c_size_t]
        L.hth_ref_gf8_mul.restype = ctypes.c_uint32
        L.hth_ref_gf8_mul.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.hth_ref_encode_batch.argtypes = [ctypes.c_uint32, ctypes.c_uint32, u64p, u64p, ctypes.c_size_t]
        L.hth_ref_ehc.argtypes = [ctypes.c_uint32, ctypes.c_uint32, u64p, u64p, u64p]
        L.hth_ref_hash_words.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                         u64p, u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_int, u64p]
        L.hth_ref_hash.argtypes = [u64p, ctypes.c_size_t, u8p, ctypes.c_uint64, ctypes.c_uint32, u8p]
        L.hth_ref_hash_batch.argtypes = [u64p, ctypes.c_size_t, u8p, u64p, u64p, ctypes.c_uint64,
                                         ctypes.c_uint32, u8p, ctypes.c_uint32]
        L.hth_ref_mul_counts.argtypes = [u64p]
        L.hth_ref_entropy_words_b.restype = ctypes.c_uint64
        L.hth_ref_entropy_words_b.argtypes = [ctypes.c_uint32]
        L.hth_ref_entropy_offset_b.restype = ctypes.c_int64
        L.hth_ref_entropy_offset_b.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.hth_ref_expand_seed_b.argtypes = [ctypes.c_uint64, ctypes.c_uint32, u64p]
        L.hth_ref_hash_b.argtypes = [u64p, ctypes.c_size_t, u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, u8p]
        L.hth_ref_hash_batch_b.argtypes = [u64p, ctypes.c_size_t, u8p, u64p, u64p, ctypes.c_uint64,
                                           ctypes.c_uint32, ctypes.c_uint32, u8p, ctypes.c_uint32]
        L.hth_ref_tab_words.restype = ctypes.c_size_t
        L.hth_ref_tab_words.argtypes = [ctypes.c_uint32]
        L.hth_ref_tab_expand.argtypes = [ctypes.c_uint64, ctypes.c_uint32, u64p]
        L.hth_ref_hash64_b.argtypes = [u64p, ctypes.c_size_t, u64p, ctypes.c_size_t, u8p, ctypes.c_uint64,
                                       ctypes.c_uint32, ctypes.c_uint32, u64p]
        L.hth_ref_hash64_batch_b.argtypes = [u64p, ctypes.c_size_t, u64p, ctypes.c_size_t, u8p, u64p, u64p,
                                             ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, u64p,
                                             ctypes.c_uint32]
        _lib = L
    return _lib


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _p8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def shape(width):
    """(d, e, k, w) of one output width."""
    out = (ctypes.c_uint32 * 4)()
    if lib().hth_ref_shape(width, out):
        raise ValueError(width)
    return tuple(out)


def tables(width):
    """(P, T): the oracle's GF(8) parity matrix ((k-1) x d) and combine matrix (k x e)."""
    d, e, k, w = shape(width)
    P = np.zeros((k - 1) * d, dtype=np.uint32)
    T = np.zeros(k * e, dtype=np.uint32)
    if lib().hth_ref_tables(width, P.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                            T.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))):
        raise ValueError(width)
    return P.reshape(k - 1, d), T.reshape(k, e)


def layout(width, b=8, f=8):
    """Offsets {ehc, tree, final, tail, len, total} of one width's entropy block."""
    out = np.zeros(6, dtype=np.uint64)
    if lib().hth_ref_layout(width, b, f, _p64(out)):
        raise ValueError(width)
    return [int(x) for x in out]


def entropy_words(b=8):
    """Entropy words of the standard layout for block size b (4 or 8)."""
    return int(lib().hth_ref_entropy_words_b(b))


def entropy_offset(width, b=8):
    return int(lib().hth_ref_entropy_offset_b(width, b))


def expand_seed(user_seed, b=8):
    out = np.zeros(entropy_words(b), dtype=np.uint64)
    lib().hth_ref_expand_seed_b(ctypes.c_uint64(user_seed & (2**64 - 1)), b, _p64(out))
    return out


def nh(W, x, s):
    x = _u64(x); s = _u64(s)
    out = np.zeros_like(x)
    lib().hth_ref_nh_batch(W, _p64(x), _p64(s), _p64(out), x.size)
    return out


def gf8_mul(a, b):
    return int(lib().hth_ref_gf8_mul(a, b))


def encode(width, X, W=32):
    """X: (n, d*w) words -> (n, e*w) encoded words."""
    d, e, k, w = shape(width)
    X = _u64(X).reshape(-1, d * w)
    Y = np.zeros((X.shape[0], e * w), dtype=np.uint64)
    if lib().hth_ref_encode_batch(width, W, _p64(X), _p64(Y), X.shape[0]):
        raise ValueError
    return Y


def ehc(width, X, S_ehc, W=32):
    d, e, k, w = shape(width)
    X = _u64(X); S = _u64(S_ehc)
    z = np.zeros(k, dtype=np.uint64)
    if lib().hth_ref_ehc(width, W, _p64(X), _p64(S), _p64(z)):
        raise ValueError
    return z


def hash_words(width, entropy_block, words, n_exec=None, len_value=None, W=32, b=8, f=8, recursive=False):
    """Generic (toy-parameter) hash over data words; returns k words."""
    d, e, k, w = shape(width)
    words = _u64(words)
    ent = _u64(entropy_block)
    if n_exec is None:
        n_exec = words.size // (b * d * w)
    if len_value is None:
        len_value = words.size
    out = np.zeros(k, dtype=np.uint64)
    wp = _p64(words) if words.size else ctypes.POINTER(ctypes.c_uint64)()
    rc = lib().hth_ref_hash_words(width, W, b, f, _p64(ent), wp, words.size, n_exec,
                                  len_value & (2**64 - 1), int(recursive), _p64(out))
    if rc:
        raise ValueError("hth_ref_hash_words rejected its arguments")
    return out


def hash_bytes(entropy, data, width, b=8):
    """The real family (block size b) on one byte string; returns width bytes."""
    ent = _u64(entropy)
    data = np.ascontiguousarray(np.frombuffer(bytes(data), dtype=np.uint8) if isinstance(data, (bytes, bytearray)) else data, dtype=np.uint8)
    out = np.zeros(width, dtype=np.uint8)
    dp = _p8(data) if data.size else ctypes.POINTER(ctypes.c_uint8)()
    if lib().hth_ref_hash_b(_p64(ent), ent.size, dp, data.size, width, b, _p8(out)):
        raise ValueError("hth_ref_hash rejected its arguments")
    return out


def hash_batch(entropy, data, offsets, lengths, width, nthreads=1, b=8):
    """Many strings of one buffer (block size b); returns (count, width) uint8."""
    ent = _u64(entropy)
    data = np.ascontiguousarray(data, dtype=np.uint8)
    offsets = _u64(offsets); lengths = _u64(lengths)
    count = offsets.size
    out = np.zeros((count, width), dtype=np.uint8)
    if count:
        assert int((offsets + lengths).max()) <= data.size
    dp = _p8(data) if data.size else ctypes.POINTER(ctypes.c_uint8)()
    if lib().hth_ref_hash_batch_b(_p64(ent), ent.size, dp, _p64(offsets), _p64(lengths), count,
                                  width, b, _p8(out), nthreads):
        raise ValueError("hth_ref_hash_batch rejected its arguments")
    return out


def mul_counts():
    out = np.zeros(5, dtype=np.uint64)
    lib().hth_ref_mul_counts(_p64(out))
    return dict(zip(("ehc", "tree", "final", "tail", "length"), (int(x) for x in out)))


def tab_words(width):
    """Words of the tabulation tables for inner width c: (c + 1) * 256."""
    n = int(lib().hth_ref_tab_words(width))
    if not n:
        raise ValueError(width)
    return n


def tab_expand(user_seed, width):
    """Tabulation tables from splitmix64 started at user_seed, shape (c + 1, 256)."""
    out = np.zeros(tab_words(width), dtype=np.uint64)
    if lib().hth_ref_tab_expand(ctypes.c_uint64(user_seed & (2**64 - 1)), width, _p64(out)):
        raise ValueError(width)
    return out.reshape(width + 1, 256)


def hash64(entropy, tables, data, width, b=8):
    """The composed 64-bit hash of one byte string (simple tabulation of the
    string itself when it has at most `width` bytes, else of its HalftimeHash
    value); returns an int."""
    ent = _u64(entropy)
    tab = _u64(tables).ravel()
    data = np.ascontiguousarray(np.frombuffer(bytes(data), dtype=np.uint8) if isinstance(data, (bytes, bytearray)) else data, dtype=np.uint8)
    out = np.zeros(1, dtype=np.uint64)
    dp = _p8(data) if data.size else ctypes.POINTER(ctypes.c_uint8)()
    if lib().hth_ref_hash64_b(_p64(ent), ent.size, _p64(tab), tab.size, dp, data.size, width, b, _p64(out)):
        raise ValueError("hth_ref_hash64 rejected its arguments")
    return int(out[0])


def hash64_batch(entropy, tables, data, offsets, lengths, width, nthreads=1, b=8):
    """The composed 64-bit hash of many strings of one buffer; returns (count,) uint64."""
    ent = _u64(entropy)
    tab = _u64(tables).ravel()
    data = np.ascontiguousarray(data, dtype=np.uint8)
    offsets = _u64(offsets); lengths = _u64(lengths)
    count = offsets.size
    out = np.zeros(count, dtype=np.uint64)
    if count:
        assert int((offsets + lengths).max()) <= data.size
    dp = _p8(data) if data.size else ctypes.POINTER(ctypes.c_uint8)()
    if lib().hth_ref_hash64_batch_b(_p64(ent), ent.size, _p64(tab), tab.size, dp, _p64(offsets), _p64(lengths),
                                    count, width, b, _p64(out), nthreads):
        raise ValueError("hth_ref_hash64_batch rejected its arguments")
    return out
