"""The C ABI library loads, exports every symbol include/hth.h declares, and
rejects bad host-side arguments before touching the GPU.  No compute calls."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hth.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hth_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2104_08865_amd import hth
    if not os.path.exists(hth.LIB_PATH):
        from paper_2104_08865_amd import build
        build.build()
    return hth.lib()


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("hth_expand_seed", "hth_hash_batch", "hth_seed_free", "hth_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2104_08865_amd import hth
    out = subprocess.run(["nm", "-D", "--defined-only", hth.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (hth_[a-z0-9_]+)\b", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    assert set(hth.SYMBOLS) <= exported


def test_entropy_words(lib):
    assert lib.hth_entropy_words() == 2688 + 3980 + 5245 + 6456


def test_host_side_rejections(lib):
    from paper_2104_08865_amd import hth
    p = ctypes.c_void_p(1)
    rc = lib.hth_hash_batch(p, p, p, p, 1, p, 17, None)
    assert rc == hth.HTH_E_INVALID and b"out_width" in lib.hth_last_error()
    rc = lib.hth_hash_batch(None, p, p, p, 1, p, 16, None)
    assert rc == hth.HTH_E_INVALID and b"seed" in lib.hth_last_error()
    assert lib.hth_set_tuning(20, 0, 0, 5) == hth.HTH_E_INVALID
    assert lib.hth_set_tuning(16, 0, 0, 9) == hth.HTH_E_INVALID
    assert lib.hth_set_tuning(16, 0, 3, 2) == hth.HTH_E_INVALID
    h = ctypes.c_void_p()
    assert lib.hth_seed_from_entropy(None, 18369, ctypes.byref(h), None) == hth.HTH_E_INVALID
    assert lib.hth_expand_seed(1, None, None) == hth.HTH_E_INVALID
    assert lib.hth_seed_free(None) == hth.HTH_OK


def test_gpu_path_does_not_touch_the_oracle():
    """The product package never imports, links or loads the oracle, and the
    oracle never includes the product's sources."""
    pkg = os.path.join(ROOT, "paper_2104_08865_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b|hth_ref_|libhth_ref|hth_oracle", text, re.M), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".h", ".py")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert not re.search(r'^\s*(import|from)\s+paper_2104_08865_amd|^\s*#\s*include\s*[<"][^>"]*(hth_family|hth_kernels|hth\.h)',
                                 text, re.M), f


def test_serve_config_rejections(lib):
    """hth_serve_create validates its limits before any device allocation."""
    from paper_2104_08865_amd import hth
    h = ctypes.c_void_p()
    seed = ctypes.c_void_p(1)  # never dereferenced: every case fails first
    assert lib.hth_serve_create(None, seed, ctypes.byref(h)) == hth.HTH_E_INVALID
    assert lib.hth_serve_create(ctypes.byref(hth.ServeConfig()), seed, None) == hth.HTH_E_INVALID
    cases = [
        (dict(max_device_bytes=1 << 20, max_request_bytes=2 << 20), b"max_request_bytes"),
        (dict(host_stage_bytes=1 << 20), b"max_request_bytes"),  # default 16 MiB requests
        (dict(slots=9), b"slots"),
        (dict(max_batch_bytes=(1 << 36) + 1), b"max_batch_bytes"),
        (dict(max_batch_requests=(1 << 22) + 1), b"max_batch_requests"),
        (dict(max_outstanding=(1 << 24) + 1), b"max_outstanding"),
    ]
    for cfg, word in cases:
        rc = lib.hth_serve_create(ctypes.byref(hth.ServeConfig(**cfg)), seed, ctypes.byref(h))
        assert rc == hth.HTH_E_INVALID and word in lib.hth_last_error(), cfg
    rc = lib.hth_serve_create(ctypes.byref(hth.ServeConfig()), None, ctypes.byref(h))
    assert rc == hth.HTH_E_INVALID and b"seed" in lib.hth_last_error()
    t = ctypes.c_uint64()
    assert lib.hth_serve_submit(None, None, 0, 16, ctypes.byref(t)) == hth.HTH_E_INVALID
    assert lib.hth_serve_destroy(None) == hth.HTH_OK


def test_block_size_entry_points(lib):
    """The 256-bit block family's sizes and argument checks (no device use)."""
    from paper_2104_08865_amd import hth
    assert lib.hth_entropy_words_b(8) == lib.hth_entropy_words()
    # per width [e*w][k*140][k*140*4][4*d*w + k - 1][k], widths 16, 24, 32, 40
    shapes = {16: (6, 7, 2), 24: (7, 9, 3), 32: (7, 10, 4), 40: (5, 9, 5)}
    assert lib.hth_entropy_words_b(4) == sum(e * 3 + k * 140 * 5 + 4 * d * 3 + k - 1 + k
                                             for d, e, k in shapes.values())
    assert lib.hth_entropy_words_b(5) == 0
    h = ctypes.c_void_p()
    assert lib.hth_expand_seed_b(1, 5, ctypes.byref(h), None) == hth.HTH_E_INVALID
    words = (ctypes.c_uint64 * 10229)()
    assert lib.hth_seed_from_entropy_b(words, 10229, 8, ctypes.byref(h), None) == hth.HTH_E_INVALID
    assert lib.hth_seed_from_entropy_b(words, 10229, 3, ctypes.byref(h), None) == hth.HTH_E_INVALID
    assert lib.hth_seed_block_words(None) == 0


def test_stream_argument_checks(lib):
    """hth_stream_* reject bad arguments before any device use."""
    from paper_2104_08865_amd import hth
    h = ctypes.c_void_p()
    assert lib.hth_stream_create(None, 24, ctypes.byref(h)) == hth.HTH_E_INVALID
    assert lib.hth_stream_create(ctypes.c_void_p(1), 24, None) == hth.HTH_E_INVALID
    assert lib.hth_stream_update(None, None, 0, None) == hth.HTH_E_INVALID
    assert lib.hth_stream_final(None, None, None) == hth.HTH_E_INVALID
    n = ctypes.c_size_t()
    assert lib.hth_stream_save(None, None, ctypes.byref(n), None) == hth.HTH_E_INVALID
    assert lib.hth_stream_length(None) == 0
    assert lib.hth_stream_free(None) == hth.HTH_OK


def test_composition_entry_points(lib, oracle_lib):
    """hth_tab_words / hth_tab_expand on the host (the tables equal the
    oracle's splitmix64 expansion) and hth_hash_batch64's host-side checks."""
    import numpy as np
    from paper_2104_08865_amd import hth
    for w in (16, 24, 32, 40):
        assert lib.hth_tab_words(w) == (w + 1) * 256
        t = np.zeros((w + 1) * 256, dtype=np.uint64)
        assert lib.hth_tab_expand(3, w, ctypes.c_void_p(t.ctypes.data), t.size) == hth.HTH_OK
        assert (t == oracle_lib.tab_expand(3, w).ravel()).all()
        assert lib.hth_tab_expand(3, w, ctypes.c_void_p(t.ctypes.data), t.size - 1) == hth.HTH_E_INVALID
    assert lib.hth_tab_words(20) == 0
    assert lib.hth_tab_expand(3, 20, None, 0) == hth.HTH_E_INVALID
    assert lib.hth_tab_expand(3, 16, None, 17 * 256) == hth.HTH_E_INVALID
    p, q = ctypes.c_void_p(8), ctypes.c_void_p(12)
    assert lib.hth_hash_batch64(p, None, p, p, p, 1, p, 16, None) == hth.HTH_E_INVALID
    assert b"tables" in lib.hth_last_error()
    assert lib.hth_hash_batch64(p, q, p, p, p, 1, p, 16, None) == hth.HTH_E_INVALID
    assert lib.hth_hash_batch64(p, p, p, p, p, 1, q, 16, None) == hth.HTH_E_INVALID
    assert b"aligned" in lib.hth_last_error()
    assert lib.hth_hash_batch64(p, p, p, p, p, 1, p, 20, None) == hth.HTH_E_INVALID
    assert lib.hth_hash_batch64(None, p, p, p, p, 1, p, 16, None) == hth.HTH_E_INVALID
    assert lib.hth_hash_batch64(p, None, None, None, None, 0, None, 16, None) == hth.HTH_OK
