"""Python binding of libhth (argument marshalling only).

Every step of the hash runs in the HIP kernels of libhth.so; this module
only loads the library, converts torch tensors to pointers and passes the
current torch stream.  It raises if the library has not been built (there is
no fallback path).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhth.so")

HTH_OK = 0
HTH_E_INVALID = -1
HTH_E_OOM = -2
HTH_E_HIP = -3
HTH_E_BUSY = -4
HTH_E_TOO_LARGE = -5

WIDTHS = (16, 24, 32, 40)

# Exported symbols declared in include/hth.h (checked by the CPU test suite).
SYMBOLS = (
    "hth_last_error", "hth_entropy_words", "hth_expand_seed", "hth_seed_from_entropy",
    "hth_seed_entropy", "hth_seed_free", "hth_hash_batch", "hth_hash_batch_timed", "hth_reserve",
    "hth_batch_check", "hth_set_tuning", "hth_batch_graph_create", "hth_batch_graph_launch",
    "hth_batch_graph_check", "hth_batch_graph_free", "hth_serve_create", "hth_serve_submit",
    "hth_serve_poll", "hth_serve_wait", "hth_serve_wait_many", "hth_serve_replay", "hth_serve_stats",
    "hth_serve_reset_stats", "hth_serve_destroy", "hth_serve_pause", "hth_read_probe", "hth_entropy_words_b",
    "hth_expand_seed_b", "hth_seed_from_entropy_b", "hth_seed_block_words", "hth_stream_create",
    "hth_stream_update", "hth_stream_final", "hth_stream_reset", "hth_stream_save", "hth_stream_load",
    "hth_stream_length", "hth_stream_free", "hth_tab_words", "hth_tab_expand", "hth_hash_batch64",
    "hth_hash_batch_noalloc", "hth_serve_submit_pinned", "hth_serve_replay_pinned", "hth_stream_update_gather",
)


def _require_pinned(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.device.type == "cpu" and t.dtype == torch.uint8 and t.is_contiguous()
            and (t.numel() == 0 or t.is_pinned())):
        raise ValueError("expected a contiguous pinned CPU uint8 torch tensor")


def pinned_bytes(data):
    """A pinned CPU uint8 torch tensor holding a copy of `data` (a uint8 numpy
    array or bytes), for Server.submit_pinned and Server.replay(pinned=True)."""
    import torch
    src = np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray)) else np.asarray(data, np.uint8)
    t = torch.empty(src.size, dtype=torch.uint8, pin_memory=True)
    if src.size:
        t.numpy()[:] = src
    return t


class ServeConfig(ctypes.Structure):
    """hth_serve_config (zero fields take the library's defaults)."""
    _fields_ = [("max_device_bytes", ctypes.c_uint64), ("host_stage_bytes", ctypes.c_uint64),
                ("max_request_bytes", ctypes.c_uint64), ("max_batch_bytes", ctypes.c_uint64),
                ("max_batch_requests", ctypes.c_uint32), ("slots", ctypes.c_uint32),
                ("max_outstanding", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ServeReport(ctypes.Structure):
    """hth_serve_report."""
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("deferred", ctypes.c_uint64),
                ("busy", ctypes.c_uint64), ("batches", ctypes.c_uint64), ("bytes", ctypes.c_uint64),
                ("elapsed_s", ctypes.c_double), ("gbps", ctypes.c_double), ("latency_p50_us", ctypes.c_double),
                ("latency_p99_us", ctypes.c_double), ("latency_max_us", ctypes.c_double),
                ("latency_mean_us", ctypes.c_double), ("mean_batch_requests", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}

_lib = None


class HthError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"libhth error {status}: {message}")
        self.status = status


def lib():
    """Load libhth.so (built by paper_2104_08865_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2104_08865_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        u64 = ctypes.c_uint64
        u32 = ctypes.c_uint32
        L.hth_last_error.restype = ctypes.c_char_p
        L.hth_entropy_words.restype = ctypes.c_size_t
        L.hth_expand_seed.argtypes = [u64, ctypes.POINTER(vp), vp]
        L.hth_seed_from_entropy.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(vp), vp]
        L.hth_seed_entropy.argtypes = [vp, vp, ctypes.c_size_t]
        L.hth_seed_free.argtypes = [vp]
        L.hth_hash_batch.argtypes = [vp, vp, vp, vp, u64, vp, u32, vp]
        L.hth_hash_batch_timed.argtypes = [vp, vp, vp, vp, u64, vp, u32, vp, vp, vp]
        L.hth_hash_batch_noalloc.argtypes = [vp, vp, vp, vp, u64, vp, u32, vp]
        L.hth_reserve.argtypes = [u64, vp]
        L.hth_batch_check.argtypes = [vp]
        L.hth_set_tuning.argtypes = [u32, u32, u32, u32]
        L.hth_batch_graph_create.argtypes = [vp, vp, vp, vp, u64, vp, u32, ctypes.POINTER(vp)]
        L.hth_batch_graph_launch.argtypes = [vp, vp]
        L.hth_batch_graph_check.argtypes = [vp, vp]
        L.hth_batch_graph_free.argtypes = [vp]
        L.hth_serve_create.argtypes = [ctypes.POINTER(ServeConfig), vp, ctypes.POINTER(vp)]
        L.hth_serve_submit.argtypes = [vp, vp, u64, u32, ctypes.POINTER(u64)]
        L.hth_serve_poll.argtypes = [vp, u64, vp]
        L.hth_serve_wait.argtypes = [vp, u64, vp]
        L.hth_serve_wait_many.argtypes = [vp, vp, u64, vp, u32]
        L.hth_serve_replay.argtypes = [vp, vp, vp, vp, vp, vp, u64, u32, vp]
        L.hth_serve_submit_pinned.argtypes = [vp, vp, u64, u32, ctypes.POINTER(u64)]
        L.hth_serve_replay_pinned.argtypes = [vp, vp, vp, vp, vp, vp, u64, u32, vp]
        L.hth_serve_stats.argtypes = [vp, ctypes.POINTER(ServeReport)]
        L.hth_serve_reset_stats.argtypes = [vp]
        L.hth_serve_destroy.argtypes = [vp]
        L.hth_serve_pause.argtypes = [vp, ctypes.c_int32]
        L.hth_read_probe.argtypes = [vp, u64, vp, u32, vp]
        L.hth_entropy_words_b.argtypes = [u32]
        L.hth_expand_seed_b.argtypes = [u64, u32, ctypes.POINTER(vp), vp]
        L.hth_seed_from_entropy_b.argtypes = [vp, ctypes.c_size_t, u32, ctypes.POINTER(vp), vp]
        L.hth_seed_block_words.argtypes = [vp]
        L.hth_stream_create.argtypes = [vp, u32, ctypes.POINTER(vp)]
        L.hth_stream_update.argtypes = [vp, vp, u64, vp]
        L.hth_stream_update_gather.argtypes = [vp, vp, vp, ctypes.c_uint32, vp]
        L.hth_stream_final.argtypes = [vp, vp, vp]
        L.hth_stream_reset.argtypes = [vp, vp]
        L.hth_stream_save.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t), vp]
        L.hth_stream_load.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.hth_stream_length.argtypes = [vp]
        L.hth_stream_free.argtypes = [vp]
        L.hth_tab_words.argtypes = [u32]
        L.hth_tab_expand.argtypes = [u64, u32, vp, ctypes.c_size_t]
        L.hth_hash_batch64.argtypes = [vp, vp, vp, vp, vp, u64, vp, u32, vp]
        for name in SYMBOLS[2:]:
            getattr(L, name).restype = ctypes.c_int32
        L.hth_entropy_words_b.restype = ctypes.c_size_t
        L.hth_seed_block_words.restype = ctypes.c_uint32
        L.hth_stream_length.restype = ctypes.c_uint64
        L.hth_tab_words.restype = ctypes.c_size_t
        for name in ("hth_expand_seed", "hth_seed_from_entropy", "hth_seed_entropy", "hth_seed_free",
                     "hth_hash_batch", "hth_hash_batch_timed", "hth_reserve", "hth_batch_check", "hth_set_tuning",
                     "hth_batch_graph_create", "hth_batch_graph_launch", "hth_batch_graph_check",
                     "hth_batch_graph_free"):
            getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(rc):
    if rc != HTH_OK:
        raise HthError(rc, lib().hth_last_error().decode(errors="replace"))


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def entropy_words(block_words=8):
    """Entropy words of a seed of the family with `block_words` (8 or 4)."""
    return int(lib().hth_entropy_words_b(block_words))


class Seed:
    """A device-resident seed (the family member's entropy words)."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    @property
    def block_words(self):
        return int(lib().hth_seed_block_words(self._h))

    def entropy(self):
        out = np.zeros(entropy_words(self.block_words), dtype=np.uint64)
        _check(lib().hth_seed_entropy(self._h, out.ctypes.data, out.size))
        return out

    def free(self):
        if self._h is not None and _lib is not None:
            lib().hth_seed_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def expand_seed(user_seed, stream=None, block_words=8):
    """splitmix64 expansion of a user seed into the family with
    `block_words` words per block (8, the default, or 4)."""
    h = ctypes.c_void_p()
    _check(lib().hth_expand_seed_b(ctypes.c_uint64(user_seed & (2**64 - 1)), block_words, ctypes.byref(h),
                                   _stream(stream)))
    return Seed(h)


def seed_from_entropy(words, stream=None, block_words=8):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    h = ctypes.c_void_p()
    _check(lib().hth_seed_from_entropy_b(w.ctypes.data, w.size, block_words, ctypes.byref(h), _stream(stream)))
    # the upload reads host memory owned by the library; nothing to keep here
    return Seed(h)


def reserve(max_count, stream=None):
    _check(lib().hth_reserve(max_count, _stream(stream)))


def set_tuning(out_width, waves_per_cu=0, min_task_level=0, max_task_level=5):
    """Grid size and task-size range of the batched kernel for one width."""
    _check(lib().hth_set_tuning(out_width, waves_per_cu, min_task_level, max_task_level))


def batch_check(stream=None):
    _check(lib().hth_batch_check(_stream(stream)))


class Timer:
    """A pair of HIP events (via the HIP runtime) around the hashing kernels
    (or any enqueued work, with record_start / record_stop)."""

    _hip = None

    def __init__(self):
        if Timer._hip is None:
            Timer._hip = ctypes.CDLL("libamdhip64.so")
            Timer._hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
            Timer._hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
            Timer._hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
            Timer._hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
            Timer._hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.start = ctypes.c_void_p()
        self.stop = ctypes.c_void_p()
        if Timer._hip.hipEventCreate(ctypes.byref(self.start)) or Timer._hip.hipEventCreate(ctypes.byref(self.stop)):
            raise RuntimeError("hipEventCreate failed")

    def record_start(self, stream=None):
        if Timer._hip.hipEventRecord(self.start, _stream(stream)):
            raise RuntimeError("hipEventRecord failed")

    def record_stop(self, stream=None):
        if Timer._hip.hipEventRecord(self.stop, _stream(stream)):
            raise RuntimeError("hipEventRecord failed")

    def elapsed_ms(self):
        ms = ctypes.c_float()
        if Timer._hip.hipEventSynchronize(self.stop) or Timer._hip.hipEventElapsedTime(ctypes.byref(ms), self.start, self.stop):
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def __del__(self):
        try:
            Timer._hip.hipEventDestroy(self.start)
            Timer._hip.hipEventDestroy(self.stop)
        except Exception:
            pass


def hash_batch_noalloc(seed, data, offsets, lengths, out_width, out, stream=None):
    """hash_batch through hth_hash_batch_noalloc: the library allocates
    nothing (its scratch is a static device array of the GPU); `out` must be
    a preallocated (count, out_width) uint8 CUDA tensor."""
    import torch
    if data.dtype != torch.uint8 or not data.is_cuda:
        raise TypeError("data must be a uint8 CUDA tensor")
    for t in (offsets, lengths):
        if t.dtype not in (torch.int64, torch.uint64) or not t.is_cuda or not t.is_contiguous():
            raise TypeError("offsets and lengths must be contiguous int64 CUDA tensors")
    count = offsets.numel()
    if lengths.numel() != count:
        raise ValueError("offsets and lengths differ in size")
    if out.dtype != torch.uint8 or not out.is_cuda or not out.is_contiguous() or out.numel() < count * out_width:
        raise TypeError("out must be a contiguous uint8 CUDA tensor of count * out_width bytes")
    dp = data.data_ptr() if data.numel() else offsets.data_ptr()
    _check(lib().hth_hash_batch_noalloc(seed.handle, ctypes.c_void_p(dp), ctypes.c_void_p(offsets.data_ptr()),
                                        ctypes.c_void_p(lengths.data_ptr()), count, ctypes.c_void_p(out.data_ptr()),
                                        out_width, _stream(stream)))
    return out


def hash_batch(seed, data, offsets, lengths, out_width, out=None, stream=None, timer=None):
    """Hash strings data[offsets[i] : offsets[i] + lengths[i]] on the GPU.

    data: uint8 CUDA tensor; offsets, lengths: int64 CUDA tensors (read as
    unsigned); returns (count, out_width) uint8 CUDA tensor."""
    import torch
    if data.dtype != torch.uint8 or not data.is_cuda:
        raise TypeError("data must be a uint8 CUDA tensor")
    for t in (offsets, lengths):
        if t.dtype not in (torch.int64, torch.uint64) or not t.is_cuda or not t.is_contiguous():
            raise TypeError("offsets and lengths must be contiguous int64 CUDA tensors")
    count = offsets.numel()
    if lengths.numel() != count:
        raise ValueError("offsets and lengths differ in size")
    if out is None:
        out = torch.empty((count, out_width), dtype=torch.uint8, device=data.device)
    dp = data.data_ptr() if data.numel() else offsets.data_ptr()
    args = (seed.handle, ctypes.c_void_p(dp), ctypes.c_void_p(offsets.data_ptr()),
            ctypes.c_void_p(lengths.data_ptr()), count, ctypes.c_void_p(out.data_ptr()), out_width, _stream(stream))
    if timer is None:
        _check(lib().hth_hash_batch(*args))
    else:
        _check(lib().hth_hash_batch_timed(*args, timer.start, timer.stop))
    return out


def tab_words(inner_width):
    """Words of the tabulation tables of the composed 64-bit hash: (c + 1) * 256."""
    n = int(lib().hth_tab_words(inner_width))
    if not n:
        raise HthError(HTH_E_INVALID, f"inner width {inner_width} is not 16/24/32/40")
    return n


def tab_tables(user_seed, inner_width, device="cuda"):
    """Tabulation tables from splitmix64 started at user_seed (pick one
    independent of the hashing seed's), as an int64 tensor on `device`."""
    import torch
    host = np.zeros(tab_words(inner_width), dtype=np.uint64)
    _check(lib().hth_tab_expand(ctypes.c_uint64(user_seed & (2**64 - 1)), inner_width,
                                ctypes.c_void_p(host.ctypes.data), host.size))
    return torch.from_numpy(host.view(np.int64)).to(device)


def hash_batch64(seed, tables, data, offsets, lengths, inner_width, out=None, stream=None):
    """The composed 64-bit hash of data[offsets[i] : offsets[i] + lengths[i]]:
    simple tabulation of the string itself when it has at most inner_width
    bytes, else of its HalftimeHash value of that width.  tables: int64 CUDA
    tensor from tab_tables; returns an int64 CUDA tensor of count values
    (read the bits as unsigned)."""
    import torch
    if data.dtype != torch.uint8 or not data.is_cuda:
        raise TypeError("data must be a uint8 CUDA tensor")
    for t in (offsets, lengths, tables):
        if t.dtype not in (torch.int64, torch.uint64) or not t.is_cuda or not t.is_contiguous():
            raise TypeError("offsets, lengths and tables must be contiguous int64 CUDA tensors")
    if tables.numel() != tab_words(inner_width):
        raise ValueError(f"tables hold {tables.numel()} words, width {inner_width} needs {tab_words(inner_width)}")
    count = offsets.numel()
    if lengths.numel() != count:
        raise ValueError("offsets and lengths differ in size")
    if out is None:
        out = torch.empty(count, dtype=torch.int64, device=data.device)
    dp = data.data_ptr() if data.numel() else offsets.data_ptr()
    _check(lib().hth_hash_batch64(seed.handle, ctypes.c_void_p(tables.data_ptr()), ctypes.c_void_p(dp),
                                  ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(lengths.data_ptr()), count,
                                  ctypes.c_void_p(out.data_ptr()), inner_width, _stream(stream)))
    return out


def read_probe(data, sink_words=2048, stream=None, timer=None):
    """Stream-read a 16-byte aligned uint8 CUDA tensor once (the device's
    achievable HBM read rate); returns the sink tensor."""
    import torch
    sink = torch.zeros(sink_words, dtype=torch.int64, device=data.device)
    if timer is not None:
        timer.record_start(stream)
    _check(lib().hth_read_probe(ctypes.c_void_p(data.data_ptr()), data.numel(), ctypes.c_void_p(sink.data_ptr()),
                                sink_words, _stream(stream)))
    if timer is not None:
        timer.record_stop(stream)
    return sink


class BatchGraph:
    """A captured hth_hash_batch (planner + hashing kernel) for repeated launches.

    The tensors passed here must stay alive (and keep their storage) as long
    as the graph is used; their contents may change between launches."""

    def __init__(self, seed, data, offsets, lengths, out_width, out=None):
        import torch
        count = offsets.numel()
        if out is None:
            out = torch.empty((count, out_width), dtype=torch.uint8, device=data.device)
        self.out = out
        self._keep = (seed, data, offsets, lengths)
        h = ctypes.c_void_p()
        dp = data.data_ptr() if data.numel() else offsets.data_ptr()
        _check(lib().hth_batch_graph_create(seed.handle, ctypes.c_void_p(dp), ctypes.c_void_p(offsets.data_ptr()),
                                            ctypes.c_void_p(lengths.data_ptr()), count,
                                            ctypes.c_void_p(out.data_ptr()), out_width, ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().hth_batch_graph_launch(self._h, _stream(stream)))
        return self.out

    def check(self, stream=None):
        _check(lib().hth_batch_graph_check(self._h, _stream(stream)))

    def free(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            lib().hth_batch_graph_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """A serving loop (hth_serve_*): submit host byte strings, collect hashes.

    Requests are admitted by device memory and batched on the GPU as they
    arrive; results equal hth_hash_batch's for the same bytes and width."""

    def __init__(self, seed, **config):
        self._seed = seed  # the server reads the seed's device words
        cfg = ServeConfig(**config)
        h = ctypes.c_void_p()
        _check(lib().hth_serve_create(ctypes.byref(cfg), seed.handle, ctypes.byref(h)))
        self._h = h
        self._pinned = []  # pinned buffers whose bytes requests may still read

    def submit(self, data, out_width):
        """Submit bytes (bytes, bytearray or a uint8 numpy array); returns
        the ticket, or None when the server is busy (staging full or too
        many uncollected results)."""
        buf = np.ascontiguousarray(np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray))
                                   else data, dtype=np.uint8)
        t = ctypes.c_uint64()
        rc = lib().hth_serve_submit(self._h, ctypes.c_void_p(buf.ctypes.data if buf.size else 0), buf.size,
                                    out_width, ctypes.byref(t))
        if rc == HTH_E_BUSY:
            return None
        _check(rc)
        return t.value

    def submit_pinned(self, data, out_width):
        """Submit the bytes of a pinned CPU uint8 torch tensor (contiguous)
        without copying them: the server reads them when it hashes the
        request, so the tensor must stay unchanged until the result is
        collected (the server keeps a reference until it is closed).
        Returns the ticket, or None when too many results are uncollected."""
        _require_pinned(data)
        self._pinned.append(data)
        t = ctypes.c_uint64()
        rc = lib().hth_serve_submit_pinned(self._h, ctypes.c_void_p(data.data_ptr() if data.numel() else 0),
                                           data.numel(), out_width, ctypes.byref(t))
        if rc == HTH_E_BUSY:
            return None
        _check(rc)
        return t.value

    def poll(self, ticket):
        """The result bytes if ready, else None."""
        out = (ctypes.c_uint8 * 40)()
        rc = lib().hth_serve_poll(self._h, ticket, out)
        if rc == HTH_E_BUSY:
            return None
        _check(rc)
        return bytes(out)

    def wait(self, ticket, out_width):
        out = (ctypes.c_uint8 * 40)()
        _check(lib().hth_serve_wait(self._h, ticket, out))
        return bytes(out)[:out_width]

    def wait_many(self, tickets):
        """Results of many tickets as an (n, 40) uint8 array (a row holds
        its request's out_width bytes, then zeros)."""
        t = np.ascontiguousarray(tickets, dtype=np.uint64)
        out = np.zeros((t.size, 40), dtype=np.uint8)
        _check(lib().hth_serve_wait_many(self._h, ctypes.c_void_p(t.ctypes.data), t.size,
                                         ctypes.c_void_p(out.ctypes.data), 40))
        return out

    def replay(self, base, offsets, lengths, widths, arrival_ns, threads=1, pinned=False):
        """Submit request i (base[offsets[i]:][:lengths[i]], widths[i]) at
        arrival_ns[i] after the call starts, from `threads` client threads;
        returns the tickets.  pinned: base is a pinned CPU uint8 torch
        tensor whose bytes are hashed in place (hth_serve_replay_pinned; it
        must stay unchanged until the results are collected), else bytes
        are copied into the server's staging (any uint8 array)."""
        if pinned:
            _require_pinned(base)
            self._pinned.append(base)
            base_ptr = ctypes.c_void_p(base.data_ptr())
        else:
            base = np.ascontiguousarray(base, dtype=np.uint8)
            base_ptr = ctypes.c_void_p(base.ctypes.data)
        o = np.ascontiguousarray(offsets, dtype=np.uint64)
        n = np.ascontiguousarray(lengths, dtype=np.uint64)
        w = np.ascontiguousarray(widths, dtype=np.uint32)
        a = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
        tickets = np.zeros(o.size, dtype=np.uint64)
        ptr = lambda x: ctypes.c_void_p(x.ctypes.data)
        fn = lib().hth_serve_replay_pinned if pinned else lib().hth_serve_replay
        _check(fn(self._h, base_ptr, ptr(o), ptr(n), ptr(w), ptr(a), o.size, threads, ptr(tickets)))
        return tickets

    def pause(self, paused=True):
        """Hold (or release) batching; submitted requests queue meanwhile."""
        _check(lib().hth_serve_pause(self._h, 1 if paused else 0))

    def stats(self):
        r = ServeReport()
        _check(lib().hth_serve_stats(self._h, ctypes.byref(r)))
        return r.as_dict()

    def reset_stats(self):
        _check(lib().hth_serve_reset_stats(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            h, self._h = self._h, None
            _check(lib().hth_serve_destroy(h))
        self._h = None
        self._pinned = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream:
    """One string hashed from pieces appended over time (hth_stream_*); the
    value equals hash_batch's for the concatenation of the pieces."""

    def __init__(self, seed, out_width):
        self._seed = seed
        self.out_width = out_width
        h = ctypes.c_void_p()
        _check(lib().hth_stream_create(seed.handle, out_width, ctypes.byref(h)))
        self._h = h

    def update(self, data, stream=None):
        """Append a uint8 CUDA tensor (it must stay alive until the work
        enqueued on the stream completes)."""
        import torch
        if data.dtype != torch.uint8 or not data.is_cuda or not data.is_contiguous():
            raise TypeError("data must be a contiguous uint8 CUDA tensor")
        _check(lib().hth_stream_update(self._h, ctypes.c_void_p(data.data_ptr() if data.numel() else 0),
                                       data.numel(), _stream(stream)))
        return self

    def update_gather(self, pieces, stream=None):
        """Append a list of uint8 CUDA tensors in order, their blocks hashed
        together (hth_stream_update_gather; same value as updating with each
        in turn).  The tensors must stay alive until the work enqueued on the
        stream completes."""
        import torch
        for d in pieces:
            if d.dtype != torch.uint8 or not d.is_cuda or not d.is_contiguous():
                raise TypeError("pieces must be contiguous uint8 CUDA tensors")
        n = len(pieces)
        ptrs = (ctypes.c_void_p * max(n, 1))(*[d.data_ptr() if d.numel() else 0 for d in pieces])
        lens = (ctypes.c_uint64 * max(n, 1))(*[d.numel() for d in pieces])
        _check(lib().hth_stream_update_gather(self._h, ptrs, lens, n, _stream(stream)))
        return self

    def final(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.out_width, dtype=torch.uint8, device="cuda")
        _check(lib().hth_stream_final(self._h, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def reset(self, stream=None):
        _check(lib().hth_stream_reset(self._h, _stream(stream)))

    def save(self, stream=None):
        """The state as bytes (a checkpoint)."""
        n = ctypes.c_size_t()
        _check(lib().hth_stream_save(self._h, None, ctypes.byref(n), _stream(stream)))
        buf = (ctypes.c_uint8 * n.value)()
        _check(lib().hth_stream_save(self._h, buf, ctypes.byref(n), _stream(stream)))
        return bytes(buf)

    def load(self, state, stream=None):
        buf = (ctypes.c_uint8 * len(state)).from_buffer_copy(state)
        _check(lib().hth_stream_load(self._h, buf, len(state), _stream(stream)))

    def __len__(self):
        return int(lib().hth_stream_length(self._h))

    def free(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            lib().hth_stream_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
