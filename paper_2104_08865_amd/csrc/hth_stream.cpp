// libhth streaming (hth_stream_* of include/hth.h): one string hashed from
// pieces appended over time, with the same value hth_hash_batch gives for
// the whole string.
//
// The state is the stack of the tree construction (Eq. (3)): at most 7
// pending items per level, each k x b words, plus the bytes of the
// execution still being filled.  Because tree keys depend only on the level,
// the subtree over an aligned block of 8^L executions (starting at a
// multiple of 8^L) is the same function of its bytes wherever the block
// sits.  An update is therefore cut into maximal aligned blocks; the
// hashing kernel in root mode computes every block's root in one launch
// (the blocks are its strings), and a one-wave kernel pushes, in order, the
// execution completed from the carried bytes (hashing it itself) and the
// roots onto the device-resident stack.  A gathered update takes several
// pieces in one call: the blocks inside each piece and the executions that
// straddle two pieces (assembled in a small buffer) are hashed in one
// root-mode launch, so pieces too small to fill the device alone fill it
// together; a group's push runs on the stream object's own HIP stream,
// beside the next group's work.  Finishing hashes the pending items with
// the final keys, the pending bytes as the tail and the length.  This file
// only plans blocks, orders launches and moves bytes; all hash arithmetic is
// in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include "hth_host.h"
#include "hth_kernels.h"

using namespace hth::host;

namespace {

constexpr int kLevelsMax = 20;
// Aligned blocks of one update: at most 7 per level on the way up to the
// alignment of the largest block and 7 per level on the way down (with room
// to spare).
constexpr uint32_t kMaxRoots = 2 * 7 * kLevelsMax + 8;
static_assert(kMaxRoots + 1 <= hth::kStreamTable, "one piece's blocks and join fit a table");
static_assert(kLevelsMax == hth::kStreamLevels, "stack levels");
constexpr uint32_t kMaxExecBytes = 8 * 8 * 7 * 3;  // largest execution (b = 8, d = 7, w = 3)
constexpr uint32_t kSaveMagic = 0x48544853;         // "HTHS"
constexpr uint32_t kSaveVersion = 1;

struct SaveHeader {
  uint32_t magic, version, width, block;
  uint64_t executions, total_len;
  uint32_t carry_len, reserved;
};

size_t align_to(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct hth_stream {
  const hth_seed* seed = nullptr;
  uint32_t width = 0, block = 8, xb = 0;
  uint64_t executions = 0;  // full executions absorbed
  uint64_t total_len = 0;   // bytes appended
  uint32_t carry_len = 0;   // bytes of the execution being filled
  void* mem = nullptr;      // device state
  uint64_t* stack = nullptr;
  uint32_t* counts = nullptr;
  uint8_t* carry = nullptr;
  uint64_t* roots = nullptr;
  uint64_t* d_off = nullptr;  // [kStreamTable] block offsets
  uint64_t* d_len = nullptr;  // [kStreamTable] block lengths
  uint32_t* d_lev = nullptr;  // [kStreamTable] block levels
  uint8_t* joins = nullptr;   // [kGatherMax][xb] executions that straddle pieces
  uint64_t* roots2 = nullptr;  // gathered groups alternate between (roots, d_lev) and these
  uint32_t* d_lev2 = nullptr;
  // A gathered group's push runs on `side` (a stream of the library's own,
  // default priority), so it overlaps the next group's table, planner and
  // hashing launch on the caller's stream: ev_main[b] orders a push after
  // its group's launch, ev_push[b] a group's table kernel after the push
  // that last read buffer b.  Everything else that touches the stack waits
  // for the last push first (join_side).
  hipStream_t side = nullptr;
  hipEvent_t ev_main[2] = {nullptr, nullptr}, ev_push[2] = {nullptr, nullptr};
  uint64_t groups = 0;        // gathered groups so far (group k uses buffer k % 2)
  bool push_pending = false;  // a push on `side` the caller's stream has not waited for
  hipEvent_t last_push = nullptr;
  Workspace ws;
};

namespace {

hth_status stream_fail(hipError_t e, const char* what) { return hip_fail(e, what); }

// Root-mode hashing of the n blocks of the table (bytes relative to base);
// roots to `roots`.  waves: an upper bound of their tasks.
hth_status launch_blocks(hth_stream* st, const uint8_t* base, uint32_t n, uint64_t waves, uint64_t* roots,
                         hipStream_t stream) {
  if (n == 0) return HTH_OK;
  return enqueue_batch(st->seed, base, st->d_off, st->d_len, n, nullptr, st->width, st->ws, stream, nullptr, nullptr,
                       waves, roots);
}

// The caller's stream waits for the last push on the side stream (before
// anything that reads or writes the stack, the counts, the carried bytes or
// buffer 0).
hth_status join_side(hth_stream* st, hipStream_t stream) {
  if (!st->push_pending) return HTH_OK;
  hipError_t e = hipEventQuery(st->last_push);  // (done: nothing to wait for)
  if (e == hipErrorNotReady) e = hipStreamWaitEvent(stream, st->last_push, 0);
  if (e != hipSuccess) return stream_fail(e, "hth_stream: wait for the previous push");
  st->push_pending = false;
  return HTH_OK;
}

void destroy_side(hth_stream* st) {
  for (int b = 0; b < 2; ++b) {
    if (st->ev_main[b]) (void)hipEventDestroy(st->ev_main[b]);
    if (st->ev_push[b]) (void)hipEventDestroy(st->ev_push[b]);
  }
  if (st->side) (void)hipStreamDestroy(st->side);
}

// The pieces appended in groups (hth_stream_update_gather; a plain update is a
// group of one piece).  Arguments are checked by the callers.
hth_status append_groups(hth_stream* st, const uint8_t* const* pieces, const uint64_t* lens, uint32_t count,
                         hipStream_t stream) {
  // (under stream capture every push stays on the captured stream)
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t ce = hipStreamIsCapturing(stream, &cap);
  if (ce != hipSuccess) return stream_fail(ce, "hth_stream update: capture status");
  const bool on_side = cap == hipStreamCaptureStatusNone;
  if (!on_side) {
    hth_status js = join_side(st, stream);
    if (js != HTH_OK) return js;
  }
  const uint64_t xb = st->xb;
  for (uint32_t i = 0; i < count;) {
    // a group: the carried bytes, then pieces while their table fits
    hth::GatherArgs g{};
    g.e0 = st->executions;
    g.xb = (uint32_t)xb;
    g.seg[0] = st->carry;
    g.seg_len[0] = st->carry_len;
    g.nseg = 1;
    g.joins = st->joins;
    g.carry = st->carry;
    g.off = st->d_off;
    g.len = st->d_len;
    const int bsel = (int)(st->groups % 2);  // the group's roots and levels
    uint64_t* const roots = bsel ? st->roots2 : st->roots;
    g.lev = bsel ? st->d_lev2 : st->d_lev;
    hth::GatherWalk w(xb, st->executions, st->carry_len);
    uint32_t n = 0;  // table entries of the pieces taken (without the joins after the last)
    uint64_t waves = 0, bytes = 0;
    auto trailing = [](hth::GatherWalk f) {  // joins after the last piece's blocks
      uint32_t c = 0;
      f.finish([&](uint32_t, uint64_t) { ++c; });
      return c;
    };
    for (; i < count && g.nseg <= hth::kGatherMax; ++i) {
      if (lens[i] == 0) continue;
      hth::GatherWalk t = w;
      uint32_t tn = n;
      uint64_t tw = waves;
      t.piece(
          pieces[i], lens[i],
          [&](uint64_t, int L, const uint8_t*) {
            ++tn;
            tw += task_bound(xb << (3 * L), st->width, st->block);
          },
          [&](uint32_t, uint64_t) {
            ++tn;
            ++tw;
          });
      if (tn + trailing(t) > hth::kStreamTable) break;  // (one piece alone always fits: kMaxRoots + 1 entries)
      g.w_at[g.nseg] = w.at;  // (the walk before the piece, for the table kernel)
      g.w_next[g.nseg] = w.next;
      g.w_nj[g.nseg] = w.nj;
      g.w_first[g.nseg] = n;
      g.seg[g.nseg] = pieces[i];
      g.seg_len[g.nseg] = lens[i];
      ++g.nseg;
      w = t;
      n = tn;
      waves = tw;
      bytes += lens[i];
    }
    if (g.nseg == 1) {
      if (i < count) return fail(HTH_E_INVALID, "hth_stream update: piece %u does not fit a table", i);
      break;  // (only empty pieces were left)
    }
    const uint32_t nt = trailing(w);
    g.w_at[g.nseg] = w.at;
    g.w_next[g.nseg] = w.next;
    g.w_nj[g.nseg] = w.nj;
    g.w_first[g.nseg] = n;
    g.nj = w.nj + nt;
    n += nt;
    waves += nt;
    const uint64_t nfull = w.at / xb;
    g.nfull = nfull;
    // table offsets from the lowest address the hashing kernel reads
    uintptr_t lo = reinterpret_cast<uintptr_t>(st->joins);
    for (uint32_t k = 1; k < g.nseg; ++k) lo = std::min(lo, reinterpret_cast<uintptr_t>(g.seg[k]));
    g.base = reinterpret_cast<const uint8_t*>(lo);
    // (the levels of buffer bsel were last read by the push two groups back)
    // (a wait across queues costs the stream ≈ 10 us even when the event has
    // long completed: it is enqueued only if the push is still running)
    hipError_t e = hipSuccess;
    if (on_side && (e = hipEventQuery(st->ev_push[bsel])) == hipErrorNotReady)
      e = hipStreamWaitEvent(stream, st->ev_push[bsel], 0);
    if (e == hipSuccess) e = hth::launch_stream_gather(g, stream);
    if (e != hipSuccess) return stream_fail(e, "hth_stream update: table");
    if (n) {
      hth_status s = launch_blocks(st, g.base, n, waves, roots, stream);
      if (s != HTH_OK) return s;
      hipStream_t ps = stream;
      if (on_side) {  // the push after this group's launch, beside the next group's work
        e = hipEventRecord(st->ev_main[bsel], stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(st->side, st->ev_main[bsel], 0);
        if (e != hipSuccess) return stream_fail(e, "hth_stream update: order the push");
        ps = st->side;
      }
      const uint64_t* ent = st->seed->d_words + hth::entropy_offset_of(st->width, st->block);
      e = hth::launch_stream_push(st->width, st->block, ent, roots, g.lev, n, st->stack, st->counts, ps);
      if (e == hipSuccess && on_side) e = hipEventRecord(st->ev_push[bsel], st->side);
      if (e != hipSuccess) return stream_fail(e, "hth_stream update: push launch");
      if (on_side) {
        st->last_push = st->ev_push[bsel];
        st->push_pending = true;
      }
      ++st->groups;
    }
    const uint64_t all = st->carry_len + bytes;
    st->executions += nfull;
    st->carry_len = (uint32_t)(all - nfull * xb);
    st->total_len += bytes;
  }
  return HTH_OK;
}

}  // namespace

extern "C" {

hth_status hth_stream_create(const hth_seed* seed, uint32_t out_width, hth_stream** out) {
  if (!out) return fail(HTH_E_INVALID, "hth_stream_create: out is null");
  *out = nullptr;
  if (!seed) return fail(HTH_E_INVALID, "hth_stream_create: seed is null");
  if (!width_ok(out_width)) return fail(HTH_E_INVALID, "hth_stream_create: out_width %u", out_width);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != seed->device)
    return fail(HTH_E_INVALID, "hth_stream_create: seed lives on device %d, current is %d", seed->device, dev);
  hth_stream* st = new (std::nothrow) hth_stream;
  if (!st) return fail(HTH_E_OOM, "hth_stream_create: host allocation");
  st->seed = seed;
  st->width = out_width;
  st->block = seed->block;
  st->xb = hth::exec_bytes_of(out_width, seed->block);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_to(off + bytes, 256);
    return at;
  };
  const size_t o_stack = take((size_t)hth::kStackWords * 8);
  const size_t o_counts = take(32 * 4);
  const size_t o_carry = take(kMaxExecBytes);
  const size_t o_roots = take((size_t)hth::kStreamTable * hth::kMaxK * 8 * 8);
  const size_t o_off = take(hth::kStreamTable * 8);
  const size_t o_len = take(hth::kStreamTable * 8);
  const size_t o_lev = take(hth::kStreamTable * 4);
  const size_t o_joins = take((size_t)hth::kGatherMax * kMaxExecBytes);
  const size_t o_roots2 = take((size_t)hth::kStreamTable * hth::kMaxK * 8 * 8);
  const size_t o_lev2 = take(hth::kStreamTable * 4);
  e = hipMalloc(&st->mem, off);
  if (e == hipSuccess) e = hipMemset(st->mem, 0, off);
  if (e != hipSuccess) {
    if (st->mem) (void)hipFree(st->mem);
    delete st;
    return hip_fail(e, "hth_stream_create: state allocation");
  }
  char* b = static_cast<char*>(st->mem);
  st->stack = reinterpret_cast<uint64_t*>(b + o_stack);
  st->counts = reinterpret_cast<uint32_t*>(b + o_counts);
  st->carry = reinterpret_cast<uint8_t*>(b + o_carry);
  st->roots = reinterpret_cast<uint64_t*>(b + o_roots);
  st->d_off = reinterpret_cast<uint64_t*>(b + o_off);
  st->d_len = reinterpret_cast<uint64_t*>(b + o_len);
  st->d_lev = reinterpret_cast<uint32_t*>(b + o_lev);
  st->joins = reinterpret_cast<uint8_t*>(b + o_joins);
  st->roots2 = reinterpret_cast<uint64_t*>(b + o_roots2);
  st->d_lev2 = reinterpret_cast<uint32_t*>(b + o_lev2);
  e = hipStreamCreateWithFlags(&st->side, hipStreamNonBlocking);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipEventCreateWithFlags(&st->ev_main[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st->ev_push[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    destroy_side(st);
    (void)hipFree(st->mem);
    delete st;
    return hip_fail(e, "hth_stream_create: side stream");
  }
  hth_status s = ws_alloc(st->ws, hth::kStreamTable, nullptr);
  if (s != HTH_OK) {
    destroy_side(st);
    (void)hipFree(st->mem);
    delete st;
    return s;
  }
  *out = st;
  return HTH_OK;
}

hth_status hth_stream_update(hth_stream* st, const uint8_t* bytes, uint64_t len, hipStream_t stream) {
  if (!st) return fail(HTH_E_INVALID, "hth_stream_update: stream is null");
  if (len && !bytes) return fail(HTH_E_INVALID, "hth_stream_update: bytes is null");
  if (len == 0) return HTH_OK;
  if (st->carry_len + len < st->xb) {  // no execution completed: the bytes join the carried ones
    hipError_t e = hipMemcpyAsync(st->carry + st->carry_len, bytes, len, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return stream_fail(e, "hth_stream_update: carry copy");
    st->carry_len += (uint32_t)len;
    st->total_len += len;
    return HTH_OK;
  }
  return append_groups(st, &bytes, &len, 1, stream);  // (a group of one piece)
}

hth_status hth_stream_update_gather(hth_stream* st, const uint8_t* const* pieces, const uint64_t* lens,
                                    uint32_t count, hipStream_t stream) {
  if (!st) return fail(HTH_E_INVALID, "hth_stream_update_gather: stream is null");
  if (count == 0) return HTH_OK;
  if (!pieces || !lens) return fail(HTH_E_INVALID, "hth_stream_update_gather: pieces or lens is null");
  for (uint32_t i = 0; i < count; ++i)
    if (lens[i] && !pieces[i]) return fail(HTH_E_INVALID, "hth_stream_update_gather: piece %u is null", i);
  return append_groups(st, pieces, lens, count, stream);
}

hth_status hth_stream_final(hth_stream* st, uint8_t* out, hipStream_t stream) {
  if (!st || !out) return fail(HTH_E_INVALID, "hth_stream_final: null pointer");
  hth_status js = join_side(st, stream);
  if (js != HTH_OK) return js;
  const uint64_t* ent = st->seed->d_words + hth::entropy_offset_of(st->width, st->block);
  hipError_t e = hth::launch_stream_final(st->width, st->block, ent, st->stack, st->counts, st->carry, st->carry_len,
                                          st->total_len, out, stream);
  if (e != hipSuccess) return stream_fail(e, "hth_stream_final: launch");
  return HTH_OK;
}

hth_status hth_stream_reset(hth_stream* st, hipStream_t stream) {
  if (!st) return fail(HTH_E_INVALID, "hth_stream_reset: stream is null");
  hth_status js = join_side(st, stream);
  if (js != HTH_OK) return js;
  hipError_t e = hipMemsetAsync(st->counts, 0, 32 * 4, stream);
  if (e != hipSuccess) return stream_fail(e, "hth_stream_reset");
  st->executions = st->total_len = 0;
  st->carry_len = 0;
  return HTH_OK;
}

hth_status hth_stream_save(hth_stream* st, void* host, size_t* size, hipStream_t stream) {
  if (!st || !size) return fail(HTH_E_INVALID, "hth_stream_save: null pointer");
  const size_t need = sizeof(SaveHeader) + kLevelsMax * 4 + (size_t)hth::kStackWords * 8 + st->xb;
  if (!host) {
    *size = need;
    return HTH_OK;
  }
  if (*size < need) return fail(HTH_E_TOO_LARGE, "hth_stream_save: buffer of %zu bytes, %zu needed", *size, need);
  hth_status js = join_side(st, stream);
  if (js != HTH_OK) return js;
  SaveHeader h{kSaveMagic, kSaveVersion, st->width, st->block, st->executions, st->total_len, st->carry_len, 0};
  char* p = static_cast<char*>(host);
  std::memcpy(p, &h, sizeof h);
  hipError_t e = hipMemcpyAsync(p + sizeof h, st->counts, kLevelsMax * 4, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p + sizeof h + kLevelsMax * 4, st->stack, (size_t)hth::kStackWords * 8, hipMemcpyDeviceToHost,
                       stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p + sizeof h + kLevelsMax * 4 + (size_t)hth::kStackWords * 8, st->carry, st->xb,
                       hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return stream_fail(e, "hth_stream_save");
  *size = need;
  return HTH_OK;
}

hth_status hth_stream_load(hth_stream* st, const void* host, size_t size, hipStream_t stream) {
  if (!st || !host) return fail(HTH_E_INVALID, "hth_stream_load: null pointer");
  const size_t need = sizeof(SaveHeader) + kLevelsMax * 4 + (size_t)hth::kStackWords * 8 + st->xb;
  SaveHeader h;
  if (size < sizeof h) return fail(HTH_E_INVALID, "hth_stream_load: %zu bytes is too short", size);
  std::memcpy(&h, host, sizeof h);
  if (h.magic != kSaveMagic || h.version != kSaveVersion)
    return fail(HTH_E_INVALID, "hth_stream_load: not a saved stream state");
  if (h.width != st->width || h.block != st->block)
    return fail(HTH_E_INVALID, "hth_stream_load: state of width %u / block %u, stream is %u / %u", h.width, h.block,
                st->width, st->block);
  if (size < need || h.carry_len >= st->xb) return fail(HTH_E_INVALID, "hth_stream_load: truncated or corrupt state");
  const char* p = static_cast<const char*>(host);
  // The state must be one that appending h.executions executions produces:
  // level l of the stack holds digit l (base 8) of the execution count, and
  // the byte count is the executions' bytes plus the carried ones.  Checked
  // before anything reaches the device (the final kernel reads counts[l]
  // items of a level that has room for 7).
  uint32_t counts[kLevelsMax];
  std::memcpy(counts, p + sizeof h, sizeof counts);
  uint64_t rest = h.executions;
  for (int l = 0; l < kLevelsMax; ++l, rest /= 8)
    if (counts[l] != rest % 8)
      return fail(HTH_E_INVALID, "hth_stream_load: level %d holds %u items, %llu executions leave %llu", l, counts[l],
                  (unsigned long long)h.executions, (unsigned long long)(rest % 8));
  if (rest != 0) return fail(HTH_E_INVALID, "hth_stream_load: execution count beyond the stack's levels");
  if (h.executions > (UINT64_MAX - h.carry_len) / st->xb || h.total_len != h.executions * st->xb + h.carry_len)
    return fail(HTH_E_INVALID, "hth_stream_load: %llu bytes do not match %llu executions and %u carried bytes",
                (unsigned long long)h.total_len, (unsigned long long)h.executions, h.carry_len);
  hth_status js = join_side(st, stream);
  if (js != HTH_OK) return js;
  hipError_t e = hipMemcpyAsync(st->counts, p + sizeof h, kLevelsMax * 4, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(st->stack, p + sizeof h + kLevelsMax * 4, (size_t)hth::kStackWords * 8, hipMemcpyHostToDevice,
                       stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(st->carry, p + sizeof h + kLevelsMax * 4 + (size_t)hth::kStackWords * 8, st->xb,
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return stream_fail(e, "hth_stream_load");
  st->executions = h.executions;
  st->total_len = h.total_len;
  st->carry_len = h.carry_len;
  return HTH_OK;
}

uint64_t hth_stream_length(const hth_stream* st) { return st ? st->total_len : 0; }

hth_status hth_stream_free(hth_stream* st) {
  if (!st) return HTH_OK;
  hipError_t e = st->side ? hipStreamSynchronize(st->side) : hipSuccess;  // (a push may still run)
  destroy_side(st);
  hipError_t f0 = hipFree(st->mem);
  if (e == hipSuccess) e = f0;
  if (st->ws.mem) {
    hipError_t f = hipFree(st->ws.mem);
    if (e == hipSuccess) e = f;
  }
  delete st;
  if (e != hipSuccess) return hip_fail(e, "hth_stream_free");
  return HTH_OK;
}

}  // extern "C"
