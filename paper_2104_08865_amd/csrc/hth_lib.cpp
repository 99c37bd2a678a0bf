// libhth host side: the C ABI of include/hth.h, seed objects, per-stream
// workspaces and launch configuration.  All hashing arithmetic runs in the
// HIP kernels of hth_kernels.hip; this file only moves arguments, memory and
// launches.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hth.h"
#include "hth_host.h"
#include "hth_kernels.h"

namespace hth {
namespace host {

thread_local std::string g_err;

hth_status fail(hth_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

hth_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? HTH_E_OOM : HTH_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool width_ok(uint32_t w) { return w == 16 || w == 24 || w == 32 || w == 40; }
int width_index(uint32_t w) { return (int)(w / 8) - 2; }

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014).
void splitmix64_fill(uint64_t state, uint64_t* out, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    out[i] = z ^ (z >> 31);
  }
}

struct Tuning {
  uint32_t waves_per_cu = 0;
  uint32_t min_j = 0;
  uint32_t max_j = hth::kPlanCandidates - 1;
};

// The planner prefers the coarsest task size that still gives this many
// tasks per resident wave.
constexpr uint64_t kTasksPerWave = 2;

// Default resident waves per compute unit of the persistent grid (2 per
// SIMD): at this depth the hashing kernel already keeps enough loads in
// flight to reach the HBM read ceiling; more waves only add contention.
constexpr uint32_t kDefaultWavesPerCU = 8;

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;
Tuning g_tune[4];
std::map<std::pair<int, int>, uint32_t> g_grid;  // (device, width index + 4 for b = 4) -> persistent grid
std::map<std::pair<int, int>, uint32_t> g_tiny_grid;  // same keys -> resident tail-only waves
std::map<std::pair<int, int>, uint32_t> g_small_grid;  // same keys -> resident small-string waves

// Resident waves per compute unit of the tail-only kernel: it is light on
// registers and latency-bound, so it runs deeper than the hashing kernel.
constexpr uint32_t kTinyWavesPerCU = 32;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

hth_status ws_alloc(Workspace& w, uint64_t count, hipStream_t stream) {
  Workspace n;
  n.cap_count = count < 1024 ? 1024 : count + count / 4;
  n.cap_tasks = n.cap_count + (1ull << 19);
  if (n.cap_tasks > (1ull << 31)) n.cap_tasks = 1ull << 31;
  n.cap_accs = n.cap_tasks * 3 / 10 + 1024;
  n.cap_blocks = hth::plan_block_count(n.cap_count);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  size_t o_ctl = take(hth::kCtlWords * 4);
  size_t o_bs = take(n.cap_blocks * hth::kBlockSums * 8);
  size_t o_bp = take(n.cap_blocks * hth::kPlanPre * 8);
  size_t o_gs = take((size_t)hth::kScanGroups * hth::kBlockSums * 8);
  size_t o_ts = take(n.cap_tasks * 4);
  size_t o_st = take(n.cap_count * 4);
  size_t o_as = take(n.cap_count * 4);
  size_t o_tl = take(n.cap_count * 4);
  size_t o_sl = take(n.cap_count * 4);
  size_t o_bf = take(((size_t)hth::kMaxBuckets + 2) * 4);
  size_t o_sacc = take(n.cap_count * hth::kMaxK * 8);
  size_t o_sdone = take(n.cap_count * 4);
  size_t o_gacc = take(n.cap_accs * hth::kMaxK * 8 * 8);
  size_t o_gcnt = take(n.cap_accs * 4);
  size_t o_h = take(n.cap_count * 40);
  n.bytes = off;
  hipError_t e = hipMalloc(&n.mem, n.bytes);
  if (e != hipSuccess) return hip_fail(e, "workspace allocation");
  e = hipMemsetAsync(n.mem, 0, n.bytes, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    (void)hipFree(n.mem);
    return hip_fail(e, "workspace clear");
  }
  char* b = static_cast<char*>(n.mem);
  n.ctl = reinterpret_cast<uint32_t*>(b + o_ctl);
  n.block_sums = reinterpret_cast<uint64_t*>(b + o_bs);
  n.block_pre = reinterpret_cast<uint64_t*>(b + o_bp);
  n.group_sums = reinterpret_cast<uint64_t*>(b + o_gs);
  n.task_string = reinterpret_cast<uint32_t*>(b + o_ts);
  n.task_start = reinterpret_cast<uint32_t*>(b + o_st);
  n.acc_start = reinterpret_cast<uint32_t*>(b + o_as);
  n.tiny_list = reinterpret_cast<uint32_t*>(b + o_tl);
  n.small_list = reinterpret_cast<uint32_t*>(b + o_sl);
  n.bucket_lead = reinterpret_cast<uint32_t*>(b + o_bf);
  n.sacc = reinterpret_cast<uint64_t*>(b + o_sacc);
  n.sdone = reinterpret_cast<uint32_t*>(b + o_sdone);
  n.gacc = reinterpret_cast<uint64_t*>(b + o_gacc);
  n.gcnt = reinterpret_cast<uint32_t*>(b + o_gcnt);
  n.hbuf = reinterpret_cast<uint8_t*>(b + o_h);
  if (w.mem) {
    // the old workspace may still be in use by work queued on this stream
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      (void)hipFree(n.mem);
      return hip_fail(e, "stream synchronise before workspace growth");
    }
    (void)hipFree(w.mem);
  }
  w = n;
  return HTH_OK;
}

// Workspace for (current device, stream) with room for `count` strings.
hth_status get_ws(uint64_t count, hipStream_t stream, Workspace** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace& w = g_ws[{dev, stream}];
  if (!w.mem || w.cap_count < count) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
      return fail(HTH_E_INVALID,
                  "workspace for %llu strings must be reserved (hth_reserve) before stream capture",
                  (unsigned long long)count);
    hth_status st = ws_alloc(w, count, stream);
    if (st != HTH_OK) return st;
  }
  *out = &w;
  return HTH_OK;
}

hth_status grid_for(uint32_t width, uint32_t block, uint32_t* grid) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  const int wi = width_index(width);
  const int key = wi + (block == 4 ? 4 : 0);
  auto it = g_grid.find({dev, key});
  if (it != g_grid.end()) {
    *grid = it->second;
    return HTH_OK;
  }
  int cus = 0, per_cu = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device attribute");
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, hth::main_kernel_fn(width, block), 64, 0);
  if (e != hipSuccess) return hip_fail(e, "occupancy query");
  uint32_t wpc = per_cu > 0 ? (uint32_t)per_cu : 1;
  const uint32_t want = g_tune[wi].waves_per_cu ? g_tune[wi].waves_per_cu : kDefaultWavesPerCU;
  if (want < wpc) wpc = want;
  *grid = (uint32_t)cus * wpc;
  g_grid[{dev, key}] = *grid;
  return HTH_OK;
}

// Waves of the tail-only kernel for a batch of `count` strings: resident
// waves up to kTinyWavesPerCU per CU, and no more than its chunks.
hth_status tiny_grid_for(uint32_t width, uint32_t block, uint64_t count, uint32_t* grid) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  uint32_t full = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const int key = width_index(width) + (block == 4 ? 4 : 0);
    auto it = g_tiny_grid.find({dev, key});
    if (it != g_tiny_grid.end()) {
      full = it->second;
    } else {
      int cus = 0, per_cu = 0;
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, hth::tiny_kernel_fn(width, block), 64, 0);
      if (e != hipSuccess) return hip_fail(e, "tail-only kernel occupancy query");
      uint32_t wpc = per_cu > 0 ? (uint32_t)per_cu : 1;
      if (wpc > kTinyWavesPerCU) wpc = kTinyWavesPerCU;
      full = (uint32_t)cus * wpc;
      g_tiny_grid[{dev, key}] = full;
    }
  }
  const uint64_t chunks = (count + hth::kTinyChunk - 1) / hth::kTinyChunk;
  *grid = chunks < full ? (uint32_t)(chunks ? chunks : 1) : full;
  return HTH_OK;
}

// Waves of the small-string kernel for a batch of `count` strings: resident
// waves, and no more than pairs of strings.
hth_status small_grid_for(uint32_t width, uint32_t block, uint64_t count, uint32_t* grid) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  uint32_t full = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const int key = width_index(width) + (block == 4 ? 4 : 0);
    auto it = g_small_grid.find({dev, key});
    if (it != g_small_grid.end()) {
      full = it->second;
    } else {
      int cus = 0, per_cu = 0;
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, hth::small_kernel_fn(width, block), 64, 0);
      if (e != hipSuccess) return hip_fail(e, "small-string kernel occupancy query");
      full = (uint32_t)cus * (uint32_t)(per_cu > 0 ? per_cu : 1);
      g_small_grid[{dev, key}] = full;
    }
  }
  const uint64_t pairs = (count + 1) / 2;
  *grid = pairs < full ? (uint32_t)(pairs ? pairs : 1) : full;
  return HTH_OK;
}

}  // namespace host
}  // namespace hth

struct hth_batch_graph {
  hth::host::Workspace ws;  // private: replays of one graph must not overlap
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace hth {
namespace host {

hth_status check_batch_args(const hth_seed* seed, const uint8_t* bytes, const uint64_t* offsets,
                            const uint64_t* lengths, uint64_t count, uint8_t* out, uint32_t out_width) {
  if (!width_ok(out_width)) return fail(HTH_E_INVALID, "hth_hash_batch: out_width %u is not 16/24/32/40", out_width);
  if (!seed) return fail(HTH_E_INVALID, "hth_hash_batch: seed is null");
  if (count == 0) return HTH_OK;
  if (!bytes || !offsets || !lengths || !out) return fail(HTH_E_INVALID, "hth_hash_batch: null pointer");
  if (count > (1ull << 31)) return fail(HTH_E_INVALID, "hth_hash_batch: count %llu exceeds 2^31", (unsigned long long)count);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != seed->device) return fail(HTH_E_INVALID, "hth_hash_batch: seed lives on device %d, current is %d", seed->device, dev);
  return HTH_OK;
}

// Planner and hashing kernel of one batch on `stream`, using workspace `w`.
hth_status enqueue_batch(const hth_seed* seed, const uint8_t* bytes, const uint64_t* offsets,
                         const uint64_t* lengths, uint64_t count, uint8_t* out, uint32_t out_width, Workspace& w,
                         hipStream_t stream, hipEvent_t main_start, hipEvent_t main_stop, uint64_t max_waves,
                         uint64_t* roots, uint32_t direct_lim) {
  const uint32_t block = seed->block;
  uint32_t grid = 0;
  hth_status st = grid_for(out_width, block, &grid);
  if (st != HTH_OK) return st;
  if (max_waves && max_waves < grid) grid = (uint32_t)max_waves;
  Tuning tune;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    tune = g_tune[width_index(out_width)];
  }
  hth::PlanArgs p{};
  p.lengths = lengths;
  p.count = count;
  p.exec_bytes = hth::exec_bytes_of(out_width, block);
  p.pass_log2 = hth::pass_log2_of(block);
  p.direct_lim = direct_lim;
  // (root mode hashes every block in the main kernel: no listed small strings)
  p.small_max = roots ? 0 : hth::kSmallMax;
  p.block_sums = w.block_sums;
  p.block_pre = w.block_pre;
  p.group_sums = w.group_sums;
  p.cap_tasks = w.cap_tasks;
  p.cap_accs = w.cap_accs;
  p.min_j = tune.min_j;
  p.max_j = tune.max_j;
  p.target_tasks = (uint64_t)grid * kTasksPerWave;
  p.task_string = w.task_string;
  p.task_start = w.task_start;
  p.acc_start = w.acc_start;
  p.bucket_lead = w.bucket_lead;
  p.tiny_list = w.tiny_list;
  p.small_list = w.small_list;
  p.ctl = w.ctl;
  hipError_t e = hth::launch_plan(p, stream);
  if (e != hipSuccess) return hip_fail(e, "plan launch");

  hth::MainArgs a{};
  a.bytes = bytes;
  a.offsets = offsets;
  a.lengths = lengths;
  a.out = out;
  a.ent = seed->d_words + hth::entropy_offset_of(out_width, block);
  a.task_string = w.task_string;
  a.task_start = w.task_start;
  a.acc_start = w.acc_start;
  a.sacc = w.sacc;
  a.sdone = w.sdone;
  a.gacc = w.gacc;
  a.gcnt = w.gcnt;
  a.bucket_lead = w.bucket_lead;
  a.tiny_list = w.tiny_list;
  a.small_list = w.small_list;
  a.roots = roots;
  a.ctl = w.ctl;
  if (main_start && (e = hipEventRecord(main_start, stream)) != hipSuccess) return hip_fail(e, "event record");
  uint32_t tiny_grid = 1, small_grid = 1;
  if (!roots) {
    st = tiny_grid_for(out_width, block, count, &tiny_grid);
    if (st == HTH_OK) st = small_grid_for(out_width, block, count, &small_grid);
    if (st != HTH_OK) return st;
  }
  e = roots ? hth::launch_roots(out_width, block, a, grid, stream)
            : hth::launch_main(out_width, block, a, grid, tiny_grid, small_grid, stream);
  if (e != hipSuccess) return hip_fail(e, "main launch");
  if (main_stop && (e = hipEventRecord(main_stop, stream)) != hipSuccess) return hip_fail(e, "event record");
  return HTH_OK;
}

uint64_t task_bound(uint64_t len, uint32_t out_width, uint32_t block) {
  const uint64_t n = len / hth::exec_bytes_of(out_width, block);
  const uint64_t pass = 1ull << hth::pass_log2_of(block);
  return n ? (n + pass - 1) / pass : 1;
}

// Synchronise and read a workspace's planner status word.
hth_status check_ctl(uint32_t* ctl, hipStream_t stream) {
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronise");
  uint32_t err = 0;
  e = hipMemcpy(&err, ctl + hth::kCtlError, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "status read");
  if (err) return fail(HTH_E_TOO_LARGE, "the last batch exceeded the workspace plan limits");
  return HTH_OK;
}

}  // namespace host
}  // namespace hth

using namespace hth::host;

extern "C" {

const char* hth_last_error(void) { return g_err.c_str(); }

size_t hth_entropy_words(void) { return (size_t)hth::entropy_words_total(8); }

size_t hth_entropy_words_b(uint32_t block_words) { return (size_t)hth::entropy_words_total(block_words); }

hth_status hth_seed_from_entropy_b(const uint64_t* words, size_t n_words, uint32_t block_words, hth_seed** out,
                                   hipStream_t stream) {
  if (!out) return fail(HTH_E_INVALID, "hth_seed_from_entropy: out is null");
  *out = nullptr;
  if (block_words != 4 && block_words != 8)
    return fail(HTH_E_INVALID, "hth_seed_from_entropy: block_words %u is not 4 or 8", block_words);
  if (!words) return fail(HTH_E_INVALID, "hth_seed_from_entropy: words is null");
  if (n_words != hth_entropy_words_b(block_words))
    return fail(HTH_E_INVALID, "hth_seed_from_entropy: n_words is %zu, expected %zu", n_words,
                hth_entropy_words_b(block_words));
  hth_seed* s = new (std::nothrow) hth_seed;
  if (!s) return fail(HTH_E_OOM, "hth_seed_from_entropy: host allocation");
  s->block = block_words;
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipGetDevice");
  }
  s->host.assign(words, words + n_words);
  e = hipMalloc(&s->d_words, n_words * 8);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "seed allocation");
  }
  // the copy reads s->host, which lives as long as the seed
  e = hipMemcpyAsync(s->d_words, s->host.data(), n_words * 8, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) {
    (void)hipFree(s->d_words);
    delete s;
    return hip_fail(e, "seed upload");
  }
  *out = s;
  return HTH_OK;
}

hth_status hth_seed_from_entropy(const uint64_t* words, size_t n_words, hth_seed** out, hipStream_t stream) {
  return hth_seed_from_entropy_b(words, n_words, 8, out, stream);
}

hth_status hth_expand_seed_b(uint64_t user_seed, uint32_t block_words, hth_seed** out, hipStream_t stream) {
  if (!out) return fail(HTH_E_INVALID, "hth_expand_seed: out is null");
  if (block_words != 4 && block_words != 8)
    return fail(HTH_E_INVALID, "hth_expand_seed: block_words %u is not 4 or 8", block_words);
  std::vector<uint64_t> w(hth_entropy_words_b(block_words));
  splitmix64_fill(user_seed, w.data(), w.size());
  return hth_seed_from_entropy_b(w.data(), w.size(), block_words, out, stream);
}

hth_status hth_expand_seed(uint64_t user_seed, hth_seed** out, hipStream_t stream) {
  return hth_expand_seed_b(user_seed, 8, out, stream);
}

uint32_t hth_seed_block_words(const hth_seed* seed) { return seed ? seed->block : 0; }

hth_status hth_seed_entropy(const hth_seed* seed, uint64_t* host_words, size_t n_words) {
  if (!seed || !host_words) return fail(HTH_E_INVALID, "hth_seed_entropy: null pointer");
  if (n_words != seed->host.size()) return fail(HTH_E_INVALID, "hth_seed_entropy: n_words mismatch");
  hipError_t e = hipMemcpy(host_words, seed->d_words, n_words * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "seed download");
  return HTH_OK;
}

hth_status hth_seed_free(hth_seed* seed) {
  if (!seed) return HTH_OK;
  hipError_t e = hipFree(seed->d_words);
  delete seed;
  if (e != hipSuccess) return hip_fail(e, "seed free");
  return HTH_OK;
}

hth_status hth_reserve(uint64_t max_count, hipStream_t stream) {
  Workspace* w = nullptr;
  return get_ws(max_count ? max_count : 1, stream, &w);
}

hth_status hth_set_tuning(uint32_t out_width, uint32_t waves_per_cu, uint32_t min_task_level,
                          uint32_t max_task_level) {
  if (!width_ok(out_width)) return fail(HTH_E_INVALID, "hth_set_tuning: out_width %u", out_width);
  if (min_task_level > max_task_level || max_task_level >= (uint32_t)hth::kPlanCandidates)
    return fail(HTH_E_INVALID, "hth_set_tuning: task levels %u..%u", min_task_level, max_task_level);
  std::lock_guard<std::mutex> lk(g_mu);
  const int wi = width_index(out_width);
  g_tune[wi].waves_per_cu = waves_per_cu;
  g_tune[wi].min_j = min_task_level;
  g_tune[wi].max_j = max_task_level;
  for (auto it = g_grid.begin(); it != g_grid.end();) {
    if (it->first.second % 4 == wi) it = g_grid.erase(it);
    else ++it;
  }
  return HTH_OK;
}

hth_status hth_hash_batch(const hth_seed* seed, const uint8_t* bytes, const uint64_t* offsets,
                          const uint64_t* lengths, uint64_t count, uint8_t* out, uint32_t out_width,
                          hipStream_t stream) {
  return hth_hash_batch_timed(seed, bytes, offsets, lengths, count, out, out_width, stream, nullptr, nullptr);
}

hth_status hth_hash_batch_timed(const hth_seed* seed, const uint8_t* bytes, const uint64_t* offsets,
                                const uint64_t* lengths, uint64_t count, uint8_t* out, uint32_t out_width,
                                hipStream_t stream, hipEvent_t main_start, hipEvent_t main_stop) {
  hth_status st = check_batch_args(seed, bytes, offsets, lengths, count, out, out_width);
  if (st != HTH_OK || count == 0) return st;
  Workspace* w = nullptr;
  st = get_ws(count, stream, &w);
  if (st != HTH_OK) return st;
  return enqueue_batch(seed, bytes, offsets, lengths, count, out, out_width, *w, stream, main_start, main_stop);
}

hth_status hth_batch_graph_create(const hth_seed* seed, const uint8_t* bytes, const uint64_t* offsets,
                                  const uint64_t* lengths, uint64_t count, uint8_t* out, uint32_t out_width,
                                  hth_batch_graph** graph) {
  if (!graph) return fail(HTH_E_INVALID, "hth_batch_graph_create: graph is null");
  *graph = nullptr;
  hth_status st = check_batch_args(seed, bytes, offsets, lengths, count, out, out_width);
  if (st != HTH_OK) return st;
  if (count == 0) return fail(HTH_E_INVALID, "hth_batch_graph_create: count is 0");
  uint32_t grid = 0;
  st = grid_for(out_width, seed->block, &grid);  // fills the caches outside the capture
  if (st == HTH_OK) st = tiny_grid_for(out_width, seed->block, count, &grid);
  if (st == HTH_OK) st = small_grid_for(out_width, seed->block, count, &grid);
  if (st != HTH_OK) return st;
  hth_batch_graph* g = new (std::nothrow) hth_batch_graph;
  if (!g) return fail(HTH_E_OOM, "hth_batch_graph_create: host allocation");
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "capture stream");
  }
  st = ws_alloc(g->ws, count, cs);
  if (st == HTH_OK) {
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      st = hip_fail(e, "hipStreamBeginCapture");
    } else {
      st = enqueue_batch(seed, bytes, offsets, lengths, count, out, out_width, g->ws, cs, nullptr, nullptr);
      hipGraph_t graph_obj = nullptr;
      e = hipStreamEndCapture(cs, &graph_obj);  // always end the capture
      if (st == HTH_OK && e != hipSuccess) st = hip_fail(e, "hipStreamEndCapture");
      g->graph = graph_obj;
      if (st == HTH_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = hip_fail(e, "hipGraphInstantiate");
      }
    }
  }
  (void)hipStreamDestroy(cs);
  if (st != HTH_OK) {
    hth_batch_graph_free(g);
    return st;
  }
  *graph = g;
  return HTH_OK;
}

hth_status hth_batch_graph_launch(hth_batch_graph* graph, hipStream_t stream) {
  if (!graph || !graph->exec) return fail(HTH_E_INVALID, "hth_batch_graph_launch: graph is null");
  hipError_t e = hipGraphLaunch(graph->exec, stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return HTH_OK;
}

hth_status hth_batch_graph_check(hth_batch_graph* graph, hipStream_t stream) {
  if (!graph) return fail(HTH_E_INVALID, "hth_batch_graph_check: graph is null");
  return check_ctl(graph->ws.ctl, stream);
}

hth_status hth_batch_graph_free(hth_batch_graph* graph) {
  if (!graph) return HTH_OK;
  hipError_t e = hipSuccess;
  if (graph->exec) e = hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  if (graph->ws.mem) {
    hipError_t f = hipFree(graph->ws.mem);
    if (e == hipSuccess) e = f;
  }
  delete graph;
  if (e != hipSuccess) return hip_fail(e, "hth_batch_graph_free");
  return HTH_OK;
}

hth_status hth_read_probe(const void* buf, uint64_t bytes, uint64_t* sink, uint32_t sink_words, hipStream_t stream) {
  if (!buf || !sink || !sink_words) return fail(HTH_E_INVALID, "hth_read_probe: null pointer or empty sink");
  if (reinterpret_cast<uintptr_t>(buf) % 16) return fail(HTH_E_INVALID, "hth_read_probe: buf not 16-byte aligned");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device attribute");
  // 4 single-wave workgroups per compute unit: the rate peaks there
  uint32_t blocks = (uint32_t)cus * 4;
  if (blocks > sink_words) blocks = sink_words;
  e = hth::launch_read_probe(buf, bytes / 16, sink, blocks, stream);
  if (e != hipSuccess) return hip_fail(e, "read probe launch");
  return HTH_OK;
}

hth_status hth_batch_check(hipStream_t stream) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  uint32_t* ctl = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find({dev, stream});
    if (it != g_ws.end()) ctl = it->second.ctl;
  }
  uint32_t* na = noalloc_ctl_for(dev, stream);
  hth_status st = HTH_OK;
  if (ctl) st = check_ctl(ctl, stream);
  if (st == HTH_OK && na) st = check_ctl(na, stream);
  return st;
}

}  // extern "C"
