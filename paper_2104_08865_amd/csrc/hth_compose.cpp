// libhth host side of the composed 64-bit hash (include/hth.h): HalftimeHash
// for the strings longer than hth::kTabInline bytes, then simple tabulation
// of every string's key (§1, §7).  Argument checks and launches only; the
// arithmetic runs in hth_kernels.hip.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "../../include/hth.h"
#include "hth_host.h"
#include "hth_kernels.h"

namespace {

using namespace hth::host;

std::mutex g_tab_mu;
std::map<std::pair<int, uint32_t>, uint32_t> g_tab_grid;  // (device, width + block) -> workgroups

// Resident tabulation workgroups of the current device (each holds one LDS
// copy of the tables, so more than that only reloads them).
hth_status tab_grid(uint32_t width, uint32_t block, uint32_t* grid) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto it = g_tab_grid.find({dev, width + block});
  if (it != g_tab_grid.end()) {
    *grid = it->second;
    return HTH_OK;
  }
  int cus = 0, per_cu = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, hth::tab_kernel_fn(width, block), hth::kTabThreads, 0);
  if (e != hipSuccess) return hip_fail(e, "tabulation occupancy query");
  *grid = (uint32_t)cus * (uint32_t)(per_cu > 0 ? per_cu : 1);
  g_tab_grid[{dev, width + block}] = *grid;
  return HTH_OK;
}

}  // namespace

extern "C" {

size_t hth_tab_words(uint32_t inner_width) { return width_ok(inner_width) ? (size_t)(inner_width + 1) * 256 : 0; }

hth_status hth_tab_expand(uint64_t user_seed, uint32_t inner_width, uint64_t* words, size_t n_words) {
  if (!width_ok(inner_width)) return fail(HTH_E_INVALID, "hth_tab_expand: inner_width %u is not 16/24/32/40", inner_width);
  if (!words) return fail(HTH_E_INVALID, "hth_tab_expand: words is null");
  if (n_words != hth_tab_words(inner_width))
    return fail(HTH_E_INVALID, "hth_tab_expand: n_words %zu, the tables of width %u have %zu", n_words, inner_width,
                hth_tab_words(inner_width));
  splitmix64_fill(user_seed, words, n_words);
  return HTH_OK;
}

hth_status hth_hash_batch64(const hth_seed* seed, const uint64_t* tables, const uint8_t* bytes,
                            const uint64_t* offsets, const uint64_t* lengths, uint64_t count, uint64_t* out,
                            uint32_t inner_width, hipStream_t stream) {
  if (count && !tables) return fail(HTH_E_INVALID, "hth_hash_batch64: tables is null");
  if (count && (reinterpret_cast<uintptr_t>(tables) | reinterpret_cast<uintptr_t>(out)) % 8)
    return fail(HTH_E_INVALID, "hth_hash_batch64: tables and out must be 8-byte aligned");
  hth_status st =
      check_batch_args(seed, bytes, offsets, lengths, count, reinterpret_cast<uint8_t*>(out), inner_width);
  if (st != HTH_OK || count == 0) return st;
  uint32_t grid = 0;
  st = tab_grid(inner_width, seed->block, &grid);
  if (st != HTH_OK) return st;
  Workspace* w = nullptr;
  st = get_ws(count, stream, &w);
  if (st != HTH_OK) return st;
  // HalftimeHash of the strings longer than kTabInline bytes into the
  // workspace (shorter ones are keyed by the tabulation kernel itself)
  st = enqueue_batch(seed, bytes, offsets, lengths, count, w->hbuf, inner_width, *w, stream, nullptr, nullptr, 0,
                     nullptr, hth::kTabInline + 1);
  if (st != HTH_OK) return st;
  const uint64_t need = (count + hth::kTabThreads - 1) / hth::kTabThreads;
  if (need < grid) grid = (uint32_t)need;
  hth::TabArgs a{bytes, offsets, lengths, count, w->hbuf, tables,
                 seed->d_words + hth::entropy_offset_of(inner_width, seed->block), out};
  hipError_t e = hth::launch_tab(inner_width, seed->block, a, grid, stream);
  if (e != hipSuccess) return hip_fail(e, "tabulation launch");
  return HTH_OK;
}

}  // extern "C"
