// Host-side internals shared by the C ABI files of libhth (not installed).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/hth.h"

struct hth_seed {
  int device = 0;
  uint32_t block = 8;  // 64-bit words per block of the family (8 or 4)
  uint64_t* d_words = nullptr;
  std::vector<uint64_t> host;
};

namespace hth {
namespace host {

// Workspace of one (device, stream): planning arrays and the cross-task
// accumulators.  sacc, sdone, gacc and gcnt hold zeros between launches (the
// kernel that consumes an accumulator resets it), so a workspace is cleared
// only once, when it is allocated.
struct Workspace {
  uint64_t cap_count = 0, cap_tasks = 0, cap_accs = 0, cap_blocks = 0;
  void* mem = nullptr;
  size_t bytes = 0;
  uint32_t* ctl = nullptr;
  uint64_t* block_sums = nullptr;
  uint64_t* block_pre = nullptr;
  uint64_t* group_sums = nullptr;
  uint32_t* task_string = nullptr;
  uint32_t* task_start = nullptr;
  uint32_t* acc_start = nullptr;
  uint32_t* bucket_lead = nullptr;
  uint32_t* tiny_list = nullptr;
  uint32_t* small_list = nullptr;
  uint64_t* sacc = nullptr;
  uint32_t* sdone = nullptr;
  uint64_t* gacc = nullptr;
  uint32_t* gcnt = nullptr;
  uint8_t* hbuf = nullptr;  // [cap_count][40]: inner values of the composed 64-bit hash
};

// Error reporting: sets the thread's hth_last_error message, returns code.
hth_status fail(hth_status code, const char* fmt, ...);
hth_status hip_fail(hipError_t e, const char* what);
bool width_ok(uint32_t w);

// (Re)allocates w with room for `count` strings, zeroed; the old workspace
// is freed after `stream` drains.
hth_status ws_alloc(Workspace& w, uint64_t count, hipStream_t stream);

// Workspace for (current device, stream) with room for `count` strings
// (grown on the host; refused inside a stream capture).
hth_status get_ws(uint64_t count, hipStream_t stream, Workspace** out);

// splitmix64 outputs 1 .. n from `state` (the generator of the seed expansion).
void splitmix64_fill(uint64_t state, uint64_t* out, size_t n);

// Validates the arguments of one batch (as hth_hash_batch).
hth_status check_batch_args(const hth_seed* seed, const uint8_t* bytes, const uint64_t* offsets,
                            const uint64_t* lengths, uint64_t count, uint8_t* out, uint32_t out_width);

// Enqueues the planner and the hashing kernel of one batch on `stream`
// using workspace `w` (events optional, recorded around the hashing kernel).
// max_waves, when nonzero, caps the hashing kernel's grid: a caller that
// knows the lengths on the host passes an upper bound of the batch's tasks.
// roots, when non-null, selects root mode (every string a block of exactly
// 8^L executions; its root node, kMaxK x 8 words, goes to roots[i]; out
// is not written).  Strings shorter than direct_lim bytes are not hashed
// (their rows of out are not written).
hth_status enqueue_batch(const hth_seed* seed, const uint8_t* bytes, const uint64_t* offsets,
                         const uint64_t* lengths, uint64_t count, uint8_t* out, uint32_t out_width, Workspace& w,
                         hipStream_t stream, hipEvent_t main_start, hipEvent_t main_stop, uint64_t max_waves = 0,
                         uint64_t* roots = nullptr, uint32_t direct_lim = 0);

// Grids of the tail-only and small-string kernels for a batch of `count`
// strings (cached occupancy queries).
hth_status tiny_grid_for(uint32_t width, uint32_t block, uint64_t count, uint32_t* grid);
hth_status small_grid_for(uint32_t width, uint32_t block, uint64_t count, uint32_t* grid);

// Upper bound of the tasks a string of `len` bytes can make (at the finest
// task size) in the family with `block` words per block, for max_waves.
uint64_t task_bound(uint64_t len, uint32_t out_width, uint32_t block);

// Control words of the static workspace of hth_hash_batch_noalloc on device
// `dev` when its last call there was on `stream`, else null.
uint32_t* noalloc_ctl_for(int dev, hipStream_t stream);

}  // namespace host
}  // namespace hth
