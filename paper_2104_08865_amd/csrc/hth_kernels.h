// Interface between the HIP kernels and the host library (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hth {

constexpr int kMaxK = 5;            // largest number of output words (40 bytes)
constexpr int kPlanCandidates = 6;  // task sizes 128 * 8^j, j = 0..5

// Control words of one launch (device memory, written by the planner).
enum { kCtlNext = 0, kCtlTotal = 1, kCtlLevel = 2, kCtlError = 3, kCtlWords = 4 };

struct PlanArgs {
  const uint64_t* lengths;
  uint64_t count;
  uint32_t exec_bytes;
  uint64_t* block_sums;  // [nblocks][2 * kPlanCandidates]
  uint64_t cap_tasks, cap_accs;
  uint32_t min_j, max_j;   // task level range the planner may choose from
  uint64_t target_tasks;   // prefer the coarsest level with at least this many tasks
  uint32_t* task_string;  // [cap_tasks]
  uint32_t* task_start;   // [count]
  uint32_t* acc_start;    // [count]
  uint32_t* ctl;          // [kCtlWords]
};

struct MainArgs {
  const uint8_t* bytes;
  const uint64_t* offsets;
  const uint64_t* lengths;
  uint8_t* out;
  const uint64_t* ent;  // this width's entropy block
  const uint32_t* task_string;
  const uint32_t* task_start;
  const uint32_t* acc_start;
  uint64_t* sacc;  // [count][kMaxK], zero between launches
  uint32_t* sdone; // [count], zero between launches
  uint64_t* gacc;  // [cap_accs][kMaxK * 8], zero between launches
  uint32_t* gcnt;  // [cap_accs], zero between launches
  uint32_t* ctl;
};

const void* main_kernel_fn(uint32_t width);
uint32_t exec_bytes_of(uint32_t width);
int64_t entropy_offset_of(uint32_t width);
uint64_t entropy_words_total();
uint64_t plan_block_count(uint64_t count);
hipError_t launch_plan(const PlanArgs& p, hipStream_t stream);
hipError_t launch_main(uint32_t width, const MainArgs& a, uint32_t grid, hipStream_t stream);

}  // namespace hth
