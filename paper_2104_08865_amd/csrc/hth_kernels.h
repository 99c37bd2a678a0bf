// Interface between the HIP kernels and the host library (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hth {

constexpr int kMaxK = 5;            // largest number of output words (40 bytes)
constexpr int kPlanCandidates = 6;  // task sizes 128 * 8^j, j = 0..5

// Work distribution: the planner cuts the task list into buckets of about
// equal work (string bytes plus a per-task overhead), at most kMaxBuckets of
// at least kMinBucketBytes each.  A bucket is the run of tasks from a leader
// (the first task starting at or after a bucket boundary) up to the next
// leader, so a task longer than a bucket never leaves empty buckets behind.
// Waves take whole buckets from one device counter: one atomic per bucket,
// not per task, so runs of short strings cost one fetch between them.
constexpr uint32_t kMaxBuckets = 1u << 16;
constexpr uint64_t kMinBucketBytes = 128u << 10;
constexpr uint64_t kTaskOverheadBytes = 4096;
constexpr int kPlanSums = 3;  // per candidate task size: tasks, accumulators, work
// Per planner block: kPlanSums per candidate, then the block's tail-only and
// small strings.
constexpr int kSumTiny = kPlanCandidates * kPlanSums;
constexpr int kSumSmall = kSumTiny + 1;
constexpr int kBlockSums = kSumSmall + 1;
// Per-block prefixes of the chosen level: tasks, accumulators, work, tail-only
// and small strings.
constexpr int kPlanPre = kPlanSums + 2;
// Tail-only strings (shorter than one EHC execution) get no task: they are
// listed apart and hashed one string per lane, in chunks of kTinyChunk
// strings; wave w of the tail-only kernel takes chunks w, w + grid, ...
// Small strings (1 .. kSmallMax executions: at most one complete tree node,
// of level 1) get no task either: listed apart, one per half-wave of the
// small-string kernel.
constexpr int kTinyChunk = 64;
constexpr uint32_t kSmallMax = 8;
// Plans of more planner blocks than this get two scan kernels between their
// two steps (linear in the block count); smaller ones sum in the fill step.
// The scan cuts the blocks into at most kScanGroups runs of at least
// kScanGroupMin blocks, one workgroup each.
constexpr uint32_t kPlanScanMin = 256;
constexpr uint32_t kScanGroups = 128;
constexpr uint32_t kScanGroupMin = 64;

// Control words of one launch (device memory, written by the planner).
enum {
  kCtlNext = 0,  // next bucket to hand out
  kCtlTotal,     // number of tasks
  kCtlLevel,
  kCtlError,
  kCtlBuckets,   // number of buckets (leaders)
  kCtlTiny,      // number of tail-only strings
  kCtlBucketLo,  // bucket size in work bytes (low, high word), for the fill step
  kCtlBucketHi,
  kCtlSmall,     // number of small strings
  kCtlWords = 16
};

struct PlanArgs {
  const uint64_t* lengths;
  uint64_t count;
  uint32_t exec_bytes;
  uint32_t pass_log2;     // log2 of the executions of one pass (7 for b = 8, 8 for b = 4)
  uint32_t direct_lim;    // strings shorter than this are not hashed at all (0: every string is)
  uint32_t small_max;     // strings of 1 .. small_max executions are listed as small (0: none)
  uint64_t* block_sums;  // [kBlockSums][nblocks] (column-major)
  uint64_t* block_pre;   // [kPlanPre][nblocks]: per-block prefixes (large plans)
  uint64_t* group_sums;  // [kBlockSums][kScanGroups]: per-run sums (large plans)
  uint64_t cap_tasks, cap_accs;
  uint32_t min_j, max_j;   // task level range the planner may choose from
  uint64_t target_tasks;   // prefer the coarsest level with at least this many tasks
  uint32_t* task_string;  // [cap_tasks]: string of each task, bit 31 set on bucket leaders
  uint32_t* task_start;   // [count]
  uint32_t* acc_start;    // [count]
  uint32_t* bucket_lead;  // [kMaxBuckets]: leader task of each bucket, any order
  uint32_t* tiny_list;    // [count]: the tail-only strings
  uint32_t* small_list;   // [count]: the small strings
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
  const uint32_t* bucket_lead;
  const uint32_t* tiny_list;
  const uint32_t* small_list;
  uint64_t* roots;  // root mode only: [count][kMaxK * 8]
  uint32_t* ctl;
};

// Kernels and layouts per (output width, block size b = 4 or 8).
const void* main_kernel_fn(uint32_t width, uint32_t block);
uint32_t exec_bytes_of(uint32_t width, uint32_t block);
uint32_t pass_log2_of(uint32_t block);
int64_t entropy_offset_of(uint32_t width, uint32_t block);
uint64_t entropy_words_total(uint32_t block);
uint64_t plan_block_count(uint64_t count);
// Reads n16 16-byte pieces of buf; sink holds `blocks` words (XOR-folded).
hipError_t launch_read_probe(const void* buf, uint64_t n16, uint64_t* sink, uint32_t blocks, hipStream_t stream);
hipError_t launch_plan(const PlanArgs& p, hipStream_t stream);
// The hashing kernel with `grid` waves, then the tail-only kernel with
// `tiny_grid` waves and the small-string kernel with `small_grid` waves.
hipError_t launch_main(uint32_t width, uint32_t block, const MainArgs& a, uint32_t grid, uint32_t tiny_grid,
                       uint32_t small_grid, hipStream_t stream);
const void* tiny_kernel_fn(uint32_t width, uint32_t block);
const void* small_kernel_fn(uint32_t width, uint32_t block);

// Composition with simple tabulation: one string per thread; the string's
// key is its own bytes (lengths <= width) or its HalftimeHash value: computed
// by the tabulation kernel itself for strings of at most kTabInline bytes
// (tail-only strings of at most 8 words), read from h for longer ones (the
// planner's direct_lim is kTabInline + 1, so the hashing kernels write h for
// exactly those).
constexpr uint32_t kTabInline = 64;
struct TabArgs {
  const uint8_t* bytes;
  const uint64_t* offsets;
  const uint64_t* lengths;
  uint64_t count;
  const uint8_t* h;        // [count][width]: values of the strings longer than kTabInline bytes
  const uint64_t* tables;  // [(width + 1) * 256]
  const uint64_t* ent;     // this width's entropy block (tail and length keys)
  uint64_t* out;           // [count]
};
hipError_t launch_tab(uint32_t width, uint32_t block, const TabArgs& a, uint32_t grid, hipStream_t stream);
const void* tab_kernel_fn(uint32_t width, uint32_t block);
// Threads of one tabulation workgroup.
constexpr int kTabThreads = 1024;

// Streaming.  Root mode: every string is a block of exactly 8^L executions
// whose root node (kMaxK x 8 words, [t][j]) goes to a.roots; no tail-only
// strings.  The stack holds kLevels x 7 items of kMaxK x 8 words.
constexpr int kStackWords = 20 * 7 * kMaxK * 8;
hipError_t launch_roots(uint32_t width, uint32_t block, const MainArgs& a, uint32_t grid, hipStream_t stream);
// Pushes the nroots roots (levels[r]: the level of root r) onto the stack,
// closing full nodes upwards.
hipError_t launch_stream_push(uint32_t width, uint32_t block, const uint64_t* ent, const uint64_t* roots,
                              const uint32_t* levels, uint32_t nroots, uint64_t* stack, uint32_t* counts,
                              hipStream_t stream);

// Gathered update: a group of pieces appended with one root-mode launch.
// Segment 0 is the carried bytes, segments 1 .. nseg-1 the pieces; their
// concatenation is cut into full executions.
constexpr int kGatherMax = 64;             // pieces per group
constexpr uint32_t kStreamTable = 1024;    // table entries per launch (one planner workgroup)
constexpr int kStreamLevels = 20;          // levels of the stack
struct GatherArgs {
  uint64_t e0;                             // executions absorbed before the group
  uint32_t xb, nseg;
  const uint8_t* seg[kGatherMax + 1];
  uint64_t seg_len[kGatherMax + 1];
  const uint8_t* base;                     // table offsets are relative to this
  uint8_t* joins;                          // [kGatherMax][xb] executions that straddle segments
  uint8_t* carry;                          // segment 0; rewritten with the group's trailing bytes
  uint64_t* off;
  uint64_t* len;
  uint32_t* lev;
  // The host's walk (GatherWalk) before segment k = 1 .. nseg-1 and after
  // the last (k = nseg): the segment's start in the concatenation (w_at[0]
  // = 0, w_at[nseg] = the total), the next execution not yet emitted, the
  // joins so far and the table index of the segment's first entry; then the
  // group's joins and full executions.
  uint64_t w_at[kGatherMax + 2];
  uint64_t w_next[kGatherMax + 2];
  uint32_t w_nj[kGatherMax + 2];
  uint32_t w_first[kGatherMax + 2];
  uint32_t nj;
  uint64_t nfull;
};
static_assert(sizeof(GatherArgs) <= 4096, "a kernel argument");

// The full executions of a group's concatenation, in order, one segment at
// a time: block(x, L, at) for each maximal aligned block of 8^L executions
// lying inside one piece (x: index of its first execution, at: its first
// byte), join(j, s) for the j-th execution that straddles segments (s: its
// offset in the concatenation; at most one per segment boundary).  The host
// counts a group's table with it and the table kernel writes the table with
// it, so the two cannot disagree.
struct GatherWalk {
  uint64_t xb, e0;
  uint64_t at = 0, next = 0;  // segment start in the concatenation; next execution not yet emitted
  uint32_t nj = 0;
  __host__ __device__ GatherWalk(uint64_t xb_, uint64_t e0_, uint64_t carry_len) : xb(xb_), e0(e0_), at(carry_len) {}
  __host__ __device__ GatherWalk(uint64_t xb_, uint64_t e0_, uint64_t at_, uint64_t next_, uint32_t nj_)
      : xb(xb_), e0(e0_), at(at_), next(next_), nj(nj_) {}
  template <class Block, class Join>
  __host__ __device__ void piece(const uint8_t* p, uint64_t len, Block&& block, Join&& join) {
    const uint64_t a = (at + xb - 1) / xb, b = (at + len) / xb;  // executions inside the piece
    if (b > a) {
      for (; next < a; ++next) join(nj++, next * xb);
      for (uint64_t x = e0 + a, end = e0 + b; x < end;) {
        int L = 0;  // (powers of 8: masks and shifts, no 64-bit division)
        while (L + 1 < kStreamLevels && (x & ((1ull << (3 * (L + 1))) - 1)) == 0 && end - x >= (1ull << (3 * (L + 1))))
          ++L;
        block(x, L, p + ((x - e0) * xb - at));
        x += 1ull << (3 * L);
      }
      next = b;
    }
    at += len;
  }
  // The joins after the last piece's blocks; returns the full executions.
  template <class Join>
  __host__ __device__ uint64_t finish(Join&& join) {
    const uint64_t nfull = at / xb;
    for (; next < nfull; ++next) join(nj++, next * xb);
    return nfull;
  }
};

// Writes the table of a group (blocks and joins in order), assembles the
// joins and rewrites the carried bytes.
hipError_t launch_stream_gather(const GatherArgs& g, hipStream_t stream);
hipError_t launch_stream_final(uint32_t width, uint32_t block, const uint64_t* ent, const uint64_t* stack,
                               const uint32_t* counts, const uint8_t* tail, uint32_t tail_len, uint64_t total_len,
                               uint8_t* out, hipStream_t stream);

}  // namespace hth
