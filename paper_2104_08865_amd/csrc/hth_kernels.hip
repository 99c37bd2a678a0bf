// HalftimeHash kernels for gfx950 (MI355X).
//
// One launch hashes a whole batch of strings.  Work is cut into tasks: a task
// is an aligned range of T = 128 * 8^j full EHC executions of one string (the
// last task of a string also takes its tail, its length term and any partial
// range).  A planner (two small kernels, or one for small batches, plus two
// scan kernels for large ones) cuts the task list into buckets of about equal
// work; a persistent grid of single-wave workgroups pulls whole buckets from
// a device counter.  Strings shorter than one execution have no task: a
// separate tail-only kernel hashes them, one string per lane; strings of 1 ..
// kSmallMax executions have none either: a small-string kernel hashes them,
// one per half-wave.  The composed 64-bit hash's tabulation kernel is here
// too (it computes the value of short tail-only strings itself).
//
// Inside a task a wave works in passes of 128 executions.  Lane l = 4q + r
// (q = 0..15, r = 0..3) owns instances 2r and 2r+1 (the two 64-bit words of a
// 16-byte piece of each 64-byte block, paper §2: instance j = word j of
// every block) of the 8 consecutive executions p + 8q .. p + 8q + 7.  The
// executions reach the wave through LDS (copied from HBM by direct-to-LDS
// loads, one region of 16 executions at a time, while the previous region is
// hashed); for each execution a lane reads its blocks' pieces, runs Encode,
// Hash and Combine (§3.3, §4, §5.1) in registers, and feeds the k outputs into the
// first tree level: 8 consecutive executions of a lane form one level-1 node
// of every tree, so levels 0 and 1 need no data exchange.  Level 2 (64
// executions) is a 3-step butterfly over lanes q, q^1, q^2, q^4 of each half
// wave.  Above level 2 a node's value is the sum of one term per child (the
// NH variant of §3.2: NH of children 0..6 against their position's key plus
// child 7), so children are folded into their parent by adding their terms:
// in LDS when the parent lies inside the task, with 64-bit atomics in device
// memory when it spans tasks (the 8th arrival, found by a counter, carries
// on with the parent).  Items the stack construction of Eq. (3) leaves over
// (one per unit of each base-8 digit of the execution count) go straight into
// the final NH (§5.2).  All of these, the tail (§6.1) and the length term are
// sums mod 2^64, so their order never changes the result.  A string's last,
// partial pass spreads its executions over all lane groups instead
// (partial_pass), and the keys that pass and the tail read at lane-varying
// indices are held in LDS.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hth_family.h"
#include "hth_kernels.h"

namespace hth {

// ---------------------------------------------------------------------------
// Arithmetic helpers
// ---------------------------------------------------------------------------

// NH of one word (lo, hi) against one key (§3.2): halves added mod 2^32, one
// 32x32->64 product (v_mad_u64_u32 with the accumulate).
__device__ __forceinline__ uint64_t nh_acc(uint64_t acc, uint32_t lo, uint32_t hi, uint64_t key) {
  return acc + (uint64_t)(uint32_t)(lo + (uint32_t)key) * (uint32_t)(hi + (uint32_t)(key >> 32));
}
__device__ __forceinline__ uint64_t nh_acc(uint64_t acc, uint64_t x, uint64_t key) {
  return nh_acc(acc, (uint32_t)x, (uint32_t)(x >> 32), key);
}

// Multiply by one of the small combine coefficients with shifts and adds.
__device__ __forceinline__ uint64_t mulc(int c, uint64_t h) {
  switch (c) {
    case 0: return 0;
    case 1: return h;
    case 2: return h << 1;
    case 3: return (h << 1) + h;
    case 4: return h << 2;
    case 5: return (h << 2) + h;
    case 6: return (h << 2) + (h << 1);
    case 7: return (h << 3) - h;
    case 8: return h << 3;
    case 9: return (h << 3) + h;
    default: return h * (uint64_t)c;
  }
}

// Keys that every lane of a wave reads at the same address go through the
// scalar cache: the constant address space lets the compiler use scalar loads
// (counted apart from the vector loads of the data, so they never delay the
// data's waits) and keep the keys out of vector registers.
typedef const __attribute__((address_space(4))) uint64_t* key_ptr;
__device__ __forceinline__ key_ptr uniform_keys(const uint64_t* p) { return (key_ptr)p; }
// The same for per-string metadata read at wave-uniform indices (written
// before the launch, read-only during it).
typedef const __attribute__((address_space(4))) uint32_t* meta32_ptr;
__device__ __forceinline__ meta32_ptr smeta(const uint32_t* p) { return (meta32_ptr)p; }

// The n bytes at p (1 <= n <= 7) as a zero-padded little-endian word: the
// one or two aligned words that hold them, shifted into place (both loads
// issued at once; each word holds one of the n bytes, so neither reaches
// past the page of the bytes' allocation).  Byte-by-byte loads in a loop of
// n iterations were waited for one after another.
__device__ __forceinline__ uint64_t load_partial_word(const uint8_t* p, uint32_t n) {
  const uint32_t s = (uint32_t)(reinterpret_cast<uintptr_t>(p) & 7);
  const uint8_t* ab = p - s;  // (derived from p: the loads stay global loads)
  uint64_t lo, hi = 0;
  __builtin_memcpy(&lo, ab, 8);
  if (s + n > 8) __builtin_memcpy(&hi, ab + 8, 8);
  const uint64_t v = s ? (lo >> (8 * s)) | (hi << (64 - 8 * s)) : lo;
  return v & ((1ull << (8 * n)) - 1);
}

// A run of tail words loaded by one lane, at most one of them partial: the
// loads of every word are issued first (issue_tail_word) and the partial one
// is shifted into place afterwards (finish_tail_words), so that no wait for
// it falls between the loads (a wait inside the loop of loads held up every
// later load of the run).
struct PartialWord {
  int idx = -1;      // which word of the run is partial (-1: none)
  uint32_t sh = 0;   // its byte offset from the aligned word below it
  uint32_t n = 0;    // its bytes
  uint64_t hi = 0;   // the aligned word after it (when it reaches in)
};
__device__ __forceinline__ void issue_tail_word(const uint8_t* pw, uint64_t avail, int i, uint64_t& w,
                                                PartialWord& pp) {
  if (avail >= 8) {
    __builtin_memcpy(&w, pw, 8);
  } else {
    const uint32_t s = (uint32_t)(reinterpret_cast<uintptr_t>(pw) & 7);
    const uint8_t* ab = pw - s;
    __builtin_memcpy(&w, ab, 8);
    if (s + avail > 8) __builtin_memcpy(&pp.hi, ab + 8, 8);
    pp.idx = i;
    pp.sh = s;
    pp.n = (uint32_t)avail;
  }
}
template <int NW>
__device__ __forceinline__ void finish_tail_words(uint64_t (&w)[NW], const PartialWord& pp) {
#pragma unroll
  for (int i = 0; i < NW; ++i)
    if (i == pp.idx) {
      const uint64_t v = pp.sh ? (w[i] >> (8 * pp.sh)) | (pp.hi << (64 - 8 * pp.sh)) : w[i];
      w[i] = v & ((1ull << (8 * pp.n)) - 1);
    }
}

__device__ __forceinline__ uint4 load16(const uint8_t* p) {
  uint4 v;
  __builtin_memcpy(&v, p, 16);
  return v;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  uint32_t lo = __shfl((uint32_t)v, src);
  uint32_t hi = __shfl((uint32_t)(v >> 32), src);
  return (uint64_t)hi << 32 | lo;
}
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  uint32_t lo = __shfl_xor((uint32_t)v, m);
  uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m);
  return (uint64_t)hi << 32 | lo;
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v += shfl_xor64(v, m);
  return v;
}

// The builtin returns a signed int: widen each half as uint32_t, never as
// int, or bit 31 of the low half would be sign-extended into the high half.
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  return (uint64_t)hi << 32 | lo;
}

// Cross-task sums live in device memory that only device-scope atomic
// read-modify-writes ever touch, so they need ordering, not cache
// maintenance: the workgroup fence keeps the compiler from reordering this
// wave's atomics, and the wait makes every earlier atomic of the wave
// complete (performed where all compute units see it) before any later one
// is issued.  A device-scope fence would also write back and invalidate the
// L2, which costs far more than the hashing itself.
__device__ __forceinline__ void complete_atomics() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
}

// Number of complete nodes of level l (8^l executions each) among N executions.
__device__ __forceinline__ uint64_t nodes_at(uint64_t N, int l) { return l >= 22 ? 0 : N >> (3 * l); }

// ---------------------------------------------------------------------------
// EHC of one execution for the two instances of a lane (blocks of B words:
// block i of the execution starts 8*B*i bytes in).
// ---------------------------------------------------------------------------

// EHC state of one execution for the two instances of a lane: the parity
// words (sums over the systematic words) and the k combined outputs.  The
// systematic items can be fed in several calls, in order.
template <int WIDTH>
struct Ehc {
  static constexpr int D = Family<WIDTH>::D, K = Family<WIDTH>::K, R = K - 1, RR = R > 0 ? R : 1;
  uint64_t par0[RR][kSym], par1[RR][kSym];
  uint64_t z0[K], z1[K];
};

template <int WIDTH>
__device__ __forceinline__ void ehc_begin(Ehc<WIDTH>& s) {
#pragma unroll
  for (int r = 0; r < Ehc<WIDTH>::R; ++r)
#pragma unroll
    for (int u = 0; u < kSym; ++u) s.par0[r][u] = s.par1[r][u] = 0;
#pragma unroll
  for (int t = 0; t < Ehc<WIDTH>::K; ++t) s.z0[t] = s.z1[t] = 0;
}

// Systematic blocks K0 .. K1-1 (block k = word k % kSym of item k / kSym, in
// x[k - K0]): hash each word, add it into the parity words whose binary image
// selects it, and add T times the item's NH sum into the outputs.  An item
// may be split over two calls: T is linear, so its two partial sums are
// combined separately.
template <int WIDTH, int K0, int K1>
__device__ __forceinline__ void ehc_blocks(Ehc<WIDTH>& s, const uint4* x, key_ptr S_ehc) {
  using Fm = Family<WIDTH>;
  constexpr int K = Fm::K, R = K - 1;
  uint64_t h0 = 0, h1 = 0;
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    const int c = k / kSym, v = k % kSym;
    const uint4 w = x[k - K0];
    const uint64_t key = S_ehc[k];
    h0 = nh_acc(h0, w.x, w.y, key);
    h1 = nh_acc(h1, w.z, w.w, key);
    const uint64_t w0 = (uint64_t)w.y << 32 | w.x, w1 = (uint64_t)w.w << 32 | w.z;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < kSym; ++u)
        if (image_bit(Fm::P[r][c], u, v)) {
          s.par0[r][u] += w0;
          s.par1[r][u] += w1;
        }
    if (v == kSym - 1 || k == K1 - 1) {
#pragma unroll
      for (int t = 0; t < K; ++t) {
        s.z0[t] += mulc(Fm::T[t][c], h0);
        s.z1[t] += mulc(Fm::T[t][c], h1);
      }
      h0 = h1 = 0;
    }
  }
}

// The parity items, after every systematic item.
template <int WIDTH>
__device__ __forceinline__ void ehc_end(Ehc<WIDTH>& s, key_ptr S_ehc) {
  using Fm = Family<WIDTH>;
  constexpr int D = Fm::D, K = Fm::K, R = K - 1;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    uint64_t h0 = 0, h1 = 0;
#pragma unroll
    for (int u = 0; u < kSym; ++u) {
      const uint64_t key = S_ehc[(D + r) * kSym + u];
      h0 = nh_acc(h0, s.par0[r][u], key);
      h1 = nh_acc(h1, s.par1[r][u], key);
    }
#pragma unroll
    for (int t = 0; t < K; ++t) {
      s.z0[t] += mulc(Fm::T[t][D + r], h0);
      s.z1[t] += mulc(Fm::T[t][D + r], h1);
    }
  }
}

template <int WIDTH, int B>
__device__ __forceinline__ void ehc2_x(const uint4 (&x)[Family<WIDTH>::D * kSym], key_ptr S_ehc,
                                       uint64_t z0[], uint64_t z1[]) {
  Ehc<WIDTH> s;
  ehc_begin(s);
  ehc_blocks<WIDTH, 0, Family<WIDTH>::D * kSym>(s, x, S_ehc);
  ehc_end(s, S_ehc);
#pragma unroll
  for (int t = 0; t < Family<WIDTH>::K; ++t) {
    z0[t] = s.z0[t];
    z1[t] = s.z1[t];
  }
}

template <int WIDTH, int B>
__device__ __forceinline__ void ehc2(const uint8_t* __restrict__ eb, key_ptr S_ehc, uint64_t z0[], uint64_t z1[]) {
  uint4 x[Family<WIDTH>::D * kSym];
#pragma unroll
  for (int i = 0; i < Family<WIDTH>::D * kSym; ++i) x[i] = load16(eb + 8 * B * i);
  ehc2_x<WIDTH, B>(x, S_ehc, z0, z1);
}

// ---------------------------------------------------------------------------
// Planning kernels: tasks and cross-task accumulators per string.
// ---------------------------------------------------------------------------

// Strings of at most small_max executions get no task: tail-only strings (no
// execution) and small strings are listed apart, each kind hashed by a kernel
// of its own; tasks are counted from the executions of the other strings.
__device__ __forceinline__ uint64_t task_execs(uint64_t L, uint32_t exec_bytes, uint32_t small_max) {
  const uint64_t N = L / exec_bytes;
  return N <= small_max ? 0 : N;
}
__device__ __forceinline__ bool tail_only(uint64_t L, uint32_t exec_bytes, uint32_t direct_lim) {
  return L < exec_bytes && L >= direct_lim;
}
__device__ __forceinline__ bool small_string(uint64_t L, uint32_t exec_bytes, uint32_t small_max) {
  const uint64_t N = L / exec_bytes;
  return N >= 1 && N <= small_max;
}

// Per string and per candidate task size 2^pass_log2 * 8^j executions (a
// pass is 128 executions for b = 8, 256 for b = 4): number of tasks, and
// number of cross-task accumulators (complete nodes of levels >= j + 3).
// A tail-only string (N = 0) has no task: it is hashed from the tiny list,
// unless it is shorter than the planner's direct_lim (the composed 64-bit
// hash tabulates such strings itself; direct_lim is 0 for every other caller).
__device__ __forceinline__ void plan_counts(uint64_t N, int j, uint32_t pass_log2, uint64_t& tasks,
                                            uint64_t& accs) {
  const int shift = (int)pass_log2 + 3 * j;
  tasks = (N + (1ull << shift) - 1) >> shift;
  accs = 0;
  for (int l = j + 3; l < 22; ++l) {  // nodes per level shrink to zero
    const uint64_t n = nodes_at(N, l);
    if (!n) break;
    accs += n;
  }
}

// The smallest multiple of d > 0 that is at least x, for x < 2^53 (sums of
// string bytes): a double estimate of x / d, corrected exactly.
__device__ __forceinline__ uint64_t round_up_to(uint64_t x, uint64_t d, double inv_d) {
  uint64_t q = (uint64_t)((double)x * inv_d);
  while (q > 0 && q * d > x) --q;  // q = floor(x / d)
  while ((q + 1) * d <= x) ++q;
  return q * d == x ? x : (q + 1) * d;
}

constexpr int kPlanThreads = 256;
constexpr int kPlanPer = 4;
constexpr int kPlanBlock = kPlanThreads * kPlanPer;

constexpr int kPlanWaves = kPlanThreads / 64;
// Threads of a workgroup of the scan kernels of large plans.
constexpr int kScanThreads = 256;

// Sums of n values over a workgroup of NT threads, returned to every
// thread, with one pair of barriers for all of them.
template <int NV, int NT = kPlanThreads>
__device__ void block_sum_n(uint64_t (&v)[NV], uint64_t (*lds)[NV]) {
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v[k] += shfl_xor64(v[k], m);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[threadIdx.x >> 6][k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    uint64_t t = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += lds[i][k];
    v[k] = t;
  }
}

// Exclusive prefix sum of v over a workgroup of NT threads (thread order);
// `total` receives the workgroup's sum.
template <int NT = kPlanThreads>
__device__ uint64_t block_exclusive(uint64_t v, uint64_t* lds, uint64_t& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = shfl64(x, lane >= d ? lane - d : lane);
    if (lane >= d) x += y;
  }
  __syncthreads();
  if (lane == 63) lds[w] = x;
  __syncthreads();
  uint64_t before = 0;
  total = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    if (i < w) before += lds[i];
    total += lds[i];
  }
  return before + x - v;
}

// Exclusive prefix sums of NV values over a workgroup of NT threads (thread
// order), in place, with one pair of barriers; `total` receives the sums.
template <int NV, int NT = kPlanThreads>
__device__ void block_exclusive_n(uint64_t (&v)[NV], uint64_t (*lds)[NV], uint64_t (&total)[NV]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t x[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) x[k] = v[k];
#pragma unroll
  for (int d = 1; d < 64; d <<= 1)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const uint64_t y = shfl64(x[k], lane >= d ? lane - d : lane);
      if (lane >= d) x[k] += y;
    }
  __syncthreads();
  if (lane == 63)
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[w][k] = x[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    uint64_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
      if (i < w) before += lds[i][k];
      tot += lds[i][k];
    }
    v[k] = before + x[k] - v[k];
    total[k] = tot;
  }
}

// A thread's kPlanPer consecutive lengths from `base` (zero past count): in
// 16-byte loads when all are inside, so that a load instruction reads 1 KiB
// of consecutive lengths.
__device__ __forceinline__ void load_lengths(const uint64_t* __restrict__ lengths, uint64_t count, uint64_t base,
                                             uint64_t (&L)[kPlanPer]) {
  if (base + kPlanPer <= count) {
    __builtin_memcpy(L, lengths + base, 8 * kPlanPer);
  } else {
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i) L[i] = base + i < count ? lengths[base + i] : 0;
  }
}

// Planning step 1 for workgroup `blk`: per candidate task size, the tasks,
// accumulators and work of its kPlanBlock strings.
// `v` receives the workgroup's sums (every thread) and `L` this thread's
// lengths; the sums also go to column blk of block_sums unless it is null.
__device__ void plan_count_body(uint32_t blk, const uint64_t* __restrict__ lengths, uint64_t count,
                                uint32_t exec_bytes, uint32_t pass_log2, uint32_t direct_lim, uint32_t small_max,
                                uint64_t* __restrict__ block_sums, uint32_t* __restrict__ ctl,
                                uint64_t (&v)[kBlockSums], uint64_t (&L)[kPlanPer]) {
  __shared__ uint64_t lds[kPlanWaves][kBlockSums];
  __shared__ uint64_t lds1[kPlanWaves][2];
  // the fill kernel appends bucket leaders to this counter
  if (blk == 0 && threadIdx.x == 0) ctl[kCtlBuckets] = 0;
  const uint64_t base = (uint64_t)blk * kPlanBlock + threadIdx.x * kPlanPer;
  load_lengths(lengths, count, base, L);
  uint64_t N[kPlanPer];
  bool any = false;
#pragma unroll
  for (int i = 0; i < kPlanPer; ++i) {
    N[i] = task_execs(L[i], exec_bytes, small_max);
    any |= N[i] != 0;
  }
#pragma unroll
  for (int k = 0; k < kBlockSums; ++k) v[k] = 0;
  uint64_t tiny = 0, small = 0;
#pragma unroll
  for (int i = 0; i < kPlanPer; ++i) {
    tiny += base + i < count && tail_only(L[i], exec_bytes, direct_lim);
    small += base + i < count && small_string(L[i], exec_bytes, small_max);
  }
  // a block of listed strings only (common in batches of short keys) has no
  // tasks at any level: only its listed counts are summed
  if (!__syncthreads_or(any)) {
    uint64_t t1[2] = {tiny, small};
    block_sum_n(t1, lds1);
    v[kSumTiny] = t1[0];
    v[kSumSmall] = t1[1];
  } else {
#pragma unroll
    for (int j = 0; j < kPlanCandidates; ++j) {
      uint64_t t = 0, a = 0, w = 0;
#pragma unroll
      for (int i = 0; i < kPlanPer; ++i) {
        uint64_t ti, ai;
        plan_counts(N[i], j, pass_log2, ti, ai);
        t += ti;
        a += ai;
        w += ti ? L[i] + kTaskOverheadBytes * ti : 0;
      }
      v[j * kPlanSums + 0] = t;
      v[j * kPlanSums + 1] = a;
      v[j * kPlanSums + 2] = w;
    }
    v[kSumTiny] = tiny;
    v[kSumSmall] = small;
    block_sum_n(v, lds);
  }
  // (column-major, [kBlockSums][nblocks]: the steps that read a column over
  // many blocks read consecutive words)
  if (block_sums && threadIdx.x < kBlockSums) {
    uint64_t x = v[0];
    for (int k = 1; k < kBlockSums; ++k)
      if ((int)threadIdx.x == k) x = v[k];
    block_sums[(uint64_t)threadIdx.x * gridDim.x + blk] = x;
  }
}

// Task level and bucket size from the totals over every planner block;
// `write_ctl`: this thread also writes the launch's control words.  jsel < 0
// means that no task level fits the workspace (the launch does nothing).
__device__ void plan_choose(const uint64_t (&tot)[kBlockSums], uint64_t cap_tasks, uint64_t cap_accs,
                            uint32_t min_j, uint32_t max_j, uint64_t target_tasks, bool write_ctl,
                            uint32_t* __restrict__ ctl, int& jsel_out, uint64_t& bucket_out) {
  uint64_t tt[kPlanCandidates], ta[kPlanCandidates], tw[kPlanCandidates];
#pragma unroll
  for (int j = 0; j < kPlanCandidates; ++j) {
    tt[j] = tot[j * kPlanSums + 0];
    ta[j] = tot[j * kPlanSums + 1];
    tw[j] = tot[j * kPlanSums + 2];
  }
  // Task size: the coarsest level in [min_j, max_j] that still yields
  // target_tasks tasks (fewer cross-task merges, enough tasks to keep the
  // grid busy), else min_j; then coarser until the plan fits the workspace.
  // (unrolled over the candidates: constant register indices)
  int want = (int)min_j;
#pragma unroll
  for (int j = 0; j < kPlanCandidates; ++j)
    if (j >= (int)min_j && j <= (int)max_j && tt[j] >= target_tasks) want = j;
  int jsel = -1;
  uint64_t total_work = 0;
#pragma unroll
  for (int j = 0; j < kPlanCandidates; ++j)
    if (jsel < 0 && j >= want && tt[j] <= cap_tasks && ta[j] <= cap_accs) {
      jsel = j;
      total_work = tw[j];
    }
  // Buckets of about equal work: at most kMaxBuckets of `bucket` bytes.
  uint64_t bucket = (total_work + kMaxBuckets - 1) / kMaxBuckets;
  if (bucket < kMinBucketBytes) bucket = kMinBucketBytes;
  if (write_ctl) {
    ctl[kCtlNext] = 0;
    uint64_t ntasks = 0;
#pragma unroll
    for (int j = 0; j < kPlanCandidates; ++j)
      if (j == jsel) ntasks = tt[j];
    ctl[kCtlTotal] = (uint32_t)ntasks;
    ctl[kCtlLevel] = jsel >= 0 ? (uint32_t)jsel : 0;
    ctl[kCtlError] = jsel >= 0 ? 0 : 1;
    ctl[kCtlTiny] = jsel >= 0 ? (uint32_t)tot[kSumTiny] : 0;
    ctl[kCtlSmall] = jsel >= 0 ? (uint32_t)tot[kSumSmall] : 0;
    ctl[kCtlBucketLo] = (uint32_t)bucket;
    ctl[kCtlBucketHi] = (uint32_t)(bucket >> 32);
  }
  jsel_out = jsel;
  bucket_out = bucket;
}

// Planning step 2 for workgroup `blk` (after step 1 of every workgroup), in
// one of three modes:
//   kFillSum:    the workgroup sums the other blocks' step-1 results itself
//                (cost grows with the square of the block count: small plans);
//   kFillPre:    the scan kernel has chosen the task level and bucket size
//                (control words) and written each block's prefix;
//   kFillSingle: the only workgroup, right after its own step 1: the sums
//                and this thread's lengths come in `tot_in` and `len_in`, and
//                no other workgroup appends bucket leaders.
enum { kFillSum = 0, kFillPre = 1, kFillSingle = 2 };
template <int MODE>
__device__ void plan_fill_body(
    uint32_t blk, const uint64_t* __restrict__ lengths, uint64_t count, uint32_t exec_bytes, uint32_t pass_log2,
    uint32_t direct_lim, uint32_t small_max, const uint64_t* __restrict__ block_sums, uint32_t nblocks,
    const uint64_t* __restrict__ block_pre, const uint64_t (&tot_in)[kBlockSums],
    const uint64_t (&len_in)[kPlanPer], uint64_t cap_tasks, uint64_t cap_accs,
    uint32_t min_j, uint32_t max_j, uint64_t target_tasks, uint32_t* __restrict__ task_string,
    uint32_t* __restrict__ task_start, uint32_t* __restrict__ acc_start, uint32_t* __restrict__ bucket_lead,
    uint32_t* __restrict__ tiny_list, uint32_t* __restrict__ small_list, uint32_t* __restrict__ ctl) {
  __shared__ uint64_t lds[kPlanWaves];
  __shared__ uint64_t ldsn[kPlanWaves][kBlockSums];
  __shared__ uint64_t lds4[kPlanWaves][kPlanPre];
  __shared__ uint64_t lds2[kPlanWaves][2];
  __shared__ uint64_t lds3[kPlanWaves][kPlanSums];
  __shared__ uint32_t incl[kPlanBlock];
  __shared__ uint64_t wstart[kPlanBlock];
  __shared__ uint64_t slen[kPlanBlock];  // the block's lengths, for the task table
  const int tid = threadIdx.x;
  int jsel;
  uint64_t bucket;
  uint64_t pre[kPlanPre] = {0, 0, 0, 0, 0};
  if constexpr (MODE == kFillSingle) {
    plan_choose(tot_in, cap_tasks, cap_accs, min_j, max_j, target_tasks, tid == 0, ctl, jsel, bucket);
    if (jsel < 0) return;  // uniform over the workgroup
  } else if constexpr (MODE == kFillPre) {
    jsel = ctl[kCtlError] ? -1 : (int)ctl[kCtlLevel];
    bucket = (uint64_t)ctl[kCtlBucketLo] | (uint64_t)ctl[kCtlBucketHi] << 32;
    if (jsel < 0) return;  // uniform over the grid
    // a block with no task and no listed string writes nothing (batches of
    // keys short enough for the composed hash's direct path): its lengths
    // are not read again
    if (!(block_sums[(uint64_t)(jsel * kPlanSums) * nblocks + blk] | block_sums[(uint64_t)kSumTiny * nblocks + blk] |
          block_sums[(uint64_t)kSumSmall * nblocks + blk]))
      return;  // uniform over the workgroup
#pragma unroll
    for (int k = 0; k < kPlanPre; ++k) pre[k] = block_pre[(uint64_t)k * nblocks + blk];
  } else {
    // Totals of every candidate over all blocks (threads stride over blocks).
    uint64_t tot[kBlockSums];
#pragma unroll
    for (int k = 0; k < kBlockSums; ++k) tot[k] = 0;
    for (uint32_t b = tid; b < nblocks; b += kPlanThreads)
#pragma unroll
      for (int k = 0; k < kBlockSums; ++k) tot[k] += block_sums[(uint64_t)k * nblocks + b];
    block_sum_n(tot, ldsn);
    plan_choose(tot, cap_tasks, cap_accs, min_j, max_j, target_tasks, blk == 0 && tid == 0, ctl, jsel, bucket);
    if (jsel < 0) return;  // uniform over the grid
    // Tasks, accumulators, work and tail-only strings of the blocks before this one.
    for (uint32_t b = tid; b < blk; b += kPlanThreads) {
#pragma unroll
      for (int k = 0; k < kPlanSums; ++k) pre[k] += block_sums[(uint64_t)(jsel * kPlanSums + k) * nblocks + b];
      pre[kPlanSums] += block_sums[(uint64_t)kSumTiny * nblocks + b];
      pre[kPlanSums + 1] += block_sums[(uint64_t)kSumSmall * nblocks + b];
    }
    block_sum_n(pre, lds4);
  }
  const uint64_t task_base = pre[0];
  const uint64_t acc_base = pre[1];
  const uint64_t work_base = pre[2];
  const uint64_t tiny_base = pre[3];
  const uint64_t small_base = pre[4];

  const uint64_t base = (uint64_t)blk * kPlanBlock + tid * kPlanPer;
  uint64_t Ls[kPlanPer];
  if constexpr (MODE == kFillSingle) {
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i) Ls[i] = len_in[i];
  } else {
    load_lengths(lengths, count, base, Ls);
  }
  uint64_t tk[kPlanPer], ac[kPlanPer], wk[kPlanPer];
  uint64_t st = 0, sa = 0, sw = 0, sy = 0, sm = 0;
  bool tiny[kPlanPer], small[kPlanPer];
#pragma unroll
  for (int i = 0; i < kPlanPer; ++i) {
    tk[i] = ac[i] = wk[i] = 0;
    tiny[i] = small[i] = false;
    if (base + i < count) {
      const uint64_t L = Ls[i];
      slen[tid * kPlanPer + i] = L;
      plan_counts(task_execs(L, exec_bytes, small_max), jsel, pass_log2, tk[i], ac[i]);
      wk[i] = tk[i] ? L + kTaskOverheadBytes * tk[i] : 0;
      tiny[i] = tail_only(L, exec_bytes, direct_lim);
      small[i] = small_string(L, exec_bytes, small_max);
    }
    st += tk[i];
    sa += ac[i];
    sw += wk[i];
    sy += tiny[i];
    sm += small[i];
  }
  const bool any = __syncthreads_or(st != 0) != 0;
  uint64_t lst[2] = {sy, sm}, blk_l[2];
  block_exclusive_n(lst, lds2, blk_l);
  uint64_t ty = tiny_base + lst[0], tm = small_base + lst[1];
#pragma unroll
  for (int i = 0; i < kPlanPer; ++i) {
    if (tiny[i]) tiny_list[ty++] = (uint32_t)(base + i);
    if (small[i]) small_list[tm++] = (uint32_t)(base + i);
  }
  // a block without tasks (tail-only strings) is done: no task table
  // entries, offsets or bucket leaders (uniform over the workgroup)
  if (!any) return;
  uint64_t ex[kPlanSums] = {st, sa, sw}, blk_tot[kPlanSums];
  block_exclusive_n(ex, lds3, blk_tot);
  const uint64_t et = ex[0], blk_t = blk_tot[0];
  uint64_t run_t = task_base + et, run_a = acc_base + ex[1], run_w = work_base + ex[2];
  uint64_t loc = et;
#pragma unroll
  for (int i = 0; i < kPlanPer; ++i) {
    if (tk[i]) {  // read only for strings with tasks
      task_start[base + i] = (uint32_t)run_t;
      acc_start[base + i] = (uint32_t)run_a;
    }
    wstart[tid * kPlanPer + i] = run_w;  // work before this string
    run_t += tk[i];
    run_a += ac[i];
    run_w += wk[i];
    loc += tk[i];
    incl[tid * kPlanPer + i] = (uint32_t)loc;  // inclusive task count inside the block
  }
  __syncthreads();
  // Fill the task -> string table for this block's tasks.  A task leads a
  // bucket when a bucket boundary k * bucket falls inside its work
  // [start, end): the buckets are the runs of tasks from one leader to the
  // next, so none is empty and there are at most as many as boundaries.
  // Leaders carry bit 31 in the table and are appended to bucket_lead (in no
  // particular order) with one atomic per workgroup.
  const uint64_t first = (uint64_t)blk * kPlanBlock;
  const int nstr = (int)((count - first) < (uint64_t)kPlanBlock ? (count - first) : kPlanBlock);
  const uint64_t texec = 1ull << (pass_log2 + 3 * jsel);
  const uint64_t unit = texec * exec_bytes + kTaskOverheadBytes;  // work of a full task
  // Each thread fills a contiguous run of the block's tasks: the string of
  // its first task is found once, then only moves forward.
  const uint64_t per = (blk_t + kPlanThreads - 1) / kPlanThreads;
  const uint64_t e_lo = (uint64_t)tid * per < blk_t ? (uint64_t)tid * per : blk_t;
  const uint64_t e_hi = e_lo + per < blk_t ? e_lo + per : blk_t;
  const int tshift = (int)pass_log2 + 3 * jsel;  // log2 of a full task's executions
  const double inv_bucket = 1.0 / (double)bucket;
  uint32_t nlead = 0;
  uint64_t leads = 0;  // lead flags of this thread's first 64 tasks (bit k: task e_lo + k)
  if (e_lo < e_hi) {
    // first string whose inclusive count exceeds e_lo: the guess from the
    // average tasks per string (exact when the block's strings have equal
    // task counts), else a binary search
    int lo = (int)(e_lo * (uint64_t)nstr / blk_t);
    if (!((uint64_t)incl[lo] > e_lo && (lo == 0 || (uint64_t)incl[lo - 1] <= e_lo))) {
      lo = 0;
      int hi = nstr - 1;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((uint64_t)incl[mid] > e_lo) hi = mid;
        else lo = mid + 1;
      }
    }
    uint64_t before = lo > 0 ? incl[lo - 1] : 0;  // tasks of the block's strings before string lo
    uint64_t L = slen[lo];
    uint64_t ntk = (L / exec_bytes + (1ull << tshift) - 1) >> tshift;
    for (uint64_t e = e_lo; e < e_hi; ++e) {
      while ((uint64_t)incl[lo] <= e) {  // on to the next string with tasks
        before = incl[lo];
        ++lo;
        L = slen[lo];
        ntk = (L / exec_bytes + (1ull << tshift) - 1) >> tshift;
      }
      const uint64_t task = task_base + e;
      const uint64_t tau = e - before;
      const uint64_t w0 = wstart[lo] + tau * unit;
      const uint64_t w1 = tau + 1 < ntk ? w0 + unit : wstart[lo] + L + kTaskOverheadBytes * ntk;
      const bool lead = round_up_to(w0, bucket, inv_bucket) < w1;
      task_string[task] = (uint32_t)(first + lo) | (lead ? 0x80000000u : 0u);
      nlead += lead;
      if (lead && e - e_lo < 64) leads |= 1ull << (e - e_lo);
    }
  }
  // positions in bucket_lead: one atomic per workgroup (none when it is the
  // only one)
  uint64_t blk_lead;
  const uint64_t before = block_exclusive(nlead, lds, blk_lead);
  __shared__ uint32_t lead_base;
  if (tid == 0) {
    if constexpr (MODE == kFillSingle) {
      lead_base = 0;
      ctl[kCtlBuckets] = (uint32_t)blk_lead;
    } else {
      lead_base = blk_lead ? atomicAdd(ctl + kCtlBuckets, (uint32_t)blk_lead) : 0;
    }
  }
  __syncthreads();
  // this thread's leaders, in task order (flags past its 64th task read
  // back from the table it wrote)
  uint32_t at = lead_base + (uint32_t)before;
  if (nlead) {
    for (uint64_t e = e_lo; e < e_hi; ++e) {
      const uint64_t task = task_base + e;
      if (e - e_lo < 64 ? (leads >> (e - e_lo)) & 1 : task_string[task] >> 31) bucket_lead[at++] = (uint32_t)task;
    }
  }
}


__global__ __launch_bounds__(kPlanThreads) void plan_count_kernel(const uint64_t* __restrict__ lengths,
                                                                  uint64_t count, uint32_t exec_bytes,
                                                                  uint32_t pass_log2, uint32_t direct_lim,
                                                                  uint32_t small_max,
                                                                  uint64_t* __restrict__ block_sums,
                                                                  uint32_t* __restrict__ ctl) {
  uint64_t v[kBlockSums], L[kPlanPer];
  plan_count_body(blockIdx.x, lengths, count, exec_bytes, pass_log2, direct_lim, small_max, block_sums, ctl, v, L);
}

// Large plans, between the two steps, in two launches of one workgroup per
// run of blocks (at most kScanGroups runs of at least kScanGroupMin blocks):
// the first sums each run's step-1 results (group_sums, column-major
// [kBlockSums][ngroups]); in the second every workgroup sums the runs (the
// totals, the same in each), chooses the task level and bucket size
// (workgroup 0 writes the control words), adds the runs before its own for
// its exclusive prefix, and writes the prefixes of tasks, accumulators,
// work, tail-only and small strings of its run's blocks, kScanThreads
// blocks per round.  (One workgroup over every block took 72 us for 16,384
// blocks: a single workgroup is bound by its round trips, not by bytes.)
__device__ __forceinline__ void scan_run(uint32_t nblocks, uint32_t ngroups, uint32_t g, uint32_t& r0, uint32_t& r1) {
  const uint32_t per = (nblocks + ngroups - 1) / ngroups;
  r0 = g * per < nblocks ? g * per : nblocks;
  r1 = r0 + per < nblocks ? r0 + per : nblocks;
}

__global__ __launch_bounds__(kScanThreads) void plan_group_kernel(const uint64_t* __restrict__ block_sums,
                                                                  uint32_t nblocks,
                                                                  uint64_t* __restrict__ group_sums) {
  __shared__ uint64_t ldsn[kScanThreads / 64][kBlockSums];
  uint32_t r0, r1;
  scan_run(nblocks, gridDim.x, blockIdx.x, r0, r1);
  uint64_t tot[kBlockSums];
#pragma unroll
  for (int k = 0; k < kBlockSums; ++k) tot[k] = 0;
  for (uint32_t b = r0 + threadIdx.x; b < r1; b += kScanThreads)
#pragma unroll
    for (int k = 0; k < kBlockSums; ++k) tot[k] += block_sums[(uint64_t)k * nblocks + b];
  block_sum_n<kBlockSums, kScanThreads>(tot, ldsn);
  if (threadIdx.x < kBlockSums) {
    uint64_t x = tot[0];
#pragma unroll
    for (int k = 1; k < kBlockSums; ++k)
      if ((int)threadIdx.x == k) x = tot[k];
    group_sums[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x] = x;
  }
}

__global__ __launch_bounds__(kScanThreads) void plan_prefix_kernel(
    const uint64_t* __restrict__ block_sums, uint32_t nblocks, const uint64_t* __restrict__ group_sums,
    uint64_t cap_tasks, uint64_t cap_accs, uint32_t min_j, uint32_t max_j, uint64_t target_tasks,
    uint64_t* __restrict__ block_pre, uint32_t* __restrict__ ctl) {
  constexpr int NP = kPlanPre;
  __shared__ uint64_t ldsn[kScanThreads / 64][kBlockSums];
  __shared__ uint64_t ldsp[kScanThreads / 64][NP];
  __shared__ uint64_t ldsx[kScanThreads / 64][NP];
  const uint32_t ngroups = gridDim.x, g = blockIdx.x;
  // totals over every run (the runs' sums are few: one load per thread)
  uint64_t tot[kBlockSums];
#pragma unroll
  for (int k = 0; k < kBlockSums; ++k) tot[k] = 0;
  for (uint32_t i = threadIdx.x; i < ngroups; i += kScanThreads)
#pragma unroll
    for (int k = 0; k < kBlockSums; ++k) tot[k] += group_sums[(uint64_t)k * ngroups + i];
  block_sum_n<kBlockSums, kScanThreads>(tot, ldsn);
  int jsel;
  uint64_t bucket;
  plan_choose(tot, cap_tasks, cap_accs, min_j, max_j, target_tasks, g == 0 && threadIdx.x == 0, ctl, jsel, bucket);
  if (jsel < 0) return;  // uniform over the grid
  int col[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) col[k] = k < kPlanSums ? jsel * kPlanSums + k : k == kPlanSums ? kSumTiny : kSumSmall;
  // the runs before this one
  uint64_t pre[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) pre[k] = 0;
  for (uint32_t i = threadIdx.x; i < g; i += kScanThreads)
#pragma unroll
    for (int k = 0; k < NP; ++k) pre[k] += group_sums[(uint64_t)col[k] * ngroups + i];
  block_sum_n<NP, kScanThreads>(pre, ldsp);
  uint32_t r0, r1;
  scan_run(nblocks, ngroups, g, r0, r1);
  for (uint32_t b0 = r0; b0 < r1; b0 += kScanThreads) {  // uniform over the workgroup
    const uint32_t b = b0 + threadIdx.x;
    uint64_t x[NP], run[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) x[k] = b < r1 ? block_sums[(uint64_t)col[k] * nblocks + b] : 0;
    block_exclusive_n<NP, kScanThreads>(x, ldsx, run);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      if (b < r1) block_pre[(uint64_t)k * nblocks + b] = pre[k] + x[k];
      pre[k] += run[k];
    }
  }
}

template <bool PRE>
__global__ __launch_bounds__(kPlanThreads) void plan_fill_kernel(
    const uint64_t* __restrict__ lengths, uint64_t count, uint32_t exec_bytes, uint32_t pass_log2,
    uint32_t direct_lim, uint32_t small_max, const uint64_t* __restrict__ block_sums, uint32_t nblocks,
    const uint64_t* __restrict__ block_pre, uint64_t cap_tasks, uint64_t cap_accs,
    uint32_t min_j, uint32_t max_j, uint64_t target_tasks, uint32_t* __restrict__ task_string,
    uint32_t* __restrict__ task_start, uint32_t* __restrict__ acc_start, uint32_t* __restrict__ bucket_lead,
    uint32_t* __restrict__ tiny_list, uint32_t* __restrict__ small_list, uint32_t* __restrict__ ctl) {
  const uint64_t none[kBlockSums] = {}, none_l[kPlanPer] = {};
  plan_fill_body<PRE ? kFillPre : kFillSum>(blockIdx.x, lengths, count, exec_bytes, pass_log2, direct_lim,
                                            small_max, block_sums,
                                            nblocks, block_pre, none, none_l, cap_tasks, cap_accs, min_j, max_j,
                 target_tasks, task_string, task_start, acc_start, bucket_lead, tiny_list, small_list, ctl);
}

// Both steps in one workgroup, for batches of at most kPlanBlock strings
// (one launch instead of two): step 2 takes step 1's sums and lengths from
// registers (nothing goes through block_sums).
__global__ __launch_bounds__(kPlanThreads) void plan_single_kernel(
    const uint64_t* __restrict__ lengths, uint64_t count, uint32_t exec_bytes, uint32_t pass_log2,
    uint32_t direct_lim, uint32_t small_max, uint64_t cap_tasks, uint64_t cap_accs, uint32_t min_j, uint32_t max_j,
    uint64_t target_tasks,
    uint32_t* __restrict__ task_string, uint32_t* __restrict__ task_start, uint32_t* __restrict__ acc_start,
    uint32_t* __restrict__ bucket_lead, uint32_t* __restrict__ tiny_list, uint32_t* __restrict__ small_list,
    uint32_t* __restrict__ ctl) {
  uint64_t v[kBlockSums], L[kPlanPer];
  plan_count_body(0, lengths, count, exec_bytes, pass_log2, direct_lim, small_max, nullptr, ctl, v, L);
  plan_fill_body<kFillSingle>(0, lengths, count, exec_bytes, pass_log2, direct_lim, small_max, nullptr, 1, nullptr,
                              v, L,
                              cap_tasks, cap_accs, min_j, max_j, target_tasks, task_string, task_start, acc_start,
                              bucket_lead, tiny_list, small_list, ctl);
}

// ---------------------------------------------------------------------------
// Main kernel.
// ---------------------------------------------------------------------------

// Local accumulators for parents inside a task: levels 3 .. 3 + kMaxLocal - 1.
constexpr int kMaxLocal = kPlanCandidates;

// Lane geometry for blocks of B words.  A lane reads 16 bytes (instances 2r
// and 2r + 1) of each block, so a block takes LPB = B / 2 lanes and a wave
// has G = 64 / LPB lane groups; each lane group works through 8 consecutive
// executions (one level-1 node) per pass, so a pass is PASS = 8 G executions
// and holds NG2 = G / 8 level-2 nodes.
template <int B>
struct Geo {
  static constexpr int LPB = B / 2;
  static constexpr int G = 64 / LPB;
  static constexpr int PASS = 8 * G;
  static constexpr int NG2 = G / 8;
  static constexpr int LOG_PASS = B == 8 ? 7 : 8;
  static_assert(B == 4 || B == 8, "block size");
  static_assert(PASS == 1 << LOG_PASS, "pass size");
};

// Staging of executions in LDS.  A wave hashes a region of G executions at a
// time (one per lane group: G * XB bytes), staged in LDS in two parts: part A
// holds the first blocks of every execution, part B the rest.  A part is
// copied from HBM with 16-byte direct-to-LDS loads, non-temporal (the bytes
// are read once); then every lane reads its instance pair of its execution's
// blocks of the part back into registers, and the next part's copy is issued
// before those blocks are hashed: part B of the same region while part A is
// hashed, part A of the next region while part B is.  A wave's loads are thus
// in flight while it computes, without holding registers, and its buffer
// holds one part, so that enough waves fit in a compute unit's LDS.  Each load
// instruction fills 1 KiB of the image and its lanes read runs of contiguous
// bytes (the part of one execution): the direct pattern, 16 half-lines of 16
// executions per load instruction, reaches a lower HBM rate.
//
// Part A of an execution ends at a 128-byte line boundary of its address when
// one lies near the middle (the execution starts at a multiple of the block
// size): blocks 0 .. cA-1 with cA = C0 + shift, shift < LB (LB blocks per
// line).  A line split between the parts would be fetched from HBM twice
// (non-temporal lines do not stay in the L2 until the second part's copy).
// The registers stay static: a lane reads blocks 0 .. C0+LB-2 of part A's
// slot and blocks C0 .. XB/8B-1 of part B's slot (part B's slot starts at block
// C0; blocks below cA are not copied there) and takes each of the blocks
// C0 .. C0+LB-2 from whichever part copied it.  The EHC is fed block by block
// (ehc_blocks), so the split may fall inside an item.  In the image,
// execution q of the region takes a slot of an odd number of blocks (padded),
// so that the lane groups reading one block of consecutive executions in one
// LDS access fall into different banks.
//
// In a full pass, lane group q hashes executions p + 8q + e in regions e = 0 ..
// 7, so execution g + 1 follows execution g in the same lane's next region.
// When g ends inside a line, part B also copies the blocks of g + 1 that
// complete the line (cout of them), the lane keeps them in registers and the
// next region's part A skips them (cin), so that line is fetched once too.
typedef __attribute__((address_space(3))) void* lds_void_ptr;
typedef __attribute__((address_space(3))) uint8_t lds_u8;  // the buffer, as an LDS pointer
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(3))) u32x4 lds_u4;
typedef const __attribute__((address_space(3))) uint32_t lds_u32;
constexpr int kLoadNT = 2;  // cache policy of the copies: non-temporal

template <int WIDTH, int B>
struct Parts {
  static constexpr int BB = 8 * B;                       // bytes per block
  static constexpr int LB = 128 / BB;                    // blocks per 128-byte line
  static constexpr int NBLK = Family<WIDTH>::D * kSym;   // blocks per execution
  static constexpr int C0 = (NBLK - LB + 2) / 2;         // part A has C0 .. C0+LB-1 blocks
  static constexpr int LX = LB - 1;                      // blocks that may move between parts
  static constexpr int NA = C0 + LX;                     // blocks read from part A's slot
  static constexpr int NB = NBLK - C0 + LX;              // blocks read from part B's slot (with
                                                         // the successor's first blocks)
  static constexpr int slot(int nb) { return nb % 2 ? nb : nb + 1; }
  static constexpr int SA = slot(NA), SB = slot(NB);     // blocks per execution slot
  static constexpr int BYTES = 1024 * (SA > SB ? SA : SB);  // G * slot * BB: the buffer
  static_assert(Geo<B>::G * BB == 1024, "a region's block row is one 1 KiB load");
  static_assert(NA <= NBLK && NB - LX >= LB, "parts");
};

// Blocks from address `at` up to the next line boundary (0 when `at` is not
// at a block boundary: then every block straddles two lines anyway).
template <int B>
__device__ __forceinline__ uint32_t blocks_to_line(const uint8_t* at) {
  constexpr uint32_t BB = 8 * B;
  const uint32_t a = (uint32_t)reinterpret_cast<uintptr_t>(at) & 127u;
  return a % BB ? 0 : ((128u - a) % 128u) / BB;
}

// Blocks of part A of the execution at address `at`: C0 plus the blocks up to
// the next line boundary, when the execution starts at a block boundary.
template <int WIDTH, int B>
__device__ __forceinline__ uint32_t part_a_blocks(const uint8_t* at) {
  using P = Parts<WIDTH, B>;
  const uint32_t a = (uint32_t)reinterpret_cast<uintptr_t>(at) & 127u;
  if (a % P::BB) return P::C0;
  return P::C0 + ((128u - (a + P::BB * P::C0) % 128u) % 128u) / P::BB;
}

// This lane's index, opaque to the compiler: per-lane addresses derived from it
// are recomputed where they are used instead of being hoisted out of the task
// loop and held in registers for the whole kernel (which spilled).
__device__ __forceinline__ uint32_t opaque_lane() {
  uint32_t l = threadIdx.x;
  asm volatile("" : "+v"(l));
  return l;
}

// Waits for this wave's outstanding vector memory operations (the copies into
// LDS among them: vmcnt(0)), or for its LDS reads and scalar loads
// (lgkmcnt(0)); the other counters are left at their maximum (gfx9 encoding:
// vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).  The compiler
// schedules no memory operation across either wait, and values already in
// registers (the keys) stay there.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }
__device__ __forceinline__ void wait_lgkm() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Copy one part of the first nq executions of a region (execution q at base +
// q * qs in HBM) into slots of S blocks.  Part A: blocks lo .. cA-1 (lo = cin
// blocks already in registers) to slot positions lo ..; part B: blocks cA ..
// NBLK-1+cout (the last cout of them the successor's, contiguous in HBM) to
// slot positions cA - C0 ..  Padding, blocks of the other part and executions
// past nq are not copied.  UNI: a full pass's region, whose G executions lie
// a multiple of 128 bytes apart (same line alignment, one cA for all).
//
// The copies read from 4-byte-aligned addresses: when the executions start sh
// = base mod 4 bytes past a 4-byte boundary (the same sh for all: they lie
// multiples of 64 bytes apart), slot byte w holds execution byte w - sh of the
// part, one more piece is copied at the part's end, and read_slot shifts the
// bytes back into place.  (A direct-to-LDS copy from an address that is not a
// multiple of 4 costs far more than one from an aligned address, and so does
// an LDS read at such an offset: strings packed back to back took 1.18-1.20
// ms either way where the same strings on 8-byte boundaries took 1.03.)  Only
// part A copies the extra piece: its bytes are the execution's own (part B
// follows), while past part B may lie the end of the string and of its
// allocation's last page; part B's last word is loaded into a register
// instead (region_ehc).  So every piece copied holds only words that hold
// bytes of the executions.  Such strings start mid-block, so cA = C0 and no
// blocks are carried (cin = cout = 0), and the slots' padding (at least one
// block past each part) holds the extra piece.
template <int WIDTH, int B, bool PART_B, bool UNI>
__device__ __forceinline__ void stage_part(const uint8_t* __restrict__ base, uint32_t qs, uint32_t nq,
                                           uint32_t cnt, lds_u8* stage) {
  using P = Parts<WIDTH, B>;
  constexpr uint32_t S = PART_B ? P::SB : P::SA;
  constexpr uint32_t SLOT = S * P::BB;
  constexpr uint32_t FIRST = PART_B ? P::C0 : 0;  // block at slot position 0
  // copied bytes of a slot: [wlo, whi) (uniform when UNI)
  const uint32_t ca_u = UNI ? part_a_blocks<WIDTH, B>(base) : 0;
  const uint32_t sh = (uint32_t)reinterpret_cast<uintptr_t>(base) & 3u;  // (uniform)
  const uint8_t* const abase = base - sh;
  const uint32_t wext = sh && !PART_B ? 16u : 0u;
  const uint32_t lane = opaque_lane();
#pragma unroll
  for (int i = 0; i < (int)S; ++i) {
    const uint32_t o = 1024u * i + 16u * lane;
    const uint32_t q = o / SLOT, w = o - q * SLOT;
    const uint32_t ca = UNI ? ca_u : part_a_blocks<WIDTH, B>(base + q * qs);
    const uint32_t wlo = (PART_B ? ca - P::C0 : cnt) * P::BB;
    const uint32_t whi = PART_B ? (P::NBLK - P::C0 + cnt) * P::BB : ca * P::BB;
    if (w >= wlo && w < whi + wext && (UNI || q < nq))
      __builtin_amdgcn_global_load_lds((const void*)(abase + (q * qs + FIRST * P::BB + w)),
                                       (lds_void_ptr)(stage + 1024 * i), 16, 0, kLoadNT);
  }
}

// This lane's instance pair of N blocks of its execution's slot (S blocks),
// whose bytes start sh < 4 bytes into the slot (see stage_part): an aligned
// 16-byte read and the next word, shifted right by sh bytes (bytes read past
// the slot's copied ones are not used; the stage buffer has a guard word
// past its last slot).  KLAST >= 0: the word after block KLAST of the lane
// group's last lane is `elast` (loaded from HBM: the slot holds no copy).
template <int B, int N, int S, int KLAST = -1>
__device__ __forceinline__ void read_slot(const lds_u8* stage, uint32_t sh, uint4 (&x)[N], uint32_t elast = 0) {
  const uint32_t lane = opaque_lane();
  const int q = lane / Geo<B>::LPB, r = lane % Geo<B>::LPB;
  const lds_u8* at = stage + q * (S * 8 * B) + 16 * r;
  if (sh == 0) {  // (uniform) aligned strings: one read per block
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const u32x4 v = *(lds_u4*)(at + 8 * B * k);
      x[k] = make_uint4(v.x, v.y, v.z, v.w);
    }
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const u32x4 v = *(lds_u4*)(at + 8 * B * k);
      uint32_t e = *(lds_u32*)(at + 8 * B * k + 16);
      if (k == KLAST && r == Geo<B>::LPB - 1) e = elast;
      x[k] = make_uint4(__builtin_amdgcn_alignbyte(v.y, v.x, sh), __builtin_amdgcn_alignbyte(v.z, v.y, sh),
                        __builtin_amdgcn_alignbyte(v.w, v.z, sh), __builtin_amdgcn_alignbyte(e, v.w, sh));
    }
  }
}

// Part A of the region whose execution q starts at base + q * qs (nq
// executions), without its first cin blocks.
template <int WIDTH, int B>
__device__ __forceinline__ void stage_first(const uint8_t* base, uint32_t qs, uint32_t nq, uint32_t cin,
                                            lds_u8* stage) {
  if (qs == 8u * Layout<WIDTH, B>::exec_bytes)
    stage_part<WIDTH, B, false, true>(base, qs, nq, cin, stage);
  else
    stage_part<WIDTH, B, false, false>(base, qs, nq, cin, stage);
}

// Blocks of a full pass's region e that complete the last line of each of its
// executions (copied with the region, kept for region e + 1).
template <int WIDTH, int B>
__device__ __forceinline__ uint32_t carry_blocks(const uint8_t* str, uint64_t p, int e) {
  constexpr uint64_t XB = Layout<WIDTH, B>::exec_bytes;
  // (b = 4: up to three blocks of 32 bytes stay in registers; the kernels
  // fit them without spilling, 206-254 VGPRs)
  return e < 7 ? blocks_to_line<B>(str + (p + e + 1) * XB) : 0;  // (uniform over the region)
}

// EHC of this lane's execution of a region whose part A is being copied (as
// stage_first, skipping cin blocks that are in xc); part B also copies the
// first cout blocks of every execution's successor, which go to xc for the
// next region.  `next` is the next region (part A skipping ncin blocks, or
// whole), copied while part B of this one is hashed.  Lanes whose
// execution is past nq hash stale bytes (their results are not used).  Called
// by the whole wave; cin, cout, ncin uniform, at most LB - 1.  UNI: a full
// pass's region (see stage_part).  `hook` (when call_hook, uniform) runs once
// part A has been read and part B's copy issued.
struct NextStage;
template <int WIDTH, int B>
__device__ __forceinline__ void stage_issue(const NextStage& n, uint32_t cin, lds_u8* stage);

struct NoHook {
  __device__ void operator()() const {}
};

template <int WIDTH, int B, bool UNI, class Hook = NoHook>
__device__ __forceinline__ void region_ehc(lds_u8* stage, const uint8_t* base, uint32_t qs, uint32_t nq,
                                           uint32_t cin, uint32_t cout, const NextStage& next, uint32_t ncin,
                                           uint4 (&xc)[Parts<WIDTH, B>::LX > 0 ? Parts<WIDTH, B>::LX : 1],
                                           key_ptr S_ehc, uint64_t z0[], uint64_t z1[], const Hook& hook = Hook(),
                                           bool call_hook = false) {
  using P = Parts<WIDTH, B>;
  constexpr int LX = P::LX;  // blocks C0 .. C0+LX-1 may come from either part
  Ehc<WIDTH> s;
  ehc_begin(s);
  const uint32_t ca = part_a_blocks<WIDTH, B>(base + (opaque_lane() / Geo<B>::LPB) * qs);
  const uint32_t sh = (uint32_t)reinterpret_cast<uintptr_t>(base) & 3u;
  uint4 xe[LX > 0 ? LX : 1];  // part A's copies of blocks C0 .. C0+LX-1
  uint32_t eb = 0;             // (sh > 0) the word holding the execution's last bytes
  {
    uint4 x[P::NA];
    wait_vm();
    read_slot<B, P::NA, P::SA>(stage, sh, x);
    wait_lgkm();
    stage_part<WIDTH, B, true, UNI>(base, qs, nq, cout, stage);
    if (sh) {  // (uniform) read by the lane that shifts the last block's bytes
      const uint32_t l = opaque_lane(), q = l / Geo<B>::LPB;
      if (l % Geo<B>::LPB == Geo<B>::LPB - 1 && (UNI || q < nq))
        eb = *reinterpret_cast<const uint32_t*>(base - sh + q * qs + P::NBLK * P::BB);
    }
    if (call_hook) hook();  // (e.g. the string's tail loads, in flight with part B)
#pragma unroll
    for (int k = 0; k < LX; ++k) xe[k] = x[P::C0 + k];
#pragma unroll
    for (int k = 0; k < LX; ++k)
      if ((uint32_t)k < cin) x[k] = xc[k];
    ehc_blocks<WIDTH, 0, P::C0>(s, x, S_ehc);
  }
  {
    uint4 x[P::NB];
    wait_vm();
    read_slot<B, P::NB, P::SB, P::NBLK - P::C0 - 1>(stage, sh, x, eb);
    wait_lgkm();
    stage_issue<WIDTH, B>(next, ncin, stage);
#pragma unroll
    for (int k = 0; k < LX; ++k) {
      if ((uint32_t)(P::C0 + k) < ca) x[k] = xe[k];
      xc[k] = x[P::NB - LX + k];
    }
    ehc_blocks<WIDTH, P::C0, P::NBLK>(s, x, S_ehc);
  }
  ehc_end(s, S_ehc);
#pragma unroll
  for (int t = 0; t < Family<WIDTH>::K; ++t) {
    z0[t] = s.z0[t];
    z1[t] = s.z1[t];
  }
}

// A region to copy next: nq executions (0: nothing), execution q at base + q
// * qs.
struct NextStage {
  const uint8_t* base;
  uint32_t qs;
  uint32_t nq;
};

// Issue the copy of region n (part A, skipping cin blocks in registers).
// Uniform.
template <int WIDTH, int B>
__device__ __forceinline__ void stage_issue(const NextStage& n, uint32_t cin, lds_u8* stage) {
  if (n.nq) stage_first<WIDTH, B>(n.base, n.qs, n.nq, cin, stage);
}

// The first region of a task hashing executions g0 .. of a string of N
// executions at str: a full pass's first region, or the first region of its
// last, partial pass.
template <int WIDTH, int B>
__device__ __forceinline__ NextStage first_region(const uint8_t* str, uint64_t L, uint64_t g0) {
  using Gm = Geo<B>;
  constexpr uint64_t XB = Layout<WIDTH, B>::exec_bytes;
  const uint64_t N = L / XB;
  if (N - g0 >= (uint64_t)Gm::PASS) return {str + g0 * XB, 8 * (uint32_t)XB, (uint32_t)Gm::G};
  const uint32_t nv = (uint32_t)(N - g0);
  return {str + g0 * XB, (uint32_t)XB, nv < (uint32_t)Gm::G ? nv : (uint32_t)Gm::G};
}

// The task after the current one in its bucket, when its string's metadata
// has been read (no bucket boundary in between): its first region is copied
// while the current task's last region is hashed.  The region is worked out
// only there, so that the metadata loads are not waited for earlier.
struct TaskNext {
  bool have;
  const uint8_t* bytes;
  uint64_t off, L, tau, texec;
};

template <int WIDTH, int B>
__device__ __forceinline__ NextStage task_next_region(const TaskNext& t) {
  if (!t.have) return {nullptr, 0, 0};
  return first_region<WIDTH, B>(t.bytes + t.off, t.L, t.tau * t.texec);
}

template <int WIDTH>
struct Ctx {
  static constexpr int K = Family<WIDTH>::K;
  const uint64_t* __restrict__ ent;
  uint64_t N;
  uint32_t j;  // task size PASS * 8^j executions
  uint64_t acc_base;
  uint64_t* gacc;
  uint32_t* gcnt;
  uint64_t* roots;  // root mode: this string's root node, [K][8] words
  // LDS copies (per wave) of the keys of tree levels 0 and 1: tree keys
  // [t][l * 7 + pos], final keys [t][(l * 7 + pos) * B + j]
  const uint64_t* ltree;
  const uint64_t* lfin;
};

// Offset of the accumulator of node `parent` at level l among one string's
// cross-task accumulators (levels j + 3 and up, complete nodes only).
__device__ __forceinline__ uint64_t acc_index(uint64_t N, uint32_t j, int l, uint64_t parent) {
  uint64_t off = 0;
  for (int m = (int)j + 3; m < l; ++m) off += nodes_at(N, m);
  return off + parent;
}

// Fold one complete node of level l (index n within the string), held by
// lanes 0 .. LPB-1 (instances 2r, 2r+1 of every tree), into the tree above
// it.  Called by the whole wave; all control flow is wave-uniform.
template <int WIDTH, int B, bool ROOTS>
__device__ __forceinline__ void fold_up(const Ctx<WIDTH>& c, int l, uint64_t n, uint64_t v0[], uint64_t v1[], uint64_t F[],
                        uint64_t (*lacc)[Family<WIDTH>::K][B]) {
  constexpr int K = Family<WIDTH>::K;
  using Ly = Layout<WIDTH, B>;
  const int lane = threadIdx.x;
  const bool owner = lane < Geo<B>::LPB;
  const int j0 = 2 * lane, j1 = 2 * lane + 1;
  for (;;) {
    const uint64_t parent = n >> 3;
    const int pos = (int)(n & 7);
    if (parent >= nodes_at(c.N, l + 1)) {
      // the parent is incomplete: this node is a leftover item (l, pos)
      if (owner) {
        if constexpr (ROOTS) {
          // a block of 8^L executions: its only leftover is its root
#pragma unroll
          for (int t = 0; t < K; ++t) {
            c.roots[t * kBlock + j0] = v0[t];
            c.roots[t * kBlock + j1] = v1[t];
          }
        } else {
#pragma unroll
          for (int t = 0; t < K; ++t) {
            const uint64_t* kf = c.ent + Ly::fin + ((t * kLevels + l) * (kFan - 1) + pos) * B;
            F[t] = nh_acc(F[t], v0[t], kf[j0]);
            F[t] = nh_acc(F[t], v1[t], kf[j1]);
          }
        }
      }
      return;
    }
    uint64_t term0[K], term1[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      if (pos < kFan - 1) {
        const uint64_t key = c.ent[Ly::tree + (t * kLevels + l) * (kFan - 1) + pos];
        term0[t] = nh_acc(0, v0[t], key);
        term1[t] = nh_acc(0, v1[t], key);
      } else {
        term0[t] = v0[t];
        term1[t] = v1[t];
      }
    }
    if (l + 1 <= (int)c.j + 2) {
      // parent inside the task: children arrive in order
      const int li = l + 1 - 3;
      if (owner) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
          lacc[li][t][j0] += term0[t];
          lacc[li][t][j1] += term1[t];
        }
      }
      if (pos != kFan - 1) return;
      if (owner) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
          v0[t] = lacc[li][t][j0];
          v1[t] = lacc[li][t][j1];
          lacc[li][t][j0] = 0;
          lacc[li][t][j1] = 0;
        }
      }
      ++l;
      n = parent;
      continue;
    }
    // parent spans tasks: add the terms to its device accumulator
    const uint64_t idx = c.acc_base + acc_index(c.N, c.j, l + 1, parent);
    uint64_t* acc = c.gacc + idx * (uint64_t)(kMaxK * kBlock);
    if (owner) {
#pragma unroll
      for (int t = 0; t < K; ++t) {
        __hip_atomic_fetch_add(acc + t * kBlock + j0, term0[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(acc + t * kBlock + j1, term1[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    complete_atomics();
    uint32_t old = 0;
    if (lane == 0) old = __hip_atomic_fetch_add(c.gcnt + idx, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    old = uniform(old);
    if (old != kFan - 1) return;
    // the 8th child: every sibling's terms are in; read and clear the
    // accumulator and its counter (they stay zero for the next launch)
    complete_atomics();
    if (owner) {
#pragma unroll
      for (int t = 0; t < K; ++t) {
        v0[t] = __hip_atomic_exchange(acc + t * kBlock + j0, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v1[t] = __hip_atomic_exchange(acc + t * kBlock + j1, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __hip_atomic_store(c.gcnt + idx, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_wave_barrier();
    ++l;
    n = parent;
  }
}

// The last pass of a string, nv < PASS executions starting at execution p:
// execution p + G e + q goes to lane group q (e = 0 .. ceil(nv/G) - 1), so
// the executions spread over all G lane groups (a lane does at most
// ceil(nv/G) of them instead of up to 8).  Execution G e + q is child q mod 8
// of level-1 node NG2 e + q/8; the 8 children of a node sit in 8 adjacent
// lane groups and are summed across lanes.  Complete level-1 nodes either
// join a complete level-2 node (its children arrive over 8/NG2 consecutive
// steps, from the lane groups q = 0, 8, 16, ...) or are leftover items of
// level 1; the executions of the incomplete level-1 node are leftover items
// of level 0.  Called by the whole wave (nv uniform).
template <int WIDTH, int B, bool ROOTS, class Hook = NoHook>
__device__ __forceinline__ void partial_pass(const Ctx<WIDTH>& c, const uint8_t* __restrict__ str, uint64_t p, uint32_t nv,
                             uint64_t F[], uint64_t (*lacc)[Family<WIDTH>::K][B], lds_u8* stage, bool staged,
                             const TaskNext& tn, const Hook& first_hook = Hook(), bool call_hook = false) {
  using Ly = Layout<WIDTH, B>;
  using Gm = Geo<B>;
  constexpr int K = Family<WIDTH>::K;
  constexpr uint64_t XB = Ly::exec_bytes;
  constexpr uint32_t kPer2 = 8 / Gm::NG2;  // steps that feed one level-2 node
  const int lane = threadIdx.x;
  const int q = lane / Gm::LPB, r = lane % Gm::LPB;
  const int h = q >> 3, pos0 = q & 7;
  const uint32_t full1 = nv / 8;   // complete level-1 nodes of the pass
  const uint32_t full2 = nv / 64;  // complete level-2 nodes (fewer than NG2)
  uint64_t k0[K];                  // level-0 key of this lane's child position
#pragma unroll
  for (int t = 0; t < K; ++t) k0[t] = pos0 < kFan - 1 ? c.ltree[t * 2 * (kFan - 1) + pos0] : 0;
  uint64_t s0[K], s1[K];  // terms of the current level-2 node (lanes of pos0 == 0)
#pragma unroll
  for (int t = 0; t < K; ++t) s0[t] = s1[t] = 0;
  const uint32_t steps = (nv + Gm::G - 1) / Gm::G;
  // step e's region: the contiguous executions p + G e .. p + G e + G - 1
  // (fewer in the last step)
  auto nq_of = [&](uint32_t e) {
    return nv - Gm::G * e < (uint32_t)Gm::G ? nv - Gm::G * e : (uint32_t)Gm::G;
  };
  auto base_of = [&](uint32_t e) { return str + (p + (uint64_t)Gm::G * e) * XB; };
  auto region = [&](uint32_t e) -> NextStage { return {base_of(e), (uint32_t)XB, nq_of(e)}; };
  // (region 0 may have been copied ahead, by the previous task or pass)
  if (!staged) stage_issue<WIDTH, B>(region(0), 0, stage);
  uint4 xc[Parts<WIDTH, B>::LX > 0 ? Parts<WIDTH, B>::LX : 1];  // (no carried blocks here)
  for (uint32_t e = 0; e < steps; ++e) {
    const uint32_t i = Gm::G * e + (uint32_t)q;  // execution within the pass
    const uint32_t m = Gm::NG2 * e + (uint32_t)h;  // its level-1 node
    const uint32_t g = e / kPer2;                // that node's level-2 parent (uniform)
    const bool node_full = m < full1;
    uint64_t t0[K], t1[K];
#pragma unroll
    for (int t = 0; t < K; ++t) t0[t] = t1[t] = 0;
    uint64_t z0[K], z1[K];
    // the next region: this pass's next step, else the next task's first
    const NextStage nx = e + 1 < steps ? region(e + 1) : task_next_region<WIDTH, B>(tn);
    const NextStage cur = region(e);
    region_ehc<WIDTH, B, false>(stage, cur.base, cur.qs, cur.nq, 0, 0, nx, 0, xc, uniform_keys(c.ent + Ly::ehc), z0,
                                z1);
    // (after the region: inside it, the loads' registers would come on top of
    // the parts')
    if (call_hook && e == 0) first_hook();
    if (i < nv) {
      if (node_full) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
          t0[t] = pos0 < kFan - 1 ? nh_acc(0, z0[t], k0[t]) : z0[t];
          t1[t] = pos0 < kFan - 1 ? nh_acc(0, z1[t], k0[t]) : z1[t];
        }
      } else if constexpr (ROOTS) {
        // a block of one execution: the execution is the root
#pragma unroll
        for (int t = 0; t < K; ++t) {
          c.roots[t * kBlock + 2 * r] = z0[t];
          c.roots[t * kBlock + 2 * r + 1] = z1[t];
        }
      } else {
        // child of the incomplete level-1 node: leftover item (0, pos0)
#pragma unroll
        for (int t = 0; t < K; ++t) {
          const uint64_t* kf = c.lfin + (t * 2 * (kFan - 1) + pos0) * B;
          F[t] = nh_acc(F[t], z0[t], kf[2 * r]);
          F[t] = nh_acc(F[t], z1[t], kf[2 * r + 1]);
        }
      }
    }
    // sum the 8 children of each level-1 node (q mod 8 = lane bits above r)
#pragma unroll
    for (int t = 0; t < K; ++t) {
#pragma unroll
      for (int msk = Gm::LPB; msk < 8 * Gm::LPB; msk <<= 1) {
        t0[t] += shfl_xor64(t0[t], msk);
        t1[t] += shfl_xor64(t1[t], msk);
      }
    }
    if (pos0 == 0 && node_full) {
      if (g < full2) {
        // child m mod 8 of level-2 node g
#pragma unroll
        for (int t = 0; t < K; ++t) {
          if ((m & 7) < (uint32_t)kFan - 1) {
            const uint64_t key = c.ltree[t * 2 * (kFan - 1) + (kFan - 1) + (m & 7)];
            s0[t] = nh_acc(s0[t], t0[t], key);
            s1[t] = nh_acc(s1[t], t1[t], key);
          } else {
            s0[t] += t0[t];
            s1[t] += t1[t];
          }
        }
      } else if constexpr (ROOTS) {
        // a block of 8 executions: its level-1 node is the root
#pragma unroll
        for (int t = 0; t < K; ++t) {
          c.roots[t * kBlock + 2 * r] = t0[t];
          c.roots[t * kBlock + 2 * r + 1] = t1[t];
        }
      } else {
        // complete level-1 node with an incomplete parent: leftover (1, m mod 8)
#pragma unroll
        for (int t = 0; t < K; ++t) {
          const uint64_t* kf = c.lfin + (t * 2 * (kFan - 1) + (kFan - 1) + (m & 7)) * B;
          F[t] = nh_acc(F[t], t0[t], kf[2 * r]);
          F[t] = nh_acc(F[t], t1[t], kf[2 * r + 1]);
        }
      }
    }
    if (e % kPer2 == kPer2 - 1 && g < full2) {
      // all children of level-2 node g are in: sum the lane groups q = 8h
      // into lanes 0 .. LPB-1 and fold it up
#pragma unroll
      for (int t = 0; t < K; ++t) {
#pragma unroll
        for (int msk = 8 * Gm::LPB; msk < 64; msk <<= 1) {
          s0[t] += shfl_xor64(s0[t], msk);
          s1[t] += shfl_xor64(s1[t], msk);
        }
      }
      fold_up<WIDTH, B, ROOTS>(c, 2, (p >> 6) + g, s0, s1, F, lacc);
#pragma unroll
      for (int t = 0; t < K; ++t) s0[t] = s1[t] = 0;
    }
  }
}

// One tail-only string: its tail words hashed with the Toeplitz keys of
// §6.1 plus the length term, by one lane.
template <int WIDTH, int B>
__device__ __forceinline__ void tiny_one(const MainArgs& a, const uint64_t* ltail, uint32_t s, uint64_t L,
                                         uint64_t off) {
  using Ly = Layout<WIDTH, B>;
  constexpr int K = Family<WIDTH>::K;
  const uint8_t* __restrict__ str = a.bytes + off;
  uint64_t F[K];
#pragma unroll
  for (int t = 0; t < K; ++t) F[t] = 0;
  // whole 128-byte groups: eight independent 16-byte loads, then 16 words
  uint64_t m = 0;
  for (; 8 * m + 128 <= L; m += 16) {
    uint64_t w[16];
#pragma unroll
    for (int c = 0; c < 8; ++c) __builtin_memcpy(&w[2 * c], str + 8 * m + 16 * c, 16);
#pragma unroll
    for (int c = 0; c < 16; ++c)
#pragma unroll
      for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], w[c], ltail[t + m + c]);
  }
  // the rest (under 128 bytes): up to 15 whole words and a zero-padded last
  // word, every load issued before the first is used
  const uint64_t rem = L - 8 * m;
  const uint32_t nw = (uint32_t)(rem / 8), nb = (uint32_t)(rem % 8);
  const uint8_t* __restrict__ rp = str + 8 * m;
  uint64_t w[15];
#pragma unroll
  for (int j = 0; j < 15; ++j) {
    w[j] = 0;
    if ((uint32_t)j < nw) __builtin_memcpy(&w[j], rp + 8 * j, 8);
  }
  const uint64_t last = nb ? load_partial_word(rp + 8 * nw, nb) : 0;
#pragma unroll
  for (int j = 0; j < 15; ++j)
    if ((uint32_t)j < nw) {
#pragma unroll
      for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], w[j], ltail[t + m + j]);
    }
  if (nb) {
#pragma unroll
    for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], last, ltail[t + m + nw]);
  }
  uint8_t* o = a.out + (uint64_t)s * WIDTH;
#pragma unroll
  for (int t = 0; t < K; ++t) {
    const uint64_t v = nh_acc(F[t], L, ltail[Ly::len - Ly::tail + t]);
    __builtin_memcpy(o + 8 * t, &v, 8);
  }
}

// A small string (1 .. kSmallMax executions, at most 15) per half-wave.  The half's
// lane groups take the executions in rounds (lane group q: executions q, q +
// QH, ..., QH lane groups per half), each hashing the EHC of its instance
// pair (§3.3, loaded directly).  With 8 executions or more, executions 0 .. 7
// form the one complete level-1 node (Eq. (3)): their terms (§3.2's variant:
// NH against the level-0 key of their position, the 8th raw) are summed over
// the node's 8 lane groups and the node goes to the final NH as the leftover
// at level 1, position 0; every other execution is a leftover at level 0,
// position i mod 8 (§5.2).  The half's lanes add the tail words (Toeplitz
// keys, §6.1) and the length term, and a half-wave sum gives the output.
// `valid` is false for a half without a string.  Called by the whole wave.
template <int WIDTH, int B>
__device__ __forceinline__ void small_half(const MainArgs& a, const uint64_t* ltree0, const uint64_t* lfin0,
                                           const uint64_t* lfin1, const uint64_t* ltail, bool valid, uint32_t s,
                                           uint64_t L, uint64_t off) {
  using Ly = Layout<WIDTH, B>;
  constexpr int K = Family<WIDTH>::K;
  constexpr uint64_t XB = Ly::exec_bytes;
  constexpr int LPB = Geo<B>::LPB;
  constexpr int QH = 32 / LPB;                          // lane groups per half
  constexpr int ROUNDS = ((int)kSmallMax + QH - 1) / QH;
  static_assert(kSmallMax < 2 * kFan, "at most one complete level-1 node");
  const int l32 = threadIdx.x & 31;
  const int q = l32 / LPB, r = l32 % LPB;
  const uint8_t* __restrict__ str = a.bytes + off;
  const uint64_t N = L / XB;
  const bool node = N >= (uint64_t)kFan;  // executions 0 .. 7 form a level-1 node
  uint64_t F[K];
#pragma unroll
  for (int t = 0; t < K; ++t) F[t] = 0;
  // tail words m0 .. m0 + R - 1 (R <= XB / 8 <= 6 * 32), the last one
  // zero-padded, loaded to its last byte only; issued before the
  // executions' loads, so that both are in flight together
  const uint64_t tb = N * XB, rem = L - tb;
  const uint64_t R = (rem + 7) / 8;
  uint64_t w[6];
  PartialWord pp;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const uint64_t m = (uint64_t)l32 + 32 * i;
    w[i] = 0;
    if (valid && m < R) issue_tail_word(str + tb + 8 * m, rem - 8 * m, i, w[i], pp);
  }
#pragma unroll
  for (int rd = 0; rd < ROUNDS; ++rd) {
    const int i = rd * QH + q;  // execution of this lane group
    const int pos = i & 7;
    uint64_t t0[K], t1[K];      // terms of the level-1 node's children
#pragma unroll
    for (int t = 0; t < K; ++t) t0[t] = t1[t] = 0;
    if (valid && (uint64_t)i < N) {
      uint64_t z0[K], z1[K];
      ehc2<WIDTH, B>(str + (uint64_t)i * XB + 16 * r, uniform_keys(a.ent + Ly::ehc), z0, z1);
      if (node && i < kFan) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
          t0[t] = pos < kFan - 1 ? nh_acc(0, z0[t], ltree0[t * (kFan - 1) + pos]) : z0[t];
          t1[t] = pos < kFan - 1 ? nh_acc(0, z1[t], ltree0[t * (kFan - 1) + pos]) : z1[t];
        }
      } else {
#pragma unroll
        for (int t = 0; t < K; ++t) {
          const uint64_t* kf = lfin0 + (t * (kFan - 1) + pos) * B;
          F[t] = nh_acc(F[t], z0[t], kf[2 * r]);
          F[t] = nh_acc(F[t], z1[t], kf[2 * r + 1]);
        }
      }
    }
    if (rd == 0) {
      // the node's 8 children are lane groups 0 .. 7 of the half's first
      // round: sum them, then lane group 0 adds the node's final NH
#pragma unroll
      for (int t = 0; t < K; ++t) {
#pragma unroll
        for (int msk = LPB; msk < 8 * LPB; msk <<= 1) {
          t0[t] += shfl_xor64(t0[t], msk);
          t1[t] += shfl_xor64(t1[t], msk);
        }
      }
      if (valid && node && q == 0) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
          F[t] = nh_acc(F[t], t0[t], lfin1[t * B + 2 * r]);
          F[t] = nh_acc(F[t], t1[t], lfin1[t * B + 2 * r + 1]);
        }
      }
    }
  }
  finish_tail_words(w, pp);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const uint64_t m = (uint64_t)l32 + 32 * i;
    if (valid && m < R) {
#pragma unroll
      for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], w[i], ltail[t + m]);
    }
  }
  if (valid && l32 == 0) {
#pragma unroll
    for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], L, ltail[Ly::len - Ly::tail + t]);
  }
#pragma unroll
  for (int t = 0; t < K; ++t)
#pragma unroll
    for (int m = 1; m < 32; m <<= 1) F[t] += shfl_xor64(F[t], m);
  if (valid && l32 < K) {
    uint64_t v = F[0];
#pragma unroll
    for (int t = 1; t < K; ++t)
      if (l32 == t) v = F[t];
    __builtin_memcpy(a.out + (uint64_t)s * WIDTH + 8 * l32, &v, 8);
  }
}

// Tail-only strings (shorter than one execution: §6.1's tail and the length
// term, no tree), one string per lane, in chunks of kTinyChunk strings: wave
// w takes chunks w, w + grid, ...  A tail-only string costs at most a few
// dozen loads, so static shares balance, and no wave queues on a counter (one
// device atomic per chunk serialised millions of short strings).  A separate
// kernel: inside the hashing kernel this code cost the full passes 3-10 %
// (register allocation of the whole kernel), while a launch costs a few
// microseconds.  The list entry of the chunk two rounds ahead and the
// offset and length of the next round's string are loaded before the
// current string is hashed, so a string costs one exposed memory round trip
// instead of three.
template <int WIDTH, int B>
__global__ __launch_bounds__(64) void tiny_kernel(MainArgs a) {
  using Ly = Layout<WIDTH, B>;
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const uint32_t ntiny = uniform(a.ctl[kCtlTiny]);
  // the Toeplitz tail keys and the length keys, read at lane-varying indices
  // for every string, in LDS (one copy per wave)
  constexpr int NTAIL = (int)(Ly::len + Family<WIDTH>::K - Ly::tail);
  __shared__ uint64_t ltail[NTAIL];
  if ((uint64_t)blockIdx.x * kTinyChunk >= ntiny) return;  // no chunk for this wave
  for (int i = threadIdx.x; i < NTAIL; i += 64) ltail[i] = a.ent[Ly::tail + i];
  __syncthreads();
  const uint32_t G = gridDim.x;
  auto entry = [&](uint64_t k) -> uint32_t {
    const uint64_t idx = k * kTinyChunk + threadIdx.x;
    return idx < ntiny ? a.tiny_list[idx] : kNone;
  };
  uint64_t k = blockIdx.x;
  uint32_t s = entry(k), s1 = entry(k + G);
  uint64_t L = 0, off = 0;
  if (s != kNone) {
    L = a.lengths[s];
    off = a.offsets[s];
  }
  for (; k * kTinyChunk < ntiny; k += G) {
    const uint32_t s2 = entry(k + 2 * (uint64_t)G);
    uint64_t L1 = 0, off1 = 0;
    if (s1 != kNone) {
      L1 = a.lengths[s1];
      off1 = a.offsets[s1];
    }
    if (s != kNone) tiny_one<WIDTH, B>(a, ltail, s, L, off);
    s = s1;
    s1 = s2;
    L = L1;
    off = off1;
  }
}

// Small strings (1 .. kSmallMax executions, listed by the planner), one per
// half-wave: wave w takes the pairs w, w + grid, ... of the list.  The list
// entries of the pair two rounds ahead and the offset and length of the next
// round's pair are loaded before the current pair is hashed, so a pair costs
// one exposed memory round trip (its bytes) instead of three.
template <int WIDTH, int B>
__global__ __launch_bounds__(64) void small_kernel(MainArgs a) {
  using Ly = Layout<WIDTH, B>;
  constexpr int K = Family<WIDTH>::K;
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const uint32_t nsmall = uniform(a.ctl[kCtlSmall]);
  // Toeplitz tail keys, length keys and the final keys of level 0, read at
  // lane-varying indices, in LDS (one copy per wave)
  constexpr int NTAIL = (int)(Ly::len + K - Ly::tail);
  __shared__ uint64_t ltail[NTAIL];
  __shared__ uint64_t ltree0[K * (kFan - 1)];    // tree keys of level 0
  __shared__ uint64_t lfin0[K * (kFan - 1) * B];  // final keys of level 0
  __shared__ uint64_t lfin1[K * B];               // final keys of level 1, position 0
  if ((uint64_t)blockIdx.x * 2 >= nsmall) return;  // no pair for this wave
  for (int i = threadIdx.x; i < NTAIL; i += 64) ltail[i] = a.ent[Ly::tail + i];
  for (int i = threadIdx.x; i < K * (kFan - 1); i += 64)
    ltree0[i] = a.ent[Ly::tree + (i / (kFan - 1)) * kLevels * (kFan - 1) + i % (kFan - 1)];
  for (int i = threadIdx.x; i < K * (kFan - 1) * B; i += 64)
    lfin0[i] = a.ent[Ly::fin + (i / ((kFan - 1) * B)) * kLevels * (kFan - 1) * B + i % ((kFan - 1) * B)];
  for (int i = threadIdx.x; i < K * B; i += 64)
    lfin1[i] = a.ent[Ly::fin + (i / B) * kLevels * (kFan - 1) * B + (kFan - 1) * B + i % B];
  __syncthreads();
  const uint32_t G = gridDim.x;
  const int half = threadIdx.x >> 5;
  // this half's list entry of pair k
  auto entry = [&](uint64_t k) -> uint32_t {
    const uint64_t idx = 2 * k + half;
    return idx < nsmall ? a.small_list[idx] : kNone;
  };
  uint64_t k = blockIdx.x;
  uint32_t s = entry(k), s1 = entry(k + G);
  uint64_t L = 0, off = 0;
  if (s != kNone) {
    L = a.lengths[s];
    off = a.offsets[s];
  }
  for (; 2 * k < nsmall; k += G) {
    const uint32_t s2 = entry(k + 2 * (uint64_t)G);
    uint64_t L1 = 0, off1 = 0;
    if (s1 != kNone) {
      L1 = a.lengths[s1];
      off1 = a.offsets[s1];
    }
    small_half<WIDTH, B>(a, ltree0, lfin0, lfin1, ltail, s != kNone, s, L, off);
    s = s1;
    s1 = s2;
    L = L1;
    off = off1;
  }
}

// Composition of HalftimeHash with a short-input family (§1: a universe-
// collapsing family reduces long strings to short values that a short-input
// family hashes as if they were the input; §7: pairing HalftimeHash with a
// fast short-input family).  The short-input family is simple tabulation:
// C + 1 byte characters, one table of 256 random words per character, the
// result the XOR of the characters' entries.  A string of at most C bytes is
// its own key (zero-padded, separator character = its length); a longer
// string's key is its C-byte HalftimeHash value with separator 255.
//
// One workgroup of kTabThreads per resident slot shares one LDS copy of the
// tables ((C + 1) * 2 KiB) and of the Toeplitz tail and length keys; its
// threads take strings with a grid stride.  A string of at most kTabInline
// bytes is keyed here from its own bytes: as they are (at most C bytes), or
// through its HalftimeHash value, which for a string shorter than one
// execution is the tail and length terms alone (§6.1; at most 8 words); a
// longer string's value comes from h.  Bytes are read as the aligned 8-byte
// words that hold them (never a word without one of the string's bytes, so
// never past the page of its allocation) and shifted into place.  Two-deep
// pipeline: while string i is tabulated, the words (or the h row) of string
// i + stride and the offset and length of string i + 2 stride are in flight.
template <int C, int B>
__global__ __launch_bounds__(kTabThreads) void tab_kernel(TabArgs a) {
  using Ly = Layout<C, B>;
  constexpr int K = Family<C>::K;
  constexpr int NA = kTabInline / 8 + 1;  // aligned words that hold kTabInline bytes at any alignment
  constexpr int NTAIL = (int)(Ly::len + K - Ly::tail);
  static_assert(K * 8 == C, "one output word per 8 bytes");
  static_assert(kTabInline < (uint32_t)Ly::exec_bytes, "inline strings are tail-only");
  static_assert(NA >= K + 1, "a direct key's words");
  __shared__ uint64_t T[(C + 1) * 256];
  __shared__ uint64_t ltail[NTAIL];
  for (int i = threadIdx.x; i < (C + 1) * 256; i += kTabThreads) T[i] = a.tables[i];
  for (int i = threadIdx.x; i < NTAIL; i += kTabThreads) ltail[i] = a.ent[Ly::tail + i];
  const uint64_t stride = (uint64_t)gridDim.x * kTabThreads;
  struct Meta {
    uint64_t L = 0, off = 0;
  };
  auto fetch = [&](uint64_t i, Meta& m) {
    if (i < a.count) {
      m.L = a.lengths[i];
      m.off = a.offsets[i];
    }
  };
  // the aligned words of an inline string, or the h row of a longer one
  auto words_of = [&](uint64_t i, const Meta& m, uint64_t (&A)[NA]) {
#pragma unroll
    for (int j = 0; j < NA; ++j) A[j] = 0;
    if (i >= a.count) return;
    if (m.L > kTabInline) {
      const uint64_t* h = reinterpret_cast<const uint64_t*>(a.h + i * C);
#pragma unroll
      for (int j = 0; j < K; ++j) A[j] = h[j];
    } else if (m.L) {
      const uintptr_t p = reinterpret_cast<uintptr_t>(a.bytes + m.off);
      const uint64_t* w = reinterpret_cast<const uint64_t*>(p & ~(uintptr_t)7);
      const uint64_t last = ((p & 7) + m.L - 1) / 8;
#pragma unroll
      for (int j = 0; j < NA; ++j)
        if ((uint64_t)j <= last) A[j] = w[j];
    }
  };
  uint64_t s = (uint64_t)blockIdx.x * kTabThreads + threadIdx.x;
  Meta m0, m1;
  fetch(s, m0);
  fetch(s + stride, m1);
  uint64_t A0[NA];
  words_of(s, m0, A0);
  __syncthreads();
  for (; s < a.count; s += stride) {
    Meta m2;
    fetch(s + 2 * stride, m2);
    uint64_t A1[NA];
    words_of(s + stride, m1, A1);
    const uint64_t L = m0.L;
    uint64_t w[K];
    uint32_t sep = 255;
    if (L > kTabInline) {
#pragma unroll
      for (int j = 0; j < K; ++j) w[j] = A0[j];
    } else {
      // word j of the string (bytes 8j .. 8j + 7, zero past its end)
      const uint32_t sh = 8 * (uint32_t)(reinterpret_cast<uintptr_t>(a.bytes + m0.off) & 7);
      auto word = [&](int j) -> uint64_t {
        if (8 * (uint64_t)j >= L) return 0;
        uint64_t x = sh ? (A0[j] >> sh) | (A0[j + 1] << (64 - sh)) : A0[j];
        const uint64_t rem = L - 8 * (uint64_t)j;
        if (rem < 8) x &= (1ull << (8 * rem)) - 1;
        return x;
      };
      if (L <= (uint64_t)C) {
#pragma unroll
        for (int j = 0; j < K; ++j) w[j] = word(j);
        sep = (uint32_t)L;
      } else {
        // tail-only HalftimeHash value: Toeplitz tail words, then the length
        uint64_t F[K];
#pragma unroll
        for (int t = 0; t < K; ++t) F[t] = 0;
#pragma unroll
        for (int j = 0; j < NA - 1; ++j) {
          if (8 * (uint64_t)j < L) {
            const uint64_t x = word(j);
#pragma unroll
            for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], x, ltail[t + j]);
          }
        }
#pragma unroll
        for (int t = 0; t < K; ++t) w[t] = nh_acc(F[t], L, ltail[Ly::len - Ly::tail + t]);
      }
    }
    uint64_t z = T[C * 256 + sep];
#pragma unroll
    for (int i = 0; i < C; ++i) z ^= T[i * 256 + (uint32_t)((w[i / 8] >> (8 * (i % 8))) & 0xFF)];
    a.out[s] = z;
    m0 = m1;
    m1 = m2;
#pragma unroll
    for (int j = 0; j < NA; ++j) A0[j] = A1[j];
  }
}

// ROOTS: root mode (streaming): every string is a block of exactly 8^L
// executions and its root node goes to a.roots instead of a hash to a.out.
template <int WIDTH, int B, bool ROOTS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void hash_main_kernel(MainArgs a) {
  using Fm = Family<WIDTH>;
  using Ly = Layout<WIDTH, B>;
  using Gm = Geo<B>;
  constexpr int K = Fm::K;
  constexpr uint64_t XB = Ly::exec_bytes;
  __shared__ uint64_t lacc[kMaxLocal][K][B];
  // Keys read at lane-varying indices by every short string and every
  // string's last pass (tree and final keys of levels 0 and 1, the Toeplitz
  // tail keys and the length keys), copied to LDS once per wave: they leave
  // the chain of dependent memory round trips of a short task.
  constexpr int NT0 = 2 * (kFan - 1);
  constexpr int NTAIL = (int)(Ly::len + K - Ly::tail);
  __shared__ uint64_t ltree[K * NT0];
  __shared__ uint64_t lfin[K * NT0 * B];
  __shared__ uint64_t ltail[NTAIL];
  // this wave's region of staged executions
  __shared__ __attribute__((aligned(1024))) uint8_t stage_buf[Parts<WIDTH, B>::BYTES + 16];  // (+ guard, read_slot)
  lds_u8* const stage = (lds_u8*)stage_buf;

  const int lane = threadIdx.x;
  const int q = lane / Gm::LPB, r = lane % Gm::LPB;
  for (int i = lane; i < K * NT0; i += 64)
    ltree[i] = a.ent[Ly::tree + (i / NT0) * kLevels * (kFan - 1) + i % NT0];
  for (int i = lane; i < K * NT0 * B; i += 64)
    lfin[i] = a.ent[Ly::fin + (i / (NT0 * B)) * kLevels * (kFan - 1) * B + i % (NT0 * B)];
  for (int i = lane; i < NTAIL; i += 64) ltail[i] = a.ent[Ly::tail + i];
  __syncthreads();
  const uint32_t nb = uniform(a.ctl[kCtlBuckets]);
  const uint32_t jlev = uniform(a.ctl[kCtlLevel]);
  const uint64_t texec = (uint64_t)Gm::PASS << (3 * jlev);
  const uint64_t* __restrict__ ent = a.ent;

  // each owner lane (0 .. LPB-1) only ever touches its own two instances' slots
  if (lane < Gm::LPB) {
    for (int li = 0; li < kMaxLocal; ++li)
#pragma unroll
      for (int t = 0; t < K; ++t) lacc[li][t][2 * lane] = lacc[li][t][2 * lane + 1] = 0;
  }

  // Whole buckets from one counter: a bucket runs from its leader task up
  // to the next leader (bit 31 of the task table) or the last task; a wave
  // leaves once the counter ran past the last bucket.
  const uint32_t ntasks_all = uniform(a.ctl[kCtlTotal]);
  uint32_t task = 0;
  bool fetch = true, first = true;
  // metadata of the next task's string, read while the current task runs
  bool have_next = false;
  uint32_t pf_s = 0, pf_ts = 0, pf_as = 0;
  uint64_t pf_off = 0, pf_L = 0;
  // the current task's first region was copied ahead by the previous task
  bool staged = false;
  for (;;) {
    __builtin_amdgcn_wave_barrier();
    if (fetch) {
      if (first) {
        // a batch with fewer buckets than waves: most waves leave on a
        // plain read instead of queueing on the counter's atomic
        first = false;
        uint32_t seen = 0;
        if (lane == 0) seen = __hip_atomic_load(a.ctl + kCtlNext, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (uniform(seen) >= nb) break;
      }
      uint32_t k = 0;
      if (lane == 0) k = atomicAdd(a.ctl + kCtlNext, 1u);
      k = uniform(k);
      if (k >= nb) break;
      task = uniform(a.bucket_lead[k]);
      fetch = false;
      have_next = false;
      staged = false;
      continue;  // (an empty bucket would fetch again)
    }
    uint32_t s, ts, as;
    uint64_t off, L;
    if (have_next) {
      s = pf_s;
      ts = pf_ts;
      as = pf_as;
      off = pf_off;
      L = pf_L;
    } else {
      s = smeta(a.task_string)[task] & 0x7FFFFFFFu;
      ts = smeta(a.task_start)[s];
      as = smeta(a.acc_start)[s];
      off = uniform_keys(a.offsets)[s];
      L = uniform_keys(a.lengths)[s];
    }
    // next task's entry: whether it leads another bucket; if not, its
    // string's metadata is read now and used next time round
    const uint32_t next_entry = task + 1 < ntasks_all ? smeta(a.task_string)[task + 1] : 0x80000000u;
    have_next = (next_entry >> 31) == 0;
    if (have_next) {
      pf_s = next_entry;
      pf_ts = smeta(a.task_start)[pf_s];
      pf_as = smeta(a.acc_start)[pf_s];
      pf_off = uniform_keys(a.offsets)[pf_s];
      pf_L = uniform_keys(a.lengths)[pf_s];
    }
    const uint64_t tau = task - ts;
    const uint64_t N = L / XB;
    const uint64_t ntask = N ? (N + texec - 1) / texec : 1;
    const uint8_t* __restrict__ str = a.bytes + off;
    // the next task of the bucket, whose first region this task copies ahead
    const TaskNext tn{have_next, a.bytes, pf_off, pf_L, (uint64_t)(task + 1) - pf_ts, texec};

    Ctx<WIDTH> c{ent, N, jlev, ntask > 1 ? (uint64_t)as : 0, a.gacc, a.gcnt,
                 ROOTS ? a.roots + (uint64_t)s * (kMaxK * kBlock) : nullptr, ltree, lfin};
    uint64_t F[K];
#pragma unroll
    for (int t = 0; t < K; ++t) F[t] = 0;

    // The string's tail words (§6.1: words N XB / 8 .., at most XB / 8 <= 3 *
    // 64 of them, the last one zero-padded), loaded to its last byte only, in
    // flight while the last pass's first region is hashed (issued after that
    // region's bytes have arrived, so that waiting for them never holds up a
    // region).
    uint64_t tw[3];
    PartialWord tpp;
    auto load_tail = [&]() {
      const uint64_t tb = N * XB, rem = L - tb, R = (rem + 7) / 8;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const uint64_t m = (uint64_t)lane + 64 * i;
        tw[i] = 0;
        if (m < R) issue_tail_word(str + tb + 8 * m, rem - 8 * m, i, tw[i], tpp);
      }
    };

    // (at widths 32 and 40, and in the b = 4 family, the registers of the early loads made the
    // hashing kernel spill: there the tail words are loaded at task start,
    // or after the passes)
    constexpr bool kEarlyTail = K <= 3 && B == 8;
    if (N < Gm::PASS) {
      // a string of fewer than PASS executions (one task): one partial pass
      if (N) {
        if (!kEarlyTail) load_tail();
        partial_pass<WIDTH, B, ROOTS>(c, str, 0, (uint32_t)N, F, lacc, stage, staged, tn, load_tail, kEarlyTail);
      } else {
        stage_issue<WIDTH, B>(task_next_region<WIDTH, B>(tn), 0, stage);
        load_tail();
      }
      finish_tail_words(tw, tpp);
      const uint64_t R = (L - N * XB + 7) / 8;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const uint64_t m = (uint64_t)lane + 64 * i;
        if (m < R) {
#pragma unroll
          for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], tw[i], ltail[t + m]);
        }
      }
      if (lane == 0) {
#pragma unroll
        for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], L, ltail[Ly::len - Ly::tail + t]);
      }
    } else {
      const uint64_t g0 = tau * texec;
      const uint64_t g1 = g0 + texec < N ? g0 + texec : N;
      // the first region of a first full pass is copied ahead
      constexpr uint32_t QS = 8 * (uint32_t)XB;  // lane group stride of a full pass's region
      if (!staged && N - g0 >= (uint64_t)Gm::PASS) stage_first<WIDTH, B>(str + g0 * XB, QS, Gm::G, 0, stage);
      uint4 xc[Parts<WIDTH, B>::LX > 0 ? Parts<WIDTH, B>::LX : 1];  // blocks carried between regions
      bool pstaged = staged;  // the next pass's first region is copied
      bool tail_loaded = false;
      for (uint64_t p = g0; p < g1; p += Gm::PASS) {
        if (N - p < Gm::PASS) {
          // the string's last, partial pass (in the string's last task: the
          // tail words are loaded with its first region)
          tail_loaded = kEarlyTail && tau == ntask - 1;
          partial_pass<WIDTH, B, ROOTS>(c, str, p, (uint32_t)(N - p), F, lacc, stage, pstaged, tn, load_tail,
                                        tail_loaded);
          break;
        }
        // full pass: lane group q takes the 8 consecutive executions
        // p + 8q .. p + 8q + 7, i.e. all children of level-1 node p/8 + q;
        // region e holds executions p + 8q + e of every lane group
        uint64_t a0[K], a1[K];
#pragma unroll
        for (int t = 0; t < K; ++t) a0[t] = a1[t] = 0;
        // the region after this pass's last step: the next pass's first (a
        // full pass, or the last, partial one) if this task has one, else
        // the next task's first (uniform)
        const bool more = p + Gm::PASS < g1;
        for (int e = 0; e < 8; ++e) {
          const uint32_t cin = e > 0 ? carry_blocks<WIDTH, B>(str, p, e - 1) : 0;
          const uint32_t cout = carry_blocks<WIDTH, B>(str, p, e);
          const NextStage nx = e < 7 ? NextStage{str + (p + e + 1) * XB, QS, (uint32_t)Gm::G}
                               : more ? first_region<WIDTH, B>(str, L, p + Gm::PASS)
                                      : task_next_region<WIDTH, B>(tn);
          uint64_t z0[K], z1[K];
          region_ehc<WIDTH, B, true>(stage, str + (p + e) * XB, QS, Gm::G, cin, cout, nx, e < 7 ? cout : 0, xc,
                               uniform_keys(ent + Ly::ehc), z0, z1);
          // level 0 of every tree: child e of this lane's level-1 node
          if (e < kFan - 1) {
#pragma unroll
            for (int t = 0; t < K; ++t) {
              const uint64_t key = uniform_keys(ent)[Ly::tree + (t * kLevels) * (kFan - 1) + e];
              a0[t] = nh_acc(a0[t], z0[t], key);
              a1[t] = nh_acc(a1[t], z1[t], key);
            }
          } else {
#pragma unroll
            for (int t = 0; t < K; ++t) {
              a0[t] += z0[t];
              a1[t] += z1[t];
            }
          }
        }
        // level 1 -> level 2: lane group q holds level-1 node p/8 + q, child
        // pos1 of level-2 node p/64 + q/8
        const int pos1 = q & 7;
        uint64_t n0[K], n1[K];
#pragma unroll
        for (int t = 0; t < K; ++t) {
          uint64_t t0, t1;
          if (pos1 < kFan - 1) {
            // (HH16 runs its full passes faster with this key from the
            // cache hierarchy than from LDS, the other widths slower:
            // measured per width)
            const uint64_t key = WIDTH == 16 ? ent[Ly::tree + (t * kLevels + 1) * (kFan - 1) + pos1]
                                             : ltree[t * NT0 + (kFan - 1) + pos1];
            t0 = nh_acc(0, a0[t], key);
            t1 = nh_acc(0, a1[t], key);
          } else {
            t0 = a0[t];
            t1 = a1[t];
          }
#pragma unroll
          for (int msk = Gm::LPB; msk < 8 * Gm::LPB; msk <<= 1) {
            t0 += shfl_xor64(t0, msk);
            t1 += shfl_xor64(t1, msk);
          }
          n0[t] = t0;
          n1[t] = t1;
        }
        // lanes 8 g LPB + r (lane group q = 8g) hold level-2 node p/64 + g;
        // each is brought to lanes 0 .. LPB-1 and folded up (fold_up may
        // overwrite its argument arrays, so it gets copies)
#pragma unroll
        for (int g = 0; g < Gm::NG2; ++g) {
          uint64_t b0[K], b1[K];
#pragma unroll
          for (int t = 0; t < K; ++t) {
            b0[t] = g ? shfl64(n0[t], r + 8 * Gm::LPB * g) : n0[t];
            b1[t] = g ? shfl64(n1[t], r + 8 * Gm::LPB * g) : n1[t];
          }
          fold_up<WIDTH, B, ROOTS>(c, 2, (p >> 6) + g, b0, b1, F, lacc);
        }
        pstaged = true;  // (the next pass's first region was issued in step 7)
      }

      if (tau == ntask - 1) {
        // tail (§6.1): words m0 .. m0+R-1, output t keyed by S_tail[t + m]
        if (!tail_loaded) load_tail();
        finish_tail_words(tw, tpp);
        const uint64_t R = (L - N * XB + 7) / 8;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const uint64_t m = (uint64_t)lane + 64 * i;
          if (m < R) {
#pragma unroll
            for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], tw[i], ltail[t + m]);
          }
        }
        if (lane == 0) {
#pragma unroll
          for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], L, ltail[Ly::len - Ly::tail + t]);
        }
      }
    }

    if constexpr (!ROOTS) {
#pragma unroll
      for (int t = 0; t < K; ++t) F[t] = wave_sum64(F[t]);

      uint8_t* o = a.out + (uint64_t)s * WIDTH;
      if (ntask == 1) {
        if (lane < K) {
          uint64_t v = F[0];
#pragma unroll
          for (int t = 1; t < K; ++t)
            if (lane == t) v = F[t];
          __builtin_memcpy(o + 8 * lane, &v, 8);
        }
      } else {
        uint64_t* sacc = a.sacc + (uint64_t)s * kMaxK;
        if (lane < K) {
          uint64_t v = F[0];
#pragma unroll
          for (int t = 1; t < K; ++t)
            if (lane == t) v = F[t];
          __hip_atomic_fetch_add(sacc + lane, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        complete_atomics();
        uint32_t old = 0;
        if (lane == 0) old = __hip_atomic_fetch_add(a.sdone + s, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        old = uniform(old);
        if (old == ntask - 1) {
          // last task of the string: read and clear the sums and the counter
          complete_atomics();
          if (lane < K) {
            uint64_t v = __hip_atomic_exchange(sacc + lane, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_memcpy(o + 8 * lane, &v, 8);
            __hip_atomic_store(a.sdone + s, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
    }
    // every lane finishes the task here, before the next one starts; the
    // last region of every task copied the next one's first (when known)
    ++task;
    fetch = (next_entry >> 31) != 0;
    staged = have_next;
    __builtin_amdgcn_wave_barrier();
  }

}

// ---------------------------------------------------------------------------
// Streaming: the stack of Eq. (3) kept on the device between updates.
// stack[l][i][t][j] (l < kLevels, i < 7, t < kMaxK, j < 8) holds the i-th
// pending item of level l; counts[l] how many are pending.  One wave; lane
// t * B + j owns word (t, j) of every item.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t* stack_at(uint64_t* stack, int l, int i) {
  return stack + ((uint64_t)l * (kFan - 1) + i) * (kMaxK * kBlock);
}

// Push the nroots roots of consecutive aligned blocks, in order (root r at
// level levels[r]): an item joins its level; the 8th completes the node
// sum_{i<7} NH(item_i, S_tree[t][l][i]) + item_7, which is pushed one level
// up.  The occupied levels of the stack and the tree keys are held in LDS
// while the kernel runs (copied in, and the stack back, with many loads in
// flight), and the roots are loaded kAhead at a time, one chunk ahead of the
// pushes.
template <int WIDTH, int B>
__global__ __launch_bounds__(64) void stream_push_kernel(const uint64_t* __restrict__ ent,
                                                         const uint64_t* __restrict__ roots,
                                                         const uint32_t* __restrict__ levels, uint32_t nroots,
                                                         uint64_t* __restrict__ stack, uint32_t* __restrict__ counts) {
  using Ly = Layout<WIDTH, B>;
  constexpr int K = Family<WIDTH>::K;
  constexpr int IW = kMaxK * kBlock;  // words per stack item, [t][j]
  constexpr int kBatch = 16;          // words per lane in flight when copying
  constexpr int kKeys = K * kLevels * (kFan - 1);     // tree keys [t][level][i]
  constexpr int kAhead = 16;                           // roots per chunk
  __shared__ uint64_t lst[kLevels * (kFan - 1) * IW];
  __shared__ uint64_t lkey[kKeys];
  const int lane = threadIdx.x;
  const bool mine = lane < K * B;
  const int t = lane / B, j = lane % B, w = t * kBlock + j;
  uint32_t cnt = lane < kLevels ? counts[lane] : 0;  // lane l holds counts[l]
  auto used_words = [&]() {  // the levels up to the highest occupied one
    const uint64_t occ = __ballot(cnt != 0);
    return occ ? (64 - __clzll((long long)occ)) * (kFan - 1) * IW : 0;
  };
  const int nin = used_words();
  for (int i = lane; i < kKeys; i += 64) lkey[i] = ent[Ly::tree + i];
  for (int base = 0; base < nin; base += 64 * kBatch) {
    uint64_t buf[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int f = base + u * 64 + lane;
      buf[u] = f < nin ? stack[f] : 0;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int f = base + u * 64 + lane;
      if (f < nin) lst[f] = buf[u];
    }
  }
  __syncthreads();
  // one item into level l, closing full nodes upwards (each lane handles its
  // own word w of every item, so no cross-lane LDS traffic)
  auto push = [&](int l, uint64_t v) {
    for (;;) {
      const uint32_t c = (uint32_t)__shfl((int)cnt, l);
      if (c < kFan - 1) {
        if (mine) lst[(l * (kFan - 1) + (int)c) * IW + w] = v;
        if (lane == l) cnt = c + 1;
        return;
      }
      uint64_t node = v;
      if (mine) {
        for (int i = 0; i < kFan - 1; ++i)
          node = nh_acc(node, lst[(l * (kFan - 1) + i) * IW + w], lkey[(t * kLevels + l) * (kFan - 1) + i]);
      }
      if (lane == l) cnt = 0;
      v = node;
      ++l;
    }
  };
  // roots: chunk c + 1 in flight while chunk c is pushed (lane u of the
  // chunk's level word holds root c + u's level)
  uint64_t cur[kAhead], nxt[kAhead];
  uint32_t lcur = 0, lnxt = 0;
  auto load_chunk = [&](uint32_t c, uint64_t(&v)[kAhead], uint32_t& lv) {
#pragma unroll
    for (int u = 0; u < kAhead; ++u) v[u] = mine && c + u < nroots ? roots[(uint64_t)(c + u) * IW + w] : 0;
    lv = lane < kAhead && c + lane < nroots ? levels[c + lane] : 0;
  };
  if (nroots) load_chunk(0, cur, lcur);
  for (uint32_t c = 0; c < nroots; c += kAhead) {
    if (c + kAhead < nroots) load_chunk(c + kAhead, nxt, lnxt);
#pragma unroll
    for (int u = 0; u < kAhead; ++u)
      if (c + u < nroots) push(__shfl((int)lcur, u), cur[u]);
#pragma unroll
    for (int u = 0; u < kAhead; ++u) cur[u] = nxt[u];
    lcur = lnxt;
  }
  // occupied levels back to the device stack, and the counts
  const int nout = used_words();
  for (int base = 0; base < nout; base += 64 * kBatch) {
    uint64_t buf[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int f = base + u * 64 + lane;
      buf[u] = f < nout ? lst[f] : 0;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int f = base + u * 64 + lane;
      if (f < nout) stack[f] = buf[u];
    }
  }
  if (lane < kLevels) counts[lane] = cnt;
}

// The table of a gathered group (GatherWalk): thread k = 1 .. nseg-1 walks
// the executions of piece k from the state the host's walk had before it
// (its entries start at w_first[k]), thread nseg the joins after the last
// piece; then each wave copies the bytes of every fourth join into its slot,
// and every thread some of the group's trailing bytes (after its last full
// execution, fewer than one execution) into the carry buffer.  The old
// carried bytes (segment 0) are all read before the barrier that precedes
// that write.
static_assert(kStreamLevels == kLevels, "the stack's levels are the tree's");
__global__ __launch_bounds__(256) void stream_gather_kernel(GatherArgs g) {
  constexpr uint32_t kThreads = 256;
  constexpr int kRest = (8 * 8 * 7 * 3 + kThreads - 1) / kThreads;  // trailing bytes per thread (b = 8, d = 7, w = 3)
  static_assert(kGatherMax + 1 < (int)kThreads, "a thread per segment");
  __shared__ uint64_t js[kGatherMax];         // the joins' offsets in the concatenation
  __shared__ uint64_t segat[kGatherMax + 2];  // segment starts, then the total
  __shared__ const uint8_t* segp[kGatherMax + 1];
  const uint32_t tid = threadIdx.x;
  const uint64_t xb = g.xb;
  if (tid <= g.nseg) segat[tid] = g.w_at[tid];
  if (tid < g.nseg) segp[tid] = g.seg[tid];
  if (tid >= 1 && tid <= g.nseg) {
    const uintptr_t b = reinterpret_cast<uintptr_t>(g.base);
    uint32_t i = g.w_first[tid];
    auto block = [&](uint64_t, int L, const uint8_t* at) {
      g.off[i] = reinterpret_cast<uintptr_t>(at) - b;
      g.len[i] = xb << (3 * L);
      g.lev[i] = (uint32_t)L;
      ++i;
    };
    auto join = [&](uint32_t j, uint64_t s) {
      js[j] = s;
      g.off[i] = reinterpret_cast<uintptr_t>(g.joins + j * xb) - b;
      g.len[i] = xb;
      g.lev[i] = 0;
      ++i;
    };
    GatherWalk w(xb, g.e0, g.w_at[tid], g.w_next[tid], g.w_nj[tid]);
    if (tid < g.nseg)
      w.piece(g.seg[tid], g.seg_len[tid], block, join);
    else
      w.finish(join);
  }
  __syncthreads();
  const uint64_t nj = g.nj, r0 = g.nfull * xb, total = segat[g.nseg];
  // joins: a wave per join, each lane's segment moving forward with its bytes
  const uint32_t lane = tid % 64, wave = tid / 64;
  for (uint64_t j = wave; j < nj; j += kThreads / 64) {
    uint32_t k = 0;
    for (uint64_t i = lane; i < xb; i += 64) {
      const uint64_t s = js[j] + i;  // (< total)
      while (s >= segat[k + 1]) ++k;
      g.joins[j * xb + i] = segp[k][s - segat[k]];
    }
  }
  uint8_t rest[kRest];
  uint32_t k = 0;
#pragma unroll
  for (int u = 0; u < kRest; ++u) {
    const uint64_t s = r0 + u * kThreads + tid;
    if (s < total) {
      while (s >= segat[k + 1]) ++k;
      rest[u] = segp[k][s - segat[k]];
    } else {
      rest[u] = 0;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kRest; ++u) {
    const uint64_t s = r0 + u * kThreads + tid;
    if (s < total) g.carry[s - r0] = rest[u];
  }
}

// The hash of everything pushed so far plus the pending tail bytes: the
// final NH over the pending items (§5.2), the Toeplitz tail (§6.1) and the
// length term, as the batch kernel computes them.
template <int WIDTH, int B>
__global__ __launch_bounds__(64) void stream_final_kernel(const uint64_t* __restrict__ ent,
                                                          const uint64_t* __restrict__ stack,
                                                          const uint32_t* __restrict__ counts,
                                                          const uint8_t* __restrict__ tail, uint32_t tail_len,
                                                          uint64_t total_len, uint8_t* __restrict__ out) {
  using Ly = Layout<WIDTH, B>;
  constexpr int K = Family<WIDTH>::K;
  const int lane = threadIdx.x;
  uint64_t F[K];
#pragma unroll
  for (int t = 0; t < K; ++t) F[t] = 0;
  // pending items: lane t * B + j hashes word (t, j) of each
  if (lane < K * B) {
    const int t = lane / B, j = lane % B;
    for (int l = 0; l < kLevels; ++l) {
      const uint32_t c = counts[l];
      for (uint32_t i = 0; i < c; ++i) {
        const uint64_t key = ent[Ly::fin + ((t * kLevels + l) * (kFan - 1) + i) * B + j];
        const uint64_t v = nh_acc(0, stack_at(const_cast<uint64_t*>(stack), l, (int)i)[t * kBlock + j], key);
#pragma unroll
        for (int u = 0; u < K; ++u)
          if (u == t) F[u] += v;
      }
    }
  }
  // tail words, lane m, m + 64, ...
  const uint32_t R = (tail_len + 7) / 8;
  for (uint32_t m = lane; m < R; m += 64) {
    uint64_t w = 0;
    if (8 * m + 8 <= tail_len) {
      __builtin_memcpy(&w, tail + 8 * m, 8);
    } else {
      w = load_partial_word(tail + 8 * m, tail_len - 8 * m);
    }
#pragma unroll
    for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], w, ent[Ly::tail + t + m]);
  }
  if (lane == 0) {
#pragma unroll
    for (int t = 0; t < K; ++t) F[t] = nh_acc(F[t], total_len, ent[Ly::len + t]);
  }
#pragma unroll
  for (int t = 0; t < K; ++t) F[t] = wave_sum64(F[t]);
  if (lane < K) {
    uint64_t v = F[0];
#pragma unroll
    for (int t = 1; t < K; ++t)
      if (lane == t) v = F[t];
    __builtin_memcpy(out + 8 * lane, &v, 8);
  }
}

// ---------------------------------------------------------------------------
// Read-bandwidth probe: the achievable HBM read rate on this device, the
// ceiling the hashing kernel is compared with.  Every 16-byte piece of the
// buffer is read once: each single-wave workgroup streams its own contiguous
// share, 16 non-temporal 16-byte loads per lane in flight (1 KiB contiguous
// per load instruction; the fastest form measured on this GPU, about 7 TB/s,
// against about 6.3 TB/s for plain loads), and folds it into an XOR that is
// written out, so no load is dead.
// ---------------------------------------------------------------------------

constexpr int kProbeUnroll = 16;

__global__ __launch_bounds__(64) void read_probe_kernel(const uint4* __restrict__ p, uint64_t n16,
                                                        uint64_t* __restrict__ sink) {
  typedef unsigned int v4 __attribute__((ext_vector_type(4)));
  const uint64_t nw = gridDim.x;
  const uint64_t per = (n16 / 64 + nw - 1) / nw * 64;  // pieces per wave, a multiple of 64
  const uint64_t b = blockIdx.x * per;
  const uint64_t e = b + per < n16 ? b + per : n16;
  const v4* __restrict__ q = reinterpret_cast<const v4*>(p);
  uint32_t x = 0;
  uint64_t i = b + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * 64 < e; i += kProbeUnroll * 64) {
    v4 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(q + i + u * 64);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) x ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < e; i += 64) {
    const v4 a = __builtin_nontemporal_load(q + i);
    x ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  for (int m = 32; m >= 1; m >>= 1) x ^= __shfl_xor(x, m);
  if (threadIdx.x == 0) atomicXor(reinterpret_cast<unsigned int*>(sink + blockIdx.x), x);
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------

// Instantiates fn<W, B> for the runtime (width, block) pair.
#define HTH_DISPATCH(width, block, ...)                              \
  do {                                                               \
    if ((block) == 8) {                                              \
      switch (width) {                                               \
        case 16: { constexpr int W = 16, Bk = 8; __VA_ARGS__; } break; \
        case 24: { constexpr int W = 24, Bk = 8; __VA_ARGS__; } break; \
        case 32: { constexpr int W = 32, Bk = 8; __VA_ARGS__; } break; \
        case 40: { constexpr int W = 40, Bk = 8; __VA_ARGS__; } break; \
      }                                                              \
    } else if ((block) == 4) {                                       \
      switch (width) {                                               \
        case 16: { constexpr int W = 16, Bk = 4; __VA_ARGS__; } break; \
        case 24: { constexpr int W = 24, Bk = 4; __VA_ARGS__; } break; \
        case 32: { constexpr int W = 32, Bk = 4; __VA_ARGS__; } break; \
        case 40: { constexpr int W = 40, Bk = 4; __VA_ARGS__; } break; \
      }                                                              \
    }                                                                \
  } while (0)

const void* main_kernel_fn(uint32_t width, uint32_t block) {
  const void* f = nullptr;
  HTH_DISPATCH(width, block, f = reinterpret_cast<const void*>(&hash_main_kernel<W, Bk, false>));
  return f;
}

const void* tiny_kernel_fn(uint32_t width, uint32_t block) {
  const void* f = nullptr;
  HTH_DISPATCH(width, block, f = reinterpret_cast<const void*>(&tiny_kernel<W, Bk>));
  return f;
}

const void* small_kernel_fn(uint32_t width, uint32_t block) {
  const void* f = nullptr;
  HTH_DISPATCH(width, block, f = reinterpret_cast<const void*>(&small_kernel<W, Bk>));
  return f;
}

const void* tab_kernel_fn(uint32_t width, uint32_t block) {
  const void* f = nullptr;
  HTH_DISPATCH(width, block, f = reinterpret_cast<const void*>(&tab_kernel<W, Bk>));
  return f;
}

hipError_t launch_tab(uint32_t width, uint32_t block, const TabArgs& a, uint32_t grid, hipStream_t stream) {
  bool known = false;
  HTH_DISPATCH(width, block, {
    hipLaunchKernelGGL((tab_kernel<W, Bk>), dim3(grid), dim3(kTabThreads), 0, stream, a);
    known = true;
  });
  if (!known) return hipErrorInvalidValue;
  return hipGetLastError();
}

uint32_t exec_bytes_of(uint32_t width, uint32_t block) {
  uint32_t x = 0;
  HTH_DISPATCH(width, block, x = Layout<W, Bk>::exec_bytes);
  return x;
}

uint32_t pass_log2_of(uint32_t block) { return block == 4 ? Geo<4>::LOG_PASS : Geo<8>::LOG_PASS; }

int64_t entropy_offset_of(uint32_t width, uint32_t block) {
  return block == 4 ? width_offset<4>((int)width) : block == 8 ? width_offset<8>((int)width) : -1;
}
uint64_t entropy_words_total(uint32_t block) {
  return block == 4 ? entropy_words<4>() : block == 8 ? entropy_words<8>() : 0;
}

hipError_t launch_plan(const PlanArgs& p, hipStream_t stream) {
  const uint32_t nblocks = (uint32_t)((p.count + kPlanBlock - 1) / kPlanBlock);
  const bool scan = nblocks > kPlanScanMin;
  if (nblocks == 1) {
    hipLaunchKernelGGL(plan_single_kernel, dim3(1), dim3(kPlanThreads), 0, stream, p.lengths, p.count, p.exec_bytes,
                       p.pass_log2, p.direct_lim, p.small_max, p.cap_tasks, p.cap_accs, p.min_j, p.max_j, p.target_tasks, p.task_string,
                       p.task_start, p.acc_start, p.bucket_lead, p.tiny_list, p.small_list, p.ctl);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(plan_count_kernel, dim3(nblocks), dim3(kPlanThreads), 0, stream, p.lengths, p.count,
                     p.exec_bytes, p.pass_log2, p.direct_lim, p.small_max, p.block_sums, p.ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (scan) {
    uint32_t ngroups = (nblocks + kScanGroupMin - 1) / kScanGroupMin;
    if (ngroups > kScanGroups) ngroups = kScanGroups;
    hipLaunchKernelGGL(plan_group_kernel, dim3(ngroups), dim3(kScanThreads), 0, stream, p.block_sums, nblocks,
                       p.group_sums);
    hipLaunchKernelGGL(plan_prefix_kernel, dim3(ngroups), dim3(kScanThreads), 0, stream, p.block_sums, nblocks,
                       (const uint64_t*)p.group_sums, p.cap_tasks, p.cap_accs, p.min_j, p.max_j, p.target_tasks,
                       p.block_pre, p.ctl);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (scan)
    hipLaunchKernelGGL(plan_fill_kernel<true>, dim3(nblocks), dim3(kPlanThreads), 0, stream, p.lengths, p.count,
                       p.exec_bytes, p.pass_log2, p.direct_lim, p.small_max, p.block_sums, nblocks, (const uint64_t*)p.block_pre,
                       p.cap_tasks, p.cap_accs, p.min_j, p.max_j, p.target_tasks, p.task_string, p.task_start,
                       p.acc_start, p.bucket_lead, p.tiny_list, p.small_list, p.ctl);
  else
    hipLaunchKernelGGL(plan_fill_kernel<false>, dim3(nblocks), dim3(kPlanThreads), 0, stream, p.lengths, p.count,
                       p.exec_bytes, p.pass_log2, p.direct_lim, p.small_max, p.block_sums, nblocks, (const uint64_t*)nullptr,
                       p.cap_tasks, p.cap_accs, p.min_j, p.max_j, p.target_tasks, p.task_string, p.task_start,
                       p.acc_start, p.bucket_lead, p.tiny_list, p.small_list, p.ctl);
  return hipGetLastError();
}

hipError_t launch_main(uint32_t width, uint32_t block, const MainArgs& a, uint32_t grid, uint32_t tiny_grid,
                       uint32_t small_grid, hipStream_t stream) {
  // the hashing kernel, then the tail-only and the small strings
  bool known = false;
  HTH_DISPATCH(width, block, {
    hipLaunchKernelGGL((hash_main_kernel<W, Bk, false>), dim3(grid), dim3(64), 0, stream, a);
    hipLaunchKernelGGL((tiny_kernel<W, Bk>), dim3(tiny_grid), dim3(64), 0, stream, a);
    hipLaunchKernelGGL((small_kernel<W, Bk>), dim3(small_grid), dim3(64), 0, stream, a);
    known = true;
  });
  if (!known) return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_roots(uint32_t width, uint32_t block, const MainArgs& a, uint32_t grid, hipStream_t stream) {
  bool known = false;
  HTH_DISPATCH(width, block, {
    hipLaunchKernelGGL((hash_main_kernel<W, Bk, true>), dim3(grid), dim3(64), 0, stream, a);
    known = true;
  });
  if (!known) return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_stream_push(uint32_t width, uint32_t block, const uint64_t* ent, const uint64_t* roots,
                              const uint32_t* levels, uint32_t nroots, uint64_t* stack, uint32_t* counts,
                              hipStream_t stream) {
  bool known = false;
  HTH_DISPATCH(width, block, {
    hipLaunchKernelGGL((stream_push_kernel<W, Bk>), dim3(1), dim3(64), 0, stream, ent, roots, levels, nroots, stack,
                       counts);
    known = true;
  });
  if (!known) return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_stream_gather(const GatherArgs& g, hipStream_t stream) {
  hipLaunchKernelGGL(stream_gather_kernel, dim3(1), dim3(256), 0, stream, g);
  return hipGetLastError();
}

hipError_t launch_stream_final(uint32_t width, uint32_t block, const uint64_t* ent, const uint64_t* stack,
                               const uint32_t* counts, const uint8_t* tail, uint32_t tail_len, uint64_t total_len,
                               uint8_t* out, hipStream_t stream) {
  bool known = false;
  HTH_DISPATCH(width, block, {
    hipLaunchKernelGGL((stream_final_kernel<W, Bk>), dim3(1), dim3(64), 0, stream, ent, stack, counts, tail,
                       tail_len, total_len, out);
    known = true;
  });
  if (!known) return hipErrorInvalidValue;
  return hipGetLastError();
}

uint64_t plan_block_count(uint64_t count) { return (count + kPlanBlock - 1) / kPlanBlock; }

hipError_t launch_read_probe(const void* buf, uint64_t n16, uint64_t* sink, uint32_t blocks, hipStream_t stream) {
  hipLaunchKernelGGL(read_probe_kernel, dim3(blocks), dim3(64), 0, stream,
                     reinterpret_cast<const uint4*>(buf), n16, sink);
  return hipGetLastError();
}

}  // namespace hth
