// hth_hash_batch_noalloc: the batched hash for callers that cannot allocate
// device memory.  The planner's arrays and the cross-task accumulators that
// hth_hash_batch keeps in a per-stream workspace live here in one static
// device array per GPU, `scratch`, of fixed size; the call runs the same
// planner and kernels as hth_hash_batch on it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/hth.h"
#include "hth_host.h"
#include "hth_kernels.h"

namespace {

using hth::host::Workspace;

// Limits of the static workspace (the planner chooses coarser tasks when a
// batch would need more tasks or accumulators; with these limits that only
// happens above about 10^14 bytes of strings in one batch, reachable only with
// overlapping strings, and is then reported by hth_batch_check).
constexpr uint64_t kNaCount = HTH_NOALLOC_MAX_COUNT;
constexpr uint64_t kNaTasks = kNaCount + (1u << 16);
constexpr uint64_t kNaAccs = 8192;
constexpr uint64_t kNaBlocks = (kNaCount + 1023) / 1024;

constexpr size_t up256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kOffCtl = 0;
constexpr size_t kOffBs = kOffCtl + up256(hth::kCtlWords * 4);
constexpr size_t kOffBp = kOffBs + up256(kNaBlocks * hth::kBlockSums * 8);
constexpr size_t kOffGs = kOffBp + up256(kNaBlocks * hth::kPlanPre * 8);
constexpr size_t kOffTs = kOffGs + up256((size_t)hth::kScanGroups * hth::kBlockSums * 8);
constexpr size_t kOffSt = kOffTs + up256(kNaTasks * 4);
constexpr size_t kOffAs = kOffSt + up256(kNaCount * 4);
constexpr size_t kOffTl = kOffAs + up256(kNaCount * 4);
constexpr size_t kOffSl = kOffTl + up256(kNaCount * 4);
constexpr size_t kOffBl = kOffSl + up256(kNaCount * 4);
constexpr size_t kOffSacc = kOffBl + up256(((size_t)hth::kMaxBuckets + 2) * 4);
constexpr size_t kOffSdone = kOffSacc + up256(kNaCount * hth::kMaxK * 8);
constexpr size_t kOffGacc = kOffSdone + up256(kNaCount * 4);
constexpr size_t kOffGcnt = kOffGacc + up256(kNaAccs * hth::kMaxK * 8 * 8);
constexpr size_t kNaBytes = kOffGcnt + up256(kNaAccs * 4);
static_assert(kNaBytes == HTH_NOALLOC_SCRATCH_BYTES, "scratch size in include/hth.h");

// The static workspace.  Its name is a host-side stand-in in host code: the
// device address of each GPU's copy comes from hipGetSymbolAddress.
__device__ __align__(256) uint8_t scratch[kNaBytes];

constexpr int kMaxDevices = 64;
std::mutex g_na_mu;
uint8_t* g_na_ptr[kMaxDevices];        // device address of scratch, per device
hipStream_t g_na_stream[kMaxDevices];  // stream of the last call, per device
bool g_na_used[kMaxDevices];

__global__ void na_clear_kernel(uint4* p, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0, 0, 0, 0);
}

// This device's scratch address; on the first call on a device, looks it up
// and enqueues a clear (a kernel, so that the call stays capturable).
hth_status na_scratch(int dev, hipStream_t stream, uint8_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return hth::host::fail(HTH_E_INVALID, "hth_hash_batch_noalloc: device %d", dev);
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hth::host::hip_fail(e, "hipGetSymbolAddress(scratch)");
    hipLaunchKernelGGL(na_clear_kernel, dim3(256), dim3(256), 0, stream, static_cast<uint4*>(p), kNaBytes / 16);
    e = hipGetLastError();
    if (e != hipSuccess) return hth::host::hip_fail(e, "scratch clear");
    g_na_ptr[dev] = static_cast<uint8_t*>(p);
  }
  g_na_stream[dev] = stream;
  g_na_used[dev] = true;
  *out = g_na_ptr[dev];
  return HTH_OK;
}

Workspace na_workspace(uint8_t* b) {
  Workspace w;
  w.cap_count = kNaCount;
  w.cap_tasks = kNaTasks;
  w.cap_accs = kNaAccs;
  w.cap_blocks = kNaBlocks;
  w.mem = b;
  w.bytes = kNaBytes;
  w.ctl = reinterpret_cast<uint32_t*>(b + kOffCtl);
  w.block_sums = reinterpret_cast<uint64_t*>(b + kOffBs);
  w.block_pre = reinterpret_cast<uint64_t*>(b + kOffBp);
  w.group_sums = reinterpret_cast<uint64_t*>(b + kOffGs);
  w.task_string = reinterpret_cast<uint32_t*>(b + kOffTs);
  w.task_start = reinterpret_cast<uint32_t*>(b + kOffSt);
  w.acc_start = reinterpret_cast<uint32_t*>(b + kOffAs);
  w.tiny_list = reinterpret_cast<uint32_t*>(b + kOffTl);
  w.small_list = reinterpret_cast<uint32_t*>(b + kOffSl);
  w.bucket_lead = reinterpret_cast<uint32_t*>(b + kOffBl);
  w.sacc = reinterpret_cast<uint64_t*>(b + kOffSacc);
  w.sdone = reinterpret_cast<uint32_t*>(b + kOffSdone);
  w.gacc = reinterpret_cast<uint64_t*>(b + kOffGacc);
  w.gcnt = reinterpret_cast<uint32_t*>(b + kOffGcnt);
  w.hbuf = nullptr;
  return w;
}

}  // namespace

namespace hth {
namespace host {

uint32_t* noalloc_ctl_for(int dev, hipStream_t stream) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_used[dev] || g_na_stream[dev] != stream) return nullptr;
  return reinterpret_cast<uint32_t*>(g_na_ptr[dev] + kOffCtl);
}

}  // namespace host
}  // namespace hth

extern "C" hth_status hth_hash_batch_noalloc(const hth_seed* seed, const uint8_t* bytes, const uint64_t* offsets,
                                             const uint64_t* lengths, uint64_t count, uint8_t* out,
                                             uint32_t out_width, hipStream_t stream) {
  if (count > kNaCount)
    return hth::host::fail(HTH_E_TOO_LARGE, "hth_hash_batch_noalloc: count %llu exceeds the static workspace's %llu",
                           (unsigned long long)count, (unsigned long long)kNaCount);
  hth_status st = hth::host::check_batch_args(seed, bytes, offsets, lengths, count, out, out_width);
  if (st != HTH_OK || count == 0) return st;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hth::host::hip_fail(e, "hipGetDevice");
  uint8_t* b = nullptr;
  st = na_scratch(dev, stream, &b);
  if (st != HTH_OK) return st;
  Workspace w = na_workspace(b);
  return hth::host::enqueue_batch(seed, bytes, offsets, lengths, count, out, out_width, w, stream, nullptr, nullptr);
}
