// Composition of HalftimeHash with a short-input family (§1: a universe-
// collapsing family reduces long strings to short values that a short-input
// family hashes as if they were the input; §7: pairing HalftimeHash with a
// fast short-input family).  The short-input family is simple tabulation:
// c + 1 byte characters, one table of 256 random words per character, the
// result the XOR of the characters' entries.  A string of at most c bytes is
// its own key (zero-padded, separator character = its length); a longer
// string's key is its c-byte HalftimeHash value with separator 255.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hth_kernels.h"

namespace hth {
namespace {

// One workgroup of kTabThreads per compute unit shares one LDS copy of the
// tables ((c + 1) * 2 KiB); its threads take strings with a grid stride,
// loading the next string's offset, length and HalftimeHash value (every row
// of h exists; a short string's row is simply not used) while the current
// one is tabulated.
template <int C>
__global__ __launch_bounds__(kTabThreads) void tab_kernel(TabArgs a) {
  constexpr int NW = C / 8;
  __shared__ uint64_t T[(C + 1) * 256];
  for (int i = threadIdx.x; i < (C + 1) * 256; i += kTabThreads) T[i] = a.tables[i];
  const uint64_t stride = (uint64_t)gridDim.x * kTabThreads;
  auto fetch = [&](uint64_t i, uint64_t& L, uint64_t& off, uint64_t (&hv)[NW]) {
    if (i < a.count) {
      L = a.lengths[i];
      off = a.offsets[i];
      const uint64_t* h = reinterpret_cast<const uint64_t*>(a.h + i * C);
#pragma unroll
      for (int j = 0; j < NW; ++j) hv[j] = h[j];
    }
  };
  uint64_t s = (uint64_t)blockIdx.x * kTabThreads + threadIdx.x;
  uint64_t L = 0, off = 0, hv[NW];
  fetch(s, L, off, hv);
  __syncthreads();
  for (; s < a.count; s += stride) {
    uint64_t Ln = 0, offn = 0, hn[NW];
    fetch(s + stride, Ln, offn, hn);
    uint64_t w[NW];
    uint32_t sep;
    if (L <= (uint64_t)C) {
      // the string itself, zero-padded (unrolled: constant register indices)
      const uint8_t* p = a.bytes + off;
#pragma unroll
      for (int j = 0; j < NW; ++j) w[j] = 0;
#pragma unroll
      for (int i = 0; i < C; ++i)
        if ((uint64_t)i < L) w[i / 8] |= (uint64_t)p[i] << (8 * (i % 8));
      sep = (uint32_t)L;
    } else {
#pragma unroll
      for (int j = 0; j < NW; ++j) w[j] = hv[j];
      sep = 255;
    }
    uint64_t z = T[C * 256 + sep];
#pragma unroll
    for (int i = 0; i < C; ++i) z ^= T[i * 256 + (uint32_t)((w[i / 8] >> (8 * (i % 8))) & 0xFF)];
    a.out[s] = z;
    L = Ln;
    off = offn;
#pragma unroll
    for (int j = 0; j < NW; ++j) hv[j] = hn[j];
  }
}

}  // namespace

const void* tab_kernel_fn(uint32_t width) {
  switch (width) {
    case 16: return reinterpret_cast<const void*>(&tab_kernel<16>);
    case 24: return reinterpret_cast<const void*>(&tab_kernel<24>);
    case 32: return reinterpret_cast<const void*>(&tab_kernel<32>);
    case 40: return reinterpret_cast<const void*>(&tab_kernel<40>);
    default: return nullptr;
  }
}

hipError_t launch_tab(uint32_t width, const TabArgs& a, uint32_t grid, hipStream_t stream) {
  switch (width) {
    case 16: hipLaunchKernelGGL(tab_kernel<16>, dim3(grid), dim3(kTabThreads), 0, stream, a); break;
    case 24: hipLaunchKernelGGL(tab_kernel<24>, dim3(grid), dim3(kTabThreads), 0, stream, a); break;
    case 32: hipLaunchKernelGGL(tab_kernel<32>, dim3(grid), dim3(kTabThreads), 0, stream, a); break;
    case 40: hipLaunchKernelGGL(tab_kernel<40>, dim3(grid), dim3(kTabThreads), 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace hth
