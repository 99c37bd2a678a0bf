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
// tables ((c + 1) * 2 KiB); its threads take strings with a grid stride in a
// two-deep pipeline: while string i is tabulated, the bytes of string
// i + stride (a short one's own bytes; every row of h exists, a short
// string's row is simply not used) and the offset, length and HalftimeHash
// value of string i + 2 stride are in flight.
template <int C>
__global__ __launch_bounds__(kTabThreads) void tab_kernel(TabArgs a) {
  constexpr int NW = C / 8;
  __shared__ uint64_t T[(C + 1) * 256];
  for (int i = threadIdx.x; i < (C + 1) * 256; i += kTabThreads) T[i] = a.tables[i];
  const uint64_t stride = (uint64_t)gridDim.x * kTabThreads;
  struct Meta {
    uint64_t L = 0, off = 0, hv[NW] = {};
  };
  auto fetch = [&](uint64_t i, Meta& m) {
    if (i < a.count) {
      m.L = a.lengths[i];
      m.off = a.offsets[i];
      const uint64_t* h = reinterpret_cast<const uint64_t*>(a.h + i * C);
#pragma unroll
      for (int j = 0; j < NW; ++j) m.hv[j] = h[j];
    }
  };
  // the key's characters 0 .. C-1: a short string's zero-padded bytes (one
  // load per byte, all issued together), else the inner value
  auto bytes_of = [&](const Meta& m, uint8_t (&by)[C]) {
#pragma unroll
    for (int i = 0; i < C; ++i) by[i] = (uint64_t)i < m.L && m.L <= (uint64_t)C ? a.bytes[m.off + i] : 0;
  };
  uint64_t s = (uint64_t)blockIdx.x * kTabThreads + threadIdx.x;
  Meta m0, m1;
  fetch(s, m0);
  fetch(s + stride, m1);
  uint8_t b0[C];
  bytes_of(m0, b0);
  __syncthreads();
  for (; s < a.count; s += stride) {
    Meta m2;
    fetch(s + 2 * stride, m2);
    uint8_t b1[C];
    bytes_of(m1, b1);
    uint64_t w[NW];
    uint32_t sep;
    if (m0.L <= (uint64_t)C) {
#pragma unroll
      for (int j = 0; j < NW; ++j) w[j] = 0;
#pragma unroll
      for (int i = 0; i < C; ++i) w[i / 8] |= (uint64_t)b0[i] << (8 * (i % 8));
      sep = (uint32_t)m0.L;
    } else {
#pragma unroll
      for (int j = 0; j < NW; ++j) w[j] = m0.hv[j];
      sep = 255;
    }
    uint64_t z = T[C * 256 + sep];
#pragma unroll
    for (int i = 0; i < C; ++i) z ^= T[i * 256 + (uint32_t)((w[i / 8] >> (8 * (i % 8))) & 0xFF)];
    a.out[s] = z;
    m0 = m1;
    m1 = m2;
#pragma unroll
    for (int i = 0; i < C; ++i) b0[i] = b1[i];
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
