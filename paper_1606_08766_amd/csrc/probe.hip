// Bandwidth probes (measurement support): a read-only kernel and a copy
// kernel over device memory, both moving 16 bytes per lane per access with
// several independent accesses in flight per thread.  Their measured rates
// are the practical HBM ceilings against which the sort's passes are read.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/rsort.h"
#include "internal.hpp"

namespace rs {

constexpr int kProbeThreads = 256, kProbeUnroll = 4;

// Reads every 16-byte word of src once; each block writes one word (the xor
// of what it read) to out[blockIdx.x] so the loads cannot be dropped.
__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const uint4* src, uint64_t words, uint32_t* out) {
  uint32_t acc = 0;
  const uint64_t stride = (uint64_t)gridDim.x * kProbeThreads * kProbeUnroll;
  for (uint64_t base = (uint64_t)blockIdx.x * kProbeThreads * kProbeUnroll + threadIdx.x; base < words;
       base += stride) {
    uint4 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; u++) {
      const uint64_t i = base + (uint64_t)u * kProbeThreads;
      v[u] = i < words ? src[i] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < kProbeUnroll; u++) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (int d = 32; d > 0; d >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, d, 64);
  __shared__ uint32_t s[kProbeThreads / 64];
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0;
    for (int w = 0; w < kProbeThreads / 64; w++) a ^= s[w];
    out[blockIdx.x] = a;
  }
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const uint4* src, uint4* dst, uint64_t words) {
  const uint64_t stride = (uint64_t)gridDim.x * kProbeThreads * kProbeUnroll;
  for (uint64_t base = (uint64_t)blockIdx.x * kProbeThreads * kProbeUnroll + threadIdx.x; base < words;
       base += stride) {
    uint4 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; u++) {
      const uint64_t i = base + (uint64_t)u * kProbeThreads;
      if (i < words) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < kProbeUnroll; u++) {
      const uint64_t i = base + (uint64_t)u * kProbeThreads;
      if (i < words) dst[i] = v[u];
    }
  }
}

}  // namespace rs

extern "C" int rsort_bandwidth_probe(int kind, const void* src, void* dst, uint64_t bytes, void* stream) {
  if ((kind != 0 && kind != 1) || !src || !dst || (bytes & 15) || (((uintptr_t)src | (uintptr_t)dst) & 15))
    return RSORT_EINVAL;
  if (bytes == 0) return RSORT_OK;
  const uint64_t words = bytes / 16;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>((words + rs::kProbeThreads * rs::kProbeUnroll - 1) / (rs::kProbeThreads * rs::kProbeUnroll),
                            (uint64_t)rs::num_cu_cached() * 8));
  hipStream_t st = (hipStream_t)stream;
  if (kind == 0)
    hipLaunchKernelGGL(rs::k_probe_read, dim3(grid), dim3(rs::kProbeThreads), 0, st, (const uint4*)src, words,
                       (uint32_t*)dst);
  else
    hipLaunchKernelGGL(rs::k_probe_copy, dim3(grid), dim3(rs::kProbeThreads), 0, st, (const uint4*)src,
                       (uint4*)dst, words);
  return hipPeekAtLastError() == hipSuccess ? RSORT_OK : RSORT_EDEVICE;
}
