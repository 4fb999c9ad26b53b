// Gather / scatter kernels that pack many small sort requests into one
// segmented sort (used by the sort server): one launch copies every
// request's keys into the packed input, one launch copies every request's
// sorted keys and permutation back.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.hpp"

namespace rs {

template <typename T>
__global__ __launch_bounds__(256) void k_batch_in(const BatchEntry* tab, uint32_t count, T* packed) {
  for (uint32_t r = blockIdx.x; r < count; r += gridDim.x) {
    const BatchEntry e = tab[r];
    const T* s = (const T*)e.src;
    T* d = packed + e.off;
    for (uint64_t j = threadIdx.x; j < e.n; j += blockDim.x) d[j] = s[j];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_batch_out(const BatchEntry* tab, uint32_t count, const T* keys,
                                                   const uint32_t* perm) {
  for (uint32_t r = blockIdx.x; r < count; r += gridDim.x) {
    const BatchEntry e = tab[r];
    T* dk = (T*)e.dst_keys;
    for (uint64_t j = threadIdx.x; j < e.n; j += blockDim.x) dk[j] = keys[e.off + j];
    if (e.dst_perm)
      for (uint64_t j = threadIdx.x; j < e.n; j += blockDim.x) e.dst_perm[j] = perm[e.off + j];
  }
}

int enqueue_batch_in(const BatchEntry* tab_dev, uint32_t count, uint32_t key_bytes, void* packed, hipStream_t st) {
  const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>(count, num_cu_cached() * 4));
  if (key_bytes == 8)
    RS_LAUNCH(k_batch_in<uint64_t>, g, 256, st, tab_dev, count, (uint64_t*)packed);
  else
    RS_LAUNCH(k_batch_in<uint32_t>, g, 256, st, tab_dev, count, (uint32_t*)packed);
  return 0;
}

int enqueue_batch_out(const BatchEntry* tab_dev, uint32_t count, uint32_t key_bytes, const void* keys,
                      const uint32_t* perm, hipStream_t st) {
  const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>(count, num_cu_cached() * 4));
  if (key_bytes == 8)
    RS_LAUNCH(k_batch_out<uint64_t>, g, 256, st, tab_dev, count, (const uint64_t*)keys, perm);
  else
    RS_LAUNCH(k_batch_out<uint32_t>, g, 256, st, tab_dev, count, (const uint32_t*)keys, perm);
  return 0;
}

}  // namespace rs
