// Binary-tree approximate median with a single reduction (paper Section 3.2)
// as a device primitive over many independent problems.
//
// Window entries are (value, class) with class 0 = below everything,
// 1 = real value, 2 = above everything; they are compared by class first.
// Level 0 computes every leaf's window from its (unsorted) slice by ranking
// the slice's values; level l merges sibling windows and keeps the middle k;
// the root picks one of its two middle entries by its coin.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace rs {

struct MWin {
  uint64_t v;
  uint32_t cls;
  uint32_t pad;
};

__device__ __forceinline__ bool mw_less(const MWin& a, const MWin& b) {
  if (a.cls != b.cls) return a.cls < b.cls;
  return a.cls == 1 && a.v < b.v;
}

// One thread per (problem, leaf).
__global__ void k_med_leaf(const uint64_t* vals, uint64_t per_problem, const uint64_t* leaf_off, uint32_t log2_p,
                           uint32_t k, const uint8_t* coins, uint32_t num_problems, MWin* win, int32_t* status) {
  const uint64_t p = 1ull << log2_p;
  const uint64_t total = p * num_problems;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t q = g >> log2_p, l = g & (p - 1);
    const uint64_t a = leaf_off[q * (p + 1) + l], b = leaf_off[q * (p + 1) + l + 1];
    MWin* w = win + g * k;
    if (b < a || b - a > 64 || b > per_problem) {
      atomicCAS(status, 0, -1);
      for (uint32_t i = 0; i < k; i++) w[i] = MWin{0, 1, 0};
      continue;
    }
    const uint32_t m = (uint32_t)(b - a);
    const uint64_t* x = vals + q * per_problem + a;
    uint32_t h = m / 2;
    if (m & 1) h += coins[q * (p + 1) + l] ? 1u : 0u;
    // window position i holds the slice element of rank h - k/2 + i
    for (uint32_t i = 0; i < k; i++) {
      const int r = (int)h - (int)(k / 2) + (int)i;
      w[i] = MWin{0, r < 0 ? 0u : 2u, 0};
    }
    for (uint32_t i = 0; i < m; i++) {
      uint32_t r = 0;
      for (uint32_t j = 0; j < m; j++) r += x[j] < x[i] ? 1u : 0u;
      const int slot = (int)r - ((int)h - (int)(k / 2));
      if (slot >= 0 && slot < (int)k) w[slot] = MWin{x[i], 1u, 0};
    }
  }
}

// One thread per (problem, parent node, entry of the two children windows).
__global__ void k_med_merge(const MWin* in, MWin* out, uint64_t parents_per_problem, uint32_t num_problems,
                            uint32_t k) {
  const uint64_t total = parents_per_problem * num_problems * 2 * k;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t node = g / (2 * k);  // global parent index (problem-major)
    const uint32_t e = (uint32_t)(g % (2 * k));
    const MWin* A = in + (2 * node) * k;
    const MWin* B = in + (2 * node + 1) * k;
    MWin x;
    uint32_t pos;
    if (e < k) {
      x = A[e];
      uint32_t c = 0;  // entries of B strictly below x
      for (uint32_t t = 0; t < k; t++) c += mw_less(B[t], x) ? 1u : 0u;
      pos = e + c;
    } else {
      x = B[e - k];
      uint32_t c = 0;  // entries of A not above x (ties: A first)
      for (uint32_t t = 0; t < k; t++) c += mw_less(x, A[t]) ? 0u : 1u;
      pos = (e - k) + c;
    }
    if (pos >= k / 2 && pos < k / 2 + k) out[node * k + (pos - k / 2)] = x;
  }
}

__global__ void k_med_root(const MWin* win, const uint8_t* coins, uint64_t p, uint32_t num_problems, uint32_t k,
                           uint64_t* out) {
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < num_problems; q += gridDim.x * blockDim.x) {
    const uint32_t c = coins[q * (p + 1) + p] ? 1u : 0u;
    const MWin r = win[(uint64_t)q * k + (k / 2 - 1 + c)];
    out[2 * q] = r.cls == 1 ? r.v : 0ull;
    out[2 * q + 1] = r.cls == 1 ? 0ull : (r.cls == 0 ? 1ull : 2ull);
  }
}

size_t median_tree_workspace(uint32_t log2_p, uint32_t k, uint32_t num_problems) {
  const uint64_t p = 1ull << log2_p;
  return 256 + 2 * (size_t)p * num_problems * k * sizeof(MWin);
}

int enqueue_median_tree(const uint64_t* vals, uint64_t per_problem, const uint64_t* leaf_off, uint32_t log2_p,
                        uint32_t k, const uint8_t* coins, uint32_t num_problems, uint64_t* out, void* ws,
                        size_t ws_bytes, hipStream_t st) {
  if (num_problems == 0) return 0;
  if (ws_bytes < median_tree_workspace(log2_p, k, num_problems)) return -2;
  const uint64_t p = 1ull << log2_p;
  int32_t* status = (int32_t*)ws;
  MWin* w0 = (MWin*)((char*)ws + 256);
  MWin* w1 = w0 + p * num_problems * k;
  const uint32_t cu = num_cu_cached();
  auto grid = [&](uint64_t work) { return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((work + 255) / 256, cu * 8ull)); };
  RS_LAUNCH(k_med_leaf, grid(p * num_problems), 256, st, vals, per_problem, leaf_off, log2_p, k, coins, num_problems,
            w0, status);
  MWin* a = w0;
  MWin* b = w1;
  for (uint64_t parents = p / 2; parents >= 1; parents /= 2) {
    RS_LAUNCH(k_med_merge, grid(parents * num_problems * 2 * k), 256, st, a, b, parents, num_problems, k);
    std::swap(a, b);
  }
  RS_LAUNCH(k_med_root, grid(num_problems), 256, st, a, coins, p, num_problems, k, out);
  return 0;
}

}  // namespace rs
