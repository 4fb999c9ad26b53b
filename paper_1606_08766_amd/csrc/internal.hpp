// Host-side interfaces between the translation units of librsort.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "engine.hpp"

namespace rs {

struct Tuning {
  uint32_t oversample = 32;   // samples per bucket
  uint32_t target = 6144;     // bucket size a level aims for (at most cap / 2)
  uint32_t cap = 12288;       // largest bucket sorted in LDS
  uint32_t max_levels = 4;
  uint32_t rfis_max = 64;     // classes with upper bound <= rfis_max use RFIS
  uint32_t rquick_max = 1;    // classes with upper bound <= rquick_max use RQuick
  uint64_t seed = 0x5EED5EED12345678ull;
  uint32_t tile_log2 = 13;  // scatter tile: 2^tile_log2 keys
  uint32_t force_fallback = 0;
  uint32_t extra_levels = 0;  // sample-sort levels beyond the fewest needed
  uint32_t class_shape = 0;   // bit c: class c uses its alternative workgroup shape
};

Tuning& tuning();

// Enqueue a full sort.  seg_off == nullptr means one segment [0, n).
// Returns 0, -1 (bad argument), -2 (workspace too small), -3 (launch failed).
int enqueue_sort(int kt, const void* keys_in, const uint32_t* pay_in, const uint64_t* seg_off, uint32_t num_segs,
                 uint64_t n, void* keys_out, uint32_t* perm_out, uint32_t* pay_out, void* ws, size_t ws_bytes,
                 hipStream_t st);
size_t workspace_bytes(int kt, uint64_t n, uint32_t num_segs, bool pay);

// Per-class local sorts (final segments of class c, read from the class list
// in the workspace).  Merge sort: engine.hip; RFIS / RQuick: small.hip.
template <typename K, bool F32, bool PAY>
int launch_merge_class(int c, const Work& w, const K* kin, const uint32_t* pay_in, K* kout, uint32_t* perm_out,
                       uint32_t* pay_out, uint64_t cap_c, hipStream_t st);
template <typename K, bool F32, bool PAY>
int launch_rfis_class(int c, const Work& w, const K* kin, const uint32_t* pay_in, K* kout, uint32_t* perm_out,
                      uint32_t* pay_out, uint64_t cap_c, hipStream_t st);
template <typename K, bool F32, bool PAY>
int launch_rquick_class(int c, const Work& w, const K* kin, const uint32_t* pay_in, K* kout, uint32_t* perm_out,
                        uint32_t* pay_out, uint64_t cap_c, hipStream_t st);

// Segments the word sorts handed over (merge sort of words, then pair sort),
// launched once after all classes (local.hip).
template <typename K, bool F32, bool PAY>
int launch_local_fallbacks(const Work& w, uint32_t cap, const K* kin, const uint32_t* pay_in, K* kout,
                           uint32_t* perm_out, uint32_t* pay_out, hipStream_t st);

// Global-memory fallback sort of final segments longer than cap (local.hip).
template <typename K, bool F32, bool PAY>
int launch_oversize(const Work& w, const K* kin, const uint32_t* pay_in, K* kout, uint32_t* perm_out,
                    uint32_t* pay_out, uint64_t cap_c, hipStream_t st);

// Sort of up to 2^36 keys with 64-bit positions (wide.hip).
size_t wide_workspace_bytes(int kt, uint64_t n);
int enqueue_wide(int kt, const void* keys_in, uint64_t n, void* keys_out, uint64_t* perm_out, void* ws,
                 size_t ws_bytes, hipStream_t st);

// Device binary-tree median (median.hip).
size_t median_tree_workspace(uint32_t log2_p, uint32_t k, uint32_t num_problems);
int enqueue_median_tree(const uint64_t* vals, uint64_t per_problem, const uint64_t* leaf_off, uint32_t log2_p,
                        uint32_t k, const uint8_t* coins, uint32_t num_problems, uint64_t* out, void* ws,
                        size_t ws_bytes, hipStream_t st);

// Hypercube quicksort with workgroups as PEs (rquick_mw.hip).
bool rquick_mw_shape_ok(uint64_t n, uint32_t log2_p, uint32_t k);
size_t rquick_mw_workspace(uint64_t n, uint32_t log2_p);
int enqueue_rquick_mw(bool f32, const uint32_t* keys_in, uint64_t n, uint32_t log2_p, uint32_t k, int tie_break,
                      uint64_t seed, uint32_t* keys_out, uint32_t* perm_out, uint32_t* load_out, void* ws,
                      size_t ws_bytes, hipStream_t st);

// One request of a packed batch (sort server): source keys, destination
// keys / permutation, length and offset inside the packed arrays.
struct BatchEntry {
  const void* src;
  void* dst_keys;
  uint32_t* dst_perm;
  uint64_t n;
  uint64_t off;
};
int enqueue_batch_in(const BatchEntry* tab_dev, uint32_t count, uint32_t key_bytes, void* packed, hipStream_t st);
int enqueue_batch_out(const BatchEntry* tab_dev, uint32_t count, uint32_t key_bytes, const void* keys,
                      const uint32_t* perm, hipStream_t st);

uint32_t num_cu_cached();
uint32_t class_max(int c);  // upper bound of final-bucket size class c

}  // namespace rs

namespace rs {
// Kernel timing (measurement support): when enabled, every launch made
// through RS_LAUNCH is bracketed by HIP events on its stream.
bool timing_enabled();
void timing_before(hipStream_t st);
void timing_after(const char* tag, hipStream_t st);
}  // namespace rs

#define RS_LAUNCH(kern, grid, block, stream, ...) RS_LAUNCH_TAGGED(kern, #kern, grid, block, stream, __VA_ARGS__)

// Same, with an explicit timing tag (for launches whose shape is a template
// parameter of the launching function).
#define RS_LAUNCH_TAGGED(kern, tag, grid, block, stream, ...)                                 \
  do {                                                                                        \
    const bool rs_t_ = ::rs::timing_enabled();                                                \
    if (rs_t_) ::rs::timing_before((hipStream_t)(stream));                                    \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, (hipStream_t)(stream), __VA_ARGS__); \
    if (hipPeekAtLastError() != hipSuccess) return -3;                                        \
    if (rs_t_) ::rs::timing_after(tag, (hipStream_t)(stream));                                \
  } while (0)
