// Internal layout shared by the host driver and the kernels of the
// multilevel sample sort engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

constexpr int kMaxLogK = 9;               // at most 512 buckets per level
constexpr int kMaxK = 1 << kMaxLogK;
constexpr int kMaxLevels = 8;
constexpr int kNumClasses = 10;           // final-bucket size classes (see the class table in engine.hip)
constexpr uint32_t kMaxOversample = 32;
// A segment's keys are handled in aligned groups of 2^group_log2 keys (a
// power of two between kGroupMinLog2 and kGroupMaxLog2, chosen per call so
// that the groups of n keys occupy the whole GPU), each by one workgroup;
// histograms and offsets are kept per (bucket, group), so the count and
// scatter passes may use different tile sizes inside a group.
constexpr uint32_t kGroupMinLog2 = 12, kGroupMaxLog2 = 17;

// A segment that the current level splits.
struct BigSeg {
  uint64_t start;  // global position of the first element
  uint64_t ubase;  // position of the user segment start (input-sourced levels: idx = pos - ubase)
  uint32_t len;    // number of elements
  uint32_t logk;   // this segment is split into 1 << logk buckets
};

// A bucket (or a whole user segment) that is sorted in one workgroup.
struct FinalSeg {
  uint64_t start;
  uint32_t len;
  uint32_t src;  // low byte: 0 caller input (positions implicit), 1 buffer A, 2 buffer B;
                 // kPairsFlag: handed from the word sort to the pair sort;
                 // kMergeFlag: handed from the binned word sort to the merged one
};
constexpr uint32_t kPairsFlag = 0x100;
constexpr uint32_t kMergeFlag = 0x200;

// Control block at the start of the workspace (all counters device-side).
struct Ctl {
  int32_t status;                  // RSORT_OK or a device-detected error
  uint32_t levels;                 // levels enqueued by the host
  uint32_t big_count[2];           // ping-pong lists of segments to split
  uint32_t total_groups;           // tile groups of the current level
  uint32_t total_counts;           // entries of the current level's count matrix
  uint32_t scan_next;              // next chunk of the count matrix to scan (chained scan)
  uint32_t runs;                   // (tile, bucket) runs the first level's scatter wrote
  uint32_t glog;                   // log2 keys per tile group of the levels after the first (0: as planned)
  uint32_t ids0;                   // 1: the first level (one segment) passes bucket ids from count to scatter
  uint32_t class_in[kNumClasses];  // segmented calls: user segments at the front of each class list
  uint32_t queue[2][8];            // per-XCD tile-group queues of the count and scatter passes
  uint32_t class_count[kNumClasses];  // final segments per size class (last = oversize)
  uint32_t level_max[kMaxLevels];  // largest bucket created per level
  uint32_t level_buckets[kMaxLevels];
  uint64_t class_keys[kNumClasses];  // keys routed to each size class
  // diagnostics of level 0, segment 0
  uint32_t l0_k;
  uint32_t pad0;
  uint64_t l0_spl_key[kMaxK];      // ordinal keys, sorted
  uint32_t l0_spl_pos[kMaxK];
  uint32_t l0_bucket[kMaxK];
};

// Pointers into the workspace for one call.
struct Work {
  Ctl* ctl;
  BigSeg* big[2];
  uint32_t* group_base;  // [big_max + 1] first tile group of each segment
  uint32_t* count_base;  // [big_max + 1]
  void* tree_key;        // [big_max * kMaxK] (K), node t of segment s at s*kMaxK + t
  uint32_t* tree_idx;
  uint32_t* counts;      // [count_max]
  uint32_t* offsets;     // [count_max]
  uint64_t* scan_flags;  // [scan_blocks] chained-scan status of each chunk of the count matrix
  uint32_t* scan_part;   // [scan_blocks] chunk sums of the reduce-then-scan
  FinalSeg* cls[kNumClasses];     // per size class lists
  uint64_t cls_cap[kNumClasses];
  uint32_t* buf_rec[2];  // A, B: [n] element records (ordinal key, position; see BufView)
  uint32_t* buf_pay[2];  // [n] (payload calls only)
  uint8_t* ids;          // [2 n] bucket of each element of a buffer level (see bucket ids below)
  uint64_t big_max, count_max, scan_blocks, n;
  uint32_t group_log2;   // log2 of the keys per tile group
  uint32_t spread;       // 1: the plan has extra levels, and segments spread their buckets over them
};

// Bucket ids of a level that reads a buffer: the count pass stores the
// bucket of the element at buffer position p of a segment starting at s in
// the segment's own byte range [2 s, 2 s + 2 len) of ids: one byte at 2 s + (p - s)
// when the segment has at most 256 buckets, else two at 2 s + 2 (p - s).  The
// scatter reads them instead of classifying again.
__device__ __forceinline__ void put_bucket_id(uint8_t* ids, uint64_t s, uint64_t r, uint32_t logk, uint32_t b) {
  if (logk <= 8)
    ids[2 * s + r] = (uint8_t)b;
  else
    ((uint16_t*)(ids + 2 * s))[r] = (uint16_t)b;
}
__device__ __forceinline__ uint32_t get_bucket_id(const uint8_t* ids, uint64_t s, uint64_t r, uint32_t logk) {
  return logk <= 8 ? (uint32_t)ids[2 * s + r] : (uint32_t)((const uint16_t*)(ids + 2 * s))[r];
}

// The element buffers of the levels interleave each element's ordinal key
// and input position in one record of 32-bit words (key low, key high for
// 64-bit keys, then the position), so that one memory instruction moves a
// whole element; a scatter writes half as many partial lines as with
// separate key and position arrays.
template <typename K>
struct BufView {
  static constexpr int W = (int)(sizeof(K) / 4) + 1;  // words per record
  uint32_t* p;
  __device__ __forceinline__ K key(uint64_t i) const {
    const uint32_t* r = p + i * W;
    if constexpr (sizeof(K) == 8)
      return ((uint64_t)r[1] << 32) | r[0];
    else
      return r[0];
  }
  __device__ __forceinline__ uint32_t idx(uint64_t i) const { return p[i * W + W - 1]; }
  __device__ __forceinline__ void get(uint64_t i, K& k, uint32_t& v) const {
    const uint32_t* r = p + i * W;
    if constexpr (sizeof(K) == 8) {
      const uint32_t a = r[0], b = r[1], c = r[2];
      k = ((uint64_t)b << 32) | a;
      v = c;
    } else {
      const uint32_t a = r[0], c = r[1];
      k = a;
      v = c;
    }
  }
  __device__ __forceinline__ void put(uint64_t i, K k, uint32_t v) const {
    uint32_t* r = p + i * W;
    r[0] = (uint32_t)k;
    if constexpr (sizeof(K) == 8) r[1] = (uint32_t)((uint64_t)k >> 32);
    r[W - 1] = v;
  }
};
template <typename K>
__device__ __forceinline__ BufView<K> buf_view(const Work& w, int b) {
  return BufView<K>{w.buf_rec[b]};
}

// Launcher flag (or-ed into the class index): sort the whole input of a
// plain call as one segment in a single launch.  The kernels then receive a
// negative class argument.
constexpr int kDirect = 0x100;
// Launcher flag: no sample-sort level ran, so every final segment lies in the
// caller's input (positions implicit) and the class kernels need no table of
// positions.
constexpr int kInputOnly = 0x200;
// Launcher flag: final segments of both kinds (a segmented call where some
// user segments were split by levels): the class kernels run once for the
// input segments and once for the buffer segments.
constexpr int kMixed = 0x400;

// Final segments of class cls (cls < 0: the direct single-segment mode).
__device__ __forceinline__ uint32_t final_count(const Work& w, int cls) {
  if (cls < 0) return 1u;
  return (uint32_t)min((uint64_t)w.ctl->class_count[cls], w.cls_cap[cls]);
}
__device__ __forceinline__ FinalSeg final_at(const Work& w, int cls, uint32_t q) {
  if (cls < 0) return FinalSeg{0ull, (uint32_t)w.n, 0u};
  return w.cls[cls][q];
}
// In the direct mode no reset kernel runs: the first thread clears the status
// and statistics of the workspace.
__device__ __forceinline__ void direct_reset(const Work& w, int cls) {
  if (cls < 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    w.ctl->status = 0;
    w.ctl->levels = 0;
    w.ctl->l0_k = 0;
    for (int c = 0; c < kNumClasses; c++) {
      w.ctl->class_count[c] = 0;
      w.ctl->class_keys[c] = 0;
    }
  }
}

}  // namespace rs
