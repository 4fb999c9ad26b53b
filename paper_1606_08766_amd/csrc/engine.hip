// Multilevel sample sort engine (paper Appendix G: robust multi-level sample
// sort, RAMS) for one GPU, plus the LDS sort of its final buckets.
//
// One level splits every "big" segment (more than `cap` elements) into
// k = 2^logk buckets:
//   splitters  draw a*k random sample positions per segment, gather
//              (key, position) pairs, sort them in LDS and keep every a-th
//              as a splitter (positions break key ties, Appendix G);
//   count      classify every element with a branchless descent of the
//              splitter tree held in LDS (a Super Scalar Sample Sort style
//              classifier; a key equal to a splitter key is resolved by the
//              positions) and histogram buckets per tile;
//   scan       exclusive prefix sum of the [segment][bucket][tile] counts;
//   scatter    re-classify, rank inside (tile, bucket) with LDS atomics,
//              stage the tile in LDS grouped by bucket and write contiguous
//              runs: the paper's all-to-all exchange becomes a scatter
//              through HBM at prefix-sum offsets.
// Buckets at most `cap` long become final segments and are sorted, one
// workgroup each, in LDS; the rest are split again at the next level.
// Everything is sized on the device: no bucket size returns to the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>

#include "device.hpp"
#include "engine.hpp"
#include "internal.hpp"

namespace rs {

// Size classes of final segments (upper bounds); the last is "oversize".
__constant__ uint32_t c_class_max[kNumClasses] = {64, 256, 1024, 2048, 3072, 4096, 6144, 8192, 12288, 0xFFFFFFFFu};
static const uint32_t h_class_max[kNumClasses] = {64, 256, 1024, 2048, 3072, 4096, 6144, 8192, 12288, 0xFFFFFFFFu};

uint32_t class_max(int c) { return (c >= 0 && c < kNumClasses) ? h_class_max[c] : 0u; }

// cmin: the smallest class used.  A sort with few final buckets routes them
// all to one or two large classes, so that they run in one launch that fills
// the GPU instead of several nearly idle ones.
__device__ __forceinline__ uint32_t class_of(uint32_t len, uint32_t cap, uint32_t force_fallback, uint32_t cmin) {
  if (len > cap || (force_fallback && len > 64)) return kNumClasses - 1;
  uint32_t c = cmin;
  while (len > c_class_max[c]) c++;
  return c;
}

// log2 of the bucket count for a segment of len keys that still has `left`
// levels (this one included) to reach buckets of about `target` keys: the
// 2^lq buckets needed are shared out over the levels the segment needs, the
// upper levels taking the smaller share (fewer buckets where the data is
// largest keeps the scatter's runs long).  Only a plan with extra levels
// (`spread`) spreads them over more levels than the fewest that reach the
// target, at least 4 buckets per level; otherwise a segment of a batch that
// needs one level takes one, however many the batch's largest needs.
__device__ __forceinline__ uint32_t logk_for(uint32_t len, uint32_t target, uint32_t left, uint32_t spread) {
  const uint32_t q = (len + target - 1) / target;  // buckets wanted
  const uint32_t lq = q <= 1 ? 0u : 32u - __clz(q - 1);
  const uint32_t need = (lq + kMaxLogK - 1) / kMaxLogK;
  const uint32_t fewest = max(need, 1u);
  const uint32_t lv = left < need ? left : (spread ? max(fewest, min(left, lq / 2)) : fewest);
  uint32_t lk = lv > 1 ? lq / lv : lq;
  lk = lk < 1u ? 1u : lk;
  return lk > (uint32_t)kMaxLogK ? (uint32_t)kMaxLogK : lk;
}

__device__ __forceinline__ void set_status(Ctl* ctl, int32_t code) { atomicCAS(&ctl->status, 0, code); }

// A compile-time flag passed to a generic lambda.
template <bool B>
struct BoolC {
  static constexpr bool value = B;
};

// A value the caller knows to be the same in every lane (read from LDS, say),
// moved to a scalar register.
__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  return ((uint64_t)uniform((uint32_t)(x >> 32)) << 32) | uniform((uint32_t)x);
}

// The chained scan's per-chunk status words start at zero on every level.
__device__ __forceinline__ void scan_flags_clear(const Work& w, uint32_t t, uint32_t nt) {
  for (uint64_t i = t; i < w.scan_blocks; i += nt) w.scan_flags[i] = 0ull;
}


// Routing of a block's segments to the list of segments to split (index
// kNumClasses) or to the final lists by size class, aggregated per block:
// slots are counted in LDS (one LDS atomic per list and wave), then one
// global atomic per list and block reserves them.  Every thread of the block
// calls once per iteration of a block-uniform loop; `lds` is zeroed before
// the first call (route_lds_init) and is left zeroed.
struct RouteLds {
  uint32_t cnt[kNumClasses + 1];
  uint32_t base[kNumClasses + 1];
  unsigned long long keys[kNumClasses];
};

__device__ __forceinline__ void route_lds_init(RouteLds& L) {
  if (threadIdx.x <= (unsigned)kNumClasses) {
    L.cnt[threadIdx.x] = 0;
    if (threadIdx.x < (unsigned)kNumClasses) L.keys[threadIdx.x] = 0;
  }
  __syncthreads();
}

__device__ __forceinline__ void route(const Work& w, RouteLds& L, uint32_t* big_counter, BigSeg* big_list,
                                      bool active, bool to_big, uint64_t start, uint64_t ubase, uint32_t len,
                                      uint32_t src, uint32_t cap, uint32_t ff, uint32_t target, uint32_t left,
                                      uint32_t cmin) {
  const uint32_t c = (active && !to_big) ? class_of(len, cap, ff, cmin) : 0u;
  const uint32_t dest = to_big ? (uint32_t)kNumClasses : c;
  const uint32_t li = wave_append(L.cnt, dest, active);
  // keys per class (statistics): one LDS atomic per distinct class per wave
  const bool af = active && !to_big;
  uint64_t pending = __ballot(af);
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t k = __shfl(c, leader, kWave);
    const bool mine = af && c == k;
    uint64_t sum = mine ? (uint64_t)len : 0ull;
    for (int d = kWave / 2; d > 0; d >>= 1) sum += __shfl_xor(sum, d, kWave);
    if (lane_id() == (uint32_t)leader) atomicAdd(&L.keys[k], (unsigned long long)sum);
    pending &= ~__ballot(mine);
  }
  __syncthreads();
  if (threadIdx.x <= (unsigned)kNumClasses) {
    const uint32_t t = threadIdx.x, n = L.cnt[t];
    uint32_t* ctr = t == (uint32_t)kNumClasses ? big_counter : &w.ctl->class_count[t];
    L.base[t] = n ? atomicAdd(ctr, n) : 0u;
    if (t < (uint32_t)kNumClasses && L.keys[t]) atomicAdd((unsigned long long*)&w.ctl->class_keys[t], L.keys[t]);
    L.cnt[t] = 0;
    if (t < (uint32_t)kNumClasses) L.keys[t] = 0;
  }
  __syncthreads();
  if (active) {
    const uint32_t i = L.base[dest] + li;
    if (to_big) {
      if (i < w.big_max)
        big_list[i] = BigSeg{start, ubase, len, logk_for(len, target, left, w.spread)};
      else
        set_status(w.ctl, -3);  // capacity bound violated: internal error
    } else {
      if (i < w.cls_cap[c])
        w.cls[c][i] = FinalSeg{start, len, src};
      else
        set_status(w.ctl, -3);
    }
  }
}

// ---------------------------------------------------------------------------
__global__ void k_reset(Ctl* ctl, uint32_t levels) {
  uint32_t* p = reinterpret_cast<uint32_t*>(ctl);
  const uint32_t nw = (uint32_t)(offsetof(Ctl, l0_spl_key) / 4);
  for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) p[i] = (i == 1) ? levels : 0u;
}

// Route every user segment: split it (big list 0) or sort it directly.
__global__ void k_init(Work w, const uint64_t* seg_off, uint32_t num_segs, uint64_t n_total, uint32_t cap,
                       uint32_t target, uint32_t levels, uint32_t ff, uint32_t cmin) {
  __shared__ RouteLds L;
  route_lds_init(L);
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t s0 = blockIdx.x * blockDim.x; s0 < num_segs; s0 += stride) {
    const uint32_t s = s0 + threadIdx.x;
    bool active = s < num_segs;
    uint64_t a = 0, b = 0;
    if (active) {
      a = seg_off ? seg_off[s] : 0ull;
      b = seg_off ? seg_off[s + 1] : n_total;
      if (b < a || b > n_total || (s == 0 && a != 0) || (s + 1 == num_segs && b != n_total) ||
          b - a >= 0xFFFFFFFFull) {
        set_status(w.ctl, -1);
        active = false;
      }
    }
    const uint32_t len = active ? (uint32_t)(b - a) : 0u;
    active = active && len > 0;
    route(w, L, &w.ctl->big_count[0], w.big[0], active, len > cap && levels > 0, a, a, len, 0u, cap, ff, target,
          levels, cmin);
  }
}

// The splitter kernel's shape: up to kSplThreads * kSplItems samples per segment.
constexpr int kSplThreads = 1024, kSplItems = 8;  // (a = 32 at k = 256, 16 at 512)
constexpr uint32_t kStartThreads = 256;

// A plain sort's start in one launch: reset the control block, route the one
// segment [0, n) (split it, or sort it in its class), and plan level 0 when
// it is split (one segment: its tile groups and count-matrix base are
// immediate).  With `staged` (a split sort of at least kSplThreads *
// kSplItems keys), the workgroups also draw the first level's sample, the
// same a0 * k positions the splitter kernel would, and store the (raw key,
// position) records at the front of buffer B, which the first level does
// not touch before its scatter: the random loads are spread over many CUs
// instead of coming from the splitter kernel's one workgroup.
template <typename K>
__global__ __launch_bounds__(kStartThreads) void k_start_plain(Work w, uint64_t n, uint32_t cap, uint32_t target,
                                                              uint32_t levels, uint32_t ff, uint32_t cmin,
                                                              const K* in_keys, uint32_t a0, uint64_t seed,
                                                              int staged) {
  if (staged) {
    const uint32_t logk = logk_for((uint32_t)n, target, levels, w.spread);
    const uint32_t S = min(a0, (uint32_t)(kSplThreads * kSplItems) >> logk) << logk;
    const uint32_t j = blockIdx.x * kStartThreads + threadIdx.x;
    if (j < S) {
      // level 0, segment start 0: the stream and position of k_splitters
      const uint64_t r = rand_at(seed, 0ull, j);
      const uint64_t pos = ((r >> 32) * n) >> 32;
      BufView<K>{w.buf_rec[1]}.put(j, in_keys[pos], (uint32_t)pos);
    }
    if (blockIdx.x != 0) return;
  }
  uint32_t* p = reinterpret_cast<uint32_t*>(w.ctl);
  const uint32_t nw = (uint32_t)(offsetof(Ctl, l0_spl_key) / 4);
  for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) p[i] = (i == 1) ? levels : 0u;
  if (levels > 0) scan_flags_clear(w, threadIdx.x, blockDim.x);
  __syncthreads();
  if (threadIdx.x != 0 || n == 0) return;
  const uint32_t len = (uint32_t)n;
  if (len > cap && levels > 0) {
    const uint32_t logk = logk_for(len, target, levels, w.spread);
    w.big[0][0] = BigSeg{0ull, 0ull, len, logk};
    const uint32_t ng = (uint32_t)((n + (1ull << w.group_log2) - 1) >> w.group_log2);
    w.group_base[0] = 0;
    w.group_base[1] = ng;
    w.count_base[0] = 0;
    w.count_base[1] = ng << logk;
    w.ctl->big_count[0] = 1;
    w.ctl->total_groups = ng;
    w.ctl->total_counts = ng << logk;
  } else {
    const uint32_t c = class_of(len, cap, ff, cmin);
    w.cls[c][0] = FinalSeg{0ull, len, 0u};
    w.ctl->class_count[c] = 1;
    w.ctl->class_keys[c] = n;
  }
}

// Per level: tile groups and count-matrix bases of the segments to split.
// glog_small (levels after the first of a plain sort; 0 otherwise): when the
// first level's scatter wrote runs of fewer than kShortRun keys on average
// (keys spread over all buckets of every tile), this level's groups hold
// 2^glog_small keys instead of 2^group_log2, and the count and scatter passes
// read the choice from ctl->glog.
constexpr int kPlanThreads = 1024;
constexpr uint32_t kShortRun = 128;
__global__ __launch_bounds__(kPlanThreads) void k_plan(Work w, int lev, uint32_t glog_small) {
  __shared__ uint32_t tmp[kPlanThreads / kWave + 1];
  __shared__ uint32_t s_glog;
  const int cur = lev & 1;
  const uint32_t m = (uint32_t)min((uint64_t)w.ctl->big_count[cur], w.big_max);
  const BigSeg* B = w.big[cur];
  // the first level of a segmented call: the class lists hold only the
  // user segments routed so far (k_init); the levels append theirs after
  if (lev == 0 && threadIdx.x < (unsigned)kNumClasses) w.ctl->class_in[threadIdx.x] = w.ctl->class_count[threadIdx.x];
  if (threadIdx.x == 0) {
    const uint32_t runs = w.ctl->runs;
    const bool short_runs = glog_small && runs && w.n / runs < kShortRun;
    s_glog = short_runs ? glog_small : w.group_log2;
    if (glog_small) w.ctl->glog = s_glog;
  }
  __syncthreads();
  const uint32_t glog = s_glog;
  uint32_t ct = 0, cc = 0;
  for (uint32_t base = 0; base < m; base += kPlanThreads) {
    const uint32_t i = base + threadIdx.x;
    uint32_t nt = 0, nc = 0;
    if (i < m) {
      nt = (uint32_t)(((uint64_t)B[i].len + (1u << glog) - 1) >> glog);  // groups
      nc = nt << B[i].logk;
    }
    uint32_t tt, tc;
    const uint32_t et = block_excl_scan<kPlanThreads>(nt, tmp, &tt);
    const uint32_t ec = block_excl_scan<kPlanThreads>(nc, tmp, &tc);
    if (i < m) {
      w.group_base[i] = ct + et;
      w.count_base[i] = cc + ec;
    }
    ct += tt;
    cc += tc;
  }
  if (threadIdx.x < 16) w.ctl->queue[threadIdx.x >> 3][threadIdx.x & 7] = 0;
  scan_flags_clear(w, threadIdx.x, kPlanThreads);
  if (threadIdx.x == 0) {
    w.ctl->scan_next = 0;
    w.group_base[m] = ct;
    w.count_base[m] = cc;
    w.ctl->total_groups = ct;
    w.ctl->total_counts = cc;
    w.ctl->big_count[cur ^ 1] = 0;
  }
}

// Splitter selection: one workgroup per segment.  S = a << logk sample
// positions drawn uniformly (with replacement) from the segment; the
// (key, position) pairs are sorted in LDS and every a-th becomes a splitter.
// The k-1 splitters are stored as an implicit binary search tree: node t at
// depth d, index q = t - 2^d within its depth, holds splitter number
// (2q+1) * 2^(logk-1-d) (1-based, in sorted order).
constexpr uint32_t kSplRankBudget = 64;  // compares per sample the ranking path may take
// first-level bucket ids when at least 1 / kDupIdsDiv of the splitter keys
// equal their predecessor
constexpr uint32_t kDupIdsDiv = 16;

template <typename K, bool F32, bool SRC_IN, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_splitters(Work w, int lev, const K* in_keys, int src_buf,
                                                       uint32_t a, uint64_t seed, int ids_ok, int staged) {
  constexpr int N = THREADS * ITEMS;
  constexpr int NP = lpad_size(N);
  constexpr int LB = 31 - __builtin_clz((unsigned)(N / 8));  // bins of the ranking path
  constexpr int PL = (1 << LB) / kWave;
  static_assert(PL >= 1, "one bin per lane at least");
  __shared__ uint32_t s_lo[NP];
  __shared__ uint32_t s_hi[sizeof(K) == 8 ? NP : 1];
  __shared__ uint32_t s_v[NP];
  __shared__ uint32_t s_bin[(1 << LB) + 1];
  __shared__ uint32_t s_red[6 * (THREADS / kWave)];
  __shared__ uint32_t s_cost;
  __shared__ K s_spl[kMaxK];  // level 0, segment 0: the sorted splitter keys
  __shared__ uint32_t s_dup;
  const LdsArr<K> sa{s_lo, s_hi, s_v, nullptr};
  const int cur = lev & 1;
  const uint32_t m = (uint32_t)min((uint64_t)w.ctl->big_count[cur], w.big_max);
  const BufView<K> bv{SRC_IN ? nullptr : w.buf_rec[src_buf]};
  K* tkey = (K*)w.tree_key;
  for (uint32_t s = blockIdx.x; s < m; s += gridDim.x) {
    const BigSeg bs = w.big[cur][s];
    // a samples per bucket, fewer when a * k would exceed the LDS sample
    const uint32_t ae = min(a, (uint32_t)(THREADS * ITEMS) >> bs.logk);
    const uint32_t S = ae << bs.logk;
    K k[ITEMS];
    uint32_t v[ITEMS], p[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t j = threadIdx.x * ITEMS + i;
      if (SRC_IN && staged && j < S) {
        // drawn by k_start_plain (the same positions), stored in order
        BufView<K>{w.buf_rec[1]}.get(j, k[i], v[i]);
      } else if (j < S) {
        const uint64_t r = rand_at(seed, ((uint64_t)lev << 40) ^ bs.start, j);
        const uint64_t pos = bs.start + (((r >> 32) * (uint64_t)bs.len) >> 32);
        if constexpr (SRC_IN) {
          k[i] = in_keys[pos];  // raw bits; mapped below once all loads are issued
          v[i] = (uint32_t)(pos - bs.ubase);
        } else {
          bv.get(pos, k[i], v[i]);
        }
      } else {
        k[i] = KMax<K>::v;
        v[i] = kPadIdx;
      }
      p[i] = 0;
    }
    if constexpr (SRC_IN && F32) {
#pragma unroll
      for (int i = 0; i < ITEMS; i++)
        if (threadIdx.x * ITEMS + i < S) k[i] = ord_of<K, F32>(k[i]);
    }
    const uint32_t kk = 1u << bs.logk;
    // The splitters are the samples of rank j * ae - 1 (j = 1 .. kk - 1) in
    // (key, position) order.  Ranks come from bins, as in the word sort:
    // samples are counted into bins by the top bits of (key - min) (or, for a
    // narrow key range, key offset then position bits), and a sample's rank
    // is its bin's start plus the number of smaller samples in its bin.  If
    // that would cost more than kRankBudget compares per sample, the samples
    // are merge sorted instead.
    bool ranked = false;
    {
      K kmn = KMax<K>::v, kmx = K(0);
      uint32_t imn = ~0u, imx = 0u;
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        if (threadIdx.x * ITEMS + i < S) {
          kmn = k[i] < kmn ? k[i] : kmn;
          kmx = k[i] > kmx ? k[i] : kmx;
          imn = min(imn, v[i]);
          imx = max(imx, v[i]);
        }
      }
      for (int b = threadIdx.x; b <= (1 << LB); b += THREADS) s_bin[b] = 0;
      const Range4 br = block_range<K, THREADS>(kmn, kmx, imn, imx, s_red, threadIdx.x);
      kmn = (K)br.kmn;
      const uint64_t kr = (uint64_t)((K)br.kmx - kmn);
      const int rb = kr ? 64 - __clzll((long long)kr) : 0;
      BinMap bm;
      const bool narrow = rb < LB;  // bins: key offset, then the top bits of the position
      if (narrow) {
        const uint32_t ib = LB - rb, ir = br.imx - br.imn;
        const int ibits = ir ? 32 - __clz(ir) : 0;
        bm = BinMap{(uint64_t)br.imn, 32u, ib, (uint32_t)max(ibits - (int)ib, 0), (1u << ib) - 1u};
      } else {
        bm = BinMap{0ull, (uint32_t)(rb - LB), 0u, 0u, 0u};
      }
      auto bin_of = [&](K key, uint32_t idx) -> uint32_t {
        const uint64_t off = (uint64_t)(K)(key - kmn);
        return bm(narrow ? (off << 32) | idx : off);
      };
      uint32_t r[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        r[i] = 0;
        if (threadIdx.x * ITEMS + i < S) r[i] = atomicAdd(&s_bin[bin_of(k[i], v[i])], 1u);
      }
      __syncthreads();
      if (threadIdx.x < kWave) {  // one wave scans the bins and sums their squared sizes
        uint64_t acc = 0;
        for (int q = 0; q < PL; q++) {
          const uint32_t x = s_bin[threadIdx.x * PL + q];
          acc += ((uint64_t)(x * x) << 32) | x;
        }
        const uint64_t inc = wave_incl_scan<uint64_t>(acc);
        uint32_t e = (uint32_t)(inc - acc);
        for (int q = 0; q < PL; q++) {
          const uint32_t x = s_bin[threadIdx.x * PL + q];
          s_bin[threadIdx.x * PL + q] = e;
          e += x;
        }
        if (threadIdx.x == kWave - 1) {
          s_bin[1 << LB] = S;
          s_cost = (uint32_t)(inc >> 32);
        }
      }
      __syncthreads();
      if (s_cost <= kSplRankBudget * S) {  // uniform
        ranked = true;
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
          if (threadIdx.x * ITEMS + i < S) sa.put(s_bin[bin_of(k[i], v[i])] + r[i], k[i], v[i]);
        }
        __syncthreads();
        for (uint32_t pq = threadIdx.x; pq < S; pq += THREADS) {
          const K key = sa.key(pq);
          const uint32_t idx = s_v[pq];
          const uint32_t db = bin_of(key, idx);
          const uint32_t s0 = s_bin[db], s1 = s_bin[db + 1];
          // samples are drawn with replacement: equal samples are ranked by
          // their place in the bin, so that every rank is taken once
          uint32_t less = 0;
          for (uint32_t q = s0; q < s1; q++) {
            const K kq = sa.key(q);
            const uint32_t iq = s_v[q];
            less += (pair_less(kq, iq, key, idx) || (kq == key && iq == idx && q < pq)) ? 1u : 0u;
          }
          const uint32_t rank = s0 + less;
          if ((rank + 1) % ae == 0) {
            const uint32_t j = (rank + 1) / ae;
            if (j < kk) {
              const uint32_t node = (j | kk) >> (__builtin_ctz(j) + 1);
              tkey[(uint64_t)s * kMaxK + node] = key;
              w.tree_idx[(uint64_t)s * kMaxK + node] = idx;
              if (lev == 0 && s == 0) {
                w.ctl->l0_spl_key[j - 1] = (uint64_t)key;
                w.ctl->l0_spl_pos[j - 1] = idx;
                s_spl[j - 1] = key;
              }
            }
          }
        }
      }
    }
    if (!ranked) {
      lds_merge_sort<K, THREADS, ITEMS, false>(k, v, p, sa);
#pragma unroll
      for (int i = 0; i < ITEMS; i++) sa.put(lpad(threadIdx.x * ITEMS + i), k[i], v[i]);
      __syncthreads();
      for (uint32_t node = threadIdx.x + 1; node < kk; node += THREADS) {
        const uint32_t d = 31u - __clz(node);
        const uint32_t q = node - (1u << d);
        const uint32_t j = (2u * q + 1u) << (bs.logk - 1u - d);
        const uint32_t r = j * ae - 1u;
        tkey[(uint64_t)s * kMaxK + node] = sa.key(lpad(r));
        w.tree_idx[(uint64_t)s * kMaxK + node] = s_v[lpad(r)];
      }
      if (lev == 0 && s == 0) {
        for (uint32_t j = threadIdx.x + 1; j < kk; j += THREADS) {
          w.ctl->l0_spl_key[j - 1] = (uint64_t)sa.key(lpad(j * ae - 1u));
          w.ctl->l0_spl_pos[j - 1] = s_v[lpad(j * ae - 1u)];
          s_spl[j - 1] = sa.key(lpad(j * ae - 1u));
        }
      }
    }
    if (lev == 0 && s == 0 && threadIdx.x == 0) w.ctl->l0_k = kk;
    if (lev == 0 && m == 1 && ids_ok) {  // uniform
      // Keys that tie a splitter cost the (key, position) descent.  When the
      // one first-level segment's splitters repeat keys (few distinct keys),
      // its count stores each key's bucket for the scatter, which then
      // skips the second classification; otherwise the scatter classifies
      // again, cheaper than writing and reading the ids.
      if (threadIdx.x == 0) s_dup = 0;
      __syncthreads();
      uint32_t d = 0;
      for (uint32_t j = threadIdx.x + 1; j + 1 < kk; j += THREADS) d += s_spl[j] == s_spl[j - 1] ? 1u : 0u;
      if (d) atomicAdd(&s_dup, d);
      __syncthreads();
      if (threadIdx.x == 0) w.ctl->ids0 = s_dup * kDupIdsDiv >= kk ? 1u : 0u;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Classification of a thread's ITEMS elements with the splitter tree in LDS.
// tk holds 2k entries: node t of the implicit tree (t in [1, k)) at tk[t],
// and below them a leaf row, tk[k + b] = the b-th smallest splitter key for
// b < k - 1 and tk[2k - 1] = the largest (see tree_to_lds).  ti holds the
// positions of the tree nodes.  Levels are the outer loop so the ITEMS
// lookups of a level are independent.  The descent compares keys only and
// walks byte offsets into tk (one shift-add per level, no index scaling).
// It ends at the leaf k + b where b is the number of splitter keys strictly
// below the key, so the key can only equal a splitter key on its path if it
// equals that leaf's (the smallest splitter key >= key; the last leaf repeats
// the largest splitter key, which a key in bucket k - 1 exceeds).  Such an
// element is classified again comparing (key, position) pairs (the tie-break
// of Appendix G: positions are looked at only when keys are equal).  `pairs`
// (uniform over the wave, kept by the caller across tiles) skips the key-only
// descent for a tile after one in which every element of the wave tied, as
// on inputs of few distinct keys.
// Result: bucket = number of splitters strictly below (key, position).
template <typename K, int ITEMS, typename IdxFn>
__device__ __forceinline__ void classify_batch(const K* tk, const uint32_t* ti, uint32_t logk, const K (&key)[ITEMS],
                                               const bool (&valid)[ITEMS], IdxFn idx_of, uint32_t (&b)[ITEMS],
                                               bool& pairs) {
  constexpr uint32_t KB = (uint32_t)sizeof(K);
  const uint32_t kk = 1u << logk;
  // level-major descent comparing (key, position) for the elements in m
  auto pair_descent = [&](const bool (&m)[ITEMS], uint32_t (&q)[ITEMS]) {
    uint32_t id[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      id[i] = m[i] ? idx_of(i) : 0u;  // positions first (independent loads)
      q[i] = 1;
    }
    for (uint32_t l = 0; l < logk; l++) {
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const K t = tk[q[i]];
        const uint32_t u = ti[q[i]];
        q[i] = 2u * q[i] + ((key[i] > t) | ((key[i] == t) & (id[i] > u)) ? 1u : 0u);
      }
    }
  };
  uint32_t j[ITEMS];
  if (pairs) {  // uniform
    // every element of this wave's previous tile tied: the (key, position)
    // descent alone gives the bucket.  A splitter key equals the key exactly
    // when one of the two splitters around the result does (the leaf row
    // holds them), which decides the mode of the next tile.
    pair_descent(valid, j);
    bool untied = false;
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const bool t = key[i] == tk[j[i]] || (j[i] > kk && key[i] == tk[j[i] - 1]);
      untied = untied | (valid[i] & !t);
    }
    pairs = !__any(untied);
  } else {
    const char* tb = reinterpret_cast<const char*>(tk);
    uint32_t a[ITEMS];  // byte offset of the current node
#pragma unroll
    for (int i = 0; i < ITEMS; i++) a[i] = KB;
    for (uint32_t l = 0; l < logk; l++) {
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const K t = *reinterpret_cast<const K*>(tb + a[i]);
        a[i] = 2u * a[i] + (key[i] > t ? KB : 0u);
      }
    }
    K leaf[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) leaf[i] = *reinterpret_cast<const K*>(tb + a[i]);
    bool eq[ITEMS];
    bool tie = false, untied = false;
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      eq[i] = (key[i] == leaf[i]) & valid[i];
      tie = tie | eq[i];
      untied = untied | (valid[i] & !eq[i]);
      j[i] = a[i] / KB;
    }
    if (__any(tie)) {
      uint32_t q[ITEMS];
      pair_descent(eq, q);
#pragma unroll
      for (int i = 0; i < ITEMS; i++) j[i] = eq[i] ? q[i] : j[i];
    }
    pairs = !__any(untied);
  }
#pragma unroll
  for (int i = 0; i < ITEMS; i++) b[i] = j[i] - kk;
}

// Copies the splitter tree of segment s (2^logk buckets) from global memory
// into tk[1, k) / ti[1, k) and fills tk's leaf row tk[k, 2k) (see
// classify_batch): splitter j (1-based, in sorted order) is tree node
// (j | k) >> (ctz(j) + 1).  Called by every thread; the caller synchronizes.
template <typename K, int THREADS>
__device__ __forceinline__ void tree_to_lds(const Work& w, uint32_t s, uint32_t logk, K* tk, uint32_t* ti) {
  const K* tkey = (const K*)w.tree_key;
  const uint32_t kk = 1u << logk;
  const uint64_t o = (uint64_t)s * kMaxK;
  for (uint32_t i = threadIdx.x + 1; i < kk; i += THREADS) {
    tk[i] = tkey[o + i];
    ti[i] = w.tree_idx[o + i];
    const uint32_t node = (i | kk) >> (__builtin_ctz(i) + 1);
    tk[kk + i - 1] = tkey[o + node];
  }
  if (threadIdx.x == 0 && kk > 1) tk[2 * kk - 1] = tkey[o + (((kk - 1) | kk) >> 1)];
}

__device__ __forceinline__ uint32_t find_seg(const uint32_t* base, uint32_t m, uint32_t tile) {
  uint32_t lo = 0, hi = m;  // base[0] = 0 <= tile < base[m]
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (base[mid] <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Work queue of tile groups, XCD-aware: workgroups are dispatched round-robin
// over the 8 XCDs, so workgroup g runs on XCD g % 8.  Each XCD owns a
// contiguous share of the groups, and its workgroups take the next group of
// that share from the XCD's own counter: neighbouring groups write
// neighbouring parts of each bucket's output run (which then meet in the same
// L2), consecutive groups of a workgroup mostly belong to the same segment
// (whose splitter tree then stays in LDS), and a workgroup that finishes
// early takes more, so uneven segments do not leave a tail of idle CUs.
struct GroupQueue {
  uint32_t* ctr;
  uint32_t lo, hi;
  __device__ __forceinline__ GroupQueue(uint32_t* q, uint32_t G) {
    const uint32_t x = blockIdx.x & 7u;
    lo = (uint32_t)(((uint64_t)G * x) >> 3);
    hi = (uint32_t)(((uint64_t)G * (x + 1)) >> 3);
    ctr = q + x;
  }
  // Called by every thread; returns the next group, or hi when the share is
  // done.  The caller's group loop must pass a __syncthreads before the next
  // call (slot is rewritten there).  An empty share (a level with no work,
  // as the host launches for a batch whose segments all fit the local sort)
  // takes no atomic: a thousand workgroups on eight counters serialise.
  __device__ __forceinline__ uint32_t next(uint32_t* slot) {
    if (threadIdx.x == 0) {
      const uint32_t g = lo < hi ? lo + atomicAdd(ctr, 1u) : hi;
      *slot = g < hi ? g : hi;
    }
    __syncthreads();
    return *slot;
  }
};

// Keys per tile group (log2) of level lev: as the host planned it, unless the
// level's plan chose smaller groups (k_plan).
__device__ __forceinline__ uint32_t group_log2_of(const Work& w, int lev) {
  if (lev == 0) return w.group_log2;  // (no load on the first level)
  const uint32_t g = w.ctl->glog;
  return g ? g : w.group_log2;
}

// Segment a tile group belongs to, cached in LDS by the group loops below.
struct SegCache {
  uint32_t s, gb, gb_end, cb, seg0, logk;
  uint64_t start, ubase;
  uint32_t len, pad;
};

// Make sc describe the segment holding `group` (reloading its splitter tree
// into tk/ti) if the group lies outside the cached segment.  Contains
// __syncthreads(); called by every thread of the block.
template <typename K, int THREADS>
__device__ __forceinline__ void seg_for_group(const Work& w, int cur, uint32_t m, uint32_t group, SegCache& sc,
                                              K* tk, uint32_t* ti, bool need_seg0) {
  if (group >= sc.gb && group < sc.gb_end) return;  // uniform: sc is in LDS
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t s = find_seg(w.group_base, m, group);
    const BigSeg bs = w.big[cur][s];
    sc.s = s;
    sc.gb = w.group_base[s];
    sc.gb_end = w.group_base[s + 1];
    sc.cb = w.count_base[s];
    sc.seg0 = need_seg0 ? w.offsets[sc.cb] : 0u;
    sc.logk = bs.logk;
    sc.start = bs.start;
    sc.ubase = bs.ubase;
    sc.len = bs.len;
  }
  __syncthreads();
  tree_to_lds<K, THREADS>(w, sc.s, sc.logk, tk, ti);
  __syncthreads();
}

// Occupancy: 32-bit keys fit eight waves per SIMD (at most 64 VGPRs); the
// 64-bit instances spill at that bound and keep what the compiler chooses
// (the first level's count got faster on tied keys but 2 us slower on the
// latency path, the buffer level's slower on every input).
template <typename K, bool F32, bool SRC_IN, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS, sizeof(K) == 4 ? 8 : 1) void k_count(Work w, int lev, const K* in_keys,
                                                                          int src_buf) {
  constexpr uint32_t TILE = THREADS * ITEMS;
  static_assert(TILE <= (1u << kGroupMinLog2), "tiles divide a group");
  const uint32_t GT = (1u << group_log2_of(w, lev)) / TILE;  // tiles per group
  __shared__ K tk[2 * kMaxK];
  __shared__ uint32_t ti[kMaxK];
  __shared__ uint32_t hist[kMaxK];
  __shared__ SegCache sc;
  const int cur = lev & 1;
  const uint32_t m = (uint32_t)min((uint64_t)w.ctl->big_count[cur], w.big_max);
  const uint32_t G = w.ctl->total_groups;
  const BufView<K> bv{SRC_IN ? nullptr : w.buf_rec[src_buf]};
  // bucket ids for the scatter: always on a level that reads a buffer; on
  // the first level when its splitters chose so (ids0)
  const bool put_ids = !SRC_IN || (w.ids != nullptr && w.ctl->ids0 != 0u);
  const uint32_t lane = lane_id();
  if (threadIdx.x == 0) {
    sc.gb = 1;
    sc.gb_end = 0;  // empty: forces a load
  }
  for (uint32_t i = threadIdx.x; i < kMaxK; i += THREADS) hist[i] = 0;
  __syncthreads();
  __shared__ uint32_t s_group;
  GroupQueue gq(w.ctl->queue[0], G);
  bool pairs = false;  // classification mode of this wave's next tile
  for (uint32_t group = gq.next(&s_group); group < gq.hi; group = gq.next(&s_group)) {
    seg_for_group<K, THREADS>(w, cur, m, group, sc, tk, ti, false);
    // the segment's fields are uniform: kept in scalar registers
    const uint32_t gl = group - uniform(sc.gb);
    const uint32_t slen = uniform(sc.len), slogk = uniform(sc.logk);
    const uint64_t sstart = uniform64(sc.start);
    const uint32_t nt = (slen + TILE - 1) / TILE;
    const uint32_t t_end = min(nt, (gl + 1) * GT);
    // place of a thread's item i in a tile: striped over the block, or (a
    // level that reads a buffer) striped over the thread's wave
    const uint32_t wbase = (threadIdx.x & ~(uint32_t)(kWave - 1)) * ITEMS, wl = threadIdx.x & (kWave - 1);
    auto place = [&](int i) -> uint32_t {
      return SRC_IN ? i * THREADS + threadIdx.x : wbase + i * kWave + wl;
    };
    // the group's histogram accumulates over its tiles
    for (uint32_t tl = gl * GT; tl < t_end; tl++) {
      const uint64_t base = sstart + (uint64_t)tl * TILE;
      const uint32_t cnt = min(TILE, slen - tl * TILE);
      K key[ITEMS];
      bool valid[ITEMS];
      // every lane loads (lanes past the tile's end reload its last key), so
      // the loads are issued back to back without branches.  A level that
      // reads a buffer gives each wave ITEMS * 64 consecutive elements, so
      // that its byte ids form one contiguous run.
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const uint32_t jj = place(i);
        valid[i] = jj < cnt;
        const uint32_t jc = min(jj, cnt - 1u);
        if constexpr (SRC_IN)
          key[i] = in_keys[base + jc];
        else
          key[i] = bv.key(base + jc);
      }
      if constexpr (SRC_IN && F32) {
#pragma unroll
        for (int i = 0; i < ITEMS; i++) key[i] = ord_of<K, F32>(key[i]);
      }
      uint32_t b[ITEMS];
      const uint64_t ub = sc.ubase;
      classify_batch<K, ITEMS>(tk, ti, slogk, key, valid,
                               [&](int i) -> uint32_t {
                                 const uint64_t pos = base + place(i);
                                 if constexpr (SRC_IN)
                                   return (uint32_t)(pos - ub);
                                 else
                                   return bv.idx(pos);
                               },
                               b, pairs);
      if (put_ids) {
#pragma unroll
        for (int i = 0; i < ITEMS; i++)
          if (valid[i]) put_bucket_id(w.ids, sstart, (uint64_t)tl * TILE + place(i), slogk, b[i]);
      }
      // One atomic per wave when all its elements fall into one bucket
      // (skewed inputs).  A wave's valid elements are a prefix of its lanes,
      // so lane 0 holds one whenever any lane does.
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const uint32_t b0 = uniform(b[i]);
        if (__ballot(valid[i] && b[i] != b0) == 0) {
          const uint32_t nv = (uint32_t)__popcll(__ballot(valid[i]));
          if (lane == 0 && nv) atomicAdd(&hist[b0], nv);
        } else if (valid[i]) {
          atomicAdd(&hist[b[i]], 1u);
        }
      }
    }
    __syncthreads();
    const uint32_t kk = 1u << sc.logk;
    const uint32_t ng = sc.gb_end - sc.gb;
    for (uint32_t bb = threadIdx.x; bb < kk; bb += THREADS) {
      w.counts[sc.cb + bb * ng + gl] = hist[bb];
      hist[bb] = 0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Exclusive scan of counts[0 .. total_counts) into offsets in one launch: a
// chained scan with decoupled look-back.  Workgroups take chunks of
// kScanChunk counts in order from a counter; each publishes its chunk's sum
// at once and, after looking back at its predecessors' published sums (or
// inclusive prefixes), its inclusive prefix.  A chunk's predecessors are held
// by workgroups that are already running, so every wait ends; the wait is
// bounded all the same (status set to an internal error after kScanSpinMax
// polls).  Status word of chunk c: flag << 32 | value, flag 1 = the chunk's
// sum, 2 = the inclusive prefix through the chunk; zeroed before each level.
// Sums are taken modulo 2^32: offsets are only ever subtracted from offsets
// of the same segment, which is shorter than 2^32.
constexpr int kScanThreads = 256, kScanItems = 16, kScanChunk = kScanThreads * kScanItems;
constexpr uint32_t kScanSpinMax = 1u << 26;
constexpr uint64_t kChainedScanMax = 1u << 20;  // larger count matrices use reduce-then-scan

__global__ __launch_bounds__(kScanThreads) void k_scan(Work w) {
  __shared__ uint32_t tmp[kScanThreads / kWave + 1];
  __shared__ uint32_t s_chunk, s_prefix;
  const uint32_t M = w.ctl->total_counts;
  const uint32_t nb = (M + kScanChunk - 1) / kScanChunk;
  for (;;) {
    if (threadIdx.x == 0) s_chunk = atomicAdd(&w.ctl->scan_next, 1u);
    __syncthreads();
    const uint32_t c = s_chunk;
    if (c >= nb) break;
    const uint32_t b0 = c * kScanChunk + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
#pragma unroll
    for (int q = 0; q < kScanItems / 4; q++) {
      const uint32_t j = b0 + 4 * q;
      if (j + 4 <= M) {
        const uint4 x = *reinterpret_cast<const uint4*>(w.counts + j);  // j % 4 == 0: 16-byte aligned
        v[4 * q] = x.x;
        v[4 * q + 1] = x.y;
        v[4 * q + 2] = x.z;
        v[4 * q + 3] = x.w;
      } else {
#pragma unroll
        for (int r = 0; r < 4; r++) v[4 * q + r] = j + r < M ? w.counts[j + r] : 0u;
      }
    }
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) sum += v[i];
    uint32_t tot;
    uint32_t e = block_excl_scan<kScanThreads>(sum, tmp, &tot);
    if (threadIdx.x == 0) {
      uint32_t prefix = 0;
      if (c == 0) {
        __hip_atomic_store(&w.scan_flags[0], (2ull << 32) | tot, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_store(&w.scan_flags[c], (1ull << 32) | tot, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t j = c - 1, spins = 0;
        for (;;) {
          const uint64_t st =
              __hip_atomic_load(&w.scan_flags[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          const uint32_t flag = (uint32_t)(st >> 32);
          if (flag == 0) {
            if (++spins > kScanSpinMax) {
              set_status(w.ctl, -3);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          prefix += (uint32_t)st;
          if (flag == 2 || j == 0) break;
          j--;
        }
        __hip_atomic_store(&w.scan_flags[c], (2ull << 32) | (uint32_t)(prefix + tot), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
      s_prefix = prefix;
    }
    __syncthreads();
    e += s_prefix;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
      const uint32_t x = v[i];
      v[i] = e;
      e += x;
    }
#pragma unroll
    for (int q = 0; q < kScanItems / 4; q++) {
      const uint32_t j = b0 + 4 * q;
      if (j + 4 <= M) {
        *reinterpret_cast<uint4*>(w.offsets + j) = make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
      } else {
#pragma unroll
        for (int r = 0; r < 4; r++)
          if (j + r < M) w.offsets[j + r] = v[4 * q + r];
      }
    }
    __syncthreads();  // s_chunk / s_prefix are rewritten next
  }
}

// Large count matrices: reduce-then-scan in three launches (partial sums of
// chunks, a one-workgroup scan of the partials, the down-sweep), which for
// thousands of chunks beats waiting on the chunks' predecessors.
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(Work w) {
  __shared__ uint32_t tmp[kScanThreads / kWave + 1];
  const uint32_t M = w.ctl->total_counts;
  const uint32_t nb = (M + kScanChunk - 1) / kScanChunk;
  for (uint32_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
    uint32_t s = 0;
    const uint64_t base = (uint64_t)blk * kScanChunk;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
      const uint64_t j = base + i * kScanThreads + threadIdx.x;
      if (j < M) s += w.counts[j];
    }
    uint32_t tot;
    block_excl_scan<kScanThreads>(s, tmp, &tot);
    if (threadIdx.x == 0) w.scan_part[blk] = tot;
  }
}

constexpr int kScanTopThreads = 1024;
__global__ __launch_bounds__(kScanTopThreads) void k_scan_partials(Work w) {
  __shared__ uint32_t tmp[kScanTopThreads / kWave + 1];
  const uint32_t M = w.ctl->total_counts;
  const uint32_t nb = (M + kScanChunk - 1) / kScanChunk;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nb; base += kScanTopThreads) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < nb ? w.scan_part[i] : 0u;
    uint32_t tot;
    const uint32_t e = block_excl_scan<kScanTopThreads>(v, tmp, &tot);
    if (i < nb) w.scan_part[i] = carry + e;
    carry += tot;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(Work w) {
  __shared__ uint32_t tmp[kScanThreads / kWave + 1];
  const uint32_t M = w.ctl->total_counts;
  const uint32_t nb = (M + kScanChunk - 1) / kScanChunk;
  for (uint32_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
    const uint64_t base = (uint64_t)blk * kScanChunk + (uint64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
      v[i] = (base + i < M) ? w.counts[base + i] : 0u;
      s += v[i];
    }
    uint32_t e = block_excl_scan<kScanThreads>(s, tmp, nullptr) + w.scan_part[blk];
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
      if (base + i < M) w.offsets[base + i] = e;
      e += v[i];
    }
  }
}

// Exclusive scan of a tile histogram: one value per thread, non-zero only
// in the first kMaxK threads (the bins).  Rows of 16 lanes are scanned with
// DPP row shifts, rows are joined through lane reads, and the at most
// kMaxK / 64 bin waves through LDS (tmp: kMaxK / 64 words), with one
// barrier.  Called by every thread of the block.
__device__ __forceinline__ uint32_t bins_excl_scan(uint32_t v, uint32_t* tmp) {
  constexpr uint32_t NW = kMaxK / kWave;
  const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
  uint32_t inc = v;
  inc += dpp_u32<0x111>(inc);  // row_shr:1 (lanes without a source add 0)
  inc += dpp_u32<0x112>(inc);  // row_shr:2
  inc += dpp_u32<0x114>(inc);  // row_shr:4
  inc += dpp_u32<0x118>(inc);  // row_shr:8
  const uint32_t r0 = lane_u32(inc, 15), r1 = lane_u32(inc, 31), r2 = lane_u32(inc, 47);
  const uint32_t row = lane >> 4;
  inc += (row > 0 ? r0 : 0u) + (row > 1 ? r1 : 0u) + (row > 2 ? r2 : 0u);
  if (w < NW && lane == kWave - 1) tmp[w] = inc;
  __syncthreads();
  uint32_t off = 0;
  for (uint32_t q = 0; q < w && q < NW; q++) off += tmp[q];
  return off + inc - v;
}

// Buckets of the finished level lev: split again or sort in LDS.  This reads
// only the level's bucket bounds (offsets) and segment list, written before
// its scatter, and writes only the next level's segment list, the class
// lists and statistics, none of which the scatter reads; so the scatter's
// workgroups do it first, each taking (segment, bucket) pairs first, first +
// stride, ... of the m * kMaxK, instead of one more dependent launch.
// Called by every thread of the block (route synchronizes it).
struct LevelEnd {
  uint32_t cap, target, last, dst_code, ff, left, cmin;
};
__device__ __forceinline__ void level_end(const Work& w, int lev, const LevelEnd& a, RouteLds& L, uint64_t first,
                                          uint64_t stride) {
  const int cur = lev & 1;
  const uint32_t m = (uint32_t)min((uint64_t)w.ctl->big_count[cur], w.big_max);
  const uint64_t total = (uint64_t)m * kMaxK;
  for (uint64_t g0 = first; g0 < total; g0 += stride) {
    const uint64_t g = g0 + threadIdx.x;
    bool active = g < total;
    const uint32_t s = active ? (uint32_t)(g / kMaxK) : 0u, b = (uint32_t)(g % kMaxK);
    BigSeg bs{0, 0, 0, 1};
    uint32_t len = 0, lo = 0;
    if (active) {
      bs = w.big[cur][s];
      const uint32_t kk = 1u << bs.logk;
      active = b < kk;
      if (active) {
        const uint32_t ng = w.group_base[s + 1] - w.group_base[s];
        const uint32_t cb = w.count_base[s];
        const uint32_t seg0 = w.offsets[cb];
        lo = w.offsets[cb + b * ng] - seg0;
        const uint32_t hi = (b + 1 < kk) ? w.offsets[cb + (b + 1) * ng] - seg0 : bs.len;
        len = hi - lo;
        if (lev == 0 && s == 0) w.ctl->l0_bucket[b] = len;
      }
    }
    if (lev < kMaxLevels) {
      // per-wave maximum and count, then one atomic per wave
      uint32_t mx = len, nz = (active && len) ? 1u : 0u;
      for (int d = kWave / 2; d > 0; d >>= 1) {
        mx = max(mx, (uint32_t)__shfl_xor(mx, d, kWave));
        nz += (uint32_t)__shfl_xor(nz, d, kWave);
      }
      if (lane_id() == 0) {
        if (mx) atomicMax(&w.ctl->level_max[lev], mx);
        if (nz) atomicAdd(&w.ctl->level_buckets[lev], nz);
      }
    }
    active = active && len > 0;
    route(w, L, &w.ctl->big_count[cur ^ 1], w.big[cur ^ 1], active, len > a.cap && !a.last, bs.start + lo, bs.ubase,
          len, a.dst_code, a.cap, a.ff, a.target, a.left, a.cmin);
  }
}

// ---------------------------------------------------------------------------
// Scatter: classify, rank inside (tile, bucket), stage by bucket in LDS and
// write each bucket's run contiguously to the destination buffer.
template <typename K, bool F32, bool SRC_IN, bool PAY, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_scatter(Work w, int lev, const K* in_keys, const uint32_t* in_pay,
                                                     int src_buf, int dst_buf, int count_runs, LevelEnd le) {
  constexpr uint32_t TILE = THREADS * ITEMS;  // the host launches tiles no larger than a group
  const uint32_t GT = (1u << group_log2_of(w, lev)) / TILE;  // tiles per group
  static_assert(THREADS >= kMaxK, "one histogram bin per thread");
  static_assert(TILE <= (1u << 23), "ranks fit 23 bits");
  __shared__ K tk[2 * kMaxK];
  __shared__ uint32_t ti[kMaxK];
  __shared__ uint32_t hist[kMaxK];
  __shared__ uint64_t gdelta[kMaxK];
  __shared__ uint32_t tmp[THREADS / kWave + 1];
  __shared__ SegCache sc;
  __shared__ K stage[TILE];
  __shared__ uint32_t stage32[TILE];
  __shared__ uint16_t stage_b[TILE];

  const int cur = lev & 1;
  const uint32_t m = (uint32_t)min((uint64_t)w.ctl->big_count[cur], w.big_max);
  const uint32_t G = w.ctl->total_groups;
  const BufView<K> bv{SRC_IN ? nullptr : w.buf_rec[src_buf]};
  const uint32_t* bpay = SRC_IN ? in_pay : w.buf_pay[src_buf];
  const BufView<K> dv{w.buf_rec[dst_buf]};
  uint32_t* dpay = w.buf_pay[dst_buf];
  // the first level reads the count pass's bucket ids when it stored them
  // (see k_count), loaded before any store; the host allows first-level ids
  // only for calls without a payload
  const bool ids0 = SRC_IN && !PAY && w.ids != nullptr && w.ctl->ids0 != 0u;
  const uint32_t lane = lane_id();
  if (threadIdx.x == 0) {
    sc.gb = 1;
    sc.gb_end = 0;  // empty: forces a load
  }
  if (threadIdx.x < kMaxK) hist[threadIdx.x] = 0;
  {
    __shared__ RouteLds L;
    route_lds_init(L);  // (its barrier also orders the stores above)
    level_end(w, lev, le, L, (uint64_t)blockIdx.x * THREADS, (uint64_t)gridDim.x * THREADS);
  }

  __shared__ uint32_t s_group;
  GroupQueue gq(w.ctl->queue[1], G);
  bool pairs = false;  // classification mode of this wave's next tile
  uint32_t runs = 0;   // runs this thread's bucket got, summed once at the end
  for (uint32_t group = gq.next(&s_group); group < gq.hi; group = gq.next(&s_group)) {
    seg_for_group<K, THREADS>(w, cur, m, group, sc, tk, ti, true);
    const uint32_t gl = group - sc.gb;
    const uint32_t ng = sc.gb_end - sc.gb;
    const uint32_t kk = 1u << sc.logk;
    const uint32_t t_end = min((sc.len + TILE - 1) / TILE, (gl + 1) * GT);
    // where the group's part of bucket threadIdx.x starts; advanced by each
    // tile's count, so the tiles' runs follow each other in group order
    uint64_t run_off = 0;
    if (threadIdx.x < kk) run_off = sc.start + (uint64_t)(w.offsets[sc.cb + threadIdx.x * ng + gl] - sc.seg0);
    const BigSeg bs{sc.start, sc.ubase, sc.len, sc.logk};
    // The group's tiles, in one of two compiled forms: IDS, reading each
    // element's bucket from the count pass (every level that reads a buffer,
    // and the first level when it stored them), or classifying again.
    auto tiles = [&](auto ids_c) {
    constexpr bool IDS = !SRC_IN || decltype(ids_c)::value;
    // the group's tiles are loaded one ahead: the loads of tile tl + 1 are in
    // flight while tile tl is classified, ranked and written
    K nkey[ITEMS];
    uint32_t nidx[ITEMS], npay[ITEMS], nb[ITEMS];
    auto load_tile = [&](uint32_t tl) {
      const uint64_t base = bs.start + (uint64_t)tl * TILE;
      const uint32_t cnt = min(TILE, bs.len - tl * TILE);
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const uint32_t jj = i * THREADS + threadIdx.x;
        nkey[i] = K(0);
        nidx[i] = 0;
        npay[i] = 0;
        nb[i] = 0;
        if (jj < cnt) {
          if constexpr (SRC_IN) {
            nkey[i] = in_keys[base + jj];  // raw bits: mapped when the tile is used, so the prefetch does not wait
            nidx[i] = (uint32_t)(base + jj - bs.ubase);
            if constexpr (IDS) nb[i] = get_bucket_id(w.ids, bs.start, (uint64_t)tl * TILE + jj, bs.logk);
          } else {
            bv.get(base + jj, nkey[i], nidx[i]);
            nb[i] = get_bucket_id(w.ids, bs.start, (uint64_t)tl * TILE + jj, bs.logk);
          }
          if constexpr (PAY) npay[i] = bpay[base + jj];
        }
      }
    };
    if (gl * GT < t_end) load_tile(gl * GT);
    for (uint32_t tl = gl * GT; tl < t_end; tl++) {
      const uint32_t cnt = min(TILE, bs.len - tl * TILE);
      K key[ITEMS];
      uint32_t idx[ITEMS], pay[ITEMS], pos[ITEMS], b[ITEMS];
      bool valid[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        valid[i] = i * THREADS + threadIdx.x < cnt;
        key[i] = SRC_IN ? ord_of<K, F32>(nkey[i]) : nkey[i];
        idx[i] = nidx[i];
        pay[i] = npay[i];
        b[i] = nb[i];
      }
      if (tl + 1 < t_end) load_tile(tl + 1);
      if constexpr (!IDS)
        classify_batch<K, ITEMS>(tk, ti, bs.logk, key, valid, [&](int i) -> uint32_t { return idx[i]; }, b,
                                 pairs);
      // rank inside (tile, bucket): one LDS atomic per element, or one per wave
      // when the whole wave falls into a single bucket (skewed inputs).  A
      // wave's valid elements are a prefix of its lanes, so lane 0 holds one
      // whenever any lane does.
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const uint32_t b0 = uniform(b[i]);
        uint32_t r = 0;
        if (__ballot(valid[i] && b[i] != b0) == 0) {
          const uint64_t act = __ballot(valid[i]);
          uint32_t basev = 0;
          if (lane == 0 && act) basev = atomicAdd(&hist[b0], (uint32_t)__popcll(act));
          r = uniform(basev) + (uint32_t)__popcll(act & ((1ull << lane) - 1ull));
        } else if (valid[i]) {
          r = atomicAdd(&hist[b[i]], 1u);
        }
        pos[i] = valid[i] ? ((b[i] << 23) | r) : 0xFFFFFFFFu;  // b < 2^9, r < TILE <= 2^23
      }
      __syncthreads();
      // exclusive scan of the tile histogram -> tile-local bucket starts
      {
        const uint32_t hv = threadIdx.x < kk ? hist[threadIdx.x] : 0u;
        runs += hv != 0u ? 1u : 0u;  // one run per non-empty bucket of a tile
        const uint32_t e = bins_excl_scan(hv, tmp);
        if (threadIdx.x < kk) {
          hist[threadIdx.x] = e;
          gdelta[threadIdx.x] = run_off - e;
          run_off += hv;
        }
      }
      __syncthreads();
      // every item's bucket start is read before any is used (an element
      // past the tile's end reads bin 511, inside hist, and is not staged)
      uint32_t hb[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; i++) hb[i] = hist[pos[i] >> 23];
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        if (pos[i] != 0xFFFFFFFFu) {
          const uint32_t bb = pos[i] >> 23;
          const uint32_t p = hb[i] + (pos[i] & 0x7FFFFFu);
          pos[i] = p;
          stage[p] = key[i];
          stage32[p] = idx[i];
          stage_b[p] = (uint16_t)bb;
        }
      }
      __syncthreads();
      if (threadIdx.x < kMaxK) hist[threadIdx.x] = 0;  // ready for the next tile
      // the next tile's loads complete here, before this tile's stores are
      // issued: a wait for them after the stores would wait for the stores too
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        asm volatile("" ::"v"(nkey[i]), "v"(nidx[i]));
        if constexpr (PAY) asm volatile("" ::"v"(npay[i]));
        if constexpr (IDS) asm volatile("" ::"v"(nb[i]));
      }
      if (!PAY && cnt == TILE) {
        // a full tile: all staged reads, then all run offsets, then the
        // stores, so that no thread waits on one LDS round trip per element
        // (not with a payload: its instances have no registers to spare)
        uint32_t sb[ITEMS], si[ITEMS];
        K sk[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
          const uint32_t p = i * THREADS + threadIdx.x;
          sb[i] = stage_b[p];
          sk[i] = stage[p];
          si[i] = stage32[p];
        }
        uint64_t gd[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; i++) gd[i] = gdelta[sb[i]];
#pragma unroll
        for (int i = 0; i < ITEMS; i++) dv.put(gd[i] + i * THREADS + threadIdx.x, sk[i], si[i]);
      } else {
        for (uint32_t p = threadIdx.x; p < cnt; p += THREADS) {
          const uint64_t g = gdelta[stage_b[p]] + p;
          dv.put(g, stage[p], stage32[p]);
        }
      }
      if constexpr (PAY) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; i++)
          if (pos[i] != 0xFFFFFFFFu) stage32[pos[i]] = pay[i];
        __syncthreads();
        for (uint32_t p = threadIdx.x; p < cnt; p += THREADS) dpay[gdelta[stage_b[p]] + p] = stage32[p];
      }
      __syncthreads();
    }
    };
    if (ids0)
      tiles(BoolC<true>{});
    else
      tiles(BoolC<false>{});
  }
  // the first level's run count, read by the next level's plan (a kernel
  // argument: a load here would wait for the write-out stores first)
  if (count_runs) {
    __shared__ uint32_t s_runs;
    if (threadIdx.x == 0) s_runs = 0;
    __syncthreads();
    for (int d = kWave / 2; d > 0; d >>= 1) runs += (uint32_t)__shfl_xor((int)runs, d, kWave);
    if (lane == 0 && runs) atomicAdd(&s_runs, runs);
    __syncthreads();
    if (threadIdx.x == 0 && s_runs) atomicAdd(&w.ctl->runs, s_runs);  // one global atomic per workgroup
  }
}


// ===========================================================================
// Host side
// ===========================================================================
static Tuning g_tuning;

Tuning& tuning() { return g_tuning; }

static inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Bucket size the levels aim for: at most half the LDS capacity, so that the
// spread of bucket sizes around it stays below the capacity.
static uint32_t effective_target(const Tuning& t, uint32_t cap) {
  return std::max<uint32_t>(64u, std::min<uint32_t>(t.target, cap / 2));
}

uint32_t plan_levels(uint64_t n, const Tuning& t, uint32_t cap) {
  if (n <= cap) return 0;
  uint32_t L = 0;
  uint64_t reach = effective_target(t, cap);
  while (reach < n) {
    reach <<= kMaxLogK;
    L++;
  }
  L = std::max<uint32_t>(L, 1);
  // extra levels, while every level still gets at least 4 buckets
  uint32_t lq = 0;
  for (uint64_t q = (n + effective_target(t, cap) - 1) / effective_target(t, cap); (1ull << lq) < q;) lq++;
  for (uint32_t e = 0; e < t.extra_levels && 2 * (L + 1) <= lq; e++) L++;
  return std::min<uint32_t>(L, std::min<uint32_t>(t.max_levels, kMaxLevels));
}

uint32_t effective_cap(const Tuning& t, bool pay) {
  uint32_t cap = std::min<uint32_t>(t.cap, pay ? 8192u : 12288u);
  return std::max<uint32_t>(cap, 64u);
}

// Keys per tile group: about four groups per CU for n keys, so that a level
// over one segment still fills the GPU, within [2^13, 2^17].
static uint32_t group_log2_for(uint64_t n) {
  const uint64_t want = n / ((uint64_t)num_cu_cached() * 4);
  uint32_t lg = kGroupMinLog2;
  while (lg < kGroupMaxLog2 && (1ull << (lg + 1)) <= want) lg++;
  return lg;
}

// Tile groups of the levels after the first of a plain sort hold at most
// 2^kGroupUpLog2 keys, or 2^kGroupSmallLog2 when the first level's runs were
// short (chosen on the device, k_plan).  Such a level splits k segments of
// about n / k keys each, and with small groups the workgroups of an XCD,
// which take consecutive groups, work on neighbouring tiles of one segment
// at once, so their runs of each bucket land next to each other in HBM.  A
// new group costs a drain of the tile prefetch and a strided read of its
// bucket offsets: the first level (one segment, whose skewed inputs already
// write long runs) and segmented sorts (mostly short segments, so
// neighbouring groups seldom share one) do not recover that and keep the
// larger groups, and inputs whose runs are long already keep 2^kGroupUpLog2.
constexpr uint32_t kGroupUpLog2 = 14, kGroupSmallLog2 = 13;
static uint32_t group_log2_level(uint32_t glog0, uint32_t lev, bool segmented) {
  return (lev == 0 || segmented) ? glog0 : std::min<uint32_t>(glog0, kGroupUpLog2);
}
static uint32_t group_log2_small(uint32_t glog0, uint32_t lev, bool segmented) {
  return (lev == 0 || segmented) ? 0u : std::min<uint32_t>(glog0, kGroupSmallLog2);
}

// Workspace layout: returns total bytes; fills w (pointers relative to base).
size_t layout(int kt, uint64_t n, uint32_t num_segs, bool pay, const Tuning& t, char* base, Work* w,
              uint32_t* levels_out) {
  const uint64_t ks = kt == 1 ? 8 : 4;
  const uint32_t cap = effective_cap(t, pay);
  const uint32_t levels = plan_levels(n, t, cap);
  const uint64_t big_max = levels ? n / (cap + 1) + 1 : 0;
  const uint32_t glog = group_log2_for(n);
  const uint64_t groups_max = levels ? (n >> std::min<uint32_t>(glog, kGroupSmallLog2)) + big_max + 1 : 0;
  const uint64_t count_max = groups_max * kMaxK;
  const uint64_t scan_blocks = count_max / kScanChunk + 2;
  const uint64_t final_max = (uint64_t)num_segs + (uint64_t)levels * kMaxK * big_max + 1;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const uint64_t o_ctl = take(sizeof(Ctl));
  const uint64_t o_big0 = take(big_max * sizeof(BigSeg));
  const uint64_t o_big1 = take(big_max * sizeof(BigSeg));
  const uint64_t o_tb = take((big_max + 1) * 4);
  const uint64_t o_cb = take((big_max + 1) * 4);
  const uint64_t o_tk = take(big_max * kMaxK * ks);
  const uint64_t o_ti = take(big_max * kMaxK * 4);
  const uint64_t o_cnt = take(count_max * 4);
  const uint64_t o_off = take(count_max * 4);
  const uint64_t o_par = take(scan_blocks * 8);
  const uint64_t o_part = take(scan_blocks * 4);
  uint64_t o_cls[kNumClasses], cls_cap[kNumClasses];
  for (int c = 0; c < kNumClasses; c++) {
    const uint64_t lo = c == 0 ? 0 : h_class_max[c - 1];
    uint64_t bound = n / (lo + 1) + 1;
    if (c == kNumClasses - 1) bound = n / (std::min<uint64_t>(cap, 64) + 1) + 1;
    // a single-level plain sort may route all its (at most kMaxK) buckets to one class
    cls_cap[c] = std::min<uint64_t>(final_max, std::max<uint64_t>(bound, kMaxK + 1));
    o_cls[c] = take(cls_cap[c] * sizeof(FinalSeg));
  }
  const uint64_t nb = (levels || t.force_fallback) ? n : 0;
  const uint64_t o_ids = take(levels >= 2 ? 2 * n : 0);
  uint64_t o_bk[2], o_bp[2];
  for (int b = 0; b < 2; b++) {
    o_bk[b] = take(nb * (ks + 4));
    o_bp[b] = take(pay ? nb * 4 : 0);
  }
  if (w) {
    w->ctl = (Ctl*)(base + o_ctl);
    w->big[0] = (BigSeg*)(base + o_big0);
    w->big[1] = (BigSeg*)(base + o_big1);
    w->group_base = (uint32_t*)(base + o_tb);
    w->count_base = (uint32_t*)(base + o_cb);
    w->tree_key = base + o_tk;
    w->tree_idx = (uint32_t*)(base + o_ti);
    w->counts = (uint32_t*)(base + o_cnt);
    w->offsets = (uint32_t*)(base + o_off);
    w->scan_flags = (uint64_t*)(base + o_par);
    w->scan_part = (uint32_t*)(base + o_part);
    for (int c = 0; c < kNumClasses; c++) {
      w->cls[c] = (FinalSeg*)(base + o_cls[c]);
      w->cls_cap[c] = cls_cap[c];
    }
    for (int b = 0; b < 2; b++) {
      w->buf_rec[b] = (uint32_t*)(base + o_bk[b]);
      w->buf_pay[b] = pay ? (uint32_t*)(base + o_bp[b]) : nullptr;
    }
    w->ids = levels >= 2 ? (uint8_t*)(base + o_ids) : nullptr;
    w->big_max = big_max;
    w->group_log2 = glog;
    w->spread = t.extra_levels > 0 ? 1u : 0u;
    w->count_max = count_max;
    w->scan_blocks = scan_blocks;
    w->n = n;
  }
  if (levels_out) *levels_out = levels;
  return off;
}

static int g_num_cu = 0;
uint32_t num_cu_cached();
static int num_cu() {
  if (!g_num_cu) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess)
      g_num_cu = p.multiProcessorCount;
    else
      g_num_cu = 256;
  }
  return g_num_cu;
}

uint32_t num_cu_cached() { return (uint32_t)num_cu(); }

static inline uint32_t grid_for(uint64_t work, uint32_t per_cu) {
  const uint64_t g = std::min<uint64_t>(work, (uint64_t)num_cu() * per_cu);
  return (uint32_t)std::max<uint64_t>(g, 1);
}




// Algorithm of each size class: RFIS, RQuick or the LDS merge sort.
template <typename K, bool F32, bool PAY>
static int launch_class_sort(int c, const Work& w, const K* kin, const uint32_t* pay_in, K* kout, uint32_t* perm_out,
                             uint32_t* pay_out, uint64_t cap_c, hipStream_t st, const Tuning& t) {
  const int cb = c & 0xFF;  // c may carry kDirect
  if (h_class_max[cb] <= t.rfis_max)
    return launch_rfis_class<K, F32, PAY>(c, w, kin, pay_in, kout, perm_out, pay_out, cap_c, st);
  if (h_class_max[cb] <= t.rquick_max)
    return launch_rquick_class<K, F32, PAY>(c, w, kin, pay_in, kout, perm_out, pay_out, cap_c, st);
  return launch_merge_class<K, F32, PAY>(c, w, kin, pay_in, kout, perm_out, pay_out, cap_c, st);
}

template <typename K, bool F32, bool PAY>
static int enqueue_typed(const void* keys_in, const uint32_t* pay_in, const uint64_t* seg_off, uint32_t num_segs,
                         uint64_t n, void* keys_out, uint32_t* perm_out, uint32_t* pay_out, void* ws,
                         size_t ws_bytes, hipStream_t st) {
  const Tuning t = g_tuning;
  Work w;
  uint32_t levels = 0;
  const size_t need = layout(F32 ? 2 : (sizeof(K) == 8 ? 1 : 0), n, num_segs, PAY, t, (char*)ws, &w, &levels);
  if (ws_bytes < need) return -2;
  const uint32_t cap = effective_cap(t, PAY);
  const uint32_t a = std::min<uint32_t>(std::max<uint32_t>(t.oversample, 1), kMaxOversample);
  const uint32_t ff = t.force_fallback;
  const uint32_t target = effective_target(t, cap);
  const K* kin = (const K*)keys_in;
  K* kout = (K*)keys_out;

  if (!seg_off && levels == 0 && !ff && n <= cap) {
    // the whole input fits one workgroup: one launch, no segment lists
    int c = 0;
    while (n > h_class_max[c]) c++;
    return launch_class_sort<K, F32, PAY>(c | kDirect, w, kin, pay_in, kout, perm_out, pay_out, 1, st, t);
  }
  // A single-level plain sort with at most about two final buckets per CU
  // routes all of them to the class kernel for twice the target size (and
  // the one above it), so the local sorts run in one or two launches.
  uint32_t cmin = 0;
  if (!seg_off && levels == 1 && n <= (uint64_t)target * 2 * num_cu()) {
    const uint32_t want = std::min<uint32_t>(2 * target, cap);
    while (cmin + 2 < (uint32_t)kNumClasses && h_class_max[cmin] < want) cmin++;
  }
  // a single-level sort of few buckets (cmin > 0) is latency-bound on its
  // one-workgroup sample sort: 16 samples per bucket keep its buckets
  // within twice the target while halving that step
  const uint32_t a0 = cmin ? std::min<uint32_t>(a, 16u) : a;
  // the first level's sample drawn at the start (k_start_plain), room in buffer B
  const int staged = (!seg_off && levels > 0 && n >= (uint64_t)kSplThreads * kSplItems) ? 1 : 0;
  if (!seg_off) {
    RS_LAUNCH(k_start_plain<K>, staged ? (uint32_t)(kSplThreads * kSplItems / kStartThreads) : 1u, kStartThreads,
              st, w, n, cap, target, levels, ff, cmin, kin, a0, t.seed, staged);
  } else {
    RS_LAUNCH(k_reset, 1, 256, st, w.ctl, levels);
    RS_LAUNCH(k_init, grid_for((num_segs + 1023) / 1024, 1), 1024, st, w, seg_off, num_segs, n, cap, target, levels,
              ff, cmin);
  }

  const Work w0 = w;
  for (uint32_t lev = 0; lev < levels; lev++) {
    // the level's tile groups; scatter tiles are at most a tile group
    Work w = w0;
    w.group_log2 = group_log2_level(w0.group_log2, lev, seg_off != nullptr);
    const uint32_t glog_small = group_log2_small(w0.group_log2, lev, seg_off != nullptr);
    // the first level of a plain sort with more levels counts its runs for the next plan
    const int runs = (lev == 0 && levels > 1 && !seg_off) ? 1 : 0;
    const uint32_t tile_log2 = (t.tile_log2 == 12 || std::min(w.group_log2, glog_small ? glog_small : 99u) < 13) ? 12 : 13;
    const uint64_t groups_max = (n >> (glog_small ? glog_small : w.group_log2)) + w.big_max + 1;
    const int dst = lev & 1;
    const int src = (lev + 1) & 1;  // buffer written by the previous level
    const bool last = lev + 1 == levels;
    // the level's buckets are routed by the scatter's workgroups (level_end)
    const LevelEnd le{cap, target, last ? 1u : 0u, (uint32_t)(dst + 1), ff, levels - lev - 1, cmin};
    if (lev > 0 || seg_off) RS_LAUNCH(k_plan, 1, kPlanThreads, st, w, (int)lev, glog_small);  // level 0 of a plain sort: planned at the start
    const uint32_t gs = grid_for(w.big_max, 4);
    if (lev == 0) {
      // first-level bucket ids need the id buffer (two levels or more) and
      // are not taken by the payload scatter
      const int ids_ok = (w.ids != nullptr && !PAY) ? 1 : 0;
      RS_LAUNCH((k_splitters<K, F32, true, kSplThreads, kSplItems>), gs, kSplThreads, st, w, (int)lev, kin, src, a0,
                t.seed, ids_ok, staged);
    } else {
      RS_LAUNCH((k_splitters<K, false, false, kSplThreads, kSplItems>), gs, kSplThreads, st, w, (int)lev, kin, src, a,
                t.seed, 0, 0);
    }
    // count tiles: 512 threads x 8 keys; scatter tiles: 512 x 8 (tile_log2
    // 12) or 1024 x 8 (tile_log2 13); both walk the same groups of
    // 2^group_log2 keys.  Grids are multiples of 8 for the XCD-aware walk.
    // resident-sized grids: the workgroups take groups from the queues
    const uint32_t gt = std::max<uint32_t>(8u, grid_for(groups_max, 4) & ~7u);
    const uint32_t gs_sc = std::max<uint32_t>(8u, grid_for(groups_max, tile_log2 == 12 ? 2 : 1) & ~7u);
    if (lev == 0)
      RS_LAUNCH((k_count<K, F32, true, 512, 8>), gt, 512, st, w, (int)lev, kin, src);
    else
      RS_LAUNCH((k_count<K, false, false, 512, 8>), gt, 512, st, w, (int)lev, kin, src);
    if (w.count_max <= kChainedScanMax) {
      RS_LAUNCH(k_scan, grid_for(w.count_max / kScanChunk + 1, 4), kScanThreads, st, w);
    } else {
      const uint32_t gsc = grid_for(w.count_max / kScanChunk + 1, 8);
      RS_LAUNCH(k_scan_reduce, gsc, kScanThreads, st, w);
      RS_LAUNCH(k_scan_partials, 1, kScanTopThreads, st, w);
      RS_LAUNCH(k_scan_down, gsc, kScanThreads, st, w);
    }
    if (tile_log2 == 12) {
      if (lev == 0)
        RS_LAUNCH((k_scatter<K, F32, true, PAY, 512, 8>), gs_sc, 512, st, w, (int)lev, kin, pay_in, src, dst, runs, le);
      else
        RS_LAUNCH((k_scatter<K, false, false, PAY, 512, 8>), gs_sc, 512, st, w, (int)lev, kin, pay_in, src, dst, 0, le);
    } else {
      if (lev == 0)
        RS_LAUNCH((k_scatter<K, F32, true, PAY, 1024, 8>), gs_sc, 1024, st, w, (int)lev, kin, pay_in, src, dst, runs, le);
      else
        RS_LAUNCH((k_scatter<K, false, false, PAY, 1024, 8>), gs_sc, 1024, st, w, (int)lev, kin, pay_in, src, dst, 0, le);
    }
  }

  // final segments by size class (a class can only be non-empty if its lower
  // bound is below cap)
  for (int c = (int)cmin; c < kNumClasses - 1; c++) {
    if (c > 0 && h_class_max[c - 1] >= cap) break;
    const int kinds = levels == 0 ? kInputOnly : (num_segs > 1 ? kMixed : 0);
    const int rc = launch_class_sort<K, F32, PAY>(c | kinds, w, kin, pay_in, kout, perm_out, pay_out, w.cls_cap[c],
                                                  st, t);
    if (rc) return rc;
  }
  {
    const int rc = launch_local_fallbacks<K, F32, PAY>(w, cap, kin, pay_in, kout, perm_out, pay_out, st);
    if (rc) return rc;
  }
  {
    const int rc = launch_oversize<K, F32, PAY>(w, kin, pay_in, kout, perm_out, pay_out, w.cls_cap[kNumClasses - 1], st);
    if (rc) return rc;
  }
  return 0;
}

int enqueue_sort(int kt, const void* keys_in, const uint32_t* pay_in, const uint64_t* seg_off, uint32_t num_segs,
                 uint64_t n, void* keys_out, uint32_t* perm_out, uint32_t* pay_out, void* ws, size_t ws_bytes,
                 hipStream_t st) {
  const bool pay = pay_in && pay_out;
  if (!pay) {
    pay_in = nullptr;
    pay_out = nullptr;
  }
  switch (kt) {
    case 0:
      return pay ? enqueue_typed<uint32_t, false, true>(keys_in, pay_in, seg_off, num_segs, n, keys_out, perm_out,
                                                         pay_out, ws, ws_bytes, st)
                 : enqueue_typed<uint32_t, false, false>(keys_in, pay_in, seg_off, num_segs, n, keys_out, perm_out,
                                                          pay_out, ws, ws_bytes, st);
    case 1:
      return pay ? enqueue_typed<uint64_t, false, true>(keys_in, pay_in, seg_off, num_segs, n, keys_out, perm_out,
                                                         pay_out, ws, ws_bytes, st)
                 : enqueue_typed<uint64_t, false, false>(keys_in, pay_in, seg_off, num_segs, n, keys_out, perm_out,
                                                          pay_out, ws, ws_bytes, st);
    case 2:
      return pay ? enqueue_typed<uint32_t, true, true>(keys_in, pay_in, seg_off, num_segs, n, keys_out, perm_out,
                                                        pay_out, ws, ws_bytes, st)
                 : enqueue_typed<uint32_t, true, false>(keys_in, pay_in, seg_off, num_segs, n, keys_out, perm_out,
                                                         pay_out, ws, ws_bytes, st);
    default:
      return -1;
  }
}

size_t workspace_bytes(int kt, uint64_t n, uint32_t num_segs, bool pay) {
  return layout(kt, n, num_segs, pay, g_tuning, nullptr, nullptr, nullptr);
}

}  // namespace rs
