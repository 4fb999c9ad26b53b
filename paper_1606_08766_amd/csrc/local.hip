// LDS sorts of final segments (one workgroup per segment) and the
// global-memory fallback for segments longer than the LDS capacity.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "device.hpp"
#include "engine.hpp"
#include "internal.hpp"

namespace rs {

static inline uint32_t grid_for(uint64_t work, uint32_t per_cu) {
  const uint64_t g = std::min<uint64_t>(work, (uint64_t)num_cu_cached() * per_cu);
  return (uint32_t)std::max<uint64_t>(g, 1);
}

// Workgroup shape of a class kernel: THREADS x ITEMS elements.
template <int THREADS, int ITEMS>
struct Shape {
  static constexpr int T = THREADS, I = ITEMS;
};



// ---------------------------------------------------------------------------
// The final segments a class kernel sorts.  flag 0: segment q = blockIdx.x +
// i * gridDim.x of class cls.  Otherwise (the launches after all classes):
// every segment of every class whose src carries `flag`; each thread checks
// one segment and the flagged ones are collected in LDS (s_list holds THREADS
// entries), so that the search is parallel rather than a chain of dependent
// loads.  body(cc, q) runs on every thread of the block.
template <int THREADS, typename F>
__device__ __forceinline__ void for_each_segment(const Work& w, int cls, uint32_t flag, uint32_t* s_list,
                                                 uint32_t& s_n, F&& body, int part = 0) {
  if (!flag) {
    // part 1 / 2: a mixed call's user segments / level segments.  k_init
    // routes every user segment before any level runs, so they are the
    // first class_in entries of each class list.
    uint32_t q0 = 0, q1 = final_count(w, cls);
    if (part && cls >= 0) {
      const uint32_t nin = min(w.ctl->class_in[cls], q1);
      if (part == 1)
        q1 = nin;
      else
        q0 = nin;
    }
    for (uint32_t q = q0 + blockIdx.x; q < q1; q += gridDim.x) body(cls, q);
    return;
  }
  for (int cc = 0; cc <= kNumClasses - 2; cc++) {
    const uint32_t cnt = final_count(w, cc);
    for (uint32_t q0 = blockIdx.x * THREADS; q0 < cnt; q0 += gridDim.x * THREADS) {
      if (threadIdx.x == 0) s_n = 0;
      __syncthreads();
      const uint32_t q = q0 + threadIdx.x;
      if (q < cnt && (w.cls[cc][q].src & flag)) s_list[atomicAdd(&s_n, 1u)] = q;
      __syncthreads();
      const uint32_t n = s_n;
      for (uint32_t k = 0; k < n; k++) body(cc, s_list[k]);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Final segments of one size class: one workgroup each, sorted in LDS as
// (key, position) pairs.  FLAGGED: the segments of every class that the word
// sort below handed over (kPairsFlag); the shape then fits the largest class.
template <typename K, bool F32, bool PAY, int THREADS, int ITEMS, bool FLAGGED = false>
__global__ __launch_bounds__(THREADS) void k_local_sort(Work w, int cls, const K* in_keys, const uint32_t* in_pay,
                                                        K* keys_out, uint32_t* perm_out, uint32_t* pay_out) {
  constexpr int N = THREADS * ITEMS;
  constexpr int NP = lpad_size(N);
  __shared__ uint32_t s_lo[NP];
  __shared__ uint32_t s_hi[sizeof(K) == 8 ? NP : 1];
  __shared__ uint32_t s_v[NP];
  __shared__ uint32_t s_p[PAY ? NP : 1];
  const LdsArr<K> sa{s_lo, s_hi, s_v, s_p};
  direct_reset(w, cls);
  __shared__ uint32_t s_list[FLAGGED ? THREADS : 1];
  __shared__ uint32_t s_n;
  for_each_segment<THREADS>(w, cls, FLAGGED ? kPairsFlag : 0u, s_list, s_n, [&](int cc, uint32_t q) {
    FinalSeg f = final_at(w, cc, q);
    if (FLAGGED && !(f.src & kPairsFlag)) return;  // uniform
    f.src &= 0xFFu;
    const BufView<K> sb{f.src ? w.buf_rec[f.src - 1] : nullptr};
    const uint32_t* srcp = f.src ? w.buf_pay[f.src - 1] : in_pay;
    K k[ITEMS];
    uint32_t v[ITEMS], p[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      // thread t takes logical elements t*ITEMS+i; load striped for coalescing
      // and let the first sort round place them (any input order is valid).
      const uint32_t j = i * THREADS + threadIdx.x;
      k[i] = KMax<K>::v;
      v[i] = j < f.len ? j : kPadIdx;
      p[i] = j;
    }
    // one source per segment (uniform), so each branch issues all its loads
    // before any is used
    if (f.src) {
#pragma unroll
      for (int i = 0; i < ITEMS; i++)
        if (i * THREADS + threadIdx.x < f.len) sb.get(f.start + i * THREADS + threadIdx.x, k[i], v[i]);
    } else {
#pragma unroll
      for (int i = 0; i < ITEMS; i++)
        if (i * THREADS + threadIdx.x < f.len) k[i] = in_keys[f.start + i * THREADS + threadIdx.x];  // raw bits
    }
    if constexpr (F32) {
      if (!f.src) {
#pragma unroll
        for (int i = 0; i < ITEMS; i++)
          if (i * THREADS + threadIdx.x < f.len) k[i] = ord_of<K, F32>(k[i]);
      }
    }
    lds_merge_sort<K, THREADS, ITEMS, PAY>(k, v, p, sa);
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const int q = lpad(threadIdx.x * ITEMS + i);
      sa.put(q, k[i], v[i]);
      if constexpr (PAY) s_p[q] = p[i];
    }
    __syncthreads();
    if constexpr (PAY) {
      // the payloads are gathered before any output store (a load issued
      // after stores waits for them)
      uint32_t pv[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const uint32_t j = i * THREADS + threadIdx.x;
        pv[i] = j < f.len ? srcp[f.start + s_p[lpad(j)]] : 0u;
      }
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const uint32_t j = i * THREADS + threadIdx.x;
        if (j < f.len) {
          const int q = lpad(j);
          keys_out[f.start + j] = to_output<K, F32>(sa.key(q));
          if (perm_out) perm_out[f.start + j] = s_v[q];
          pay_out[f.start + j] = pv[i];
        }
      }
    } else {
      for (uint32_t j = threadIdx.x; j < f.len; j += THREADS) {
        const int q = lpad(j);
        keys_out[f.start + j] = to_output<K, F32>(sa.key(q));
        if (perm_out) perm_out[f.start + j] = s_v[q];
      }
    }
    __syncthreads();
  });
}

// ---------------------------------------------------------------------------
// Bins of the word sort: a segment's words are distinct, so each word's rank
// is the number of smaller words.  The words are first distributed into 2^LB
// bins by the top bits of (word - lower bound), which keeps the bins in word
// order; a word's rank is then the start of its bin plus the number of smaller
// words inside the bin, found by comparing against the bin's words only.  On
// the key distributions the sample sort leaves in a final segment (near
// uniform over its range) a bin holds about 3 to 8 words (up to 16 in the
// instances of at most 4096 words), so this takes far
// fewer steps than a merge sort's log2(len) rounds.  The ranking costs about
// the sum over the bins of size^2 compares; where that exceeds kRankBudget per
// word (runs of equal keys, keys clustered far apart) the segment is left to
// the merge sort.
constexpr uint32_t kRankBudget = 128;

// Bin phase: c holds the element words, element j = i * THREADS + t as c[i];
// elements j >= len are not used.  Counts the words of each bin (bin[0 .. S]
// are zero on entry; r receives each word's place among its bin's words, in
// no particular order), turns the counts into bin starts (bin[S] = len) and
// returns, uniformly over the block, whether the ranking fits kRankBudget.
// The first wave scans the bins (S / 64 per lane) and leaves the ranking
// cost in *cost.
template <int THREADS, int ITEMS, int LB>
__device__ __forceinline__ bool bin_count(const uint64_t (&c)[ITEMS], uint32_t len, uint32_t* bin, uint32_t* cost,
                                          int t, const BinMap& bm, uint32_t (&r)[ITEMS]) {
  constexpr int S = 1 << LB;
  constexpr int PL = S / kWave;  // bins per lane of the scanning wave
  static_assert(PL >= 1, "at least one bin per lane");
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    r[i] = 0;
    if ((uint32_t)(i * THREADS + t) < len) r[i] = atomicAdd(&bin[bm(c[i])], 1u);
  }
  __syncthreads();
  if (t < kWave) {
    // one scan of (sum of squared bin sizes, bin size): the low half gives
    // the bin starts, the high half's total the ranking cost (both fit 32 bits)
    uint64_t v = 0;
#pragma unroll 4
    for (int k = 0; k < PL; k++) {
      const uint32_t x = bin[t * PL + k];
      v += ((uint64_t)(x * x) << 32) | x;
    }
    const uint64_t inc = wave_incl_scan<uint64_t>(v);
    uint32_t e = (uint32_t)(inc - v);
#pragma unroll 4
    for (int k = 0; k < PL; k++) {  // the counts are read again: fewer registers
      const uint32_t x = bin[t * PL + k];
      bin[t * PL + k] = e;
      e += x;
    }
    if (t == kWave - 1) {
      bin[S] = len;
      *cost = (uint32_t)(inc >> 32);
    }
  }
  __syncthreads();
  return *cost <= kRankBudget * len;
}

// Rank phase, after bin_count succeeded: places the words in their bins (in
// wb, unpadded), ranks every word and writes the sorted words to lo/hi at
// lpad(rank); wb and lo/hi are the same LDS memory, and the caller
// synchronises before reading lo/hi.  wb holds at least len + 3 words (ranking
// reads up to three words past a bin's end; the three words past len are set
// to all ones, larger than any word).
template <int THREADS, int ITEMS, int LB>
__device__ __forceinline__ void bin_rank(const uint64_t (&c)[ITEMS], const uint32_t (&r)[ITEMS], uint32_t len,
                                         uint64_t* wb, uint32_t* lo, uint32_t* hi, const uint32_t* bin, int t,
                                         const BinMap& bm) {
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    if ((uint32_t)(i * THREADS + t) < len) wb[bin[bm(c[i])] + r[i]] = c[i];
  }
  if (t < 3) wb[len + t] = ~0ull;
  __syncthreads();
  // rank of the word at each position: words of later bins and the all-ones
  // words are larger, so the count may run past the bin's end
  uint32_t rk[ITEMS];
  uint64_t wv[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    const uint32_t p = i * THREADS + t;  // < N: inside wb
    const uint64_t w = wb[p];
    uint32_t db = bm(w);
    db = p < len ? db : 0u;
    const uint32_t s0 = bin[db];
    const uint32_t s1 = p < len ? bin[db + 1] : s0;
    uint32_t less = 0;
    for (uint32_t q = s0; q < s1; q += 4) {
      less += wb[q] < w ? 1u : 0u;
      less += wb[q + 1] < w ? 1u : 0u;
      less += wb[q + 2] < w ? 1u : 0u;
      less += wb[q + 3] < w ? 1u : 0u;
    }
    rk[i] = s0 + less;
    wv[i] = w;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    if ((uint32_t)(i * THREADS + t) < len) {
      const int qq = lpad((int)rk[i]);
      lo[qq] = (uint32_t)wv[i];
      hi[qq] = (uint32_t)(wv[i] >> 32);
    }
  }
}

// ---------------------------------------------------------------------------
// Final segments of one size class sorted as single 64-bit words.  With mn the
// segment's smallest key and rb the bit width of (largest key - mn), and PB
// the bit width of a slot (the element's place in the segment as stored):
//   exact words   rb + 32 (+ PB with payload) <= 64: the word
//                 (key - mn, position [, slot]) orders exactly like the
//                 (key, position) pair;
//   slot words    otherwise: the word (top 64 - PB bits of key - mn, slot);
//                 words with equal top parts (equal keys, or keys differing
//                 only in dropped low bits) come out in slot order, which is
//                 checked against their (key, position) order afterwards.
// The words are distinct.  Segments of at least 1024 elements are ordered by
// bins and ranks (bin_count, bin_rank); a segment whose ranking would cost too
// much is marked kMergeFlag and left to the MERGE instance, launched once
// after all classes with the largest class's shape, which (like the
// instances for shorter segments) sorts the words with the LDS merge sort.  A
// segment whose check finds a pair out of order is marked kPairsFlag and
// sorted by k_local_sort<FLAGGED>, launched last.  Every path produces the
// same output; words take half the LDS of pairs and one compare per step.
// SRCBUF false: the instance for segments of the caller's input only (no
// table of positions); true: for buffer segments, and for input segments too
// unless `mixed` (then the other instance takes those).
template <typename K, bool F32, bool PAY, int THREADS, int ITEMS, bool MERGE = false, bool SRCBUF = true>
__global__ __launch_bounds__(THREADS, (THREADS >= 1024 ? 8 : 1)) void k_local_words(Work w, int cls, const K* in_keys, const uint32_t* in_pay,
                                                         K* keys_out, uint32_t* perm_out, uint32_t* pay_out,
                                                         int mixed) {
  constexpr int N = THREADS * ITEMS;
  constexpr int NP = lpad_size(N);
  constexpr int PB = 32 - __builtin_clz((unsigned)(N - 1));
  constexpr uint64_t SLOT = (1ull << PB) - 1;
  constexpr int XB = PAY ? PB : 0;  // slot bits kept in exact words (payload gather)
  // bins: about four words each in a full segment, for segments long
  // enough to need them; eight in the instances of at most 4096 words, whose
  // LDS then still fits three workgroups per CU
  constexpr bool BINS = !MERGE && N >= 1024;
  constexpr int LB = 31 - __builtin_clz((unsigned)(N <= 4096 ? N / 8 : N / 4));
  // the merge sort and the output read words as two halves (lo, hi); the
  // bins see the same memory as whole words
  __shared__ uint64_t s_words[NP];
  uint32_t* const s_lo = (uint32_t*)s_words;
  uint32_t* const s_hi = s_lo + NP;
  __shared__ uint32_t s_red[6 * (THREADS / kWave)];
  __shared__ uint32_t s_bin[BINS ? (1 << LB) + 1 : 1];
  __shared__ uint32_t s_cost;
  // positions of the segment's elements by slot (for segments of a buffer),
  // loaded coalesced with the keys; SRCBUF false: every segment lies in the
  // caller's input and positions are slots
  __shared__ uint32_t s_idx[SRCBUF ? N : 1];
  static_assert(!BINS || NP >= N + 3, "room for the words read past a bin's end");
  __shared__ uint32_t s_list[MERGE ? THREADS : 1];
  __shared__ uint32_t s_n;
  for_each_segment<THREADS>(w, cls, MERGE ? kMergeFlag : 0u, s_list, s_n, [&](int cc, uint32_t q) {
    FinalSeg f = final_at(w, cc, q);
    if (MERGE && !(f.src & kMergeFlag)) return;  // uniform
    f.src &= 0xFFu;
    if (SRCBUF ? (mixed && f.src == 0) : f.src != 0) return;  // the other instance's
    // an opaque copy of the thread index: per-thread addresses are recomputed
    // per segment rather than hoisted out of the loop and kept live
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const BufView<K> sb{f.src ? w.buf_rec[f.src - 1] : nullptr};
    const uint32_t* srcp = f.src ? w.buf_pay[f.src - 1] : in_pay;
    auto idx_at = [&](uint32_t j) -> uint32_t { return (SRCBUF && f.src) ? s_idx[j] : j; };
    auto key_at = [&](uint32_t j) -> K { return f.src ? sb.key(f.start + j) : load_ord<K, F32>(in_keys, f.start + j); };
    // thread t takes slots i*THREADS+t (striped, coalesced).  All ITEMS loads
    // are issued before any is used: a use inside each guarded load would
    // wait for that load before the next one goes out.  The keys then wait
    // in the word memory until the minimum is known.
    const bool from_buf = SRCBUF && f.src;
    K kr[ITEMS];
    uint32_t ir[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      kr[i] = K(0);
      ir[i] = i * THREADS + tid;
    }
    if (from_buf) {  // uniform: one source per segment
#pragma unroll
      for (int i = 0; i < ITEMS; i++)
        if (i * THREADS + tid < f.len) sb.get(f.start + i * THREADS + tid, kr[i], ir[i]);
    } else {
#pragma unroll
      for (int i = 0; i < ITEMS; i++)
        if (i * THREADS + tid < f.len) kr[i] = in_keys[f.start + i * THREADS + tid];
    }
    K mn = KMax<K>::v, mx = K(0);
    uint32_t imn = ~0u, imx = 0u;
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t j = i * THREADS + tid;
      if (j < f.len) {
        const K key = from_buf ? kr[i] : ord_of<K, F32>(kr[i]);
        if (from_buf) s_idx[j] = ir[i];
        s_words[j] = (uint64_t)key;
        mn = key < mn ? key : mn;
        mx = key > mx ? key : mx;
        imn = min(imn, ir[i]);
        imx = max(imx, ir[i]);
      }
    }
    if constexpr (BINS) {
      for (int b = tid; b <= (1 << LB); b += THREADS) s_bin[b] = 0;
    }
    {
      // its barrier also orders the stores above before their readers
      const Range4 br = block_range<K, THREADS>(mn, mx, imn, imx, s_red, tid);
      mn = (K)br.kmn;
      mx = (K)br.kmx;
      imn = br.imn;
      imx = br.imx;
    }
    const uint64_t range = (uint64_t)(mx - mn);
    const int rb = range ? 64 - __clzll((long long)range) : 0;
    const bool exact = rb + 32 + XB <= 64;
    // slot words keep the top 64 - PB bits of (key - mn): drop low bits when
    // the key range is wider than that
    const int drop = exact ? 0 : max(rb + PB - 64, 0);
    // the order of equal word prefixes must be checked unless it is exact: no
    // key bits dropped and slots in position order (segments of the input)
    const bool check = !exact && (drop > 0 || f.src != 0);
    const int sh = exact ? 32 + XB : PB;
    uint64_t c[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t j = i * THREADS + tid;
      uint64_t low = j;
      if (exact) low = ((uint64_t)(j < f.len ? idx_at(j) : 0u) << XB) | (PAY ? j : 0u);
      c[i] = j < f.len ? (((uint64_t)((K)s_words[j] - mn) >> drop) << sh) | low : ~0ull;
    }
    if constexpr (BINS) {
      // bounds of the words: exact words are at least (position min) and at
      // most (key range, position max, all slot bits); slot words lie in
      // [0, (key range >> drop, len - 1)]
      BinMap bm;
      if (exact && rb < LB) {  // key part, then the top bits of the position
        const uint32_t ib = LB - rb, ir = imx - imn;
        const int ibits = ir ? 32 - __clz(ir) : 0;
        bm = BinMap{(uint64_t)imn << XB, (uint32_t)sh, ib, (uint32_t)(XB + max(ibits - (int)ib, 0)), (1u << ib) - 1u};
      } else {
        const uint64_t wmn = exact ? (uint64_t)imn << XB : 0ull;
        const uint64_t wmx = exact ? ((uint64_t)range << sh) | ((uint64_t)imx << XB) | (PAY ? SLOT : 0ull)
                                   : (((uint64_t)range >> drop) << PB) | (uint64_t)(f.len - 1);
        const uint64_t wr = wmx - wmn;
        const int bits = wr ? 64 - __clzll((long long)wr) : 0;
        bm = BinMap{wmn, (uint32_t)(bits > LB ? bits - LB : 0), 0u, 0u, 0u};
      }
      uint32_t r[ITEMS];
      if (!bin_count<THREADS, ITEMS, LB>(c, f.len, s_bin, &s_cost, tid, bm, r)) {
        // uniform; every thread is past its reads of this segment's LDS
        if (tid == 0) w.cls[cc][q].src = f.src | kMergeFlag;
        return;
      }
      bin_rank<THREADS, ITEMS, LB>(c, r, f.len, s_words, s_lo, s_hi, s_bin, tid, bm);
    } else {
      __syncthreads();  // every key read from the word memory
      lds_merge_sort_words<THREADS, ITEMS>(c, s_lo, s_hi, tid);
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const int qq = lpad(tid * ITEMS + i);
        s_lo[qq] = (uint32_t)c[i];
        s_hi[qq] = (uint32_t)(c[i] >> 32);
      }
    }
    __syncthreads();
    bool bad = false;
    if constexpr (!PAY) {
      for (uint32_t j = tid; j < f.len; j += THREADS) {
        const int qq = lpad(j);
        const uint64_t cj = ((uint64_t)s_hi[qq] << 32) | s_lo[qq];
        const uint32_t slot = (uint32_t)(cj & SLOT);
        uint32_t idx;
        K key;
        if (exact) {
          idx = (uint32_t)(cj >> XB);
          key = (K)(mn + (K)(cj >> sh));
        } else {
          idx = idx_at(slot);
          key = drop ? key_at(slot) : (K)(mn + (K)(cj >> sh));
          if (check && j + 1 < f.len) {
            const int qn = lpad(j + 1);
            const uint64_t cn = ((uint64_t)s_hi[qn] << 32) | s_lo[qn];
            if ((cn >> PB) == (cj >> PB)) {
              // equal prefixes: the pair order decides
              const uint32_t sn = (uint32_t)(cn & SLOT);
              if (pair_less(key_at(sn), idx_at(sn), key, idx)) bad = true;
            }
          }
        }
        keys_out[f.start + j] = to_output<K, F32>(key);
        if (perm_out) perm_out[f.start + j] = idx;
      }
    } else {
      // with a payload, gathered by slot from global memory: the thread's
      // sorted elements j = tid + k * THREADS are read (LDS, and the global
      // key and payload reads by slot) before any output store, since a load
      // issued after stores waits for them
      K okey[ITEMS];
      uint32_t oidx[ITEMS], opay[ITEMS];
#pragma unroll
      for (int k = 0; k < ITEMS; k++) {
        const uint32_t j = tid + k * THREADS;
        okey[k] = K(0);
        oidx[k] = 0;
        opay[k] = 0;
        if (j < f.len) {
          const int qq = lpad(j);
          const uint64_t cj = ((uint64_t)s_hi[qq] << 32) | s_lo[qq];
          const uint32_t slot = (uint32_t)(cj & SLOT);
          if (exact) {
            oidx[k] = (uint32_t)(cj >> XB);
            okey[k] = (K)(mn + (K)(cj >> sh));
          } else {
            oidx[k] = idx_at(slot);
            okey[k] = drop ? key_at(slot) : (K)(mn + (K)(cj >> sh));
          }
          opay[k] = srcp[f.start + slot];
        }
      }
      if (check) {  // uniform
#pragma unroll
        for (int k = 0; k < ITEMS; k++) {
          const uint32_t j = tid + k * THREADS;
          if (j + 1 < f.len) {
            const uint64_t cj = ((uint64_t)s_hi[lpad(j)] << 32) | s_lo[lpad(j)];
            const uint64_t cn = ((uint64_t)s_hi[lpad(j + 1)] << 32) | s_lo[lpad(j + 1)];
            if ((cn >> PB) == (cj >> PB)) {
              // equal prefixes: the pair order decides
              const uint32_t sn = (uint32_t)(cn & SLOT);
              if (pair_less(key_at(sn), idx_at(sn), okey[k], oidx[k])) bad = true;
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < ITEMS; k++) {
        const uint32_t j = tid + k * THREADS;
        if (j < f.len) {
          keys_out[f.start + j] = to_output<K, F32>(okey[k]);
          if (perm_out) perm_out[f.start + j] = oidx[k];
          pay_out[f.start + j] = opay[k];
        }
      }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) w.cls[cc][q].src = f.src | kPairsFlag;
  }, mixed ? (SRCBUF ? 2 : 1) : 0);
}

// ---------------------------------------------------------------------------
// Fallback for final segments longer than cap (the balance guarantee of the
// sampling holds only with high probability): bottom-up merge sort through
// global memory by one workgroup, ping-ponging between the two buffers over
// the segment's own range (that range of the other buffer is never used by
// another segment).  Slow, exact, rare.
template <typename K>
struct GRun {
  const K* k;
  const uint32_t* v;
  const uint32_t* p;
};

template <typename K, bool F32, bool PAY, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_oversize(Work w, const K* in_keys, const uint32_t* in_pay, K* keys_out,
                                                      uint32_t* perm_out, uint32_t* pay_out) {
  constexpr int C = THREADS * ITEMS;
  __shared__ K sk[C];
  __shared__ uint32_t sv[C];
  __shared__ uint32_t sp[C];
  const int cls = kNumClasses - 1;
  const uint32_t cnt = (uint32_t)min((uint64_t)w.ctl->class_count[cls], w.cls_cap[cls]);
  for (uint32_t q = blockIdx.x; q < cnt; q += gridDim.x) {
    const FinalSeg f = w.cls[cls][q];
    // buffers used: data source code f.src; first target is the other buffer
    // pass 0 writes into the buffer that does not hold the data
    int cur = f.src == 0 ? 0 : ((int)f.src - 1) ^ 1;
    const BufView<K> sb{f.src ? w.buf_rec[f.src - 1] : nullptr};
    const uint32_t* srcp = f.src ? w.buf_pay[f.src - 1] : in_pay;
    // pass 0: sort chunks of C in LDS
    for (uint32_t c0 = 0; c0 < f.len; c0 += C) {
      K k[ITEMS];
      uint32_t v[ITEMS], p[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const uint32_t j = c0 + threadIdx.x * ITEMS + i;
        if (j < f.len) {
          if (f.src) {
            sb.get(f.start + j, k[i], v[i]);
          } else {
            k[i] = in_keys[f.start + j];  // raw bits; mapped below once all loads are issued
            v[i] = j;
          }
          p[i] = PAY ? srcp[f.start + j] : 0u;
        } else {
          k[i] = KMax<K>::v;
          v[i] = kPadIdx;
          p[i] = 0;
        }
      }
      if constexpr (F32) {
        if (!f.src) {
#pragma unroll
          for (int i = 0; i < ITEMS; i++)
            if (c0 + threadIdx.x * ITEMS + i < f.len) k[i] = ord_of<K, F32>(k[i]);
        }
      }
      block_merge_sort<K, THREADS, ITEMS, PAY>(k, v, p, sk, sv, sp);
      const BufView<K> db{w.buf_rec[cur]};
      uint32_t* dp = w.buf_pay[cur];
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const uint32_t j = c0 + threadIdx.x * ITEMS + i;
        if (j < f.len) {
          db.put(f.start + j, k[i], v[i]);
          if constexpr (PAY) dp[f.start + j] = p[i];
        }
      }
      __syncthreads();
    }
    // merge passes
    for (uint32_t run = C; run < f.len; run <<= 1) {
      const BufView<K> ab{w.buf_rec[cur] + f.start * BufView<K>::W};
      const uint32_t* ap = PAY ? w.buf_pay[cur] + f.start : nullptr;
      const BufView<K> db{w.buf_rec[cur ^ 1] + f.start * BufView<K>::W};
      uint32_t* dp = PAY ? w.buf_pay[cur ^ 1] + f.start : nullptr;
      for (uint32_t o0 = 0; o0 < f.len; o0 += THREADS) {
        const uint32_t o = o0 + threadIdx.x;  // output position handled by this thread
        if (o < f.len) {
          const uint32_t first = o / (2 * run) * (2 * run);
          const uint32_t alen = min(run, f.len - first);
          const uint32_t b0 = first + alen;
          const uint32_t blen = b0 < f.len ? min(run, f.len - b0) : 0u;
          const uint32_t d = o - first;
          // number of A elements among the first d outputs (ties prefer A)
          uint32_t lo = d > blen ? d - blen : 0u, hi = d < alen ? d : alen;
          while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            const uint32_t bj = b0 + d - 1 - mid;
            if (pair_less(ab.key(bj), ab.idx(bj), ab.key(first + mid), ab.idx(first + mid)))
              hi = mid;
            else
              lo = mid + 1;
          }
          const uint32_t ai = lo, bi = d - lo;
          bool takeA;
          if (ai >= alen)
            takeA = false;
          else if (bi >= blen)
            takeA = true;
          else
            takeA = !pair_less(ab.key(b0 + bi), ab.idx(b0 + bi), ab.key(first + ai), ab.idx(first + ai));
          const uint32_t sidx = takeA ? first + ai : b0 + bi;
          db.put(o, ab.key(sidx), ab.idx(sidx));
          if constexpr (PAY) dp[o] = ap[sidx];
        }
      }
      __syncthreads();
      cur ^= 1;
    }
    // output
    const BufView<K> rb{w.buf_rec[cur] + f.start * BufView<K>::W};
    const uint32_t* rp = PAY ? w.buf_pay[cur] + f.start : nullptr;
    for (uint32_t j = threadIdx.x; j < f.len; j += THREADS) {
      keys_out[f.start + j] = to_output<K, F32>(rb.key(j));
      if (perm_out) perm_out[f.start + j] = rb.idx(j);
      if constexpr (PAY) pay_out[f.start + j] = rp[j];
    }
    __syncthreads();
  }
}

// Local sort of one class with the merge sort.  A one-segment direct sort
// runs the pair sort alone; a class list runs the word sort and then the pair
// sort over the segments the word sort handed over.
#ifndef RS_WORDS_PER_CU
#define RS_WORDS_PER_CU 64
#endif
template <typename K, bool F32, bool PAY, int T, int I>
static int merge_class_launch(int c, const Work& w, const K* kin, const uint32_t* pay_in, K* kout,
                              uint32_t* perm_out, uint32_t* pay_out, uint64_t cap_c, hipStream_t st) {
  static const std::string shape = std::to_string(T) + ", " + std::to_string(I);
  static const std::string t_pairs = "(k_local_sort<K, F32, PAY, " + shape + ">)";
  static const std::string t_words = "(k_local_words<K, F32, PAY, " + shape + ">)";
  static const std::string t_words_in = "(k_local_words<K, F32, PAY, " + shape + ", false, false>)";
  if (c & kDirect) {
    RS_LAUNCH_TAGGED((k_local_sort<K, F32, PAY, T, I>), t_pairs.c_str(), 1, T, st, w, -1, kin, pay_in, kout,
                     perm_out, pay_out);
    return 0;
  }
  // the word sort takes about one workgroup per segment (bounded); handed-over
  // segments are sorted by launch_local_fallbacks after all classes
  const int cb = c & 0xFF;
  const int mixed = (c & kMixed) ? 1 : 0;
  if (c & (kInputOnly | kMixed))  // input segments
    RS_LAUNCH_TAGGED((k_local_words<K, F32, PAY, T, I, false, false>), t_words_in.c_str(),
                     grid_for(cap_c, RS_WORDS_PER_CU), T, st, w, cb, kin, pay_in, kout, perm_out, pay_out, mixed);
  if (!(c & kInputOnly))  // buffer segments (and input ones unless mixed)
    RS_LAUNCH_TAGGED((k_local_words<K, F32, PAY, T, I>), t_words.c_str(), grid_for(cap_c, RS_WORDS_PER_CU), T, st, w,
                     cb, kin, pay_in, kout, perm_out, pay_out, mixed);
  return 0;
}

// The segments the word sorts of all classes handed over: the merge sort of
// words for those whose ranking was too costly, then the pair sort for those
// whose word order failed the check.  One resident-sized launch each, with
// the shape of the largest class a call can have.
template <typename K, bool F32, bool PAY, int T, int I>
static int fallback_launch(const Work& w, const K* kin, const uint32_t* pay_in, K* kout, uint32_t* perm_out,
                            uint32_t* pay_out, hipStream_t st) {
  static const std::string shape = std::to_string(T) + ", " + std::to_string(I);
  static const std::string t_merge = "(k_local_words<K, F32, PAY, " + shape + ", true>)";
  static const std::string t_flagged = "(k_local_sort<K, F32, PAY, " + shape + ", true>)";
  const uint32_t g = grid_for(1u << 30, 1);
  RS_LAUNCH_TAGGED((k_local_words<K, F32, PAY, T, I, true>), t_merge.c_str(), g, T, st, w, 0, kin, pay_in, kout,
                   perm_out, pay_out, 0);
  RS_LAUNCH_TAGGED((k_local_sort<K, F32, PAY, T, I, true>), t_flagged.c_str(), g, T, st, w, 0, kin, pay_in, kout,
                   perm_out, pay_out);
  return 0;
}

template <typename K, bool F32, bool PAY>
int launch_local_fallbacks(const Work& w, uint32_t cap, const K* kin, const uint32_t* pay_in, K* kout,
                           uint32_t* perm_out, uint32_t* pay_out, hipStream_t st) {
  if constexpr (!PAY) {
    if (cap > 8192) return fallback_launch<K, F32, PAY, 768, 16>(w, kin, pay_in, kout, perm_out, pay_out, st);
  }
  return fallback_launch<K, F32, PAY, 1024, 8>(w, kin, pay_in, kout, perm_out, pay_out, st);
}

template <typename K, bool F32, bool PAY>
int launch_merge_class(int c, const Work& w, const K* kin, const uint32_t* pay_in, K* kout, uint32_t* perm_out,
                       uint32_t* pay_out, uint64_t cap_c, hipStream_t st) {
  const int cb = c & 0xFF;
  auto go = [&](auto tag, uint32_t) -> int {
    constexpr int T = decltype(tag)::T, I = decltype(tag)::I;
    return merge_class_launch<K, F32, PAY, T, I>(c, w, kin, pay_in, kout, perm_out, pay_out, cap_c, st);
  };
  // alternative shapes (tuning.class_shape): twice the threads, half the keys
  // per thread, for the classes from 1024 to 8192 keys
  const bool alt = (c & kDirect) == 0 && ((tuning().class_shape >> cb) & 1u);
  switch (cb) {
    case 0: return go(Shape<64, 1>{}, 16);
    case 1: return go(Shape<64, 4>{}, 16);
    case 2: return alt ? go(Shape<512, 2>{}, 8) : go(Shape<256, 4>{}, 8);
    case 3: return alt ? go(Shape<512, 4>{}, 8) : go(Shape<256, 8>{}, 8);
    case 4: return alt ? go(Shape<768, 4>{}, 4) : go(Shape<384, 8>{}, 4);
    case 5: return alt ? go(Shape<1024, 4>{}, 3) : go(Shape<512, 8>{}, 3);
    case 6: return go(Shape<768, 8>{}, 2);
    case 7: return go(Shape<1024, 8>{}, 1);
    case 8:
      if constexpr (!PAY) return go(Shape<768, 16>{}, 1);
      break;
    default:
      break;
  }
  return 0;
}

#define RS_INST_MERGE(K, F, P)                                                                                 \
  template int launch_merge_class<K, F, P>(int, const Work&, const K*, const uint32_t*, K*, uint32_t*, uint32_t*, \
                                           uint64_t, hipStream_t);                                              \
  template int launch_local_fallbacks<K, F, P>(const Work&, uint32_t, const K*, const uint32_t*, K*, uint32_t*,   \
                                               uint32_t*, hipStream_t);
RS_INST_MERGE(uint32_t, false, false)
RS_INST_MERGE(uint32_t, true, false)
RS_INST_MERGE(uint64_t, false, false)
RS_INST_MERGE(uint32_t, false, true)
RS_INST_MERGE(uint32_t, true, true)
RS_INST_MERGE(uint64_t, false, true)


template <typename K, bool F32, bool PAY>
int launch_oversize(const Work& w, const K* kin, const uint32_t* pay_in, K* kout, uint32_t* perm_out,
                    uint32_t* pay_out, uint64_t cap_c, hipStream_t st) {
  RS_LAUNCH((k_oversize<K, F32, PAY, 256, 16>), grid_for(cap_c, 1), 256, st, w, kin, pay_in, kout, perm_out, pay_out);
  return 0;
}

#define RS_INST_OVER(K, F, P)                                                                                  \
  template int launch_oversize<K, F, P>(const Work&, const K*, const uint32_t*, K*, uint32_t*, uint32_t*, uint64_t, \
                                        hipStream_t);
RS_INST_OVER(uint32_t, false, false)
RS_INST_OVER(uint32_t, true, false)
RS_INST_OVER(uint64_t, false, false)
RS_INST_OVER(uint32_t, false, true)
RS_INST_OVER(uint32_t, true, true)
RS_INST_OVER(uint64_t, false, true)

}  // namespace rs
