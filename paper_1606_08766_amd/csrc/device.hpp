// Device primitives shared by the rsort kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace rs {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Keys.  Every kernel works on "ordinal" keys: unsigned integers whose
// unsigned order is the sort order.  u32/u64 keys are their own ordinals; an
// f32 key maps to its IEEE 754 totalOrder ordinal (negative patterns are
// bit-inverted, non-negative ones get the sign bit set), which is a bijection,
// so the original bits are restored exactly on output.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t f32_ord(uint32_t u) {
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ uint32_t f32_unord(uint32_t o) {
  return (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
}

template <typename K>
struct KMax;
template <>
struct KMax<uint32_t> {
  static constexpr uint32_t v = 0xFFFFFFFFu;
};
template <>
struct KMax<uint64_t> {
  static constexpr uint64_t v = ~0ull;
};

// Padding element: above every real (key, position) pair because real
// positions are < 2^32 - 1.
constexpr uint32_t kPadIdx = 0xFFFFFFFFu;

template <typename K>
__device__ __forceinline__ bool pair_less(K ka, uint32_t ia, K kb, uint32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

template <typename K, bool F32>
__device__ __forceinline__ K ord_of(K v) {
  if constexpr (F32) return (K)f32_ord((uint32_t)v);
  return v;
}
template <typename K, bool F32>
__device__ __forceinline__ K load_ord(const K* p, uint64_t i) {
  return ord_of<K, F32>(p[i]);
}
template <typename K, bool F32>
__device__ __forceinline__ K to_output(K o) {
  if constexpr (F32) return (K)f32_unord((uint32_t)o);
  return o;
}

// ---------------------------------------------------------------------------
// Counter-based random numbers for sample positions and coin flips:
// SplitMix64's output function applied to a counter (Steele, Lea, Flood 2014).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t rand_at(uint64_t seed, uint64_t stream, uint64_t i) {
  return mix64(seed + mix64(stream + 0x632BE59BD9B4E019ull) + (i + 1) * 0x9E3779B97F4A7C15ull);
}

// ---------------------------------------------------------------------------
// Wave / block scans.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Inclusive scan across the 64 lanes of a wave (T: 32- or 64-bit unsigned).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_up(v, d, kWave);
    if (lane >= (uint32_t)d) v += o;
  }
  return v;
}

// Exclusive block scan of one value per thread.  `tmp` holds >= THREADS/64 + 1
// values of LDS.  Returns the exclusive prefix; *total receives the block sum.
template <typename T>
struct NoDeduce {
  using type = T;
};
template <int THREADS, typename T = uint32_t>
__device__ __forceinline__ T block_excl_scan(T v, typename NoDeduce<T>::type* tmp, typename NoDeduce<T>::type* total) {
  constexpr int NW = THREADS / kWave;
  const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
  T inc = wave_incl_scan<T>(v);
  if (lane == kWave - 1) tmp[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      T t = tmp[i];
      tmp[i] = s;
      s += t;
    }
    tmp[NW] = s;
  }
  __syncthreads();
  T r = tmp[w] + inc - v;
  if (total) *total = tmp[NW];
  __syncthreads();
  return r;
}

// Wave-aggregated append: every active lane obtains a slot from
// counters[key] with one atomic per distinct key per wave.  Must be reached by
// all lanes of the wave (inactive lanes pass active = false).
__device__ __forceinline__ uint32_t wave_append(uint32_t* counters, uint32_t key, bool active) {
  uint32_t slot = 0;
  const uint32_t lane = lane_id();
  uint64_t pending = __ballot(active);
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t k = __shfl(key, leader, kWave);
    const uint64_t m = __ballot(active && key == k) & pending;
    uint32_t base = 0;
    if (lane == (uint32_t)leader) base = atomicAdd(&counters[k], (uint32_t)__popcll(m));
    base = __shfl(base, leader, kWave);
    if ((m >> lane) & 1ull) slot = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    pending &= ~m;
  }
  return slot;
}

// ---------------------------------------------------------------------------
// Register sorting network (bitonic) on ITEMS (power of two) pairs, ascending.
// The compare-exchange swaps with a mask and XORs rather than selecting
// between two array elements: a select of two array loads can be folded into
// a load at a select-computed index, which keeps the arrays out of registers.
// ---------------------------------------------------------------------------
template <typename K>
__device__ __forceinline__ void cx_swap(K& a, K& b, bool sw) {
  const K m = (K)0 - (K)(sw ? 1 : 0);
  const K x = (a ^ b) & m;
  a ^= x;
  b ^= x;
}

template <typename K, int ITEMS, bool CARRY>
__device__ __forceinline__ void reg_sort_impl(K (&k)[ITEMS], uint32_t (&v)[ITEMS], uint32_t (&p)[ITEMS]) {
#pragma unroll
  for (int size = 2; size <= ITEMS; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const int j = i ^ stride;
        if (j > i) {
          const bool asc = (i & size) == 0;
          // ascending: the smaller pair ends at i
          const bool jl = pair_less(k[j], v[j], k[i], v[i]);
          const bool sw = asc ? jl : !jl;
          cx_swap(k[i], k[j], sw);
          cx_swap(v[i], v[j], sw);
          if constexpr (CARRY) cx_swap(p[i], p[j], sw);
        }
      }
    }
  }
}

template <typename K, int ITEMS>
__device__ __forceinline__ void reg_sort(K (&k)[ITEMS], uint32_t (&v)[ITEMS]) {
  uint32_t p[ITEMS];
  reg_sort_impl<K, ITEMS, false>(k, v, p);
}

// Same network carrying a third value.
template <typename K, int ITEMS>
__device__ __forceinline__ void reg_sort3(K (&k)[ITEMS], uint32_t (&v)[ITEMS], uint32_t (&p)[ITEMS]) {
  reg_sort_impl<K, ITEMS, true>(k, v, p);
}

// ---------------------------------------------------------------------------
// Block merge sort of N = THREADS * ITEMS pairs (N need not be a power of two;
// ITEMS must be).
// On entry thread t holds logical elements t*ITEMS .. t*ITEMS+ITEMS-1 in
// k/v (and p if CARRY); on exit it holds sorted ranks t*ITEMS .. likewise.
// sk/sv/sp: LDS arrays of N entries.  Pairs must be distinct except for
// padding copies.  Each round merges adjacent sorted runs: every thread finds
// where its ITEMS outputs start with a merge-path binary search and merges
// them serially from LDS.  Ties (padding only) prefer the left run in both
// the search and the serial merge, so the two always agree.
// ---------------------------------------------------------------------------
// With GROUP < THREADS, runs never cross aligned groups of GROUP threads: each
// group of GROUP * ITEMS elements is sorted independently (GROUP must then be
// a power of two dividing THREADS).
template <typename K, int THREADS, int ITEMS, bool CARRY, int GROUP = THREADS>
__device__ __forceinline__ void block_merge_sort(K (&k)[ITEMS], uint32_t (&v)[ITEMS],
                                                 uint32_t (&p)[ITEMS], K* sk, uint32_t* sv,
                                                 uint32_t* sp) {
  constexpr int N = THREADS * ITEMS;
  if constexpr (CARRY)
    reg_sort3<K, ITEMS>(k, v, p);
  else
    reg_sort<K, ITEMS>(k, v);
  const int t = threadIdx.x;
#pragma unroll 1
  for (int run = ITEMS; run < GROUP * ITEMS; run <<= 1) {
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      sk[t * ITEMS + i] = k[i];
      sv[t * ITEMS + i] = v[i];
      if constexpr (CARRY) sp[t * ITEMS + i] = p[i];
    }
    __syncthreads();
    const int first = (t * ITEMS) & ~(2 * run - 1);
    const int a0 = first, b0 = first + run;
    const int alen = (N - a0) < run ? (N - a0) : run;
    const int blen = (N - b0) <= 0 ? 0 : ((N - b0) < run ? (N - b0) : run);
    const int d = t * ITEMS - first;
    int lo = d > blen ? d - blen : 0;
    int hi = d < alen ? d : alen;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const int bj = b0 + d - 1 - mid;
      if (pair_less(sk[bj], sv[bj], sk[a0 + mid], sv[a0 + mid]))
        hi = mid;
      else
        lo = mid + 1;
    }
    int ai = lo, bi = d - lo;
    K ka = ai < alen ? sk[a0 + ai] : K(0);
    uint32_t va = ai < alen ? sv[a0 + ai] : 0u;
    K kb = bi < blen ? sk[b0 + bi] : K(0);
    uint32_t vb = bi < blen ? sv[b0 + bi] : 0u;
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const bool takeA = ai < alen && (bi >= blen || !pair_less(kb, vb, ka, va));
      k[i] = takeA ? ka : kb;
      v[i] = takeA ? va : vb;
      if constexpr (CARRY) p[i] = takeA ? sp[a0 + ai] : sp[b0 + bi];
      if (takeA) {
        ai++;
        if (ai < alen) {
          ka = sk[a0 + ai];
          va = sv[a0 + ai];
        }
      } else {
        bi++;
        if (bi < blen) {
          kb = sk[b0 + bi];
          vb = sv[b0 + bi];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Bank-conflict-free LDS merge sort.
//
// Elements live in LDS as separate 32-bit arrays (key low word, key high word
// for u64 keys, position, optional carried value) with one pad word after
// every 32 words: logical index i is stored at i + i/32.  In the merge rounds
// lane t reads around logical index t * ITEMS / 2, and in the store phase at
// t * ITEMS; with the pad both patterns spread a wave over all 32 banks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }
__host__ __device__ constexpr int lpad_size(int n) { return n + (n >> 5) + 1; }

template <typename K>
struct LdsArr {
  uint32_t* lo;
  uint32_t* hi;  // u64 keys only
  uint32_t* v;
  uint32_t* p;   // carried value (CARRY only)
  __device__ __forceinline__ K key(int q) const {
    if constexpr (sizeof(K) == 8)
      return ((uint64_t)hi[q] << 32) | lo[q];
    else
      return lo[q];
  }
  __device__ __forceinline__ void put(int q, K k, uint32_t idx) const {
    lo[q] = (uint32_t)k;
    if constexpr (sizeof(K) == 8) hi[q] = (uint32_t)((uint64_t)k >> 32);
    v[q] = idx;
  }
};

template <typename K, int THREADS, int ITEMS, bool CARRY, int GROUP = THREADS>
__device__ __forceinline__ void lds_merge_sort(K (&k)[ITEMS], uint32_t (&v)[ITEMS], uint32_t (&p)[ITEMS],
                                               const LdsArr<K>& s) {
  constexpr int N = THREADS * ITEMS;
  if constexpr (CARRY)
    reg_sort3<K, ITEMS>(k, v, p);
  else
    reg_sort<K, ITEMS>(k, v);
  const int t = threadIdx.x;
#pragma unroll 1
  for (int run = ITEMS; run < GROUP * ITEMS; run <<= 1) {
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const int q = lpad(t * ITEMS + i);
      s.put(q, k[i], v[i]);
      if constexpr (CARRY) s.p[q] = p[i];
    }
    __syncthreads();
    const int first = (t * ITEMS) & ~(2 * run - 1);
    const int a0 = first, b0 = first + run;
    const int alen = (N - a0) < run ? (N - a0) : run;
    const int blen = (N - b0) <= 0 ? 0 : ((N - b0) < run ? (N - b0) : run);
    const int d = t * ITEMS - first;
    int lo = d > blen ? d - blen : 0;
    int hi = d < alen ? d : alen;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const int qb = lpad(b0 + d - 1 - mid), qa = lpad(a0 + mid);
      if (pair_less(s.key(qb), s.v[qb], s.key(qa), s.v[qa]))
        hi = mid;
      else
        lo = mid + 1;
    }
    int ai = lo, bi = d - lo;
    K ka = K(0), kb = K(0);
    uint32_t va = 0, vb = 0;
    if (ai < alen) {
      const int q = lpad(a0 + ai);
      ka = s.key(q);
      va = s.v[q];
    }
    if (bi < blen) {
      const int q = lpad(b0 + bi);
      kb = s.key(q);
      vb = s.v[q];
    }
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const bool takeA = ai < alen && (bi >= blen || !pair_less(kb, vb, ka, va));
      k[i] = takeA ? ka : kb;
      v[i] = takeA ? va : vb;
      if constexpr (CARRY) p[i] = s.p[lpad(takeA ? a0 + ai : b0 + bi)];
      // advance the consumed side and fetch its next element
      const int na = takeA ? ai + 1 : ai, nb = takeA ? bi : bi + 1;
      const bool more = takeA ? na < alen : nb < blen;
      if (more) {
        const int q = lpad(takeA ? a0 + na : b0 + nb);
        const K nk = s.key(q);
        const uint32_t nv = s.v[q];
        if (takeA) {
          ka = nk;
          va = nv;
        } else {
          kb = nk;
          vb = nv;
        }
      }
      ai = na;
      bi = nb;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The padded LDS merge sort for plain 64-bit words (one value per element),
// used on composite words that already encode the sort order.  Equal words
// are interchangeable.  Half the LDS of a (key, position) pair sort per
// element and one compare per step.
// ---------------------------------------------------------------------------
template <int ITEMS>
__device__ __forceinline__ void reg_sort_words(uint64_t (&c)[ITEMS]) {
#pragma unroll
  for (int size = 2; size <= ITEMS; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const int j = i ^ stride;
        if (j > i) {
          const bool asc = (i & size) == 0;
          const bool jl = c[j] < c[i];
          cx_swap(c[i], c[j], asc ? jl : !jl);
        }
      }
    }
  }
}

// t: the thread's index in the block (a caller may pass a copy the compiler
// cannot see through, so per-thread addresses are not hoisted out of its loop).
template <int THREADS, int ITEMS>
__device__ __forceinline__ void lds_merge_sort_words(uint64_t (&c)[ITEMS], uint32_t* lo, uint32_t* hi,
                                                     int t = threadIdx.x) {
  constexpr int N = THREADS * ITEMS;
  reg_sort_words<ITEMS>(c);
  auto word = [&](int q) -> uint64_t { return ((uint64_t)hi[q] << 32) | lo[q]; };
#pragma unroll 1
  for (int run = ITEMS; run < N; run <<= 1) {
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const int q = lpad(t * ITEMS + i);
      lo[q] = (uint32_t)c[i];
      hi[q] = (uint32_t)(c[i] >> 32);
    }
    __syncthreads();
    const int first = (t * ITEMS) & ~(2 * run - 1);
    const int a0 = first, b0 = first + run;
    const int alen = (N - a0) < run ? (N - a0) : run;
    const int blen = (N - b0) <= 0 ? 0 : ((N - b0) < run ? (N - b0) : run);
    const int d = t * ITEMS - first;
    int l = d > blen ? d - blen : 0;
    int h = d < alen ? d : alen;
    while (l < h) {
      const int mid = (l + h) >> 1;
      if (word(lpad(b0 + d - 1 - mid)) < word(lpad(a0 + mid)))
        h = mid;
      else
        l = mid + 1;
    }
    int ai = l, bi = d - l;
    uint64_t ca = ai < alen ? word(lpad(a0 + ai)) : 0ull;
    uint64_t cb = bi < blen ? word(lpad(b0 + bi)) : 0ull;
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const bool takeA = ai < alen && (bi >= blen || !(cb < ca));
      c[i] = takeA ? ca : cb;
      const int na = takeA ? ai + 1 : ai, nb = takeA ? bi : bi + 1;
      const bool more = takeA ? na < alen : nb < blen;
      if (more) {
        const uint64_t nc = word(lpad(takeA ? a0 + na : b0 + nb));
        if (takeA)
          ca = nc;
        else
          cb = nc;
      }
      ai = na;
      bi = nb;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Block-wide minimum and maximum of the keys and of the positions (every
// thread of the block calls, every lane active).  Lanes of a row of 16 are
// combined with DPP moves (xor 1, xor 2, then the half-row and row mirrors),
// the four rows of a wave by lane reads into scalar registers, the waves
// through LDS (one row of lanes reads the per-wave values).  The results are
// uniform and live in scalar registers.  red holds 6 * THREADS/64 words.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  return ((uint64_t)dpp_u32<CTRL>((uint32_t)(v >> 32)) << 32) | dpp_u32<CTRL>((uint32_t)v);
}
__device__ __forceinline__ uint32_t lane_u32(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int l) {
  return ((uint64_t)lane_u32((uint32_t)(v >> 32), l) << 32) | lane_u32((uint32_t)v, l);
}
struct Range4 {  // key minimum and maximum (as 64 bits), position minimum and maximum
  uint64_t kmn, kmx;
  uint32_t imn, imx;
};

template <typename K>
__device__ __forceinline__ void row_reduce(K& kmn, K& kmx, uint32_t& imn, uint32_t& imx) {
  auto step = [&](auto ctrl) {
    constexpr int C = decltype(ctrl)::value;
    K a, b;
    if constexpr (sizeof(K) == 8) {
      a = (K)dpp_u64<C>((uint64_t)kmn);
      b = (K)dpp_u64<C>((uint64_t)kmx);
    } else {
      a = (K)dpp_u32<C>((uint32_t)kmn);
      b = (K)dpp_u32<C>((uint32_t)kmx);
    }
    const uint32_t c = dpp_u32<C>(imn), d = dpp_u32<C>(imx);
    kmn = a < kmn ? a : kmn;
    kmx = b > kmx ? b : kmx;
    imn = min(imn, c);
    imx = max(imx, d);
  };
  step(std::integral_constant<int, 0xB1>{});   // quad_perm [1,0,3,2]
  step(std::integral_constant<int, 0x4E>{});   // quad_perm [2,3,0,1]
  step(std::integral_constant<int, 0x141>{});  // row_half_mirror
  step(std::integral_constant<int, 0x140>{});  // row_mirror
}

template <typename K>
__device__ __forceinline__ Range4 rows_to_scalar(K kmn, K kmx, uint32_t imn, uint32_t imx, int rows) {
  Range4 r{~0ull, 0ull, ~0u, 0u};
  for (int q = 0; q < rows; q++) {
    uint64_t a, b;
    if constexpr (sizeof(K) == 8) {
      a = lane_u64((uint64_t)kmn, 16 * q);
      b = lane_u64((uint64_t)kmx, 16 * q);
    } else {
      a = lane_u32((uint32_t)kmn, 16 * q);
      b = lane_u32((uint32_t)kmx, 16 * q);
    }
    const uint32_t c = lane_u32(imn, 16 * q), d = lane_u32(imx, 16 * q);
    r.kmn = a < r.kmn ? a : r.kmn;
    r.kmx = b > r.kmx ? b : r.kmx;
    r.imn = min(r.imn, c);
    r.imx = max(r.imx, d);
  }
  return r;
}

template <typename K, int THREADS>
__device__ __forceinline__ Range4 block_range(K kmn, K kmx, uint32_t imn, uint32_t imx, uint32_t* red, int t) {
  constexpr int NW = THREADS / kWave;
  static_assert(NW <= 16, "per-wave values fit one row");
  row_reduce<K>(kmn, kmx, imn, imx);
  const Range4 wv = rows_to_scalar<K>(kmn, kmx, imn, imx, 4);
  const int w = t / kWave, lane = t % kWave;
  if (lane == 0) {
    red[6 * w + 0] = (uint32_t)wv.kmn;
    red[6 * w + 1] = (uint32_t)(wv.kmn >> 32);
    red[6 * w + 2] = (uint32_t)wv.kmx;
    red[6 * w + 3] = (uint32_t)(wv.kmx >> 32);
    red[6 * w + 4] = wv.imn;
    red[6 * w + 5] = wv.imx;
  }
  __syncthreads();
  K a = KMax<K>::v, b = K(0);
  uint32_t c = ~0u, d = 0u;
  if (lane < NW) {
    a = (K)(((uint64_t)red[6 * lane + 1] << 32) | red[6 * lane + 0]);
    b = (K)(((uint64_t)red[6 * lane + 3] << 32) | red[6 * lane + 2]);
    c = red[6 * lane + 4];
    d = red[6 * lane + 5];
  }
  row_reduce<K>(a, b, c, d);
  return rows_to_scalar<K>(a, b, c, d, 1);
}

// ---------------------------------------------------------------------------
// Bin of a word: with d = word - lo, ((d >> a) << b) | ((d >> c) & m), a
// non-decreasing function of the word below 2^LB.  One field (m = 0): the top
// LB bits of d.  Two fields, for exact words whose key range has fewer than
// LB bits: the key part, then the top bits of (position - minimum position),
// so that buckets with few distinct keys (long runs of equal keys) still
// spread over the bins.
struct BinMap {
  uint64_t lo;
  uint32_t a, b, c, m;
  __device__ __forceinline__ uint32_t operator()(uint64_t w) const {
    const uint64_t d = w - lo;
    return ((uint32_t)(d >> a) << b) | ((uint32_t)(d >> c) & m);
  }
};

}  // namespace rs
