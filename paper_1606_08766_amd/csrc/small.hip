// Small-array sorts of the size-class dispatch: RFIS and RQuick.
//
// RFIS (paper Section 5 and Appendix F, built on fast work-inefficient
// ranking, Appendix E.1): every element is ranked against every other
// element and delivered to out[rank].  On the GPU the sqrt(p) x sqrt(p) PE
// grid collapses into one workgroup: the row/column all-gather-merges become
// "the whole array sits in LDS", the local ranking of column elements in row
// elements is each thread counting, over LDS tiles, the elements smaller than
// its own, and the column all-reduce of partial ranks is the accumulation in
// registers.  The compare table of Appendix F is lexicographic order on
// (key, row, column, position); with the explicit input position it is the
// (key, position) compare below, which makes every rank unique in 0..n-1.
//
// RQuick (paper Section 6, Algorithm 2): robust hypercube quicksort with the
// PEs mapped to the wavefronts of one workgroup and the hypercube exchange to
// LDS.  Steps per array: random redistribution of the input over the waves
// (Section 3.1), local sort of every wave's part, then for cube dimensions
// j = d-1 .. 0: approximate median of each (j+1)-dimensional subcube by the
// single-reduction binary tree (Section 3.2), split of every wave's sorted
// run at that pivot, exchange of the halves with wave i xor 2^j and merge.
// Pivots are (key, position) pairs, so equal keys split by position and
// every split is unique.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "engine.hpp"
#include "internal.hpp"

namespace rs {

// ---------------------------------------------------------------------------
// RFIS
// ---------------------------------------------------------------------------
template <typename K>
struct RankKey;
// u32 keys: (key, position) packed into one u64, compared in one instruction.
template <>
struct RankKey<uint32_t> {
  using T = uint64_t;
  static __device__ __forceinline__ T make(uint32_t k, uint32_t i) { return ((uint64_t)k << 32) | i; }
  static __device__ __forceinline__ bool less(const T& a, const T& b) { return a < b; }
};
struct Pair64 {
  uint64_t k;
  uint32_t i;
  uint32_t pad;
};
template <>
struct RankKey<uint64_t> {
  using T = Pair64;
  static __device__ __forceinline__ T make(uint64_t k, uint32_t i) { return Pair64{k, i, 0u}; }
  static __device__ __forceinline__ bool less(const T& a, const T& b) { return pair_less(a.k, a.i, b.k, b.i); }
};

template <typename K, bool F32, bool PAY, int THREADS, int NMAX>
__global__ __launch_bounds__(THREADS) void k_rfis(Work w, int cls, const K* in_keys, const uint32_t* in_pay,
                                                  K* keys_out, uint32_t* perm_out, uint32_t* pay_out) {
  using RK = RankKey<K>;
  using T = typename RK::T;
  constexpr int PER = (NMAX + THREADS - 1) / THREADS;
  __shared__ T sx[NMAX];
  __shared__ uint16_t dest[NMAX];  // dest[rank] = local index of that element
  direct_reset(w, cls);
  const uint32_t cnt = final_count(w, cls);
  for (uint32_t q = blockIdx.x; q < cnt; q += gridDim.x) {
    const FinalSeg f = final_at(w, cls, q);
    const BufView<K> sb{f.src ? w.buf_rec[f.src - 1] : nullptr};
    const uint32_t* srcp = f.src ? w.buf_pay[f.src - 1] : in_pay;
    T mine[PER];
#pragma unroll
    for (int r = 0; r < PER; r++) {
      const uint32_t j = r * THREADS + threadIdx.x;
      if (j < f.len) {
        const K key = f.src ? sb.key(f.start + j) : load_ord<K, F32>(in_keys, f.start + j);
        const uint32_t idx = f.src ? sb.idx(f.start + j) : j;
        mine[r] = RK::make(key, idx);
        sx[j] = mine[r];
      }
    }
    __syncthreads();
    // rank of each own element = number of strictly smaller elements
    uint32_t rank[PER];
#pragma unroll
    for (int r = 0; r < PER; r++) rank[r] = 0;
    uint32_t i = 0;
    for (; i + 4 <= f.len; i += 4) {
      const T x0 = sx[i], x1 = sx[i + 1], x2 = sx[i + 2], x3 = sx[i + 3];
#pragma unroll
      for (int r = 0; r < PER; r++) {
        rank[r] += RK::less(x0, mine[r]) ? 1u : 0u;
        rank[r] += RK::less(x1, mine[r]) ? 1u : 0u;
        rank[r] += RK::less(x2, mine[r]) ? 1u : 0u;
        rank[r] += RK::less(x3, mine[r]) ? 1u : 0u;
      }
    }
    for (; i < f.len; i++) {
      const T x0 = sx[i];
#pragma unroll
      for (int r = 0; r < PER; r++) rank[r] += RK::less(x0, mine[r]) ? 1u : 0u;
    }
#pragma unroll
    for (int r = 0; r < PER; r++) {
      const uint32_t j = r * THREADS + threadIdx.x;
      if (j < f.len) dest[rank[r]] = (uint16_t)j;
    }
    __syncthreads();
    // data delivery: element of rank r goes to output position r
    for (uint32_t r = threadIdx.x; r < f.len; r += THREADS) {
      const uint32_t j = dest[r];
      const T x = sx[j];
      K key;
      uint32_t idx;
      if constexpr (sizeof(K) == 4) {
        key = (K)(x >> 32);
        idx = (uint32_t)x;
      } else {
        key = x.k;
        idx = x.i;
      }
      uint32_t pv = 0;  // loaded before the stores (a load issued after stores waits for them)
      if constexpr (PAY) pv = srcp[f.start + j];
      keys_out[f.start + r] = to_output<K, F32>(key);
      if (perm_out) perm_out[f.start + r] = idx;
      if constexpr (PAY) pay_out[f.start + r] = pv;
    }
    __syncthreads();
  }
}

template <typename K, bool F32, bool PAY>
int launch_rfis_class(int c, const Work& w, const K* kin, const uint32_t* pay_in, K* kout, uint32_t* perm_out,
                      uint32_t* pay_out, uint64_t cap_c, hipStream_t st) {
  const uint64_t slots = (uint64_t)num_cu_cached() * 16;
  const bool dir = (c & kDirect) != 0;
  const int ca = dir ? -1 : (c & 0xFF);
  const uint32_t g1 = dir ? 1u : (uint32_t)std::min<uint64_t>(std::max<uint64_t>(cap_c, 1), slots);
  const uint32_t g2 = dir ? 1u : (uint32_t)std::min<uint64_t>(std::max<uint64_t>(cap_c, 1), slots / 2);
  switch (c & 0xFF) {
    case 0:
      RS_LAUNCH((k_rfis<K, F32, PAY, 64, 64>), g1, 64, st, w, ca, kin, pay_in, kout, perm_out, pay_out);
      break;
    case 1:
      RS_LAUNCH((k_rfis<K, F32, PAY, 64, 256>), g1, 64, st, w, ca, kin, pay_in, kout, perm_out, pay_out);
      break;
    case 2:
      RS_LAUNCH((k_rfis<K, F32, PAY, 256, 1024>), g2, 256, st, w, ca, kin, pay_in, kout, perm_out, pay_out);
      break;
    default:
      return launch_merge_class<K, F32, PAY>(c, w, kin, pay_in, kout, perm_out, pay_out, cap_c, st);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// RQuick
// ---------------------------------------------------------------------------
// Window entries of the median tree carry a class: 0 = below everything,
// 1 = real element, 2 = above everything (the paper's treatment of window
// positions outside a leaf's data).
template <typename K>
struct WinE {
  K key;
  uint32_t idx;
  uint32_t cls;
};
template <typename K>
__device__ __forceinline__ bool win_less(const WinE<K>& a, const WinE<K>& b) {
  if (a.cls != b.cls) return a.cls < b.cls;
  return a.cls == 1 && pair_less(a.key, a.idx, b.key, b.idx);
}

// Merge two sorted LDS sequences (a: na, b: nb) into out[0 .. na+nb) using the
// 64 lanes of one wave; lane l produces a contiguous chunk of outputs.
template <typename K, bool CARRY>
__device__ __forceinline__ void wave_merge(const K* ak, const uint32_t* av, const uint32_t* ap, uint32_t na,
                                           const K* bk, const uint32_t* bv, const uint32_t* bp, uint32_t nb, K* ok,
                                           uint32_t* ov, uint32_t* op) {
  const uint32_t m = na + nb;
  const uint32_t lane = lane_id();
  const uint32_t chunk = (m + kWave - 1) / kWave;
  uint32_t d = lane * chunk;
  if (d >= m) return;
  const uint32_t e = min(m, d + chunk);
  uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    const uint32_t bj = d - 1 - mid;
    if (pair_less(bk[bj], bv[bj], ak[mid], av[mid]))
      hi = mid;
    else
      lo = mid + 1;
  }
  uint32_t ai = lo, bi = d - lo;
  for (; d < e; d++) {
    const bool takeA = ai < na && (bi >= nb || !pair_less(bk[bi], bv[bi], ak[ai], av[ai]));
    if (takeA) {
      ok[d] = ak[ai];
      ov[d] = av[ai];
      if constexpr (CARRY) op[d] = ap[ai];
      ai++;
    } else {
      ok[d] = bk[bi];
      ov[d] = bv[bi];
      if constexpr (CARRY) op[d] = bp[bi];
      bi++;
    }
  }
}

template <typename K, bool F32, bool PAY, int THREADS, int NMAX, int WK>
__global__ __launch_bounds__(THREADS) void k_rquick(Work w, int cls, const K* in_keys, const uint32_t* in_pay,
                                                    K* keys_out, uint32_t* perm_out, uint32_t* pay_out,
                                                    uint64_t seed) {
  constexpr int P = THREADS / kWave;  // PEs of the hypercube
  constexpr int D = P == 2 ? 1 : P == 4 ? 2 : P == 8 ? 3 : P == 16 ? 4 : 0;
  static_assert(D > 0, "2..16 waves");
  constexpr int ITEMS = NMAX / THREADS;  // per-lane capacity of a wave's first part
  static_assert(ITEMS * THREADS == NMAX && (ITEMS & (ITEMS - 1)) == 0, "NMAX = THREADS * 2^i");
  static_assert(2 * WK <= kWave && (WK & 1) == 0, "window");
  __shared__ K bk[2][NMAX];
  __shared__ uint32_t bv[2][NMAX];
  __shared__ uint32_t bp[PAY ? 2 : 1][PAY ? NMAX : 1];
  __shared__ WinE<K> win[2][P][WK];
  __shared__ WinE<K> pivot[P];
  __shared__ uint32_t off[P], len[P], xs[P], noff[P], nlen[P];

  const uint32_t wv = threadIdx.x / kWave, lane = lane_id();
  direct_reset(w, cls);
  const uint32_t cnt = final_count(w, cls);
  for (uint32_t q = blockIdx.x; q < cnt; q += gridDim.x) {
    const FinalSeg f = final_at(w, cls, q);
    const BufView<K> sb{f.src ? w.buf_rec[f.src - 1] : nullptr};
    const uint32_t* srcp = f.src ? w.buf_pay[f.src - 1] : in_pay;
    const uint32_t n = f.len;
    const uint64_t rstream = f.start * 0x9E3779B97F4A7C15ull + 0x52515549434Bull;
    // stage the input in buffer 1 (coalesced)
    for (uint32_t j = threadIdx.x; j < n; j += THREADS) {
      bk[1][j] = f.src ? sb.key(f.start + j) : load_ord<K, F32>(in_keys, f.start + j);
      bv[1][j] = f.src ? sb.idx(f.start + j) : j;
    }
    if (threadIdx.x < P) {
      off[threadIdx.x] = (uint32_t)((uint64_t)threadIdx.x * n / P);
      len[threadIdx.x] = (uint32_t)((uint64_t)(threadIdx.x + 1) * n / P) - off[threadIdx.x];
    }
    __syncthreads();
    // random redistribution: slot s of the array takes element (s*M + c) mod n
    // (M prime > n, so this is a bijection); wave w owns slots [off_w, off_w + len_w)
    const uint64_t rr = rand_at(seed, rstream, 0);
    constexpr uint32_t kPrimes[4] = {4099u, 4111u, 4127u, 4129u};
    const uint32_t M = kPrimes[rr & 3];
    const uint32_t cshift = (uint32_t)((rr >> 8) % (n ? n : 1));
    K k[ITEMS];
    uint32_t v[ITEMS], p[ITEMS];
    const uint32_t o_w = off[wv], l_w = len[wv];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t r = lane * ITEMS + i;
      if (r < l_w) {
        const uint32_t src = (uint32_t)(((uint64_t)(o_w + r) * M + cshift) % n);
        k[i] = bk[1][src];
        v[i] = bv[1][src];
        p[i] = src;
      } else {
        k[i] = KMax<K>::v;
        v[i] = kPadIdx;
        p[i] = 0;
      }
    }
    __syncthreads();
    // local sort of every wave's part (runs never cross a wave)
    block_merge_sort<K, THREADS, ITEMS, PAY, kWave>(k, v, p, bk[1], bv[1], PAY ? bp[PAY ? 1 : 0] : nullptr);
    int cur = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t r = lane * ITEMS + i;
      if (r < l_w) {
        bk[0][o_w + r] = k[i];
        bv[0][o_w + r] = v[i];
        if constexpr (PAY) bp[0][o_w + r] = p[i];
      }
    }
    __syncthreads();
    for (int j = D - 1; j >= 0; j--) {
      // (a) leaf windows around each run's median
      {
        const uint32_t m = len[wv];
        uint32_t h = m / 2;
        if (m & 1) h += (uint32_t)(rand_at(seed, rstream, 16 + j * 64 + wv) & 1);
        if (lane < (uint32_t)WK) {
          const int qq = (int)h - WK / 2 + (int)lane;
          WinE<K> e;
          if (qq < 0) {
            e = WinE<K>{K(0), 0u, 0u};
          } else if ((uint32_t)qq >= m) {
            e = WinE<K>{K(0), 0u, 2u};
          } else {
            e = WinE<K>{bk[cur][off[wv] + qq], bv[cur][off[wv] + qq], 1u};
          }
          win[0][wv][lane] = e;
        }
      }
      __syncthreads();
      // (b) reduction up the binary tree of each (j+1)-subcube
      int wsel = 0;
      for (int lv = 0; lv <= j; lv++) {
        const uint32_t stride = 1u << lv;
        if ((wv & (2 * stride - 1)) == 0 && lane < 2u * WK) {
          const WinE<K>* A = win[wsel][wv];
          const WinE<K>* B = win[wsel][wv + stride];
          WinE<K> e;
          uint32_t pos;
          if (lane < (uint32_t)WK) {
            e = A[lane];
            uint32_t c = 0;
            for (int t = 0; t < WK; t++) c += win_less(B[t], e) ? 1u : 0u;
            pos = lane + c;
          } else {
            e = B[lane - WK];
            uint32_t c = 0;
            for (int t = 0; t < WK; t++) c += win_less(e, A[t]) ? 0u : 1u;  // A[t] <= e
            pos = (lane - WK) + c;
          }
          if (pos >= (uint32_t)(WK / 2) && pos < (uint32_t)(3 * WK / 2)) win[wsel ^ 1][wv][pos - WK / 2] = e;
        }
        wsel ^= 1;
        __syncthreads();
      }
      // (c) pivot of each subcube: root window element k/2 or k/2+1 by a coin
      if (lane == 0 && (wv & ((2u << j) - 1)) == 0) {
        const uint32_t coin = (uint32_t)(rand_at(seed, rstream, 4096 + j * 64 + wv) & 1);
        pivot[wv >> (j + 1)] = win[wsel][wv][WK / 2 - 1 + coin];
      }
      __syncthreads();
      // (d) split every run: x = number of elements <= pivot
      if (lane == 0) {
        const WinE<K> pv = pivot[wv >> (j + 1)];
        const uint32_t m = len[wv], o = off[wv];
        uint32_t x;
        if (pv.cls == 0)
          x = 0;
        else if (pv.cls == 2)
          x = m;
        else {
          uint32_t lo = 0, hi = m;
          while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pair_less(pv.key, pv.idx, bk[cur][o + mid], bv[cur][o + mid]))
              hi = mid;
            else
              lo = mid + 1;
          }
          x = lo;
        }
        xs[wv] = x;
      }
      __syncthreads();
      // (e) new run sizes and offsets inside each (j+1)-subcube
      if (threadIdx.x < P) {
        const uint32_t me = threadIdx.x, partner = me ^ (1u << j);
        const bool lower = (me & (1u << j)) == 0;
        const uint32_t g0 = me & ~((2u << j) - 1);
        uint32_t o = off[g0];
        // new order inside the subcube: the lower half's waves (bit j clear)
        // in wave order, then the upper half's
        for (uint32_t u = g0; u < g0 + (2u << j); u++) {
          const bool ulow = (u & (1u << j)) == 0;
          const bool before = lower ? (ulow && u < me) : (ulow || u < me);
          if (!before) continue;
          const uint32_t up = u ^ (1u << j);
          o += ulow ? xs[u] + xs[up] : (len[u] - xs[u]) + (len[up] - xs[up]);
        }
        noff[me] = o;
        nlen[me] = lower ? xs[me] + xs[partner] : (len[me] - xs[me]) + (len[partner] - xs[partner]);
      }
      __syncthreads();
      // (f) exchange with the partner wave and merge
      {
        const uint32_t me = wv, partner = wv ^ (1u << j);
        const bool lower = (me & (1u << j)) == 0;
        uint32_t a0, na, b0, nb;
        if (lower) {
          a0 = off[me];
          na = xs[me];
          b0 = off[partner];
          nb = xs[partner];
        } else {
          a0 = off[me] + xs[me];
          na = len[me] - xs[me];
          b0 = off[partner] + xs[partner];
          nb = len[partner] - xs[partner];
        }
        const uint32_t o = noff[me];
        wave_merge<K, PAY>(bk[cur] + a0, bv[cur] + a0, PAY ? bp[PAY ? cur : 0] + a0 : nullptr, na, bk[cur] + b0,
                           bv[cur] + b0, PAY ? bp[PAY ? cur : 0] + b0 : nullptr, nb, bk[cur ^ 1] + o, bv[cur ^ 1] + o,
                           PAY ? bp[PAY ? (cur ^ 1) : 0] + o : nullptr);
      }
      __syncthreads();
      if (threadIdx.x < P) {
        off[threadIdx.x] = noff[threadIdx.x];
        len[threadIdx.x] = nlen[threadIdx.x];
      }
      cur ^= 1;
      __syncthreads();
    }
    // runs are now in wave order and globally sorted
    for (uint32_t r = threadIdx.x; r < n; r += THREADS) {
      uint32_t pv = 0;  // loaded before the stores (a load issued after stores waits for them)
      if constexpr (PAY) pv = srcp[f.start + bp[cur][r]];
      keys_out[f.start + r] = to_output<K, F32>(bk[cur][r]);
      if (perm_out) perm_out[f.start + r] = bv[cur][r];
      if constexpr (PAY) pay_out[f.start + r] = pv;
    }
    __syncthreads();
  }
}

template <typename K, bool F32, bool PAY>
int launch_rquick_class(int c, const Work& w, const K* kin, const uint32_t* pay_in, K* kout, uint32_t* perm_out,
                        uint32_t* pay_out, uint64_t cap_c, hipStream_t st) {
  const uint64_t slots = (uint64_t)num_cu_cached() * 2;
  const uint64_t seed = tuning().seed;
  const bool dir = (c & kDirect) != 0;
  const int ca = dir ? -1 : (c & 0xFF);
  const uint32_t g = dir ? 1u : (uint32_t)std::min<uint64_t>(std::max<uint64_t>(cap_c, 1), slots);
  switch (c & 0xFF) {
    case 3:
      RS_LAUNCH((k_rquick<K, F32, PAY, 512, 2048, 16>), g, 512, st, w, ca, kin, pay_in, kout, perm_out, pay_out, seed);
      break;
    case 4:
    case 5:
      RS_LAUNCH((k_rquick<K, F32, PAY, 1024, 4096, 16>), g, 1024, st, w, ca, kin, pay_in, kout, perm_out, pay_out,
                seed);
      break;
    default:
      return launch_merge_class<K, F32, PAY>(c, w, kin, pay_in, kout, perm_out, pay_out, cap_c, st);
  }
  return 0;
}

#define RS_INST_SMALL(K, F, P)                                                                                  \
  template int launch_rfis_class<K, F, P>(int, const Work&, const K*, const uint32_t*, K*, uint32_t*, uint32_t*,  \
                                          uint64_t, hipStream_t);                                               \
  template int launch_rquick_class<K, F, P>(int, const Work&, const K*, const uint32_t*, K*, uint32_t*, uint32_t*, \
                                            uint64_t, hipStream_t);
RS_INST_SMALL(uint32_t, false, false)
RS_INST_SMALL(uint32_t, true, false)
RS_INST_SMALL(uint64_t, false, false)
RS_INST_SMALL(uint32_t, false, true)
RS_INST_SMALL(uint32_t, true, true)
RS_INST_SMALL(uint64_t, false, true)

}  // namespace rs
