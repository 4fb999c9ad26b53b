// Robust hypercube quicksort with workgroups as PEs (paper Section 6,
// Algorithm 2), for arrays too large for one workgroup's LDS.
//
// p = 2^d PEs; PE i owns the packed range [off[i], off[i+1]) of a word array
// in HBM.  A word is (ord(key) << 32) | input position, so words are unique
// and their order is the sort order.  Exchanges between PEs go through HBM:
// every step writes a fresh word array and offset vector (ping-pong).
//
//   1. random redistribution (Section 3.1 / Appendix C): d rounds; in round j
//      every PE splits its part into two random halves, keeps one and sends
//      the other to PE i xor 2^j;
//   2. each PE sorts its part in LDS;
//   3. for j = d-1 .. 0: the binary-tree median (Section 3.2) of every
//      (j+1)-dimensional subcube is its splitter; every PE splits its sorted
//      part into L (words <= splitter) and R; the PE with bit j clear keeps
//      both L parts of itself and its partner, the other both R parts, and
//      merges them.
//
// After the last round the parts, in PE order, are the sorted array.  Three
// ways to split a part at the splitter:
//   * by (key, position) words: L = words <= the splitter word;
//   * without tie-breaking (ablation): L = words whose key is <= the
//     splitter's key.  Equal keys never leave a common side, so the output
//     is the same; only the load balance differs;
//   * the paper's local scheme (Section 6): a part a = a_l s^m a_r, s the
//     splitter's key, keeps L = a_l s^x with x chosen so that |L| is as
//     close to |a| / 2 as possible.  Equal keys may then end on either side,
//     so the keys come out sorted but equal keys in no fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace rs {

namespace {

constexpr uint32_t kMwCap = 8192;       // largest part a PE sorts in LDS
constexpr uint32_t kMwMaxLog2P = 8;     // at most 256 PEs
constexpr uint32_t kMwMaxK = 16;        // median window
constexpr int kMwThreads = 256;
static_assert((1u << kMwMaxLog2P) <= (uint32_t)kMwThreads, "a round's planning takes one thread per PE");

// stream ids of the counter-based generator
constexpr uint64_t kStShuffle = 0x5348554600000000ull, kStLeaf = 0x4C45414600000000ull,
                   kStRoot = 0x524F4F5400000000ull;

struct MwPivot {
  uint64_t v;
  uint32_t cls;  // 0: below every word, 1: the word v, 2: above every word
  uint32_t pad;
};

template <bool F32>
__global__ __launch_bounds__(kMwThreads) void k_mw_in(const uint32_t* keys, uint32_t n, uint32_t P, uint64_t* D,
                                                      uint32_t* off, int32_t* status) {
  const uint32_t stride = gridDim.x * blockDim.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride)
    D[r] = ((uint64_t)load_ord<uint32_t, F32>(keys, r) << 32) | r;
  if (blockIdx.x == 0)
    for (uint32_t i = threadIdx.x; i <= P; i += blockDim.x) off[i] = (uint32_t)((uint64_t)i * n / P);
}

enum MwMode : int { kMwShuffle = 0, kMwWords = 1, kMwKeyOnly = 2, kMwLocal = 3 };

// Number of words of the sorted run x[0, m) that are <= lim.
__device__ __forceinline__ uint32_t count_not_above(const uint64_t* x, uint32_t m, uint64_t lim) {
  uint32_t lo = 0, hi = m;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (x[mid] <= lim)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Number of words of the sorted run x[0, m) that go to the lower side.
__device__ __forceinline__ uint32_t split_point(const uint64_t* x, uint32_t m, const MwPivot& pv, int mode) {
  if (pv.cls == 0) return 0;
  if (pv.cls == 2) return m;
  const uint64_t key_hi = pv.v | 0xFFFFFFFFull;
  if (mode == kMwWords) return count_not_above(x, m, pv.v);
  if (mode == kMwKeyOnly) return count_not_above(x, m, key_hi);
  // local scheme: x copies of the splitter key, |a_l s^x| closest to m / 2
  const uint32_t below = (pv.v >> 32) == 0 ? 0u : count_not_above(x, m, (pv.v & ~0xFFFFFFFFull) - 1);
  const uint32_t upto = count_not_above(x, m, key_hi);
  const uint32_t half = m / 2;
  return half < below ? below : (half > upto ? upto : half);
}

// Part sizes of one exchange round over dimension j, computed by every
// workgroup of the round's kernel for all P PEs: s_lo[i] = the size of PE i's
// lower piece (a shuffle keeps floor(m/2); a split round reads the split
// points the splitter kernel stored), s_m[i] = its part size, s_off = the
// exclusive scan of the new part sizes (s_off[P] = n), s_max = the largest.
__device__ void plan_round(const uint32_t* off, uint32_t P, uint32_t j, const uint32_t* split, uint32_t* s_lo,
                           uint32_t* s_m, uint32_t* s_off, uint32_t* tmp, uint32_t* s_max) {
  const bool shuffle = split == nullptr;
  const uint32_t i = threadIdx.x;
  if (i == 0) *s_max = 0;
  uint32_t m = 0, lo = 0;
  if (i < P) {
    m = off[i + 1] - off[i];
    lo = shuffle ? m / 2 : split[i];
  }
  s_lo[i] = lo;
  s_m[i] = m;
  __syncthreads();
  uint32_t nm = 0;
  if (i < P) {
    const uint32_t q = i ^ (1u << j);
    if (shuffle)
      nm = lo + (s_m[q] - s_lo[q]);
    else if (((i >> j) & 1u) == 0)
      nm = lo + s_lo[q];
    else
      nm = (m - lo) + (s_m[q] - s_lo[q]);
    atomicMax(s_max, nm);
  }
  uint32_t total = 0;
  const uint32_t e = block_excl_scan<kMwThreads>(nm, tmp, &total);
  if (i < P) s_off[i] = e;
  if (i == 0) s_off[P] = total;
  __syncthreads();
}

// The first workgroup of a round publishes the new offsets (read by the next
// kernel) and the largest part.
__device__ __forceinline__ void publish_round(const uint32_t* s_off, uint32_t s_max, uint32_t P, uint32_t* off_next,
                                              uint32_t* load_out) {
  if (blockIdx.x != 0 || blockIdx.y != 0) return;
  for (uint32_t t = threadIdx.x; t <= P; t += blockDim.x) off_next[t] = s_off[t];
  if (threadIdx.x == 0 && load_out) *load_out = s_max;
}

// Shuffle round j: PE i permutes its part by t -> (t*M + c) mod m (M a prime
// above the part size, c random), keeps the first half and sends the second
// behind its partner's kept half.  Grid: (P, chunks of the part).
__global__ __launch_bounds__(kMwThreads) void k_mw_shuffle(const uint64_t* D, const uint32_t* off,
                                                           uint32_t* off_next, uint64_t* Dn, uint32_t n, uint32_t P,
                                                           uint32_t j, uint64_t seed, uint32_t* load_out) {
  __shared__ uint32_t s_lo[kMwThreads], s_m[kMwThreads], s_off[kMwThreads + 1];
  __shared__ uint32_t tmp[kMwThreads / kWave + 1];
  __shared__ uint32_t s_max;
  plan_round(off, P, j, nullptr, s_lo, s_m, s_off, tmp, &s_max);
  publish_round(s_off, s_max, P, off_next, load_out);
  const uint32_t i = blockIdx.x, q = i ^ (1u << j);
  const uint32_t a = off[i], m = s_m[i];
  if (m == 0) return;
  const uint32_t h = s_lo[i];
  const uint64_t r = rand_at(seed, kStShuffle + j, i);
  constexpr uint32_t kPrimes[4] = {8209u, 8219u, 8221u, 8231u};  // all above kMwCap
  const uint64_t M = kPrimes[r & 3];
  const uint64_t c = (r >> 8) % m;
  const uint32_t own = s_off[i], other = s_off[q] + s_lo[q];
  for (uint32_t t = blockIdx.y * blockDim.x + threadIdx.x; t < m; t += gridDim.y * blockDim.x) {
    const uint32_t pi = (uint32_t)(((uint64_t)t * M + c) % m);
    const uint32_t dst = pi < h ? own + pi : other + (pi - h);
    if (dst < n) Dn[dst] = D[a + t];  // always true: the new parts tile [0, n)
  }
}

// Each PE sorts its part (at most kMwCap words) in LDS: bitonic network over
// the part padded to a power of two with all-ones words.
__global__ __launch_bounds__(1024) void k_mw_sort(uint64_t* D, const uint32_t* off, int32_t* status) {
  __shared__ uint64_t s[kMwCap];
  const uint32_t i = blockIdx.x;
  const uint32_t a = off[i], m = off[i + 1] - a;
  if (m > kMwCap) {
    if (threadIdx.x == 0) atomicCAS(status, 0, -1);
    return;
  }
  if (m <= 1) return;
  uint32_t np = 1;
  while (np < m) np <<= 1;
  for (uint32_t t = threadIdx.x; t < np; t += blockDim.x) s[t] = t < m ? D[a + t] : ~0ull;
  __syncthreads();
  for (uint32_t kk = 2; kk <= np; kk <<= 1) {
    for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
      for (uint32_t t = threadIdx.x; t < np; t += blockDim.x) {
        const uint32_t u = t ^ jj;
        if (u > t) {
          const uint64_t x = s[t], y = s[u];
          const bool up = (t & kk) == 0;
          if ((x > y) == up) {
            s[t] = y;
            s[u] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t t = threadIdx.x; t < m; t += blockDim.x) D[a + t] = s[t];
}

struct MwWin {
  uint64_t v;
  uint32_t cls;
};

__device__ __forceinline__ bool mwin_less(const MwWin& x, const MwWin& y) {
  if (x.cls != y.cls) return x.cls < y.cls;
  return x.cls == 1 && x.v < y.v;
}

// Splitter of every (j+1)-dimensional subcube (one workgroup each): the
// binary-tree median of its S = 2^(j+1) sorted parts with window k.  A leaf
// forwards the k words around its middle (rank floor(m/2), or the upper
// middle by a coin when m is odd), entries outside the part being the
// below-all / above-all sentinels; a node merges its children's windows and
// forwards the middle k; the root returns entry k/2 or k/2 + 1 (1-based) of
// its window by a coin.  The workgroup then stores every PE's split point
// (the size of its lower piece) for the round's merge.
__global__ __launch_bounds__(kMwThreads) void k_mw_pivot(const uint64_t* D, const uint32_t* off, uint32_t j,
                                                         uint32_t k, uint64_t seed, int mode, uint32_t* split) {
  __shared__ MwPivot s_piv;
  __shared__ uint64_t wv[2][(1u << kMwMaxLog2P) * kMwMaxK];
  __shared__ uint32_t wc[2][(1u << kMwMaxLog2P) * kMwMaxK];
  const uint32_t q = blockIdx.x, S = 2u << j, first = q * S;
  for (uint32_t g = threadIdx.x; g < S * k; g += blockDim.x) {
    const uint32_t l = g / k, e = g % k;
    const uint32_t a = off[first + l], m = off[first + l + 1] - a;
    uint32_t h = m / 2;
    if (m & 1u) h += (uint32_t)(rand_at(seed, kStLeaf + j, first + l) & 1u);
    const int r = (int)h - (int)(k / 2) + (int)e;
    wc[0][g] = r < 0 ? 0u : (r >= (int)m ? 2u : 1u);
    wv[0][g] = (r >= 0 && r < (int)m) ? D[a + r] : 0ull;
  }
  __syncthreads();
  int cur = 0;
  for (uint32_t nodes = S / 2; nodes >= 1; nodes /= 2) {
    for (uint32_t g = threadIdx.x; g < nodes * 2 * k; g += blockDim.x) {
      const uint32_t node = g / (2 * k), e = g % (2 * k);
      const uint32_t A = 2 * node * k, B = A + k;
      MwWin x;
      uint32_t pos;
      // windows are sorted: binary searches for the rank in the other one
      const bool fromA = e < k;
      const uint32_t own = fromA ? A + e : B + e - k, other = fromA ? B : A;
      x = MwWin{wv[cur][own], wc[cur][own]};
      uint32_t lo = 0, hi = k;
      while (lo < hi) {  // A entry: count of B below x; B entry: count of A not above x (ties: A first)
        const uint32_t mid = (lo + hi) >> 1;
        const MwWin y{wv[cur][other + mid], wc[cur][other + mid]};
        if (fromA ? mwin_less(y, x) : !mwin_less(x, y))
          lo = mid + 1;
        else
          hi = mid;
      }
      pos = (fromA ? e : e - k) + lo;
      if (pos >= k / 2 && pos < k / 2 + k) {
        wv[cur ^ 1][node * k + pos - k / 2] = x.v;
        wc[cur ^ 1][node * k + pos - k / 2] = x.cls;
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  if (threadIdx.x == 0) {
    const uint32_t c = (uint32_t)(rand_at(seed, kStRoot + j, q) & 1u);
    const uint32_t e = k / 2 - 1 + c;
    s_piv = MwPivot{wc[cur][e] == 1 ? wv[cur][e] : 0ull, wc[cur][e], 0};
  }
  __syncthreads();
  // every PE of the subcube splits its sorted part at the splitter
  for (uint32_t l = threadIdx.x; l < S; l += blockDim.x) {
    const uint32_t a = off[first + l], m = off[first + l + 1] - a;
    split[first + l] = split_point(D + a, m, s_piv, mode);
  }
}

// Exchange and merge of round j: PE i gathers its own and its partner's
// lower (bit j clear) or upper pieces; each word's place in the merged part
// is its index in its piece plus the number of words of the other piece
// below it.
__device__ __forceinline__ uint32_t count_below(const uint64_t* x, uint32_t m, uint64_t v) {
  uint32_t lo = 0, hi = m;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (x[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kMwThreads) void k_mw_split_merge(const uint64_t* D, const uint32_t* off,
                                                               const uint32_t* split, uint32_t* off_next,
                                                               uint64_t* Dn, uint32_t n, uint32_t P, uint32_t j,
                                                               uint32_t* load_out) {
  __shared__ uint32_t s_lo[kMwThreads], s_m[kMwThreads], s_off[kMwThreads + 1];
  __shared__ uint32_t tmp[kMwThreads / kWave + 1];
  __shared__ uint32_t s_max;
  plan_round(off, P, j, split, s_lo, s_m, s_off, tmp, &s_max);
  publish_round(s_off, s_max, P, off_next, load_out);
  const uint32_t i = blockIdx.x, q = i ^ (1u << j);
  const bool upper = ((i >> j) & 1u) != 0;
  const uint32_t mi = s_m[i], si = s_lo[i], mq = s_m[q], sq = s_lo[q];
  const uint64_t* A = D + off[i] + (upper ? si : 0u);
  const uint64_t* B = D + off[q] + (upper ? sq : 0u);
  const uint32_t na = upper ? mi - si : si, nb = upper ? mq - sq : sq;
  const uint32_t base = s_off[i];
  for (uint32_t t = blockIdx.y * blockDim.x + threadIdx.x; t < na + nb; t += gridDim.y * blockDim.x) {
    const uint64_t v = t < na ? A[t] : B[t - na];
    const uint32_t dst = base + (t < na ? t + count_below(B, nb, v) : (t - na) + count_below(A, na, v));
    if (dst < n) Dn[dst] = v;  // always true: the new parts tile [0, n)
  }
}

__global__ __launch_bounds__(kMwThreads) void k_mw_out(const uint64_t* D, const uint32_t* keys, uint32_t n,
                                                       uint32_t* keys_out, uint32_t* perm_out) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const uint32_t idx = (uint32_t)D[r];
    keys_out[r] = idx < n ? keys[idx] : 0u;  // idx < n: D holds the n input words
    if (perm_out) perm_out[r] = idx;
  }
}

struct MwLayout {
  int32_t* status;
  uint64_t* D[2];
  uint32_t* off[2];
  uint32_t* split;
  size_t bytes;
};

MwLayout mw_layout(char* base, uint64_t n, uint32_t P) {
  MwLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += (b + 255) / 256 * 256;
    return base ? base + at : nullptr;
  };
  L.status = (int32_t*)take(256);
  L.D[0] = (uint64_t*)take(n * 8);
  L.D[1] = (uint64_t*)take(n * 8);
  L.off[0] = (uint32_t*)take((P + 1) * 4);
  L.off[1] = (uint32_t*)take((P + 1) * 4);
  L.split = (uint32_t*)take(P * 4);
  L.bytes = o;
  return L;
}

}  // namespace

bool rquick_mw_shape_ok(uint64_t n, uint32_t log2_p, uint32_t k) {
  if (log2_p < 1 || log2_p > kMwMaxLog2P) return false;
  if (k < 2 || k > kMwMaxK || (k & 1u)) return false;
  if (n >= 0xFFFFFFFFull) return false;
  const uint64_t P = 1ull << log2_p;
  return (n + P - 1) / P <= kMwCap;
}

size_t rquick_mw_workspace(uint64_t n, uint32_t log2_p) { return mw_layout(nullptr, n, 1u << log2_p).bytes; }

int enqueue_rquick_mw(bool f32, const uint32_t* keys_in, uint64_t n64, uint32_t log2_p, uint32_t k, int tie_break,
                      uint64_t seed, uint32_t* keys_out, uint32_t* perm_out, uint32_t* load_out, void* ws,
                      size_t ws_bytes, hipStream_t st) {
  const uint32_t P = 1u << log2_p, d = log2_p, n = (uint32_t)n64;
  MwLayout L = mw_layout((char*)ws, n64, P);
  if (ws_bytes < L.bytes) return -2;
  const uint32_t grid = std::max<uint32_t>(1u, std::min<uint32_t>((n + kMwThreads - 1) / kMwThreads,
                                                                  num_cu_cached() * 8u));
  if (f32)
    RS_LAUNCH(k_mw_in<true>, grid, kMwThreads, st, keys_in, n, P, L.D[0], L.off[0], L.status);
  else
    RS_LAUNCH(k_mw_in<false>, grid, kMwThreads, st, keys_in, n, P, L.D[0], L.off[0], L.status);
  const MwMode split_mode = tie_break == 1 ? kMwWords : tie_break == 2 ? kMwLocal : kMwKeyOnly;
  // workgroups per PE in the data-moving kernels: about 2048 keys each
  const uint32_t chunks = (uint32_t)std::max<uint64_t>(1, (2 * ((n64 + P - 1) / P) + 2047) / 2048);
  int cur = 0;
  for (uint32_t j = 0; j < d; j++) {  // random redistribution
    RS_LAUNCH(k_mw_shuffle, dim3(P, chunks), kMwThreads, st, L.D[cur], L.off[cur], L.off[cur ^ 1], L.D[cur ^ 1], n, P,
              j, seed, (load_out && j + 1 == d) ? load_out : nullptr);
    cur ^= 1;
  }
  RS_LAUNCH(k_mw_sort, P, 1024, st, L.D[cur], L.off[cur], L.status);
  for (uint32_t r = 0; r < d; r++) {  // cube dimensions, highest first
    const uint32_t j = d - 1 - r;
    RS_LAUNCH(k_mw_pivot, P >> (j + 1), kMwThreads, st, L.D[cur], L.off[cur], j, k, seed, (int)split_mode, L.split);
    RS_LAUNCH(k_mw_split_merge, dim3(P, chunks), kMwThreads, st, L.D[cur], L.off[cur], L.split, L.off[cur ^ 1],
              L.D[cur ^ 1], n, P, j, load_out ? load_out + 1 + r : nullptr);
    cur ^= 1;
  }
  RS_LAUNCH(k_mw_out, grid, kMwThreads, st, L.D[cur], keys_in, n, keys_out, perm_out);
  return 0;
}

}  // namespace rs
