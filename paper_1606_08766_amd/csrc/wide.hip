// Sorting more than 2^32 - 1 keys: positions (the tie-break of the paper's
// robust sample sort, Appendix G, and the output permutation) are 64-bit.
//
// One top level splits the input into kWideK buckets by (key, 64-bit
// position) splitters.  Its scatter is stable: inside a bucket the elements
// keep their input order, so a bucket's local positions order its equal keys
// exactly as the global positions do, and every bucket (far below 2^32 keys)
// is then sorted by the multilevel sample sort with 32-bit local positions,
// all buckets in one segmented call.  The global position of each element
// travels beside it through the top level, and the final permutation gathers
// it: perm[r] = gpos[bucket start + local perm[r]].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "engine.hpp"
#include "internal.hpp"

namespace rs {

constexpr int kWideLogK = 8, kWideK = 1 << kWideLogK;
constexpr int kWideThreads = 1024;
constexpr uint32_t kWideTile = 1u << 16;      // elements per tile of the top level's count and scatter
constexpr int kWideSampleItems = 8;
constexpr int kWideSamples = kWideThreads * kWideSampleItems;  // 32 samples per bucket
constexpr int kWideScanThreads = 256, kWideScanItems = 16, kWideScanChunk = kWideScanThreads * kWideScanItems;

struct WideWork {
  void* seg_ws;       // workspace of the segmented sort of the buckets (first: its status word is the call's)
  size_t seg_ws_bytes;
  void* keys_buf;     // [n] keys (input bits), bucket by bucket, input order inside a bucket
  uint64_t* gpos;     // [n] input position of each element of keys_buf
  uint32_t* perm_loc; // [n] bucket-local permutation from the segmented sort
  uint32_t* counts;   // [kWideK][ntiles] elements of bucket b in tile t
  uint64_t* offs;     // same shape: exclusive prefix sum in bucket-major order
  uint64_t* partials; // scan partials
  uint64_t* seg_off;  // [kWideK + 1] bucket boundaries
  void* tkey;         // [kWideK] splitter tree: ordinal keys at nodes 1 .. kWideK - 1
  uint64_t* tpos;     // [kWideK] and their 64-bit input positions
  uint64_t n, ntiles;
};

template <typename K>
__device__ __forceinline__ bool pair_less64(K ka, uint64_t pa, K kb, uint64_t pb) {
  return ka < kb || (ka == kb && pa < pb);
}

// Splitters: kWideSamples (key, position) samples drawn with replacement at
// counter-RNG positions, ranked in LDS by counting (equal samples ordered by
// sample number, so every rank occurs once); the sample of rank j * a - 1
// becomes splitter j, stored at its node of the implicit search tree.
template <typename K, bool F32>
__global__ __launch_bounds__(kWideThreads) void k_wide_splitters(WideWork w, const K* in, uint64_t seed) {
  __shared__ K sk[kWideSamples];
  __shared__ uint64_t sp[kWideSamples];
  K k[kWideSampleItems];
  uint64_t p[kWideSampleItems];
#pragma unroll
  for (int i = 0; i < kWideSampleItems; i++) {
    const uint32_t j = threadIdx.x * kWideSampleItems + i;
    const uint64_t r = rand_at(seed, 0x57A7E5ull, j);
    p[i] = __umul64hi(r, w.n);  // uniform in [0, n)
    k[i] = in[p[i]];
  }
#pragma unroll
  for (int i = 0; i < kWideSampleItems; i++) {
    const uint32_t j = threadIdx.x * kWideSampleItems + i;
    k[i] = ord_of<K, F32>(k[i]);
    sk[j] = k[i];
    sp[j] = p[i];
  }
  __syncthreads();
  uint32_t rank[kWideSampleItems];
#pragma unroll
  for (int i = 0; i < kWideSampleItems; i++) rank[i] = 0;
  for (uint32_t q = 0; q < (uint32_t)kWideSamples; q++) {
    const K kq = sk[q];
    const uint64_t pq = sp[q];
#pragma unroll
    for (int i = 0; i < kWideSampleItems; i++) {
      const uint32_t j = threadIdx.x * kWideSampleItems + i;
      rank[i] += (pair_less64(kq, pq, k[i], p[i]) || (kq == k[i] && pq == p[i] && q < j)) ? 1u : 0u;
    }
  }
  constexpr uint32_t a = kWideSamples / kWideK;
  K* tk = (K*)w.tkey;
#pragma unroll
  for (int i = 0; i < kWideSampleItems; i++) {
    if ((rank[i] + 1) % a == 0) {
      const uint32_t j = (rank[i] + 1) / a;
      if (j < (uint32_t)kWideK) {
        const uint32_t node = (j | kWideK) >> (__builtin_ctz(j) + 1);
        tk[node] = k[i];
        w.tpos[node] = p[i];
      }
    }
  }
}

// Bucket of (key, position): the number of splitters strictly below it.
template <typename K>
__device__ __forceinline__ uint32_t wide_bucket(const K* tk, const uint64_t* tp, K key, uint64_t pos) {
  uint32_t j = 1;
#pragma unroll
  for (int l = 0; l < kWideLogK; l++) {
    const K t = tk[j];
    j = 2u * j + ((key > t) || (key == t && pos > tp[j]) ? 1u : 0u);
  }
  return j - kWideK;
}

template <typename K>
__device__ __forceinline__ void wide_load_tree(const WideWork& w, K* tk, uint64_t* tp) {
  const K* g = (const K*)w.tkey;
  for (uint32_t i = threadIdx.x + 1; i < (uint32_t)kWideK; i += blockDim.x) {
    tk[i] = g[i];
    tp[i] = w.tpos[i];
  }
}

// Count: elements per (bucket, tile).
template <typename K, bool F32>
__global__ __launch_bounds__(kWideThreads) void k_wide_count(WideWork w, const K* in) {
  __shared__ K tk[kWideK];
  __shared__ uint64_t tp[kWideK];
  __shared__ uint32_t hist[kWideK];
  wide_load_tree<K>(w, tk, tp);
  for (uint64_t t = blockIdx.x; t < w.ntiles; t += gridDim.x) {
    for (uint32_t b = threadIdx.x; b < (uint32_t)kWideK; b += kWideThreads) hist[b] = 0;
    __syncthreads();
    const uint64_t base = t * kWideTile;
    const uint32_t cnt = (uint32_t)min((uint64_t)kWideTile, w.n - base);
    for (uint32_t e = threadIdx.x; e < cnt; e += kWideThreads) {
      const K key = ord_of<K, F32>(in[base + e]);
      atomicAdd(&hist[wide_bucket<K>(tk, tp, key, base + e)], 1u);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < (uint32_t)kWideK; b += kWideThreads) w.counts[(uint64_t)b * w.ntiles + t] = hist[b];
  }
}

// Exclusive scan of the kWideK * ntiles counts into 64-bit offsets
// (reduce, scan of the partials, down-sweep), plus the bucket boundaries.
__global__ __launch_bounds__(kWideScanThreads) void k_wide_scan_reduce(WideWork w) {
  __shared__ uint64_t tmp[kWideScanThreads / kWave + 1];
  const uint64_t M = kWideK * w.ntiles;
  const uint64_t nb = (M + kWideScanChunk - 1) / kWideScanChunk;
  for (uint64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
    uint64_t s = 0;
    for (int i = 0; i < kWideScanItems; i++) {
      const uint64_t j = blk * kWideScanChunk + (uint64_t)i * kWideScanThreads + threadIdx.x;
      if (j < M) s += w.counts[j];
    }
    uint64_t tot;
    block_excl_scan<kWideScanThreads, uint64_t>(s, tmp, &tot);
    if (threadIdx.x == 0) w.partials[blk] = tot;
  }
}

__global__ __launch_bounds__(1024) void k_wide_scan_partials(WideWork w) {
  __shared__ uint64_t tmp[1024 / kWave + 1];
  const uint64_t M = kWideK * w.ntiles;
  const uint64_t nb = (M + kWideScanChunk - 1) / kWideScanChunk;
  uint64_t carry = 0;
  for (uint64_t base = 0; base < nb; base += 1024) {
    const uint64_t i = base + threadIdx.x;
    const uint64_t v = i < nb ? w.partials[i] : 0ull;
    uint64_t tot;
    const uint64_t e = block_excl_scan<1024, uint64_t>(v, tmp, &tot);
    if (i < nb) w.partials[i] = carry + e;
    carry += tot;
  }
}

__global__ __launch_bounds__(kWideScanThreads) void k_wide_scan_down(WideWork w) {
  __shared__ uint64_t tmp[kWideScanThreads / kWave + 1];
  const uint64_t M = kWideK * w.ntiles;
  const uint64_t nb = (M + kWideScanChunk - 1) / kWideScanChunk;
  for (uint64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
    const uint64_t base = blk * kWideScanChunk + (uint64_t)threadIdx.x * kWideScanItems;
    uint32_t v[kWideScanItems];
    uint64_t s = 0;
    for (int i = 0; i < kWideScanItems; i++) {
      v[i] = base + i < M ? w.counts[base + i] : 0u;
      s += v[i];
    }
    uint64_t e = block_excl_scan<kWideScanThreads, uint64_t>(s, tmp, nullptr) + w.partials[blk];
    for (int i = 0; i < kWideScanItems; i++) {
      const uint64_t j = base + i;
      if (j < M) {
        w.offs[j] = e;
        if (j % w.ntiles == 0) w.seg_off[j / w.ntiles] = e;  // first tile of bucket j / ntiles
      }
      e += v[i];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) w.seg_off[kWideK] = w.n;
}

// Stable scatter: a tile is processed in rounds of one element per thread
// in input order; inside a wave, the elements of one bucket are ranked by
// lane (lanes with equal buckets found with one ballot per bucket bit),
// across the waves of a round by wave, across rounds by round, so every
// bucket receives its elements in input order.
template <typename K, bool F32>
__global__ __launch_bounds__(kWideThreads) void k_wide_scatter(WideWork w, const K* in) {
  constexpr int NW = kWideThreads / kWave;
  __shared__ K tk[kWideK];
  __shared__ uint64_t tp[kWideK];
  __shared__ uint64_t run[kWideK];
  __shared__ uint64_t cw[NW][kWideK];
  wide_load_tree<K>(w, tk, tp);
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  K* out = (K*)w.keys_buf;
  for (uint64_t t = blockIdx.x; t < w.ntiles; t += gridDim.x) {
    for (uint32_t b = threadIdx.x; b < (uint32_t)kWideK; b += kWideThreads) run[b] = w.offs[(uint64_t)b * w.ntiles + t];
    const uint64_t base = t * kWideTile;
    const uint32_t cnt = (uint32_t)min((uint64_t)kWideTile, w.n - base);
    for (uint32_t r0 = 0; r0 < cnt; r0 += kWideThreads) {
      for (uint32_t i = threadIdx.x; i < (uint32_t)(NW * kWideK); i += kWideThreads) (&cw[0][0])[i] = 0ull;
      __syncthreads();
      const uint32_t e = r0 + threadIdx.x;
      const bool act = e < cnt;
      const uint64_t pos = base + e;
      K raw = K(0);
      uint32_t b = 0;
      if (act) {
        raw = in[pos];
        b = wide_bucket<K>(tk, tp, ord_of<K, F32>(raw), pos);
      }
      uint64_t peers = __ballot(act);
#pragma unroll
      for (int bit = 0; bit < kWideLogK; bit++) {
        const uint64_t m = __ballot(act && ((b >> bit) & 1u));
        peers &= ((b >> bit) & 1u) ? m : ~m;
      }
      const uint32_t below = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
      if (act && below == 0) cw[wv][b] = (uint64_t)__popcll(peers);
      __syncthreads();
      for (uint32_t bb = threadIdx.x; bb < (uint32_t)kWideK; bb += kWideThreads) {
        uint64_t s = run[bb];
        for (int q = 0; q < NW; q++) {
          const uint64_t c = cw[q][bb];
          cw[q][bb] = s;
          s += c;
        }
        run[bb] = s;
      }
      __syncthreads();
      if (act) {
        const uint64_t d = cw[wv][b] + below;
        out[d] = raw;
        w.gpos[d] = pos;
      }
      __syncthreads();
    }
  }
}

// perm[r] = gpos[start of r's bucket + bucket-local perm[r]].
__global__ __launch_bounds__(256) void k_wide_perm(WideWork w, uint64_t* perm_out) {
  __shared__ uint64_t so[kWideK + 1];
  for (uint32_t i = threadIdx.x; i <= (uint32_t)kWideK; i += 256) so[i] = w.seg_off[i];
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x; r < w.n; r += stride) {
    uint32_t lo = 0, hi = kWideK - 1;  // last bucket with so[b] <= r
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (so[mid] <= r)
        lo = mid;
      else
        hi = mid - 1;
    }
    perm_out[r] = w.gpos[so[lo] + w.perm_loc[r]];
  }
}

static inline uint64_t wide_align(uint64_t x) { return (x + 255) / 256 * 256; }

// Workspace layout of the wide path (bytes; fills w when base != nullptr).
size_t wide_layout(int kt, uint64_t n, char* base, WideWork* w) {
  const uint64_t ks = kt == 1 ? 8 : 4;
  const uint64_t ntiles = (n + kWideTile - 1) / kWideTile;
  const uint64_t M = (uint64_t)kWideK * ntiles;
  const uint64_t nb = (M + kWideScanChunk - 1) / kWideScanChunk + 1;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off = wide_align(off + bytes);
    return o;
  };
  const uint64_t seg_bytes = workspace_bytes(kt, n, kWideK, false);
  const uint64_t o_seg = take(seg_bytes);
  const uint64_t o_keys = take(n * ks);
  const uint64_t o_gpos = take(n * 8);
  const uint64_t o_perm = take(n * 4);
  const uint64_t o_cnt = take(M * 4);
  const uint64_t o_offs = take(M * 8);
  const uint64_t o_par = take(nb * 8);
  const uint64_t o_so = take((kWideK + 1) * 8);
  const uint64_t o_tk = take(kWideK * 8);
  const uint64_t o_tp = take(kWideK * 8);
  if (base && w) {
    w->seg_ws = base + o_seg;
    w->seg_ws_bytes = seg_bytes;
    w->keys_buf = base + o_keys;
    w->gpos = (uint64_t*)(base + o_gpos);
    w->perm_loc = (uint32_t*)(base + o_perm);
    w->counts = (uint32_t*)(base + o_cnt);
    w->offs = (uint64_t*)(base + o_offs);
    w->partials = (uint64_t*)(base + o_par);
    w->seg_off = (uint64_t*)(base + o_so);
    w->tkey = base + o_tk;
    w->tpos = (uint64_t*)(base + o_tp);
    w->n = n;
    w->ntiles = ntiles;
  }
  return off;
}

size_t wide_workspace_bytes(int kt, uint64_t n) { return wide_layout(kt, n, nullptr, nullptr); }

template <typename K, bool F32>
static int enqueue_wide_typed(int kt, const void* keys_in, uint64_t n, void* keys_out, uint64_t* perm_out, void* ws,
                              size_t ws_bytes, hipStream_t st) {
  WideWork w;
  if (ws_bytes < wide_layout(kt, n, (char*)ws, &w)) return -2;
  const K* in = (const K*)keys_in;
  const uint32_t cus = num_cu_cached();
  const uint32_t gt = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(w.ntiles, (uint64_t)cus * 2));
  const uint64_t M = (uint64_t)kWideK * w.ntiles;
  const uint32_t gs = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>((M + kWideScanChunk - 1) / kWideScanChunk, (uint64_t)cus * 8));
  RS_LAUNCH((k_wide_splitters<K, F32>), 1, kWideThreads, st, w, in, tuning().seed);
  RS_LAUNCH((k_wide_count<K, F32>), gt, kWideThreads, st, w, in);
  RS_LAUNCH(k_wide_scan_reduce, gs, kWideScanThreads, st, w);
  RS_LAUNCH(k_wide_scan_partials, 1, 1024, st, w);
  RS_LAUNCH(k_wide_scan_down, gs, kWideScanThreads, st, w);
  RS_LAUNCH((k_wide_scatter<K, F32>), gt, kWideThreads, st, w, in);
  const int rc = enqueue_sort(kt, w.keys_buf, nullptr, w.seg_off, kWideK, n, keys_out,
                              perm_out ? w.perm_loc : nullptr, nullptr, w.seg_ws, w.seg_ws_bytes, st);
  if (rc) return rc;
  if (perm_out) {
    const uint32_t gp = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, (uint64_t)cus * 8));
    RS_LAUNCH(k_wide_perm, gp, 256, st, w, perm_out);
  }
  return 0;
}

int enqueue_wide(int kt, const void* keys_in, uint64_t n, void* keys_out, uint64_t* perm_out, void* ws,
                 size_t ws_bytes, hipStream_t st) {
  switch (kt) {
    case 0:
      return enqueue_wide_typed<uint32_t, false>(kt, keys_in, n, keys_out, perm_out, ws, ws_bytes, st);
    case 1:
      return enqueue_wide_typed<uint64_t, false>(kt, keys_in, n, keys_out, perm_out, ws, ws_bytes, st);
    case 2:
      return enqueue_wide_typed<uint32_t, true>(kt, keys_in, n, keys_out, perm_out, ws, ws_bytes, st);
    default:
      return -1;
  }
}

}  // namespace rs
