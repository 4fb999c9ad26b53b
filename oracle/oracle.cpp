/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, obviously correct CPU implementations of what the GPU library
 * computes.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this library; the product path never calls it.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * What the paper fixes (Section 2, Preliminaries; Section 5 and Appendix F,
 * robust fast work-inefficient sorting; Appendix G, robust multi-level sample
 * sort):
 *   - the output is globally sorted;
 *   - keys are made unique by pairing each element with its input position and
 *     comparing pairs lexicographically (the paper simulates this implicitly,
 *     the oracle does it explicitly);
 *   - splitter classification breaks key ties with positions.
 * So for keys x[0..n) the result is the unique permutation pi of 0..n-1 with
 * (ord(x[pi(r)]), pi(r)) strictly increasing in r, where ord is the identity
 * for unsigned keys and the IEEE 754 totalOrder bit map for f32 keys.
 *
 * Functions:
 *   oracle_ord_f32        the totalOrder bit map for f32 keys
 *   oracle_sort           the definition: std::sort of (ord key, position) records
 *   oracle_sort_mt        same result with T threads (chunk sort + pairwise merges);
 *                         used for timing only
 *   oracle_segmented      oracle_sort applied per segment (segment-local positions)
 *   oracle_classify       bucket(e) = number of splitters strictly below e in
 *                         (key, position) order (Appendix G classifier with tie-break)
 *   oracle_median_tree    binary-tree approximate median with given coin flips
 *                         (Section 3.2)
 */
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

enum { KT_U32 = 0, KT_U64 = 1, KT_F32 = 2 };

struct Rec {
  uint64_t key;  // ordinal key
  uint32_t pos;  // input position (segment-local for segmented input)
};

inline bool rec_less(const Rec &a, const Rec &b) {
  return a.key < b.key || (a.key == b.key && a.pos < b.pos);
}

// IEEE 754-2008 totalOrder on binary32 bit patterns: negative values (sign bit
// set) order by decreasing magnitude bits, positive values by increasing bits,
// every negative pattern below every positive one.
inline uint32_t ord_f32(uint32_t u) { return (u & 0x80000000u) ? ~u : (u | 0x80000000u); }

inline uint64_t key_ord(int kt, const void *keys, uint64_t i) {
  if (kt == KT_U64) return ((const uint64_t *)keys)[i];
  uint32_t u = ((const uint32_t *)keys)[i];
  return kt == KT_F32 ? ord_f32(u) : u;
}

inline void key_copy(int kt, const void *src, uint64_t si, void *dst, uint64_t di) {
  if (kt == KT_U64)
    ((uint64_t *)dst)[di] = ((const uint64_t *)src)[si];
  else
    ((uint32_t *)dst)[di] = ((const uint32_t *)src)[si];
}

void build(int kt, const void *keys, uint64_t base, uint64_t n, Rec *r) {
  for (uint64_t i = 0; i < n; i++) {
    r[i].key = key_ord(kt, keys, base + i);
    r[i].pos = (uint32_t)i;
  }
}

void emit(int kt, const void *keys, const uint32_t *payload, uint64_t base, uint64_t n,
          const Rec *r, void *keys_out, uint32_t *perm_out, uint32_t *payload_out) {
  for (uint64_t j = 0; j < n; j++) {
    uint64_t src = base + r[j].pos;
    if (keys_out) key_copy(kt, keys, src, keys_out, base + j);
    if (perm_out) perm_out[base + j] = r[j].pos;
    if (payload_out && payload) payload_out[base + j] = payload[src];
  }
}

bool bad_kt(int kt) { return kt != KT_U32 && kt != KT_U64 && kt != KT_F32; }

}  // namespace

extern "C" {

uint32_t oracle_ord_f32(uint32_t bits) { return ord_f32(bits); }

/* Sort n keys: keys_out[r] = x[pi(r)], perm_out[r] = pi(r), payload_out[r] =
 * payload[pi(r)].  Any output pointer may be NULL.  Returns 0, or -1 on bad
 * arguments (unknown key type, n >= 2^32). */
int oracle_sort(int kt, const void *keys, uint64_t n, const uint32_t *payload, void *keys_out,
                uint32_t *perm_out, uint32_t *payload_out) {
  if (bad_kt(kt) || n >= (1ull << 32)) return -1;
  std::vector<Rec> r(n);
  build(kt, keys, 0, n, r.data());
  std::sort(r.begin(), r.end(), rec_less);
  emit(kt, keys, payload, 0, n, r.data(), keys_out, perm_out, payload_out);
  return 0;
}

/* Same result as oracle_sort using `threads` threads: each thread sorts one
 * chunk, then chunks are merged pairwise in a tree. */
int oracle_sort_mt(int kt, const void *keys, uint64_t n, const uint32_t *payload, void *keys_out,
                   uint32_t *perm_out, uint32_t *payload_out, int threads) {
  if (bad_kt(kt) || n >= (1ull << 32)) return -1;
  if (threads < 1) threads = 1;
  std::vector<Rec> r(n), tmp(n);
  std::vector<uint64_t> cut(threads + 1);
  for (int t = 0; t <= threads; t++) cut[t] = n * (uint64_t)t / (uint64_t)threads;
  {
    std::vector<std::thread> th;
    for (int t = 0; t < threads; t++)
      th.emplace_back([&, t] {
        for (uint64_t i = cut[t]; i < cut[t + 1]; i++) {
          r[i].key = key_ord(kt, keys, i);
          r[i].pos = (uint32_t)i;
        }
        std::sort(r.begin() + cut[t], r.begin() + cut[t + 1], rec_less);
      });
    for (auto &x : th) x.join();
  }
  // pairwise merge rounds
  std::vector<uint64_t> bounds(cut);
  Rec *src = r.data(), *dst = tmp.data();
  while (bounds.size() > 2) {
    std::vector<uint64_t> nb;
    std::vector<std::thread> th;
    size_t runs = bounds.size() - 1;
    for (size_t k = 0; k < runs; k += 2) {
      uint64_t a = bounds[k], m = bounds[k + 1], b = (k + 2 < bounds.size()) ? bounds[k + 2] : m;
      nb.push_back(a);
      th.emplace_back([=] {
        if (b == m)
          std::copy(src + a, src + m, dst + a);
        else
          std::merge(src + a, src + m, src + m, src + b, dst + a, rec_less);
      });
    }
    nb.push_back(n);
    for (auto &x : th) x.join();
    bounds.swap(nb);
    std::swap(src, dst);
  }
  emit(kt, keys, payload, 0, n, src, keys_out, perm_out, payload_out);
  return 0;
}

/* Rank of element i by its definition, in O(n):
 * #{j : ord(x_j) < ord(x_i)} + #{j < i : ord(x_j) = ord(x_i)}.
 * Returns UINT64_MAX on bad arguments. */
uint64_t oracle_rank(int kt, const void *keys, uint64_t n, uint64_t i) {
  if (bad_kt(kt) || i >= n) return ~0ull;
  const uint64_t xi = key_ord(kt, keys, i);
  uint64_t r = 0;
  for (uint64_t j = 0; j < n; j++) {
    const uint64_t xj = key_ord(kt, keys, j);
    r += (xj < xi) || (xj == xi && j < i);
  }
  return r;
}

/* Segmented sort: segment s is [offsets[s], offsets[s+1]); positions are
 * segment-local.  Offsets must be nondecreasing.  Returns 0 or -1. */
int oracle_segmented(int kt, const void *keys, const uint32_t *payload, const uint64_t *offsets,
                     uint64_t num_segs, void *keys_out, uint32_t *perm_out,
                     uint32_t *payload_out) {
  if (bad_kt(kt)) return -1;
  std::vector<Rec> r;
  for (uint64_t s = 0; s < num_segs; s++) {
    uint64_t a = offsets[s], b = offsets[s + 1];
    if (b < a || b - a >= (1ull << 32)) return -1;
    uint64_t n = b - a;
    r.resize(n);
    build(kt, keys, a, n, r.data());
    std::sort(r.begin(), r.end(), rec_less);
    emit(kt, keys, payload, a, n, r.data(), keys_out, perm_out, payload_out);
  }
  return 0;
}

/* Classification with positional tie-break: for element i with key x[i] and
 * position pos[i] (pos == NULL means pos[i] = i), bucket[i] = number of
 * splitters (skey[j], spos[j]) that are strictly smaller than (x[i], pos[i]).
 * Splitters need not be sorted.  Keys and splitter keys share type kt. */
int oracle_classify(int kt, const void *keys, const uint32_t *pos, uint64_t n, const void *skeys,
                    const uint32_t *spos, uint64_t num_spl, uint32_t *bucket_out) {
  if (bad_kt(kt)) return -1;
  for (uint64_t i = 0; i < n; i++) {
    Rec e{key_ord(kt, keys, i), pos ? pos[i] : (uint32_t)i};
    uint32_t c = 0;
    for (uint64_t j = 0; j < num_spl; j++) {
      Rec s{key_ord(kt, skeys, j), spos[j]};
      if (rec_less(s, e)) c++;
    }
    bucket_out[i] = c;
  }
  return 0;
}

/*
 * Binary-tree approximate median (Section 3.2), for p = 2^d leaves holding the
 * consecutive slices of `vals` given by leaf_off[0..p] (any lengths, already
 * in the leaf order the tree is built on).  Values are totally ordered
 * (unique) 64-bit integers; the sentinels below-everything / above-everything
 * are returned as the flags -1 / +1 in *side.
 *   leaf:     sort its slice a[1..m]; forward the window a[h-k/2+1 .. h+k/2]
 *             with h = m/2 for even m and h = floor(m/2) or ceil(m/2) by the
 *             leaf's coin for odd m; positions below 1 are -inf, above m +inf.
 *   internal: merge the two children's windows (2k values) and forward the
 *             middle window the same way (2k is even: no coin).
 *   root:     of the root's own window, return element k/2 or k/2+1 by the
 *             root coin.
 * coins: p leaf coins then 1 root coin (0 = lower, 1 = upper).
 * Returns 0, or -1 on bad arguments.
 */
int oracle_median_tree(const uint64_t *vals, const uint64_t *leaf_off, uint32_t log2_p, uint32_t k,
                       const uint8_t *coins, uint64_t *result, int32_t *side) {
  if (k == 0 || (k & 1) || log2_p > 24) return -1;
  uint64_t p = 1ull << log2_p;
  // value with class: cls 0 = -inf, 1 = real, 2 = +inf
  struct V {
    int cls;
    uint64_t v;
  };
  auto less = [](const V &a, const V &b) { return a.cls < b.cls || (a.cls == b.cls && a.v < b.v); };
  auto window = [&](const std::vector<V> &a, uint64_t h) {
    // 1-based a[h-k/2+1 .. h+k/2]
    std::vector<V> w;
    for (int64_t q = (int64_t)h - (int64_t)(k / 2) + 1; q <= (int64_t)h + (int64_t)(k / 2); q++) {
      if (q < 1)
        w.push_back(V{0, 0});
      else if (q > (int64_t)a.size())
        w.push_back(V{2, 0});
      else
        w.push_back(a[q - 1]);
    }
    return w;
  };
  std::vector<std::vector<V>> level(p);
  for (uint64_t l = 0; l < p; l++) {
    std::vector<V> a;
    for (uint64_t i = leaf_off[l]; i < leaf_off[l + 1]; i++) a.push_back(V{1, vals[i]});
    std::sort(a.begin(), a.end(), less);
    uint64_t m = a.size();
    uint64_t h = (m % 2 == 0) ? m / 2 : (coins[l] ? (m + 1) / 2 : m / 2);
    level[l] = window(a, h);
  }
  while (level.size() > 1) {
    std::vector<std::vector<V>> up(level.size() / 2);
    for (size_t i = 0; i < up.size(); i++) {
      std::vector<V> a;
      std::merge(level[2 * i].begin(), level[2 * i].end(), level[2 * i + 1].begin(),
                 level[2 * i + 1].end(), std::back_inserter(a), less);
      up[i] = window(a, a.size() / 2);
    }
    level.swap(up);
  }
  const V &r = level[0][coins[p] ? k / 2 : k / 2 - 1];
  *result = r.v;
  *side = r.cls - 1;
  return 0;
}

}  // extern "C"
