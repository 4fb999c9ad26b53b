/*
 * Seeded synthetic input generators shared by the oracle side and the GPU side.
 *
 * This file holds no sorting arithmetic: it only produces input bytes.  Both
 * the CPU oracle and the GPU library consume exactly the bytes written here,
 * so parity never depends on the generator.
 *
 * Random stream: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) in counter mode.  The i-th output of the
 * generator seeded with s is mix(s + (i + 1) * 0x9E3779B97F4A7C15), which is
 * exactly the i-th value of the published sequential generator.
 *
 * Distributions follow the one-line instance definitions of the paper's
 * experimental section (Uniform, Gaussian, DeterDupl, Zero, Reverse), with the
 * concrete formulas chosen for this library's workloads:
 *   UNIFORM    x_i = r_i                          (u32: low 32 bits of r_i)
 *   GAUSSIAN   x_i = 2^63 + llround(z_i * 2^40)   (u32: 2^31 + llround(z_i * 2^24),
 *                                                   f32: (float) z_i)
 *              z from Box-Muller over pairs (r_{2j}, r_{2j+1})
 *   ZERO       x_i = 0
 *   DETERDUPL  x_i = i mod param (param 0 means 16)
 *   REVERSE    x_i = n - 1 - i
 *   SORTED     x_i = i
 *   TOPBITS    x_i = r_i >> (64 - param)          (param 3 gives 8 distinct values)
 *   WIDEDUP    x_i = splitmix64(seed', r_i mod param) (param 0 means 300): few
 *              distinct values spread over the whole key range, seed' = seed
 *              xor 0xD1B54A32D192ED03
 * f32 keys: UNIFORM is a random 32-bit pattern (NaNs, infinities and signed
 * zeros occur); the others are the float value of the integer formula.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

enum { KT_U32 = 0, KT_U64 = 1, KT_F32 = 2 };
enum {
  D_UNIFORM = 0,
  D_GAUSSIAN = 1,
  D_ZERO = 2,
  D_DETERDUPL = 3,
  D_REVERSE = 4,
  D_SORTED = 5,
  D_TOPBITS = 6,
  D_WIDEDUP = 7,
};

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t gen_splitmix64(uint64_t seed, uint64_t i) { return mix64(seed + (i + 1) * GOLDEN); }

/* Standard normal value number i of the stream (Box-Muller on a pair). */
static inline double gauss_at(uint64_t seed, uint64_t i) {
  uint64_t j = i >> 1;
  double u1 = ((double)((gen_splitmix64(seed, 2 * j) >> 11) + 1)) * 0x1.0p-53; /* (0, 1] */
  double u2 = ((double)(gen_splitmix64(seed, 2 * j + 1) >> 11)) * 0x1.0p-53;   /* [0, 1) */
  double r = sqrt(-2.0 * log(u1));
  double a = 6.283185307179586476925286766559 * u2;
  return (i & 1) ? r * sin(a) : r * cos(a);
}

/*
 * Fill out[0..n) with keys of type kt.  The value at position i uses random
 * stream index (stream_off + i) and position-dependent formulas use i itself
 * (and n).  Returns 0 on success, -1 on bad arguments.
 */
int gen_keys(int kt, int dist, uint64_t param, uint64_t seed, uint64_t n, uint64_t stream_off,
             void *out) {
  if (kt < 0 || kt > 2 || (n && !out)) return -1;
  uint64_t dd = param ? param : 16;
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < (int64_t)n; i++) {
    uint64_t s = stream_off + (uint64_t)i;
    uint64_t v64 = 0;
    uint32_t v32 = 0;
    float vf = 0.0f;
    switch (dist) {
      case D_UNIFORM: {
        uint64_t r = gen_splitmix64(seed, s);
        v64 = r;
        v32 = (uint32_t)r;
        memcpy(&vf, &v32, 4);
        break;
      }
      case D_GAUSSIAN: {
        double z = gauss_at(seed, s);
        v64 = (uint64_t)llround(z * 0x1.0p40) + 0x8000000000000000ULL;
        v32 = (uint32_t)((uint64_t)llround(z * 0x1.0p24) + 0x80000000ULL);
        vf = (float)z;
        break;
      }
      case D_ZERO:
        break;
      case D_DETERDUPL:
        v64 = (uint64_t)i % dd;
        v32 = (uint32_t)v64;
        vf = (float)v64;
        break;
      case D_REVERSE:
        v64 = n - 1 - (uint64_t)i;
        v32 = (uint32_t)v64;
        vf = (float)v64;
        break;
      case D_SORTED:
        v64 = (uint64_t)i;
        v32 = (uint32_t)v64;
        vf = (float)v64;
        break;
      case D_TOPBITS: {
        uint64_t b = param ? param : 3;
        v64 = gen_splitmix64(seed, s) >> (64 - b);
        v32 = (uint32_t)v64;
        vf = (float)v64;
        break;
      }
      case D_WIDEDUP: {
        uint64_t m = param ? param : 300;
        v64 = gen_splitmix64(seed ^ 0xD1B54A32D192ED03ULL, gen_splitmix64(seed, s) % m);
        v32 = (uint32_t)v64;
        memcpy(&vf, &v32, 4);
        break;
      }
      default:
        break;
    }
    if (kt == KT_U64)
      ((uint64_t *)out)[i] = v64;
    else if (kt == KT_U32)
      ((uint32_t *)out)[i] = v32;
    else
      ((float *)out)[i] = vf;
  }
  if (dist < D_UNIFORM || dist > D_WIDEDUP) return -1;
  return 0;
}

/* Random u32 payload values: high 32 bits of the stream. */
int gen_payload(uint64_t seed, uint64_t n, uint64_t stream_off, uint32_t *out) {
  if (n && !out) return -1;
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < (int64_t)n; i++) out[i] = (uint32_t)(gen_splitmix64(seed, stream_off + (uint64_t)i) >> 32);
  return 0;
}

/*
 * Log-uniform sizes: size_s = floor(exp(U_s * ln(2^hi_log2) + (1 - U_s) * ln(2^lo_log2)))
 * clamped to [2^lo_log2, 2^hi_log2], with U_s uniform in [0, 1) from the stream.
 */
int gen_log_uniform_sizes(uint64_t seed, uint64_t count, double lo_log2, double hi_log2,
                          uint64_t *out) {
  if (count && !out) return -1;
  double lo = lo_log2 * 0.69314718055994530942, hi = hi_log2 * 0.69314718055994530942;
  double mn = floor(exp(lo) + 0.5), mx = floor(exp(hi) + 0.5);
  for (uint64_t s = 0; s < count; s++) {
    double u = (double)(gen_splitmix64(seed, s) >> 11) * 0x1.0p-53;
    double v = floor(exp(lo + u * (hi - lo)));
    if (v < mn) v = mn;
    if (v > mx) v = mx;
    out[s] = (uint64_t)v;
  }
  return 0;
}

/*
 * Segmented batch: segment s has keys generated with dist_of[s] from the
 * per-segment seed splitmix64(seed, s), and payload from that seed + 1.
 * offsets has count+1 entries.  Keys of type kt; payload may be NULL.
 */
int gen_segmented(int kt, uint64_t seed, uint64_t count, const uint64_t *offsets,
                  const int32_t *dist_of, uint64_t param, void *keys, uint32_t *payload) {
  if (kt < 0 || kt > 2) return -1;
  int64_t s;
  size_t w = (kt == KT_U64) ? 8 : 4;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
  for (s = 0; s < (int64_t)count; s++) {
    uint64_t a = offsets[s], b = offsets[s + 1];
    uint64_t sseed = gen_splitmix64(seed, (uint64_t)s);
    int r = 0;
    /* nested calls run serially inside the parallel region */
    uint64_t n = b - a;
    char *kp = (char *)keys + a * w;
    for (uint64_t i = 0; i < n; i++) {
      uint64_t v64 = 0;
      uint32_t v32 = 0;
      float vf = 0.0f;
      switch (dist_of[s]) {
        case D_UNIFORM: {
          uint64_t x = gen_splitmix64(sseed, i);
          v64 = x;
          v32 = (uint32_t)x;
          memcpy(&vf, &v32, 4);
          break;
        }
        case D_GAUSSIAN: {
          double z = gauss_at(sseed, i);
          v64 = (uint64_t)llround(z * 0x1.0p40) + 0x8000000000000000ULL;
          v32 = (uint32_t)((uint64_t)llround(z * 0x1.0p24) + 0x80000000ULL);
          vf = (float)z;
          break;
        }
        case D_ZERO:
          break;
        case D_DETERDUPL:
          v64 = i % (param ? param : 16);
          v32 = (uint32_t)v64;
          vf = (float)v64;
          break;
        case D_REVERSE:
          v64 = n - 1 - i;
          v32 = (uint32_t)v64;
          vf = (float)v64;
          break;
        case D_SORTED:
          v64 = i;
          v32 = (uint32_t)v64;
          vf = (float)v64;
          break;
        default:
          r = 1;
      }
      if (kt == KT_U64)
        ((uint64_t *)kp)[i] = v64;
      else if (kt == KT_U32)
        ((uint32_t *)kp)[i] = v32;
      else
        ((float *)kp)[i] = vf;
    }
    if (payload)
      for (uint64_t i = 0; i < n; i++)
        payload[a + i] = (uint32_t)(gen_splitmix64(sseed + 1, i) >> 32);
    bad |= r;
  }
  return bad ? -1 : 0;
}
