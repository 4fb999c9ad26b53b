// C ABI of librsort (declared in include/rsort.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "../../include/rsort.h"
#include "engine.hpp"
#include "internal.hpp"

namespace {

inline uint64_t key_size(int kt) { return kt == RSORT_U64 ? 8 : 4; }
inline bool valid_kt(int kt) { return kt == RSORT_U32 || kt == RSORT_U64 || kt == RSORT_F32; }

inline bool overlap(const void* a, uint64_t na, const void* b, uint64_t nb) {
  if (!a || !b || !na || !nb) return false;
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

int map_rc(int rc) {
  switch (rc) {
    case 0:
      return RSORT_OK;
    case -1:
      return RSORT_EINVAL;
    case -2:
      return RSORT_ENOMEM;
    default:
      return RSORT_EDEVICE;
  }
}

}  // namespace

extern "C" {

const char* rsort_strerror(int code) {
  switch (code) {
    case RSORT_OK:
      return "ok";
    case RSORT_PENDING:
      return "pending";
    case RSORT_EINVAL:
      return "invalid argument";
    case RSORT_ENOMEM:
      return "not enough memory (workspace or budget)";
    case RSORT_EDEVICE:
      return "device or HIP runtime error";
    case RSORT_EBUSY:
      return "busy";
    case RSORT_ENOTFOUND:
      return "unknown ticket";
    default:
      return "unknown status";
  }
}

int rsort_version(void) { return 100; }

size_t rsort_plain_workspace(rsort_key_t kt, uint64_t n) {
  if (!valid_kt(kt) || n >= 0xFFFFFFFFull) return 0;
  return rs::workspace_bytes((int)kt, n, 1, false);
}

int rsort_plain(rsort_key_t kt, const void* keys_in, uint64_t n, void* keys_out, uint32_t* perm_out, void* workspace,
                size_t workspace_bytes, void* stream) {
  if (!valid_kt(kt) || n >= 0xFFFFFFFFull) return RSORT_EINVAL;
  if (n == 0) return RSORT_OK;
  if (!keys_in || !keys_out || !workspace) return RSORT_EINVAL;
  const uint64_t kb = n * key_size(kt);
  if (overlap(keys_in, kb, keys_out, kb) || overlap(keys_in, kb, perm_out, 4 * n) ||
      overlap(keys_out, kb, perm_out, 4 * n) || overlap(workspace, workspace_bytes, keys_in, kb) ||
      overlap(workspace, workspace_bytes, keys_out, kb) || overlap(workspace, workspace_bytes, perm_out, 4 * n))
    return RSORT_EINVAL;
  return map_rc(rs::enqueue_sort((int)kt, keys_in, nullptr, nullptr, 1, n, keys_out, perm_out, nullptr, workspace,
                                 workspace_bytes, (hipStream_t)stream));
}

size_t rsort_plain64_workspace(rsort_key_t kt, uint64_t n) {
  if (!valid_kt(kt) || n > (1ull << 36)) return 0;
  return rs::wide_workspace_bytes((int)kt, n);
}

int rsort_plain64(rsort_key_t kt, const void* keys_in, uint64_t n, void* keys_out, uint64_t* perm_out,
                  void* workspace, size_t workspace_bytes, void* stream) {
  if (!valid_kt(kt) || n > (1ull << 36)) return RSORT_EINVAL;
  if (n == 0) return RSORT_OK;
  if (!keys_in || !keys_out || !workspace) return RSORT_EINVAL;
  const uint64_t kb = n * key_size(kt);
  if (overlap(keys_in, kb, keys_out, kb) || overlap(keys_in, kb, perm_out, 8 * n) ||
      overlap(keys_out, kb, perm_out, 8 * n) || overlap(workspace, workspace_bytes, keys_in, kb) ||
      overlap(workspace, workspace_bytes, keys_out, kb) || overlap(workspace, workspace_bytes, perm_out, 8 * n))
    return RSORT_EINVAL;
  return map_rc(rs::enqueue_wide((int)kt, keys_in, n, keys_out, perm_out, workspace, workspace_bytes,
                                 (hipStream_t)stream));
}

size_t rsort_rquick_mw_workspace(uint64_t n, uint32_t log2_p) {
  if (!rs::rquick_mw_shape_ok(n, log2_p, 2)) return 0;
  return rs::rquick_mw_workspace(n, log2_p);
}

int rsort_rquick_mw(rsort_key_t kt, const void* keys_in, uint64_t n, uint32_t log2_p, uint32_t k, int tie_break,
                    uint64_t seed, void* keys_out, uint32_t* perm_out, uint32_t* load_out, void* workspace,
                    size_t workspace_bytes, void* stream) {
  if ((kt != RSORT_U32 && kt != RSORT_F32) || !rs::rquick_mw_shape_ok(n, log2_p, k)) return RSORT_EINVAL;
  if (tie_break < 0 || tie_break > 2) return RSORT_EINVAL;
  if (n == 0) return RSORT_OK;
  if (!keys_in || !keys_out || !workspace) return RSORT_EINVAL;
  const uint64_t b = 4 * n, lb = 4ull * (log2_p + 1);
  if (overlap(keys_in, b, keys_out, b) || overlap(keys_in, b, perm_out, b) || overlap(keys_out, b, perm_out, b) ||
      overlap(workspace, workspace_bytes, keys_in, b) || overlap(workspace, workspace_bytes, keys_out, b) ||
      overlap(workspace, workspace_bytes, perm_out, b) || overlap(workspace, workspace_bytes, load_out, lb) ||
      overlap(load_out, lb, keys_out, b) || overlap(load_out, lb, perm_out, b))
    return RSORT_EINVAL;
  return map_rc(rs::enqueue_rquick_mw(kt == RSORT_F32, (const uint32_t*)keys_in, n, log2_p, k, tie_break, seed,
                                      (uint32_t*)keys_out, perm_out, load_out, workspace, workspace_bytes,
                                      (hipStream_t)stream));
}

size_t rsort_segmented_workspace(rsort_key_t kt, uint64_t n_total, uint32_t num_segs, int has_payload) {
  if (!valid_kt(kt) || n_total >= (1ull << 40)) return 0;
  return rs::workspace_bytes((int)kt, n_total, num_segs, has_payload != 0);
}

int rsort_segmented(rsort_key_t kt, const void* keys_in, const uint32_t* payload_in, const uint64_t* seg_offsets,
                    uint32_t num_segs, uint64_t n_total, void* keys_out, uint32_t* payload_out, uint32_t* perm_out,
                    void* workspace, size_t workspace_bytes, void* stream) {
  if (!valid_kt(kt) || n_total >= (1ull << 40)) return RSORT_EINVAL;
  if (num_segs == 0) return n_total == 0 ? RSORT_OK : RSORT_EINVAL;
  if (!seg_offsets || !workspace) return RSORT_EINVAL;
  if (n_total > 0 && (!keys_in || !keys_out)) return RSORT_EINVAL;
  if ((payload_in == nullptr) != (payload_out == nullptr)) return RSORT_EINVAL;
  const uint64_t kb = n_total * key_size(kt), pb = 4 * n_total;
  const void* outs[3] = {keys_out, payload_out, perm_out};
  const uint64_t osz[3] = {kb, pb, pb};
  for (int i = 0; i < 3; i++) {
    if (overlap(keys_in, kb, outs[i], osz[i]) || overlap(payload_in, pb, outs[i], osz[i]) ||
        overlap(workspace, workspace_bytes, outs[i], osz[i]))
      return RSORT_EINVAL;
    for (int j = i + 1; j < 3; j++)
      if (overlap(outs[i], osz[i], outs[j], osz[j])) return RSORT_EINVAL;
  }
  if (overlap(workspace, workspace_bytes, keys_in, kb) || overlap(workspace, workspace_bytes, payload_in, pb))
    return RSORT_EINVAL;
  return map_rc(rs::enqueue_sort((int)kt, keys_in, payload_in, seg_offsets, num_segs, n_total, keys_out, perm_out,
                                 payload_out, workspace, workspace_bytes, (hipStream_t)stream));
}

int rsort_workspace_status(const void* workspace, void* stream) {
  if (!workspace) return RSORT_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return RSORT_EDEVICE;
  int32_t st = 0;
  if (hipMemcpy(&st, workspace, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return RSORT_EDEVICE;
  return st;
}

int rsort_stats(const void* workspace, void* stream, uint64_t* spl_keys, uint32_t* spl_pos, uint32_t* bucket_sizes,
                uint32_t* num_buckets, uint32_t* levels, uint32_t* level_max, uint32_t* level_buckets,
                uint32_t* oversize) {
  if (!workspace) return RSORT_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return RSORT_EDEVICE;
  rs::Ctl c;
  if (hipMemcpy(&c, workspace, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) return RSORT_EDEVICE;
  const uint32_t k = c.levels ? c.l0_k : 0;
  if (num_buckets) *num_buckets = k;
  if (levels) *levels = c.levels;
  if (spl_keys)
    for (uint32_t i = 0; i + 1 < rs::kMaxK; i++) spl_keys[i] = (k && i + 1 < k) ? c.l0_spl_key[i] : 0;
  if (spl_pos)
    for (uint32_t i = 0; i + 1 < rs::kMaxK; i++) spl_pos[i] = (k && i + 1 < k) ? c.l0_spl_pos[i] : 0;
  if (bucket_sizes)
    for (uint32_t i = 0; i < rs::kMaxK; i++) bucket_sizes[i] = (i < k) ? c.l0_bucket[i] : 0;
  if (level_max)
    for (int i = 0; i < rs::kMaxLevels; i++) level_max[i] = c.level_max[i];
  if (level_buckets)
    for (int i = 0; i < rs::kMaxLevels; i++) level_buckets[i] = c.level_buckets[i];
  if (oversize) *oversize = c.class_count[rs::kNumClasses - 1];
  return c.status;
}

int rsort_class_stats(const void* workspace, void* stream, uint32_t max_classes, uint32_t* class_max,
                      uint32_t* buckets, uint64_t* keys) {
  if (!workspace) return RSORT_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return RSORT_EDEVICE;
  rs::Ctl c;
  if (hipMemcpy(&c, workspace, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) return RSORT_EDEVICE;
  const uint32_t m = std::min<uint32_t>(max_classes, rs::kNumClasses);
  for (uint32_t i = 0; i < m; i++) {
    if (class_max) class_max[i] = rs::class_max((int)i);
    if (buckets) buckets[i] = c.class_count[i];
    if (keys) keys[i] = c.class_keys[i];
  }
  return (int)rs::kNumClasses;
}

int rsort_get_tuning(rsort_tuning* out) {
  if (!out) return RSORT_EINVAL;
  const rs::Tuning& t = rs::tuning();
  out->oversample = t.oversample;
  out->target = t.target;
  out->cap = t.cap;
  out->max_levels = t.max_levels;
  out->rfis_max = t.rfis_max;
  out->rquick_max = t.rquick_max;
  out->seed = t.seed;
  out->tile_log2 = t.tile_log2;
  out->force_fallback = t.force_fallback;
  out->extra_levels = t.extra_levels + 1;
  out->class_shape = t.class_shape | 0x80000000u;
  return RSORT_OK;
}

int rsort_set_tuning(const rsort_tuning* in) {
  if (!in) return RSORT_EINVAL;
  rs::Tuning t = rs::tuning();
  if (in->oversample) {
    if (in->oversample > rs::kMaxOversample) return RSORT_EINVAL;
    t.oversample = in->oversample;
  }
  if (in->target) t.target = in->target;
  if (in->cap) {
    if (in->cap < 64) return RSORT_EINVAL;
    t.cap = in->cap;
  }
  if (in->max_levels) {
    if (in->max_levels > (uint32_t)rs::kMaxLevels) return RSORT_EINVAL;
    t.max_levels = in->max_levels;
  }
  if (in->rfis_max) t.rfis_max = in->rfis_max;
  if (in->rquick_max) t.rquick_max = in->rquick_max;
  if (in->seed) t.seed = in->seed;
  if (in->tile_log2) {
    if (in->tile_log2 != 12 && in->tile_log2 != 13) return RSORT_EINVAL;
    t.tile_log2 = in->tile_log2;
  }
  if (in->force_fallback) t.force_fallback = in->force_fallback == 1 ? 1u : 0u;
  if (in->extra_levels) {
    if (in->extra_levels > 5) return RSORT_EINVAL;
    t.extra_levels = in->extra_levels - 1;
  }
  if (in->class_shape) {
    if (!(in->class_shape & 0x80000000u)) return RSORT_EINVAL;
    t.class_shape = in->class_shape & 0x1FFu;
  }
  rs::tuning() = t;
  return RSORT_OK;
}

}  // extern "C"
