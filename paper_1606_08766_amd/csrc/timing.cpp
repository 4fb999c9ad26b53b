// Per-kernel event timing of the library's own launches (measurement only).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rsort.h"
#include "internal.hpp"

namespace rs {
namespace {
struct Rec {
  const char* tag;
  hipEvent_t a, b;
};
std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
thread_local hipEvent_t t_pending = nullptr;

hipEvent_t get_event() {
  hipEvent_t e = nullptr;
  if (!g_pool.empty()) {
    e = g_pool.back();
    g_pool.pop_back();
  } else {
    (void)hipEventCreate(&e);
  }
  return e;
}
}  // namespace

bool timing_enabled() { return g_on.load(std::memory_order_relaxed); }

void timing_before(hipStream_t st) {
  std::lock_guard<std::mutex> g(g_mu);
  t_pending = get_event();
  (void)hipEventRecord(t_pending, st);
}

void timing_after(const char* tag, hipStream_t st) {
  std::lock_guard<std::mutex> g(g_mu);
  hipEvent_t e = get_event();
  (void)hipEventRecord(e, st);
  g_recs.push_back(Rec{tag, t_pending, e});
  t_pending = nullptr;
}
}  // namespace rs

extern "C" {

int rsort_timing_begin(void) {
  std::lock_guard<std::mutex> g(rs::g_mu);
  for (auto& r : rs::g_recs) {
    rs::g_pool.push_back(r.a);
    rs::g_pool.push_back(r.b);
  }
  rs::g_recs.clear();
  rs::g_on.store(true);
  return RSORT_OK;
}

int rsort_timing_end(uint32_t max_entries, char* names, uint32_t name_len, uint32_t* launches, double* total_ms,
                     uint32_t* n_entries) {
  rs::g_on.store(false);
  if (hipDeviceSynchronize() != hipSuccess) return RSORT_EDEVICE;
  std::lock_guard<std::mutex> g(rs::g_mu);
  std::map<std::string, std::pair<uint32_t, double>> agg;
  for (auto& r : rs::g_recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return RSORT_EDEVICE;
    auto& x = agg[r.tag];
    x.first++;
    x.second += ms;
  }
  uint32_t i = 0;
  for (auto& kv : agg) {
    if (i >= max_entries) break;
    if (names && name_len) {
      std::strncpy(names + (size_t)i * name_len, kv.first.c_str(), name_len - 1);
      names[(size_t)i * name_len + name_len - 1] = 0;
    }
    if (launches) launches[i] = kv.second.first;
    if (total_ms) total_ms[i] = kv.second.second;
    i++;
  }
  if (n_entries) *n_entries = i;
  return RSORT_OK;
}

}  // extern "C"
