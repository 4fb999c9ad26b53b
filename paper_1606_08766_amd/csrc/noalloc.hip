// Plain sort into a scratch area that the library owns statically, for
// callers that cannot allocate device memory (code under stream capture,
// serving loops, hosts that forbid allocation during operation).
//
// The scratch is a file-scope device array of kScratchBytes; every GPU the
// library runs on holds its own copy until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// symbol): the first call on a device looks up that device's address of the
// array with hipGetSymbolAddress and keeps it, and every launch receives that
// address.  The sort's kernels reset every counter and status word they use
// at the start of a call, so the contents a previous call left behind do not
// matter; two calls that overlap on one device share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/rsort.h"
#include "engine.hpp"
#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = 64ull << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (nullptr on failure).
void* scratch_for_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" int rsort_plain_noalloc(rsort_key_t kt, const void* keys_in, uint64_t n, void* keys_out,
                                   uint32_t* perm_out, void* stream) {
  if (kt != RSORT_U32 && kt != RSORT_U64 && kt != RSORT_F32) return RSORT_EINVAL;
  if (n >= 0xFFFFFFFFull) return RSORT_EINVAL;
  if (n == 0) return RSORT_OK;
  // checked before any device call: sizes beyond the static scratch are refused
  const size_t need = rs::workspace_bytes((int)kt, n, 1, false);
  if (need > kScratchBytes) return RSORT_ENOMEM;
  if (!keys_in || !keys_out) return RSORT_EINVAL;
  const uint64_t kb = n * (kt == RSORT_U64 ? 8u : 4u);
  auto ov = [](const void* a, uint64_t na, const void* b, uint64_t nb) {
    if (!a || !b) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
  };
  if (ov(keys_in, kb, keys_out, kb) || ov(keys_in, kb, perm_out, 4 * n) || ov(keys_out, kb, perm_out, 4 * n))
    return RSORT_EINVAL;
  void* ws = scratch_for_current_device();
  if (!ws) return RSORT_EDEVICE;
  const int rc = rs::enqueue_sort((int)kt, keys_in, nullptr, nullptr, 1, n, keys_out, perm_out, nullptr, ws,
                                  kScratchBytes, (hipStream_t)stream);
  return rc == 0 ? RSORT_OK : rc == -1 ? RSORT_EINVAL : rc == -2 ? RSORT_ENOMEM : RSORT_EDEVICE;
}
