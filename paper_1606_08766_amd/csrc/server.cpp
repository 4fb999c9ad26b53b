// Sort server: continuous batching of sort requests on one GPU.
//
// A scheduler thread admits queued requests in arrival order while the sum of
// admitted footprints (input + output + workspace bytes) stays within the HBM
// budget and a slot (one HIP stream each) is free.  Requests admitted while
// others run are enqueued on other streams, so their kernels overlap on the
// device.  Small requests of one key type that are admitted together are
// packed into a single segmented sort (one launch sequence for the group);
// each still gets exactly the result it would get alone, because the sort
// result is a function of its own keys only.  Completion is observed with
// HIP events; a request's status includes device-detected errors.
//
// device < 0 selects a fake executor that touches no GPU: a request
// "completes" after a delay proportional to its size and its buffers are not
// touched.  It exists to test the admission, budget and ticket logic on
// machines without a GPU.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/rsort.h"
#include "internal.hpp"

namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

constexpr uint64_t kBatchMaxN = 1u << 16;     // requests up to this size may be packed
constexpr uint64_t kBatchMaxTotal = 1u << 22;  // elements per packed launch
constexpr uint32_t kBatchMaxCount = 256;
// A magic keys_in value the fake executor treats as a failing request.
constexpr uintptr_t kFakeFault = 0xBADull;

struct Req {
  rsort_request r;
  int status = RSORT_PENDING;
  uint64_t t_submit = 0, t_start = 0, t_done = 0;
  uint64_t footprint = 0;
  uint32_t batch = 1;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t event = nullptr;
  int32_t* status_host = nullptr;  // pinned
  uint64_t* off_host = nullptr;    // pinned, kBatchMaxCount + 1 segment offsets
  bool busy = false;
  std::vector<uint64_t> tickets;
  uint64_t footprint = 0;
  uint64_t fake_done_ns = 0;
  int launch_rc = RSORT_OK;
};

uint64_t key_size(int kt) { return kt == RSORT_U64 ? 8 : 4; }

}  // namespace

struct rsort_server {
  int device = 0;
  bool fake = false;
  uint64_t budget = 0;
  uint32_t max_inflight = 1;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Req> reqs;
  std::vector<Slot> slots;
  uint64_t next_ticket = 1;
  uint64_t in_use = 0, running = 0, finished = 0;
  bool stop = false;
  std::thread worker;

  uint64_t footprint(const rsort_request& r) const {
    const uint64_t ks = key_size(r.kt);
    uint64_t ws = fake ? 0 : rsort_plain_workspace(r.kt, r.n);
    // packed requests need their share of the batch buffers as well
    if (!fake && r.n <= kBatchMaxN) ws += r.n * (2 * ks + 4) + 64;
    return r.n * ks * 2 + (r.perm_out ? 4 * r.n : 0) + ws;
  }

  void run();
  bool launch(Slot& s, std::vector<uint64_t>& group);
  void complete(Slot& s);
};

// Enqueue one group (one request, or several small ones packed) on a slot.
bool rsort_server::launch(Slot& s, std::vector<uint64_t>& group) {
  const uint64_t t0 = now_ns();
  for (uint64_t t : group) {
    reqs[t].t_start = t0;
    reqs[t].batch = (uint32_t)group.size();
  }
  s.tickets = group;
  s.busy = true;
  s.launch_rc = RSORT_OK;
  if (fake) {
    uint64_t tot = 0;
    for (uint64_t t : group) {
      tot += reqs[t].r.n;
      if ((uintptr_t)reqs[t].r.keys_in == kFakeFault) s.launch_rc = RSORT_EDEVICE;
    }
    s.fake_done_ns = t0 + 20000 + tot / 4;  // 20 us + 0.25 ns per key
    return true;
  }
  const rsort_request first = reqs[group[0]].r;
  const int kt = first.kt;
  const uint64_t ks = key_size(kt);
  hipStream_t st = s.stream;
  int rc = RSORT_OK;
  void* ws = nullptr;
  if (group.size() == 1) {
    const size_t wsb = rsort_plain_workspace(first.kt, first.n);
    if (hipMallocAsync(&ws, std::max<size_t>(wsb, 256), st) != hipSuccess) rc = RSORT_EDEVICE;
    if (rc == RSORT_OK)
      rc = rsort_plain(first.kt, first.keys_in, first.n, first.keys_out, first.perm_out, ws, wsb, st);
    if (rc == RSORT_OK && hipMemcpyAsync(s.status_host, ws, 4, hipMemcpyDeviceToHost, st) != hipSuccess)
      rc = RSORT_EDEVICE;
    if (ws) (void)hipFreeAsync(ws, st);
  } else {
    // pack: keys back to back, segment offsets, one segmented sort, unpack
    const uint32_t ns = (uint32_t)group.size();
    uint64_t* off = s.off_host;  // stays untouched until this slot completes
    off[0] = 0;
    for (uint32_t i = 0; i < ns; i++) off[i + 1] = off[i] + reqs[group[i]].r.n;
    const uint64_t tot = off[ns];
    const size_t wsb = rsort_segmented_workspace((rsort_key_t)kt, tot, ns, 0);
    const size_t bytes = tot * ks * 2 + tot * 4 + (ns + 1) * 8 + 1024;
    char* buf = nullptr;
    if (hipMallocAsync((void**)&buf, bytes, st) != hipSuccess || hipMallocAsync(&ws, std::max<size_t>(wsb, 256), st) != hipSuccess)
      rc = RSORT_EDEVICE;
    char* kin = buf;
    char* kout = buf + tot * ks;
    uint32_t* perm = (uint32_t*)(buf + tot * ks * 2);
    uint64_t* doff = (uint64_t*)(buf + ((tot * ks * 2 + tot * 4 + 255) / 256) * 256);
    for (uint32_t i = 0; i < ns && rc == RSORT_OK; i++) {
      const rsort_request& r = reqs[group[i]].r;
      if (r.n && hipMemcpyAsync(kin + off[i] * ks, r.keys_in, r.n * ks, hipMemcpyDeviceToDevice, st) != hipSuccess)
        rc = RSORT_EDEVICE;
    }
    if (rc == RSORT_OK && hipMemcpyAsync(doff, off, (ns + 1) * 8, hipMemcpyHostToDevice, st) != hipSuccess)
      rc = RSORT_EDEVICE;
    if (rc == RSORT_OK)
      rc = rsort_segmented((rsort_key_t)kt, kin, nullptr, doff, ns, tot, kout, nullptr, perm, ws, wsb, st);
    for (uint32_t i = 0; i < ns && rc == RSORT_OK; i++) {
      const rsort_request& r = reqs[group[i]].r;
      if (!r.n) continue;
      if (hipMemcpyAsync(r.keys_out, kout + off[i] * ks, r.n * ks, hipMemcpyDeviceToDevice, st) != hipSuccess)
        rc = RSORT_EDEVICE;
      if (r.perm_out &&
          hipMemcpyAsync(r.perm_out, perm + off[i], r.n * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        rc = RSORT_EDEVICE;
    }
    if (rc == RSORT_OK && hipMemcpyAsync(s.status_host, ws, 4, hipMemcpyDeviceToHost, st) != hipSuccess)
      rc = RSORT_EDEVICE;
    if (buf) (void)hipFreeAsync(buf, st);
    if (ws) (void)hipFreeAsync(ws, st);
  }
  s.launch_rc = rc;
  if (hipEventRecord(s.event, st) != hipSuccess && s.launch_rc == RSORT_OK) s.launch_rc = RSORT_EDEVICE;
  return true;
}

void rsort_server::complete(Slot& s) {
  const uint64_t t = now_ns();
  int st = s.launch_rc;
  if (st == RSORT_OK && !fake) st = *s.status_host;
  for (uint64_t tk : s.tickets) {
    Req& r = reqs[tk];
    r.t_done = t;
    r.status = st;
  }
  in_use -= s.footprint;
  running -= s.tickets.size();
  finished += s.tickets.size();
  s.busy = false;
  s.tickets.clear();
  s.footprint = 0;
}

void rsort_server::run() {
  if (!fake) (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool progress = false;
    // completions
    for (Slot& s : slots) {
      if (!s.busy) continue;
      bool done;
      if (fake)
        done = now_ns() >= s.fake_done_ns;
      else {
        const hipError_t q = hipEventQuery(s.event);
        done = q != hipErrorNotReady;
        if (done && q != hipSuccess) s.launch_rc = RSORT_EDEVICE;
      }
      if (done) {
        complete(s);
        progress = true;
      }
    }
    if (progress) cv_done.notify_all();
    // admissions
    while (!queue.empty()) {
      Slot* free_slot = nullptr;
      for (Slot& s : slots)
        if (!s.busy) {
          free_slot = &s;
          break;
        }
      if (!free_slot) break;
      const uint64_t head = queue.front();
      Req& h = reqs[head];
      if (in_use + h.footprint > budget) break;  // FIFO: wait for memory
      std::vector<uint64_t> group{head};
      uint64_t fp = h.footprint, tot = h.r.n;
      queue.pop_front();
      if (!fake && h.r.n <= kBatchMaxN) {
        // pack following small requests of the same key type that also fit
        for (auto it = queue.begin(); it != queue.end() && group.size() < kBatchMaxCount;) {
          Req& c = reqs[*it];
          if (c.r.kt == h.r.kt && c.r.n <= kBatchMaxN && tot + c.r.n <= kBatchMaxTotal &&
              in_use + fp + c.footprint <= budget) {
            group.push_back(*it);
            fp += c.footprint;
            tot += c.r.n;
            it = queue.erase(it);
          } else {
            ++it;
          }
        }
      }
      in_use += fp;
      running += group.size();
      free_slot->footprint = fp;
      launch(*free_slot, group);
      progress = true;
    }
    if (stop && queue.empty() && running == 0) break;
    if (!progress) {
      if (running > 0)
        cv_sched.wait_for(lk, std::chrono::microseconds(20));
      else
        cv_sched.wait_for(lk, std::chrono::milliseconds(50));
    }
  }
}

extern "C" {

int rsort_server_create(int device, uint64_t hbm_budget_bytes, uint32_t max_inflight, rsort_server** out) {
  if (!out || max_inflight == 0 || max_inflight > 64 || hbm_budget_bytes == 0) return RSORT_EINVAL;
  rsort_server* s = new rsort_server();
  s->device = device;
  s->fake = device < 0;
  s->budget = hbm_budget_bytes;
  s->max_inflight = max_inflight;
  s->slots.resize(max_inflight);
  if (!s->fake) {
    if (hipSetDevice(device) != hipSuccess) {
      delete s;
      return RSORT_EDEVICE;
    }
    for (Slot& sl : s->slots) {
      if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&sl.event, hipEventDisableTiming) != hipSuccess ||
          hipHostMalloc((void**)&sl.status_host, 64, hipHostMallocDefault) != hipSuccess ||
          hipHostMalloc((void**)&sl.off_host, (kBatchMaxCount + 1) * 8, hipHostMallocDefault) != hipSuccess) {
        delete s;
        return RSORT_EDEVICE;
      }
    }
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return RSORT_OK;
}

int rsort_server_destroy(rsort_server* s) {
  if (!s) return RSORT_EINVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_sched.notify_all();
  if (s->worker.joinable()) s->worker.join();
  if (!s->fake) {
    for (Slot& sl : s->slots) {
      if (sl.stream) (void)hipStreamSynchronize(sl.stream);
      if (sl.event) (void)hipEventDestroy(sl.event);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.status_host) (void)hipHostFree(sl.status_host);
      if (sl.off_host) (void)hipHostFree(sl.off_host);
    }
  }
  delete s;
  return RSORT_OK;
}

int rsort_submit(rsort_server* s, const rsort_request* r, uint64_t* ticket_out) {
  if (!s || !r || !ticket_out) return RSORT_EINVAL;
  if (r->kt != RSORT_U32 && r->kt != RSORT_U64 && r->kt != RSORT_F32) return RSORT_EINVAL;
  if (r->n >= 0xFFFFFFFFull || (r->n && (!r->keys_in || !r->keys_out))) return RSORT_EINVAL;
  Req q;
  q.r = *r;
  q.t_submit = now_ns();
  {
    std::lock_guard<std::mutex> g(s->mu);
    q.footprint = s->footprint(*r);
    if (q.footprint > s->budget) return RSORT_ENOMEM;
    const uint64_t t = s->next_ticket++;
    if (r->n == 0) {
      q.status = RSORT_OK;
      q.t_start = q.t_done = q.t_submit;
      s->reqs.emplace(t, q);
      s->finished++;
    } else {
      s->reqs.emplace(t, q);
      s->queue.push_back(t);
    }
    *ticket_out = t;
  }
  s->cv_sched.notify_all();
  return RSORT_OK;
}

static void fill(const Req& q, rsort_result* out) {
  if (!out) return;
  out->status = q.status;
  out->t_submit_ns = q.t_submit;
  out->t_start_ns = q.t_start;
  out->t_done_ns = q.t_done;
  out->batch_size = q.batch;
}

int rsort_poll(rsort_server* s, uint64_t ticket, rsort_result* out) {
  if (!s) return RSORT_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return RSORT_ENOTFOUND;
  fill(it->second, out);
  return it->second.status;
}

int rsort_wait(rsort_server* s, uint64_t ticket, uint32_t timeout_ms, rsort_result* out) {
  if (!s) return RSORT_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return RSORT_ENOTFOUND;
  s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] {
    auto j = s->reqs.find(ticket);
    return j == s->reqs.end() || j->second.status != RSORT_PENDING;
  });
  it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return RSORT_ENOTFOUND;
  fill(it->second, out);
  return it->second.status;
}

int rsort_release(rsort_server* s, uint64_t ticket) {
  if (!s) return RSORT_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return RSORT_ENOTFOUND;
  if (it->second.status == RSORT_PENDING) return RSORT_EBUSY;
  s->reqs.erase(it);
  return RSORT_OK;
}

int rsort_server_counters(rsort_server* s, uint64_t* queued, uint64_t* running, uint64_t* finished,
                          uint64_t* bytes_in_use) {
  if (!s) return RSORT_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (queued) *queued = s->queue.size();
  if (running) *running = s->running;
  if (finished) *finished = s->finished;
  if (bytes_in_use) *bytes_in_use = s->in_use;
  return RSORT_OK;
}

size_t rsort_median_tree_workspace(uint32_t log2_p, uint32_t k, uint32_t num_problems) {
  if (log2_p > 24 || k < 2 || k > 32 || (k & 1)) return 0;
  return rs::median_tree_workspace(log2_p, k, num_problems);
}

int rsort_median_tree(const uint64_t* vals, uint64_t per_problem, const uint64_t* leaf_off, uint32_t log2_p,
                      uint32_t k, const uint8_t* coins, uint32_t num_problems, uint64_t* out, void* workspace,
                      size_t workspace_bytes, void* stream) {
  if (log2_p > 24 || k < 2 || k > 32 || (k & 1)) return RSORT_EINVAL;
  if (num_problems == 0) return RSORT_OK;
  if (!vals || !leaf_off || !coins || !out || !workspace) return RSORT_EINVAL;
  const int rc = rs::enqueue_median_tree(vals, per_problem, leaf_off, log2_p, k, coins, num_problems, out, workspace,
                                         workspace_bytes, (hipStream_t)stream);
  return rc == 0 ? RSORT_OK : rc == -2 ? RSORT_ENOMEM : RSORT_EDEVICE;
}

}  // extern "C"
