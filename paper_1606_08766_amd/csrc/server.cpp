// Sort server: continuous batching of sort requests on one GPU.
//
// The server reserves its HBM budget once, at creation, as a scratch arena;
// every in-flight sort takes its workspace (and, for packed batches, the
// packed buffers) from the arena with a first-fit allocator, and returns it
// when the sort's completion event has fired.  No device allocation happens
// while serving, so no launch waits on the allocator or on another stream.
//
// Requests enter one of two lanes by size.  Large requests are admitted in
// arrival order, each on its own slot (one HIP stream per slot), when their
// scratch fits the arena.  Small requests queue in the small lane; whenever a
// small-lane slot is free, the queued small requests of the head's key type
// are packed (up to the batch limits and the arena's largest free block) into
// one segmented sort: one gather launch, the sort's launches, one
// scatter-back launch.  Requests that arrive while a batch runs join the next
// batch.  Each request's result is exactly the one it would get alone: a
// sort's output depends on its own keys only.
//
// The scheduler thread takes the server lock only for bookkeeping; event
// queries and enqueueing run outside it, so client threads calling submit or
// poll never wait behind a launch sequence.
//
// device < 0 selects a fake executor that touches no GPU: the arena is
// virtual (offsets only), a request "completes" after a delay proportional to
// its size, and its buffers are not touched.  It exists to test admission,
// arena accounting and tickets on machines without a GPU.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <time.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
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

constexpr uint64_t kSmallMaxN = 1u << 20;      // requests up to this size go to the small lane
constexpr uint64_t kBatchMaxTotal = 1u << 24;  // keys per packed batch
constexpr uint32_t kBatchMaxCount = 1024;      // requests per packed batch
constexpr uint32_t kSmallSlots = 2;            // small-lane batches in flight
// Copy-table entries are split into chunks of at most kChunk keys so that the
// gather and scatter launches spread a long request over many workgroups.
constexpr uint64_t kChunk = 1u << 15;
constexpr uint32_t kTabCap = kBatchMaxCount + (uint32_t)(kBatchMaxTotal / kChunk) + 1;
constexpr uint64_t kAlign = 256;
constexpr uint64_t kNone = ~0ull;
// A magic keys_in value the fake executor treats as a failing request.
constexpr uintptr_t kFakeFault = 0xBADull;

uint64_t up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
uint64_t key_size(int kt) { return kt == RSORT_U64 ? 8 : 4; }

// Arena bytes of a packed batch of `count` requests holding `total` keys:
// packed keys in and out, packed permutation, segment offsets, copy table,
// segmented-sort workspace.
uint64_t batch_bytes(int kt, uint64_t total, uint32_t count) {
  const uint64_t ks = key_size(kt);
  const uint64_t entries = count + total / kChunk + 1;
  return 2 * up(total * ks) + up(total * 4) + up((count + 1) * 8ull) + up(entries * sizeof(rs::BatchEntry)) +
         up(std::max<uint64_t>(rsort_segmented_workspace((rsort_key_t)kt, total, count, 0), 256));
}

uint64_t plain_bytes(int kt, uint64_t n) {
  return up(std::max<uint64_t>(rsort_plain_workspace((rsort_key_t)kt, n), 256));
}

// First-fit allocator over [0, size) with coalescing of freed blocks.
struct Arena {
  uint64_t size = 0;
  std::map<uint64_t, uint64_t> free_blocks;  // offset -> length
  void init(uint64_t sz) {
    size = sz;
    free_blocks.clear();
    if (sz) free_blocks[0] = sz;
  }
  uint64_t largest() const {
    uint64_t m = 0;
    for (const auto& b : free_blocks) m = std::max(m, b.second);
    return m;
  }
  uint64_t alloc(uint64_t bytes) {
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
      if (it->second < bytes) continue;
      const uint64_t off = it->first, len = it->second;
      free_blocks.erase(it);
      if (len > bytes) free_blocks[off + bytes] = len - bytes;
      return off;
    }
    return kNone;
  }
  void release(uint64_t off, uint64_t bytes) {
    auto it = free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_blocks.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_blocks.erase(nx);
    }
    if (it != free_blocks.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_blocks.erase(it);
      }
    }
  }
};

struct Req {
  rsort_request r;
  int status = RSORT_PENDING;
  uint64_t t_submit = 0, t_start = 0, t_done = 0;
  uint64_t dev_begin = 0, dev_end = 0;  // device timestamps, ns after the server's epoch event
  uint32_t batch = 1;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t event = nullptr;
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;  // timing events around the slot's work
  int32_t* status_host = nullptr;      // pinned
  rs::BatchEntry* tab_host = nullptr;  // pinned, kTabCap entries
  uint64_t* off_host = nullptr;        // pinned, kBatchMaxCount + 1 segment offsets
  bool busy = false;
  bool small = false;
  std::vector<uint64_t> tickets;
  uint64_t scratch_off = 0, scratch_bytes = 0;
  uint64_t fake_done_ns = 0;
  int launch_rc = RSORT_OK;
};

}  // namespace

struct rsort_server {
  int device = 0;
  bool fake = false;
  char* arena_base = nullptr;  // device memory of the arena (null for the fake executor)
  hipEvent_t epoch = nullptr;  // recorded once at creation: origin of the device timestamps
  Arena arena;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<uint64_t> q_large, q_small;
  std::unordered_map<uint64_t, Req> reqs;
  std::vector<Slot> slots;
  uint64_t next_ticket = 1;
  uint64_t running = 0, finished = 0;
  uint32_t small_running = 0;
  bool stop = false;
  std::thread worker;
  FILE* log = nullptr;  // launch / completion trace (RSORT_SERVER_LOG), written by the scheduler only

  static bool is_small(const rsort_request& r) { return r.n <= kSmallMaxN; }
  static uint64_t solo_bytes(const rsort_request& r) {
    return is_small(r) ? batch_bytes(r.kt, r.n, 1) : plain_bytes(r.kt, r.n);
  }

  void run();
  void launch(Slot& s, const std::vector<rsort_request>& group);
  bool slot_done(Slot& s);
  void complete(Slot& s);
  Slot* free_slot(bool for_small);
};

Slot* rsort_server::free_slot(bool for_small) {
  // slot 0 is kept for the small lane whenever there are at least two slots
  for (size_t i = 0; i < slots.size(); i++) {
    if (slots[i].busy) continue;
    if (!for_small && i == 0 && slots.size() > 1) continue;
    return &slots[i];
  }
  return nullptr;
}

// Enqueue one group (one request, or several small ones packed) on a slot
// whose arena range is already assigned.  Runs without the server lock: it
// reads only its arguments and the slot, which belongs to the scheduler
// thread while busy.
void rsort_server::launch(Slot& s, const std::vector<rsort_request>& group) {
  s.launch_rc = RSORT_OK;
  if (fake) {
    uint64_t tot = 0;
    for (const rsort_request& r : group) tot += r.n;
    s.fake_done_ns = now_ns() + 20000 + tot / 4;  // 20 us + 0.25 ns per key
    return;
  }
  const rsort_request& first = group[0];
  const int kt = first.kt;
  const uint64_t ks = key_size(kt);
  hipStream_t st = s.stream;
  char* base = arena_base + s.scratch_off;
  int rc = RSORT_OK;
  if (hipEventRecord(s.ev_begin, st) != hipSuccess) rc = RSORT_EDEVICE;
  void* ws = nullptr;
  if (!s.small || group.size() == 1) {  // alone: no packing copies
    ws = base;
    rc = rsort_plain(first.kt, first.keys_in, first.n, first.keys_out, first.perm_out, ws, s.scratch_bytes, st);
  } else {
    // pack: one gather launch, one segmented sort, one scatter-back launch
    const uint32_t ns = (uint32_t)group.size();
    uint64_t* off = s.off_host;  // pinned; untouched until this slot completes
    rs::BatchEntry* tab = s.tab_host;
    uint32_t nt = 0;
    off[0] = 0;
    for (uint32_t i = 0; i < ns; i++) {
      const rsort_request& r = group[i];
      off[i + 1] = off[i] + r.n;
      for (uint64_t j = 0; j < r.n && nt < kTabCap; j += kChunk)
        tab[nt++] = rs::BatchEntry{(const char*)r.keys_in + j * ks, (char*)r.keys_out + j * ks,
                                   r.perm_out ? r.perm_out + j : nullptr, std::min(kChunk, r.n - j), off[i] + j};
    }
    const uint64_t tot = off[ns];
    const uint64_t entries = ns + tot / kChunk + 1;
    char* kin = base;
    char* kout = kin + up(tot * ks);
    uint32_t* perm = (uint32_t*)(kout + up(tot * ks));
    uint64_t* doff = (uint64_t*)((char*)perm + up(tot * 4));
    rs::BatchEntry* dtab = (rs::BatchEntry*)((char*)doff + up((ns + 1) * 8ull));
    ws = (char*)dtab + up(entries * sizeof(rs::BatchEntry));
    const uint64_t wsb = s.scratch_bytes - (uint64_t)((char*)ws - base);
    if (hipMemcpyAsync(doff, off, (ns + 1) * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dtab, tab, nt * sizeof(rs::BatchEntry), hipMemcpyHostToDevice, st) != hipSuccess)
      rc = RSORT_EDEVICE;
    if (rc == RSORT_OK && rs::enqueue_batch_in(dtab, nt, (uint32_t)ks, kin, st) != 0) rc = RSORT_EDEVICE;
    if (rc == RSORT_OK)
      rc = rsort_segmented((rsort_key_t)kt, kin, nullptr, doff, ns, tot, kout, nullptr, perm, ws, wsb, st);
    if (rc == RSORT_OK && rs::enqueue_batch_out(dtab, nt, (uint32_t)ks, kout, perm, st) != 0) rc = RSORT_EDEVICE;
  }
  if (rc == RSORT_OK && hipMemcpyAsync(s.status_host, ws, 4, hipMemcpyDeviceToHost, st) != hipSuccess)
    rc = RSORT_EDEVICE;
  if (rc == RSORT_OK && hipEventRecord(s.ev_end, st) != hipSuccess) rc = RSORT_EDEVICE;
  s.launch_rc = rc;
  if (hipEventRecord(s.event, st) != hipSuccess && s.launch_rc == RSORT_OK) s.launch_rc = RSORT_EDEVICE;
}

bool rsort_server::slot_done(Slot& s) {
  if (fake) return now_ns() >= s.fake_done_ns;
  const hipError_t q = hipEventQuery(s.event);
  if (q == hipErrorNotReady) return false;
  if (q != hipSuccess) s.launch_rc = RSORT_EDEVICE;
  return true;
}

// Called with the lock held, after the slot's completion event fired.
void rsort_server::complete(Slot& s) {
  const uint64_t t = now_ns();
  int st = s.launch_rc;
  if (st == RSORT_OK && !fake) st = *s.status_host;
  uint64_t db = 0, de = 0;
  if (st == RSORT_OK && !fake) {
    float a = 0.f, b = 0.f;
    if (hipEventElapsedTime(&a, epoch, s.ev_begin) == hipSuccess &&
        hipEventElapsedTime(&b, epoch, s.ev_end) == hipSuccess) {
      db = (uint64_t)((double)a * 1e6);
      de = (uint64_t)((double)b * 1e6);
    }
  }
  for (uint64_t tk : s.tickets) {
    Req& r = reqs[tk];
    r.t_done = t;
    r.dev_begin = db;
    r.dev_end = de;
    r.status = st;
    // the fake executor fails exactly the requests marked as faulty
    if (fake && (uintptr_t)r.r.keys_in == kFakeFault) r.status = RSORT_EDEVICE;
  }
  arena.release(s.scratch_off, s.scratch_bytes);
  running -= s.tickets.size();
  finished += s.tickets.size();
  if (s.small) small_running--;
  s.busy = false;
  s.small = false;
  s.tickets.clear();
  s.scratch_bytes = 0;
}

void rsort_server::run() {
  if (!fake) (void)hipSetDevice(device);
  struct Todo {
    Slot* slot;
    std::vector<rsort_request> reqs;
  };
  std::vector<Slot*> done;
  std::vector<Todo> todo;
  for (;;) {
    done.clear();
    todo.clear();
    for (Slot& s : slots)
      if (s.busy && slot_done(s)) done.push_back(&s);
    {
      std::unique_lock<std::mutex> lk(mu);
      for (Slot* s : done) complete(*s);
      if (!done.empty()) cv_done.notify_all();
      auto start = [&](Slot* sl, std::vector<uint64_t>& group, uint64_t off, uint64_t bytes, bool small) {
        const uint64_t t0 = now_ns();
        Todo td{sl, {}};
        for (uint64_t t : group) {
          Req& q = reqs[t];
          q.t_start = t0;
          q.batch = (uint32_t)group.size();
          td.reqs.push_back(q.r);
        }
        running += group.size();
        if (small) small_running++;
        sl->scratch_off = off;
        sl->scratch_bytes = bytes;
        sl->small = small;
        sl->busy = true;
        sl->tickets = group;
        todo.push_back(std::move(td));
      };
      // large lane: arrival order, one request per slot, wait for arena space
      while (!q_large.empty()) {
        Slot* sl = free_slot(false);
        if (!sl) break;
        const uint64_t head = q_large.front();
        const uint64_t bytes = plain_bytes(reqs[head].r.kt, reqs[head].r.n);
        const uint64_t off = arena.alloc(bytes);
        if (off == kNone) break;
        q_large.pop_front();
        std::vector<uint64_t> group{head};
        start(sl, group, off, bytes, false);
      }
      // small lane: pack the queued requests of the head's key type
      while (!q_small.empty() && small_running < kSmallSlots) {
        Slot* sl = free_slot(true);
        if (!sl) break;
        const uint64_t head = q_small.front();
        const rsort_request h = reqs[head].r;
        const uint64_t room = arena.largest();
        if (batch_bytes(h.kt, h.n, 1) > room) break;
        std::vector<uint64_t> group{head};
        uint64_t tot = h.n;
        q_small.pop_front();
        for (auto it = q_small.begin(); it != q_small.end() && group.size() < kBatchMaxCount;) {
          const rsort_request& c = reqs[*it].r;
          if (c.kt == h.kt && tot + c.n <= kBatchMaxTotal &&
              batch_bytes(h.kt, tot + c.n, (uint32_t)group.size() + 1) <= room) {
            group.push_back(*it);
            tot += c.n;
            it = q_small.erase(it);
          } else {
            ++it;
          }
        }
        const uint64_t bytes = batch_bytes(h.kt, tot, (uint32_t)group.size());
        const uint64_t off = arena.alloc(bytes);  // fits: bytes <= largest free block
        start(sl, group, off, bytes, true);
      }
      if (todo.empty() && done.empty()) {
        if (stop && q_large.empty() && q_small.empty() && running == 0) break;
        if (running > 0)
          cv_sched.wait_for(lk, std::chrono::microseconds(20));
        else
          cv_sched.wait_for(lk, std::chrono::milliseconds(50));
        continue;
      }
    }
    for (Todo& td : todo) {
      const uint64_t a = now_ns();
      launch(*td.slot, td.reqs);
      if (log) {
        uint64_t keys = 0;
        for (const rsort_request& r : td.reqs) keys += r.n;
        fprintf(log, "L %llu slot %d reqs %zu keys %llu kt %d enqueue_us %.1f rc %d\n", (unsigned long long)a,
                (int)(td.slot - slots.data()), td.reqs.size(), (unsigned long long)keys, td.reqs[0].kt,
                (now_ns() - a) / 1e3, td.slot->launch_rc);
      }
    }
    if (log)
      for (Slot* sl : done) fprintf(log, "D %llu slot %d\n", (unsigned long long)now_ns(), (int)(sl - slots.data()));
  }
  if (log) fclose(log);
}

static void destroy_server(rsort_server* s) {
  if (!s->fake) {
    for (Slot& sl : s->slots) {
      if (sl.stream) (void)hipStreamSynchronize(sl.stream);
      if (sl.event) (void)hipEventDestroy(sl.event);
      if (sl.ev_begin) (void)hipEventDestroy(sl.ev_begin);
      if (sl.ev_end) (void)hipEventDestroy(sl.ev_end);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.status_host) (void)hipHostFree(sl.status_host);
      if (sl.off_host) (void)hipHostFree(sl.off_host);
      if (sl.tab_host) (void)hipHostFree(sl.tab_host);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    if (s->epoch) (void)hipEventDestroy(s->epoch);
  }
  delete s;
}

extern "C" {

size_t rsort_server_request_bytes(rsort_key_t kt, uint64_t n) {
  if (kt != RSORT_U32 && kt != RSORT_U64 && kt != RSORT_F32) return 0;
  rsort_request r{kt, nullptr, n, nullptr, nullptr};
  return n ? rsort_server::solo_bytes(r) : 0;
}

int rsort_server_create(int device, uint64_t hbm_budget_bytes, uint32_t max_inflight, rsort_server** out) {
  if (!out || max_inflight == 0 || max_inflight > 64 || hbm_budget_bytes < kAlign) return RSORT_EINVAL;
  rsort_server* s = new rsort_server();
  s->device = device;
  s->fake = device < 0;
  s->slots.resize(max_inflight);
  const uint64_t size = hbm_budget_bytes / kAlign * kAlign;
  s->arena.init(size);
  if (!s->fake) {
    if (hipSetDevice(device) != hipSuccess) {
      destroy_server(s);
      return RSORT_EDEVICE;
    }
    if (hipMalloc((void**)&s->arena_base, size) != hipSuccess) {
      s->arena_base = nullptr;
      destroy_server(s);
      return RSORT_ENOMEM;
    }
    for (Slot& sl : s->slots) {
      if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&sl.event, hipEventDisableTiming) != hipSuccess ||
          hipEventCreate(&sl.ev_begin) != hipSuccess || hipEventCreate(&sl.ev_end) != hipSuccess ||
          hipHostMalloc((void**)&sl.status_host, 64, hipHostMallocDefault) != hipSuccess ||
          hipHostMalloc((void**)&sl.off_host, (kBatchMaxCount + 1) * 8, hipHostMallocDefault) != hipSuccess ||
          hipHostMalloc((void**)&sl.tab_host, kTabCap * sizeof(rs::BatchEntry), hipHostMallocDefault) !=
              hipSuccess) {
        destroy_server(s);
        return RSORT_EDEVICE;
      }
    }
    if (hipEventCreate(&s->epoch) != hipSuccess || hipEventRecord(s->epoch, s->slots[0].stream) != hipSuccess ||
        hipEventSynchronize(s->epoch) != hipSuccess) {
      destroy_server(s);
      return RSORT_EDEVICE;
    }
  }
  if (const char* path = getenv("RSORT_SERVER_LOG")) {
    s->log = fopen(path, "a");
    if (s->log)
      fprintf(s->log, "S %llu slots %u arena %llu\n", (unsigned long long)now_ns(), max_inflight,
              (unsigned long long)size);
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
  destroy_server(s);
  return RSORT_OK;
}

int rsort_submit(rsort_server* s, const rsort_request* r, uint64_t* ticket_out) {
  if (!s || !r || !ticket_out) return RSORT_EINVAL;
  if (r->kt != RSORT_U32 && r->kt != RSORT_U64 && r->kt != RSORT_F32) return RSORT_EINVAL;
  if (r->n >= 0xFFFFFFFFull || (r->n && (!r->keys_in || !r->keys_out))) return RSORT_EINVAL;
  Req q;
  q.r = *r;
  q.t_submit = now_ns();
  if (r->n && rsort_server::solo_bytes(*r) > s->arena.size) return RSORT_ENOMEM;
  {
    std::lock_guard<std::mutex> g(s->mu);
    const uint64_t t = s->next_ticket++;
    if (r->n == 0) {
      q.status = RSORT_OK;
      q.t_start = q.t_done = q.t_submit;
      s->reqs.emplace(t, q);
      s->finished++;
    } else {
      s->reqs.emplace(t, q);
      (rsort_server::is_small(*r) ? s->q_small : s->q_large).push_back(t);
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
  out->dev_begin_ns = q.dev_begin;
  out->dev_end_ns = q.dev_end;
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
  if (queued) *queued = s->q_large.size() + s->q_small.size();
  if (running) *running = s->running;
  if (finished) *finished = s->finished;
  if (bytes_in_use) {
    uint64_t fr = 0;
    for (const auto& b : s->arena.free_blocks) fr += b.second;
    *bytes_in_use = s->arena.size - fr;
  }
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
