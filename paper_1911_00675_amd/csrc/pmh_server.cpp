// Continuous-batching server for single-set signature requests.
//
// The server owns `slots` execution slots (stream, event, pinned staging,
// device buffers, work list).  At most one slot is OPEN: submissions reserve
// room in it under the lock and copy their ids/weights straight into its
// pinned staging buffer (one host copy per request, on the submitting
// thread); replayed requests, staged in pinned memory beforehand, skip that
// copy and are DMA'd to the device from where they are.  A dispatcher thread launches the open slot as soon as it holds a
// request and no copy into it is still running: host->device copy of the
// batch, the heavy-first ordering kernel, the persistent signature kernel on
// the slot's stream, device->host copy of the signatures.  The next FREE slot
// then opens, so requests that arrive while batches are on the GPU keep
// forming the next batch; several slots run concurrently.  When every slot is
// in flight, submitters wait for one to finish (back-pressure).
//
// Admission: a slot holds at most `slot_elems` elements and `slot_sets`
// requests; its device buffers are sized from the HBM budget; its persistent
// grid is limited to its share of each CU's workgroup (LDS) capacity so
// concurrent batches co-reside.  Results do not depend on batch composition:
// a signature is a pure function of the set.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pmh.h"
#include "pmh_runtime.h"

using namespace pmh;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
  uint64_t ticket = 0;
  uint32_t n = 0;
  const uint64_t* src_ids = nullptr;  // pinned source (replay), device-mapped alias: read by the copy kernel
  const double* src_w = nullptr;
  uint64_t fill_off = 0;              // element offset of the request in its slot
  uint32_t* dst_idx = nullptr;  // result destinations (replay) ...
  uint64_t* dst_id = nullptr;
  double* dst_val = nullptr;
  std::vector<uint32_t> res_idx;  // ... or owned results (submit/fetch)
  std::vector<uint64_t> res_id;
  std::vector<double> res_val;
  bool owned = false;
  int status = PMH_OK;
  double t_done = 0.0;
  std::atomic<bool> done{false};
};

enum SlotState { kFree, kOpen, kFlight };

// Copy kernels between device buffers and device-mapped pinned host memory
// (8-byte elements; dst/src pairs b and c may be null).
hipError_t copy64(const void* sa, void* da, uint64_t na, const void* sb, void* db, uint64_t nb, const void* sc,
                  void* dc, uint64_t nc, hipStream_t s) {
  CopySegs g{{(const uint32_t*)sa, (const uint32_t*)sb, (const uint32_t*)sc},
             {(uint32_t*)da, (uint32_t*)db, (uint32_t*)dc},
             {2 * na, sb ? 2 * nb : 0, sc ? 2 * nc : 0}};
  return launch_copy_words(g, s);
}

// Single-writer maximum (the dispatcher thread).
void raise_max(std::atomic<uint64_t>& a, uint64_t v) {
  if (v > a.load(std::memory_order_relaxed)) a.store(v, std::memory_order_relaxed);
}

// A batch finishes with its slowest set, so the server splits requests far
// more finely than the batched throughput forms do: sets of >= 2^11 elements
// run as 1,024-element chunks on separate workgroups (unless the context
// disables splitting).  At 50,000 requests/s of 10..10^5 elements this
// measured p99 0.5 ms against 5-25 ms with 2^15.
constexpr uint32_t kServeSplitLog2 = 11;
uint32_t serve_split(const pmh_ctx* c) { return c->tune.split_log2 > 0 ? kServeSplitLog2 : 0u; }

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  WorkBuf work;
  uint64_t* d_ids = nullptr;
  double* d_w = nullptr;
  uint64_t* d_off = nullptr;
  uint32_t* d_idx = nullptr;
  uint64_t* d_id = nullptr;
  double* d_val = nullptr;
  uint64_t* h_ids = nullptr;
  double* h_w = nullptr;
  // device-mapped aliases of the pinned buffers (the copy kernels use them)
  const uint64_t* dh_ids = nullptr;
  const double* dh_w = nullptr;
  const uint64_t* dh_off = nullptr;
  uint32_t* dh_idx = nullptr;
  uint64_t* dh_id = nullptr;
  double* dh_val = nullptr;
  uint64_t* h_off = nullptr;
  uint32_t* h_idx = nullptr;
  uint64_t* h_id = nullptr;
  double* h_val = nullptr;
  uint64_t elems_cap = 0;
  uint32_t sets_cap = 0;
  // batch assembly, guarded by the server mutex
  SlotState state = kFree;
  std::vector<Request*> batch;
  uint64_t fill = 0;
  int copying = 0;
};

void free_slot_buffers(Slot& s) {
  (void)hipFree(s.d_ids);
  (void)hipFree(s.d_w);
  (void)hipFree(s.d_off);
  (void)hipFree(s.d_idx);
  (void)hipFree(s.d_id);
  (void)hipFree(s.d_val);
  (void)hipHostFree(s.h_ids);
  (void)hipHostFree(s.h_w);
  (void)hipHostFree(s.h_off);
  (void)hipHostFree(s.h_idx);
  (void)hipHostFree(s.h_id);
  (void)hipHostFree(s.h_val);
  s.d_ids = nullptr;
  s.d_w = nullptr;
  s.d_off = nullptr;
  s.d_idx = nullptr;
  s.d_id = nullptr;
  s.d_val = nullptr;
  s.h_ids = nullptr;
  s.h_w = nullptr;
  s.h_off = nullptr;
  s.h_idx = nullptr;
  s.h_id = nullptr;
  s.h_val = nullptr;
}

int alloc_slot_buffers(Slot& s, uint64_t elems, uint32_t sets, uint32_t m) {
  const uint64_t r = (uint64_t)sets * m;
  const bool ok = hipMalloc(&s.d_ids, elems * 8) == hipSuccess && hipMalloc(&s.d_w, elems * 8) == hipSuccess &&
                  hipMalloc(&s.d_off, (sets + 1) * 8ull) == hipSuccess && hipMalloc(&s.d_idx, r * 4) == hipSuccess &&
                  hipMalloc(&s.d_id, r * 8) == hipSuccess && hipMalloc(&s.d_val, r * 8) == hipSuccess &&
                  hipHostMalloc(&s.h_ids, elems * 8, hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc(&s.h_w, elems * 8, hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc(&s.h_off, (sets + 1) * 8ull, hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc(&s.h_idx, r * 4, hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc(&s.h_id, r * 8, hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc(&s.h_val, r * 8, hipHostMallocDefault) == hipSuccess;
  void* a[6] = {};
  if (!ok || hipHostGetDevicePointer(&a[0], s.h_ids, 0) != hipSuccess ||
      hipHostGetDevicePointer(&a[1], s.h_w, 0) != hipSuccess ||
      hipHostGetDevicePointer(&a[2], s.h_off, 0) != hipSuccess ||
      hipHostGetDevicePointer(&a[3], s.h_idx, 0) != hipSuccess ||
      hipHostGetDevicePointer(&a[4], s.h_id, 0) != hipSuccess ||
      hipHostGetDevicePointer(&a[5], s.h_val, 0) != hipSuccess) {
    free_slot_buffers(s);
    return PMH_ERR_OOM;
  }
  s.dh_ids = (const uint64_t*)a[0];
  s.dh_w = (const double*)a[1];
  s.dh_off = (const uint64_t*)a[2];
  s.dh_idx = (uint32_t*)a[3];
  s.dh_id = (uint64_t*)a[4];
  s.dh_val = (double*)a[5];
  s.elems_cap = elems;
  s.sets_cap = sets;
  return PMH_OK;
}

double now_s(Clock::time_point epoch) { return std::chrono::duration<double>(Clock::now() - epoch).count(); }

}  // namespace

struct pmh_server {
  pmh_ctx* ctx = nullptr;
  std::vector<Slot> slots;
  std::mutex mu;
  std::unordered_map<uint64_t, Request*> owned;  // submit/fetch requests by ticket
  std::atomic<bool> stop{false};
  std::thread worker;
  uint64_t next_ticket = 1;
  Clock::time_point epoch;
  int per_cu = 1;
  int waves = 2;
  int in_flight = 0;
  uint64_t st_done = 0, st_max_busy = 0, st_waited = 0;  // guarded by mu
  // written by the dispatcher thread only (read by pmh_server_stats):
  // batches, largest batch, and its timing in microseconds (longest launch:
  // copies and kernels enqueued; longest finish: results handed out;
  // longest loop iteration)
  std::atomic<uint64_t> st_batches{0}, st_max_batch{0};
  std::atomic<uint64_t> st_max_launch_us{0}, st_max_finish_us{0}, st_max_iter_us{0};
  int fatal = PMH_OK;
};

namespace {

// Reserve room for the request in the open slot (opening a free one if
// needed); waits while every slot is in flight.  Returns the slot and offset.
Slot* reserve(pmh_server* S, Request* r, uint64_t* off) {
  bool waited = false;
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      Slot* open = nullptr;
      bool have_open = false;
      for (Slot& sl : S->slots)
        if (sl.state == kOpen) {
          have_open = true;
          if (sl.fill + r->n <= sl.elems_cap && sl.batch.size() < sl.sets_cap) open = &sl;
        }
      if (!have_open) {
        for (Slot& sl : S->slots)
          if (sl.state == kFree) {
            sl.state = kOpen;
            sl.fill = 0;
            sl.batch.clear();
            open = &sl;
            break;
          }
      }
      if (open) {
        *off = open->fill;
        r->fill_off = open->fill;
        open->fill += r->n;
        open->batch.push_back(r);
        open->copying++;
        if (waited) S->st_waited++;
        return open;
      }
    }
    waited = true;
    std::this_thread::yield();
  }
}

// Requests with a pinned source (r->src_ids) are not copied on the host: the
// launch copies them to the device straight from there.
void submit_internal(pmh_server* S, Request* r, const uint64_t* ids, const double* w) {
  uint64_t off = 0;
  Slot* sl = reserve(S, r, &off);
  if (r->n && !r->src_ids) {
    memcpy(sl->h_ids + off, ids, (size_t)r->n * 8);
    memcpy(sl->h_w + off, w, (size_t)r->n * 8);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  sl->copying--;
}

// Host->device copy of the batch's ids and weights: runs of requests whose
// sources are contiguous (staging, or consecutive requests of a pinned
// replay buffer) go in one copy kernel each.
int copy_in(Slot& sl) {
  const uint64_t* run_ids = nullptr;
  const double* run_w = nullptr;
  uint64_t run_dst = 0, run_len = 0;
  auto flush = [&]() -> bool {
    if (!run_len) return true;
    const bool ok = copy64(run_ids, sl.d_ids + run_dst, run_len, run_w, sl.d_w + run_dst, run_len, nullptr, nullptr, 0,
                           sl.stream) == hipSuccess;
    run_len = 0;
    return ok;
  };
  for (Request* r : sl.batch) {
    if (!r->n) continue;
    const uint64_t* si = r->src_ids ? r->src_ids : sl.dh_ids + r->fill_off;
    const double* sw = r->src_ids ? r->src_w : sl.dh_w + r->fill_off;
    if (run_len && si == run_ids + run_len && sw == run_w + run_len && r->fill_off == run_dst + run_len) {
      run_len += r->n;
      continue;
    }
    if (!flush()) return PMH_ERR_DEVICE;
    run_ids = si;
    run_w = sw;
    run_dst = r->fill_off;
    run_len = r->n;
  }
  return flush() ? PMH_OK : PMH_ERR_DEVICE;
}

void finish(pmh_server* S, Slot& sl) {
  const uint32_t m = S->ctx->m;
  const double t = now_s(S->epoch);
  for (size_t k = 0; k < sl.batch.size(); ++k) {
    Request* r = sl.batch[k];
    const uint64_t o = (uint64_t)k * m;
    if (r->owned) {
      r->res_idx.assign(sl.h_idx + o, sl.h_idx + o + m);
      r->res_id.assign(sl.h_id + o, sl.h_id + o + m);
      r->res_val.assign(sl.h_val + o, sl.h_val + o + m);
    } else {
      if (r->dst_idx) memcpy(r->dst_idx, sl.h_idx + o, m * 4);
      if (r->dst_id) memcpy(r->dst_id, sl.h_id + o, m * 8);
      if (r->dst_val) memcpy(r->dst_val, sl.h_val + o, m * 8);
    }
    r->t_done = t;
    r->done.store(true, std::memory_order_release);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  S->st_done += sl.batch.size();
  sl.batch.clear();
  sl.fill = 0;
  sl.state = kFree;
  S->in_flight--;
}

// Signatures of nb sets to the slot's pinned result buffers.
hipError_t out_copy(Slot& sl, uint64_t nb, uint32_t m) {
  const uint64_t r = nb * m;
  CopySegs g{{(const uint32_t*)sl.d_idx, (const uint32_t*)sl.d_id, (const uint32_t*)sl.d_val},
             {sl.dh_idx, (uint32_t*)sl.dh_id, (uint32_t*)sl.dh_val},
             {r, 2 * r, 2 * r}};
  return launch_copy_words(g, sl.stream);
}

int launch(pmh_server* S, Slot& sl) {
  pmh_ctx* c = S->ctx;
  const uint32_t m = c->m;
  const uint64_t nb = sl.batch.size();
  uint64_t off = 0;
  sl.h_off[0] = 0;
  for (uint64_t k = 0; k < nb; ++k) {
    off += sl.batch[k]->n;
    sl.h_off[k + 1] = off;
  }
  if (ensure_work(c, &sl.work, nb)) return PMH_ERR_OOM;
  if (copy_in(sl) != PMH_OK ||
      copy64(sl.dh_off, sl.d_off, nb + 1, nullptr, nullptr, 0, nullptr, nullptr, 0, sl.stream) != hipSuccess)
    return PMH_ERR_DEVICE;
  HashArgs a = make_args(c, sl.d_ids, sl.d_w, sl.d_off, nb, sl.d_idx, sl.d_val, sl.d_id, nullptr, &sl.work);
  a.split_log2 = serve_split(c);
  const int rc = enqueue_batched(c, a, &sl.work, sl.stream, S->per_cu, S->waves);
  if (rc) return rc;
  if (out_copy(sl, nb, m) != hipSuccess || hipEventRecord(sl.ev, sl.stream) != hipSuccess) return PMH_ERR_DEVICE;
  S->st_batches.fetch_add(1, std::memory_order_relaxed);
  raise_max(S->st_max_batch, nb);
  return PMH_OK;
}

// The first copies and kernel launches on a new stream cost milliseconds
// (hardware queue and code set-up); left to the first requests they build a
// backlog that takes over a thousand requests to drain.  One set of
// 2^split unit-weight elements (split into chunks when splitting is on) runs
// every step of launch() on the slot's stream at creation instead.
int warm_slot(pmh_server* S, Slot& sl) {
  pmh_ctx* c = S->ctx;
  const uint32_t m = c->m;
  const uint32_t sl2 = serve_split(c);
  const uint64_t n = std::min<uint64_t>(sl.elems_cap, sl2 > 0 ? (1ull << sl2) : 64);
  for (uint64_t k = 0; k < n; ++k) {
    sl.h_ids[k] = k;
    sl.h_w[k] = 1.0;
  }
  sl.h_off[0] = 0;
  sl.h_off[1] = n;
  if (copy64(sl.dh_ids, sl.d_ids, n, sl.dh_w, sl.d_w, n, sl.dh_off, sl.d_off, 2, sl.stream) != hipSuccess)
    return PMH_ERR_DEVICE;
  HashArgs a = make_args(c, sl.d_ids, sl.d_w, sl.d_off, 1, sl.d_idx, sl.d_val, sl.d_id, nullptr, &sl.work);
  a.split_log2 = sl2;
  const int rc = enqueue_batched(c, a, &sl.work, sl.stream, S->per_cu, S->waves);
  if (rc) return rc;
  // then full-size passes over the pinned buffers (the GPU's first touches
  // of their pages are slow)
  if (out_copy(sl, 1, m) != hipSuccess ||
      copy64(sl.dh_ids, sl.d_ids, sl.elems_cap, sl.dh_w, sl.d_w, sl.elems_cap, nullptr, nullptr, 0, sl.stream) !=
          hipSuccess ||
      out_copy(sl, sl.sets_cap, m) != hipSuccess || hipEventRecord(sl.ev, sl.stream) != hipSuccess ||
      hipEventSynchronize(sl.ev) != hipSuccess)
    return PMH_ERR_DEVICE;
  return PMH_OK;
}

void fail_batch(pmh_server* S, Slot& sl, int rc) {
  const double t = now_s(S->epoch);
  for (Request* r : sl.batch) {
    r->status = rc;
    r->t_done = t;
    r->done.store(true, std::memory_order_release);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  S->fatal = rc;
  sl.batch.clear();
  sl.fill = 0;
  sl.state = kFree;
  S->in_flight--;
}

void worker_loop(pmh_server* S) {
  (void)hipSetDevice(S->ctx->device);
  auto us_since = [&](double t) { return (uint64_t)((now_s(S->epoch) - t) * 1e6); };
  for (;;) {
    const double t_iter = now_s(S->epoch);
    const bool stopping = S->stop.load(std::memory_order_acquire);
    bool progressed = false;
    for (Slot& sl : S->slots) {
      if (sl.state == kFlight && hipEventQuery(sl.ev) == hipSuccess) {
        const double t0 = now_s(S->epoch);
        finish(S, sl);
        raise_max(S->st_max_finish_us, us_since(t0));
        progressed = true;
      }
    }
    Slot* go = nullptr;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (Slot& sl : S->slots)
        if (sl.state == kOpen && !sl.batch.empty() && sl.copying == 0) {
          sl.state = kFlight;  // closed to new submissions
          S->in_flight++;
          S->st_max_busy = std::max<uint64_t>(S->st_max_busy, (uint64_t)S->in_flight);
          go = &sl;
          break;
        }
    }
    if (go) {
      const double t0 = now_s(S->epoch);
      const int rc = launch(S, *go);
      raise_max(S->st_max_launch_us, us_since(t0));
      if (rc) fail_batch(S, *go, rc);
      progressed = true;
    }
    raise_max(S->st_max_iter_us, us_since(t_iter));
    if (!progressed) {
      if (stopping) {
        std::lock_guard<std::mutex> lk(S->mu);
        bool pending = S->in_flight > 0;
        for (Slot& sl : S->slots) pending |= sl.state == kOpen && !sl.batch.empty();
        if (!pending) break;
      }
      std::this_thread::yield();
    }
  }
}

}  // namespace

extern "C" {

int pmh_server_create(pmh_ctx* c, int slots, uint64_t slot_elems, uint32_t slot_sets, uint64_t hbm_budget_bytes,
                      pmh_server** out) {
  if (!c || !out || slots < 1 || slots > 16 || slot_sets < 1) return PMH_ERR_ARG;
  *out = nullptr;
  DeviceGuard g(c->device);
  // any single request (<= 2^20 elements) fits an empty slot
  uint64_t elems = std::max<uint64_t>(slot_elems, kMaxSet);
  if (hbm_budget_bytes) {
    const uint64_t per_slot = hbm_budget_bytes / (uint64_t)slots;
    const uint64_t outb = (uint64_t)slot_sets * c->m * 20 + (slot_sets + 1ull) * 8;
    if (per_slot <= outb + kMaxSet * 16) return PMH_ERR_OOM;
    elems = std::min<uint64_t>(elems, (per_slot - outb) / 16);
  }
  pmh_server* S = new (std::nothrow) pmh_server();
  if (!S) return PMH_ERR_OOM;
  S->ctx = c;
  S->epoch = Clock::now();
  S->waves = effective_waves(c);
  int occ = 1;
  uint32_t qcap = 0;
  if (occupancy(c->variant, S->waves, launch_lds(c, S->waves, &qcap), &occ) != hipSuccess || occ < 1) occ = 1;
  S->per_cu = std::max(1, occ / slots);  // each slot's share of the CUs' workgroup (LDS) capacity
  S->slots.resize(slots);
  int rc = PMH_OK;
  for (Slot& sl : S->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
      rc = PMH_ERR_DEVICE;
      break;
    }
    rc = alloc_slot_buffers(sl, elems, slot_sets, c->m);
    if (rc) break;
    rc = ensure_work(c, &sl.work, slot_sets);
    if (rc) break;
    rc = warm_slot(S, sl);
    if (rc) break;
  }
  if (rc) {
    for (Slot& sl : S->slots) {
      free_slot_buffers(sl);
      free_work(&sl.work);
      if (sl.ev) (void)hipEventDestroy(sl.ev);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete S;
    return rc;
  }
  S->worker = std::thread(worker_loop, S);
  *out = S;
  return PMH_OK;
}

int pmh_server_submit(pmh_server* S, const uint64_t* ids, const double* w, uint32_t n, uint64_t* ticket) {
  if (!S || !ticket || (n && (!ids || !w)) || n > kMaxSet) return PMH_ERR_ARG;
  Request* r = new (std::nothrow) Request();
  if (!r) return PMH_ERR_OOM;
  r->n = n;
  r->owned = true;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r->ticket = S->next_ticket++;
    S->owned[r->ticket] = r;
  }
  *ticket = r->ticket;
  submit_internal(S, r, ids, w);
  return PMH_OK;
}

int pmh_server_fetch(pmh_server* S, uint64_t ticket, uint32_t* idx, double* val, uint64_t* id) {
  if (!S) return PMH_ERR_ARG;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->owned.find(ticket);
    if (it == S->owned.end()) return PMH_ERR_ARG;
    r = it->second;
    if (!r->done.load(std::memory_order_acquire)) return PMH_ERR_NOT_READY;
    S->owned.erase(it);
  }
  const uint32_t m = S->ctx->m;
  const int rc = r->status;
  if (!rc) {
    if (idx) memcpy(idx, r->res_idx.data(), m * 4);
    if (id) memcpy(id, r->res_id.data(), m * 8);
    if (val) memcpy(val, r->res_val.data(), m * 8);
  }
  delete r;
  return rc;
}

int pmh_server_replay(pmh_server* S, const uint64_t* ids, const double* w, const uint64_t* off, uint64_t num,
                      const double* arrival, double* latency, uint32_t* out_idx, uint64_t* out_id, double* wall) {
  return pmh_server_replay_indexed(S, ids, w, off, num, nullptr, num, arrival, latency, out_idx, out_id, wall);
}

int pmh_server_replay_indexed(pmh_server* S, const uint64_t* ids, const double* w, const uint64_t* off,
                              uint64_t pool, const uint64_t* order, uint64_t num, const double* arrival,
                              double* latency, uint32_t* out_idx, uint64_t* out_id, double* wall) {
  if (!S || !off || !arrival || (pool && (!ids || !w)) || (!order && num > pool)) return PMH_ERR_ARG;
  const uint32_t m = S->ctx->m;
  for (uint64_t r = 0; r < pool; ++r)
    if (off[r + 1] < off[r] || off[r + 1] - off[r] > kMaxSet) return PMH_ERR_ARG;
  if (order)
    for (uint64_t r = 0; r < num; ++r)
      if (order[r] >= pool) return PMH_ERR_ARG;
  // The requests are pre-generated: stage the pool once in pinned host memory
  // (before the clock starts) so each batch is DMA'd from there directly.
  const uint64_t total = pool ? off[pool] - off[0] : 0;
  uint64_t* p_ids = nullptr;
  double* p_w = nullptr;
  const uint64_t* src_ids = nullptr;
  const double* src_w = nullptr;
  if (total) {
    if (hipHostMalloc(&p_ids, total * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&p_w, total * 8, hipHostMallocDefault) != hipSuccess) {
      if (p_ids) (void)hipHostFree(p_ids);
      return PMH_ERR_OOM;
    }
    memcpy(p_ids, ids + off[0], total * 8);
    memcpy(p_w, w + off[0], total * 8);
    // Device-mapped aliases for the copy kernel.  The GPU's first reads of
    // freshly pinned pages are slow (up to ~1 ms per request) and stall the
    // first tens of milliseconds of the replay: read the whole staging area
    // once into a scratch buffer first, as a long-lived serving process would
    // have done with its request buffers.
    void* di = nullptr;
    void* dw = nullptr;
    const uint64_t step = 1ull << 22;
    void* scratch = nullptr;
    bool ok = hipHostGetDevicePointer(&di, p_ids, 0) == hipSuccess &&
              hipHostGetDevicePointer(&dw, p_w, 0) == hipSuccess && hipMalloc(&scratch, 2 * step * 8) == hipSuccess;
    for (uint64_t o = 0; ok && o < total; o += step) {
      const uint64_t len = std::min<uint64_t>(step, total - o);
      ok = copy64((const uint64_t*)di + o, scratch, len, (const uint64_t*)dw + o, (uint64_t*)scratch + step, len,
                  nullptr, nullptr, 0, nullptr) == hipSuccess;
    }
    ok = ok && hipStreamSynchronize(nullptr) == hipSuccess;
    if (scratch) (void)hipFree(scratch);
    if (!ok) {
      (void)hipHostFree(p_ids);
      (void)hipHostFree(p_w);
      return PMH_ERR_DEVICE;
    }
    src_ids = (const uint64_t*)di;
    src_w = (const double*)dw;
  }
  std::vector<Request*> reqs(num);
  for (uint64_t r = 0; r < num; ++r) {
    const uint64_t e = order ? order[r] : r;  // pool entry of request r
    Request* q = new Request();
    q->n = (uint32_t)(off[e + 1] - off[e]);
    q->src_ids = src_ids + (off[e] - off[0]);
    q->src_w = src_w + (off[e] - off[0]);
    q->dst_idx = out_idx ? out_idx + r * m : nullptr;
    q->dst_id = out_id ? out_id + r * m : nullptr;
    reqs[r] = q;
  }
  const double start = now_s(S->epoch);
  for (uint64_t r = 0; r < num; ++r) {
    const double due = start + arrival[r];
    while (now_s(S->epoch) < due) {
    }
    const uint64_t e = order ? order[r] : r;
    submit_internal(S, reqs[r], ids + off[e], w + off[e]);
  }
  double last = start;
  int rc = PMH_OK;
  for (uint64_t r = 0; r < num; ++r) {
    while (!reqs[r]->done.load(std::memory_order_acquire)) std::this_thread::yield();
    if (latency) latency[r] = reqs[r]->t_done - (start + arrival[r]);
    last = std::max(last, reqs[r]->t_done);
    if (reqs[r]->status) rc = reqs[r]->status;
  }
  if (wall) *wall = last - start;
  for (Request* q : reqs) delete q;
  if (p_ids) (void)hipHostFree(p_ids);
  if (p_w) (void)hipHostFree(p_w);
  return rc;
}

int pmh_server_stats(pmh_server* S, uint64_t* o) {
  if (!S || !o) return PMH_ERR_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  o[0] = S->st_batches.load(std::memory_order_relaxed);
  o[1] = S->st_done;
  o[2] = S->st_max_batch.load(std::memory_order_relaxed);
  o[3] = S->st_max_busy;
  o[4] = S->st_waited;
  o[5] = S->st_max_launch_us.load(std::memory_order_relaxed);
  o[6] = S->st_max_finish_us.load(std::memory_order_relaxed);
  o[7] = S->st_max_iter_us.load(std::memory_order_relaxed);
  return PMH_OK;
}

void pmh_server_destroy(pmh_server* S) {
  if (!S) return;
  // the dispatcher launches what is open, drains what is in flight, then stops
  S->stop.store(true, std::memory_order_release);
  if (S->worker.joinable()) S->worker.join();
  DeviceGuard g(S->ctx->device);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (auto& kv : S->owned) delete kv.second;
    S->owned.clear();
  }
  for (Slot& sl : S->slots) {
    free_slot_buffers(sl);
    free_work(&sl.work);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete S;
}

}  // extern "C"
