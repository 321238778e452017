// Continuous-batching server for single-set signature requests.
//
// A dispatcher thread owns `slots` execution slots (stream, event, device
// buffers, pinned staging, work list).  Whenever a slot is free and requests
// are pending it admits as many as fit the slot's element capacity and the
// server's HBM budget, packs them into pinned memory, copies them to the
// device, runs the heavy-first persistent kernel on the slot's stream and
// copies the signatures back.  Several slots run at once, so requests that
// arrive while batches are on the GPU start as soon as any slot frees.  Each
// slot's persistent grid is limited to its share of the CUs' workgroup (LDS)
// capacity so concurrent batches co-reside.  Results do not depend on batch
// composition (the signature is a pure function of the set).
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
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
  const uint64_t* ids = nullptr;
  const double* w = nullptr;
  std::vector<uint64_t> own_ids;
  std::vector<double> own_w;
  uint32_t* dst_idx = nullptr;  // result destinations (replay) ...
  uint64_t* dst_id = nullptr;
  double* dst_val = nullptr;
  std::vector<uint32_t> res_idx;  // ... or owned results (submit/fetch)
  std::vector<uint64_t> res_id;
  std::vector<double> res_val;
  bool owned = false;
  double t_done = 0.0;
  std::atomic<bool> done{false};
};

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
  uint64_t* h_off = nullptr;
  uint32_t* h_idx = nullptr;
  uint64_t* h_id = nullptr;
  double* h_val = nullptr;
  uint64_t elems_cap = 0;
  uint32_t sets_cap = 0;
  std::vector<Request*> batch;
  uint64_t bytes = 0;
  bool busy = false;
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
  free_slot_buffers(s);
  const uint64_t e = elems ? elems : 1, r = (uint64_t)sets * m;
  bool ok = hipMalloc(&s.d_ids, e * 8) == hipSuccess && hipMalloc(&s.d_w, e * 8) == hipSuccess &&
            hipMalloc(&s.d_off, (sets + 1) * 8ull) == hipSuccess && hipMalloc(&s.d_idx, r * 4) == hipSuccess &&
            hipMalloc(&s.d_id, r * 8) == hipSuccess && hipMalloc(&s.d_val, r * 8) == hipSuccess &&
            hipHostMalloc(&s.h_ids, e * 8, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&s.h_w, e * 8, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&s.h_off, (sets + 1) * 8ull, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&s.h_idx, r * 4, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&s.h_id, r * 8, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&s.h_val, r * 8, hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    free_slot_buffers(s);
    return PMH_ERR_OOM;
  }
  s.elems_cap = e;
  s.sets_cap = sets;
  return PMH_OK;
}

double now_s(Clock::time_point epoch) {
  return std::chrono::duration<double>(Clock::now() - epoch).count();
}

}  // namespace

struct pmh_server {
  pmh_ctx* ctx = nullptr;
  std::vector<Slot> slots;
  uint64_t hbm_budget = 0, hbm_used = 0;
  std::mutex mu;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Request*> owned;  // submit/fetch requests by ticket
  std::atomic<bool> stop{false};
  std::thread worker;
  uint64_t next_ticket = 1;
  Clock::time_point epoch;
  int per_cu = 1;
  int waves = 4;
  std::atomic<int> busy{0};
  uint64_t st_batches = 0, st_done = 0, st_max_batch = 0, st_max_busy = 0;
  std::atomic<uint64_t> st_waited{0};
  size_t max_pending = 1u << 22;
  int fatal = PMH_OK;
};

namespace {

uint64_t request_bytes(const pmh_server* S, uint32_t n) {
  return (uint64_t)n * 16 + (uint64_t)S->ctx->m * 20 + 8;
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
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->hbm_used -= sl.bytes;
    S->st_done += sl.batch.size();
  }
  sl.batch.clear();
  sl.bytes = 0;
  sl.busy = false;
  S->busy.fetch_sub(1);
}

int launch(pmh_server* S, Slot& sl, std::vector<Request*>& b, uint64_t elems) {
  pmh_ctx* c = S->ctx;
  const uint32_t m = c->m;
  if (elems > sl.elems_cap || b.size() > sl.sets_cap) {
    (void)hipStreamSynchronize(sl.stream);
    const int rc = alloc_slot_buffers(sl, std::max<uint64_t>(elems, sl.elems_cap),
                                      std::max<uint32_t>((uint32_t)b.size(), sl.sets_cap), m);
    if (rc) return rc;
  }
  uint64_t off = 0;
  sl.h_off[0] = 0;
  for (size_t k = 0; k < b.size(); ++k) {
    memcpy(sl.h_ids + off, b[k]->ids, (size_t)b[k]->n * 8);
    memcpy(sl.h_w + off, b[k]->w, (size_t)b[k]->n * 8);
    off += b[k]->n;
    sl.h_off[k + 1] = off;
  }
  const uint64_t nb = b.size();
  if (ensure_work(c, &sl.work, nb)) return PMH_ERR_OOM;
  if (hipMemcpyAsync(sl.d_ids, sl.h_ids, off * 8, hipMemcpyHostToDevice, sl.stream) != hipSuccess ||
      hipMemcpyAsync(sl.d_w, sl.h_w, off * 8, hipMemcpyHostToDevice, sl.stream) != hipSuccess ||
      hipMemcpyAsync(sl.d_off, sl.h_off, (nb + 1) * 8, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
    return PMH_ERR_DEVICE;
  HashArgs a = make_args(c, sl.d_ids, sl.d_w, sl.d_off, nb, sl.d_idx, sl.d_val, sl.d_id, nullptr, &sl.work);
  const size_t lds = lds_bytes(c->variant, m, S->waves);
  uint64_t grid = std::min<uint64_t>((uint64_t)c->num_cu * (uint64_t)S->per_cu, nb);
  if (launch_order(a.off, nb, sl.work.order, sl.work.counter, c->status, sl.stream) != hipSuccess ||
      launch_hash(c->variant, a, S->waves, (int)grid, lds, sl.stream) != hipSuccess)
    return PMH_ERR_DEVICE;
  if (hipMemcpyAsync(sl.h_idx, sl.d_idx, nb * m * 4, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
      hipMemcpyAsync(sl.h_id, sl.d_id, nb * m * 8, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
      hipMemcpyAsync(sl.h_val, sl.d_val, nb * m * 8, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
      hipEventRecord(sl.ev, sl.stream) != hipSuccess)
    return PMH_ERR_DEVICE;
  sl.batch.swap(b);
  sl.busy = true;
  const int nbusy = S->busy.fetch_add(1) + 1;
  S->st_batches++;
  S->st_max_batch = std::max<uint64_t>(S->st_max_batch, nb);
  S->st_max_busy = std::max<uint64_t>(S->st_max_busy, (uint64_t)nbusy);
  return PMH_OK;
}

void worker_loop(pmh_server* S) {
  (void)hipSetDevice(S->ctx->device);
  while (!S->stop.load(std::memory_order_acquire)) {
    bool progressed = false;
    for (Slot& sl : S->slots) {
      if (sl.busy && hipEventQuery(sl.ev) == hipSuccess) {
        finish(S, sl);
        progressed = true;
      }
    }
    for (Slot& sl : S->slots) {
      if (sl.busy) continue;
      std::vector<Request*> b;
      uint64_t elems = 0, bytes = 0;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        while (!S->pending.empty()) {
          Request* r = S->pending.front();
          const uint64_t rb = request_bytes(S, r->n);
          if (!b.empty() && (elems + r->n > sl.elems_cap || b.size() >= sl.sets_cap)) break;
          // HBM admission: the first request of an idle server is always admitted
          if (S->hbm_used + bytes + rb > S->hbm_budget && !(b.empty() && S->hbm_used == 0)) break;
          b.push_back(r);
          S->pending.pop_front();
          elems += r->n;
          bytes += rb;
        }
        if (!b.empty()) S->hbm_used += bytes;
      }
      if (b.empty()) break;
      sl.bytes = bytes;
      const int rc = launch(S, sl, b, elems);
      if (rc) {
        // fail the batch: mark done with empty results so callers never hang
        std::lock_guard<std::mutex> lk(S->mu);
        S->fatal = rc;
        S->hbm_used -= bytes;
        for (Request* r : b) {
          r->t_done = now_s(S->epoch);
          r->done.store(true, std::memory_order_release);
        }
        continue;
      }
      progressed = true;
    }
    if (!progressed) std::this_thread::yield();
  }
  for (Slot& sl : S->slots)
    if (sl.busy) {
      (void)hipEventSynchronize(sl.ev);
      finish(S, sl);
    }
}

}  // namespace

extern "C" {

int pmh_server_create(pmh_ctx* c, int slots, uint64_t slot_elems, uint32_t slot_sets, uint64_t hbm_budget_bytes,
                      pmh_server** out) {
  if (!c || !out || slots < 1 || slots > 16 || slot_sets < 1) return PMH_ERR_ARG;
  *out = nullptr;
  DeviceGuard g(c->device);
  pmh_server* S = new (std::nothrow) pmh_server();
  if (!S) return PMH_ERR_OOM;
  S->ctx = c;
  S->hbm_budget = hbm_budget_bytes ? hbm_budget_bytes : ~0ull;
  S->epoch = Clock::now();
  S->waves = effective_waves(c);
  int occ = 1;
  if (occupancy(c->variant, S->waves, lds_bytes(c->variant, c->m, S->waves), &occ) != hipSuccess || occ < 1) occ = 1;
  S->per_cu = std::max(1, occ / slots);  // LDS/workgroup share of each slot
  S->slots.resize(slots);
  int rc = PMH_OK;
  for (Slot& sl : S->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
      rc = PMH_ERR_DEVICE;
      break;
    }
    rc = alloc_slot_buffers(sl, slot_elems, slot_sets, c->m);
    if (rc) break;
    rc = ensure_work(c, &sl.work, slot_sets);
    if (rc) break;
  }
  if (rc) {
    for (Slot& sl : S->slots) {
      free_slot_buffers(sl);
      if (sl.work.order) (void)hipFree(sl.work.order);
      if (sl.work.counter) (void)hipFree(sl.work.counter);
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
  r->own_ids.assign(ids, ids + n);
  r->own_w.assign(w, w + n);
  r->ids = r->own_ids.data();
  r->w = r->own_w.data();
  r->owned = true;
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->pending.size() >= S->max_pending) {
    delete r;
    return PMH_ERR_BUSY;
  }
  r->ticket = S->next_ticket++;
  if (S->busy.load() == (int)S->slots.size()) S->st_waited++;
  S->owned[r->ticket] = r;
  S->pending.push_back(r);
  *ticket = r->ticket;
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
  int rc = r->res_idx.size() == m ? PMH_OK : (S->fatal ? S->fatal : PMH_ERR_DEVICE);
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
  if (!S || !off || !arrival || (num && (!ids || !w))) return PMH_ERR_ARG;
  const uint32_t m = S->ctx->m;
  std::vector<Request*> reqs(num);
  for (uint64_t r = 0; r < num; ++r) {
    const uint64_t n = off[r + 1] - off[r];
    if (off[r + 1] < off[r] || n > kMaxSet) {
      for (uint64_t q = 0; q < r; ++q) delete reqs[q];
      return PMH_ERR_ARG;
    }
    Request* q = new Request();
    q->n = (uint32_t)n;
    q->ids = ids + off[r];
    q->w = w + off[r];
    q->dst_idx = out_idx ? out_idx + r * m : nullptr;
    q->dst_id = out_id ? out_id + r * m : nullptr;
    reqs[r] = q;
  }
  const double start = now_s(S->epoch);
  for (uint64_t r = 0; r < num; ++r) {
    const double due = start + arrival[r];
    while (now_s(S->epoch) < due) {
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->busy.load() == (int)S->slots.size()) S->st_waited++;
    S->pending.push_back(reqs[r]);
  }
  double last = start;
  for (uint64_t r = 0; r < num; ++r) {
    while (!reqs[r]->done.load(std::memory_order_acquire)) std::this_thread::yield();
    if (latency) latency[r] = reqs[r]->t_done - (start + arrival[r]);
    last = std::max(last, reqs[r]->t_done);
  }
  if (wall) *wall = last - start;
  for (Request* q : reqs) delete q;
  return S->fatal;
}

int pmh_server_stats(pmh_server* S, uint64_t* o) {
  if (!S || !o) return PMH_ERR_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  o[0] = S->st_batches;
  o[1] = S->st_done;
  o[2] = S->st_max_batch;
  o[3] = S->st_max_busy;
  o[4] = S->st_waited.load();
  return PMH_OK;
}

void pmh_server_destroy(pmh_server* S) {
  if (!S) return;
  S->stop.store(true, std::memory_order_release);
  if (S->worker.joinable()) S->worker.join();
  DeviceGuard g(S->ctx->device);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (Request* r : S->pending)
      if (!r->owned) r->done.store(true);
    for (auto& kv : S->owned) delete kv.second;
    S->owned.clear();
    S->pending.clear();
  }
  for (Slot& sl : S->slots) {
    free_slot_buffers(sl);
    if (sl.work.order) (void)hipFree(sl.work.order);
    if (sl.work.counter) (void)hipFree(sl.work.counter);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete S;
}

}  // extern "C"
