// Host runtime of libpmh.so: contexts, constant tables, launches, HIP-graph
// replay, estimation and the C ABI declared in include/pmh.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/pmh.h"
#include "pmh_internal.h"
#include "pmh_runtime.h"

using namespace pmh;

namespace pmh {

uint64_t host_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint32_t imax_for(uint32_t m) {
  uint32_t bits = 0;
  for (uint32_t v = m; v; v >>= 1) ++bits;
  return 6u * m * bits + 64u;  // stream cap of ProbMinHash1/3
}

DeviceGuard::DeviceGuard(int dev) {
  (void)hipGetDevice(&prev_);
  if (prev_ != dev) (void)hipSetDevice(dev);
  dev_ = dev;
}
DeviceGuard::~DeviceGuard() {
  if (prev_ != dev_) (void)hipSetDevice(prev_);
}

size_t lds_limit_bytes(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return 65536 - lds_static_bytes();
  return p.sharedMemPerBlock - lds_static_bytes();  // budget for the dynamic part
}

int max_waves(int variant) { return (variant == 2 || variant == 4) ? 8 : 4; }

int effective_waves(const pmh_ctx* c) {
  int w = c->tune.waves;
  if (w != 1 && w != 2 && w != 4 && w != 8) w = 4;
  if (w > max_waves(c->variant)) w = max_waves(c->variant);
  while (w > 1 && lds_bytes(c->variant, c->m, w) > c->lds_limit) w >>= 1;
  return w;
}

static int waves_slot(int waves) { return waves == 1 ? 0 : waves == 2 ? 1 : waves == 4 ? 2 : 3; }

// The chain queue takes the LDS left over at the register-limited occupancy
// (the workgroups per CU with a one-batch queue), in steps of 32 entries and
// up to 8 batches: a bigger queue means fewer mid-round chain passes.
void plan_queues(pmh_ctx* c) {
  for (int waves : {1, 2, 4, 8}) {
    if (waves > max_waves(c->variant)) continue;
    const uint32_t batch = batch_size(waves);
    uint32_t best = 2 * batch;
    int occ0 = 0;
    const size_t l0 = lds_bytes_q(c->variant, c->m, waves, batch);
    if (l0 <= c->lds_limit && occupancy(c->variant, waves, l0, &occ0) == hipSuccess && occ0 >= 1) {
      for (uint32_t q = 8 * batch; q >= batch; q -= 32) {
        const size_t l = lds_bytes_q(c->variant, c->m, waves, q);
        int occ = 0;
        if (l <= c->lds_limit && occupancy(c->variant, waves, l, &occ) == hipSuccess && occ >= occ0) {
          best = q;
          break;
        }
      }
    }
    c->qcap[waves_slot(waves)] = best;
  }
}

size_t launch_lds(const pmh_ctx* c, int waves, uint32_t* qcap) {
  *qcap = c->qcap[waves_slot(waves)];
  return lds_bytes_q(c->variant, c->m, waves, *qcap);
}

void free_work(WorkBuf* wb) {
  if (wb->order) (void)hipFree(wb->order);
  if (wb->small) (void)hipFree(wb->small);
  if (wb->big_prefix) (void)hipFree(wb->big_prefix);
  if (wb->big_state) (void)hipFree(wb->big_state);
  *wb = WorkBuf{};
}

int ensure_work(pmh_ctx* c, WorkBuf* wb, uint64_t num_sets) {
  (void)c;
  if (wb->cap >= num_sets && wb->order) return PMH_OK;
  uint64_t cap = std::max<uint64_t>(num_sets, 1024);
  cap = std::max<uint64_t>(cap, wb->cap * 2);
  free_work(wb);
  if (hipMalloc(&wb->order, cap * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&wb->small, 8 * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&wb->big_prefix, (cap + 1) * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&wb->big_state, cap * sizeof(uint64_t)) != hipSuccess) {
    free_work(wb);
    return PMH_ERR_OOM;
  }
  wb->cap = cap;
  return PMH_OK;
}

HashArgs make_args(const pmh_ctx* c, const uint64_t* ids, const double* w, const uint64_t* off,
                   uint64_t num_sets, uint32_t* idx, double* val, uint64_t* id, uint64_t* keys,
                   const WorkBuf* wb) {
  HashArgs a{};
  a.ids = ids;
  a.w = w;
  a.off = off;
  a.num_sets = num_sets;
  a.out_idx = idx;
  a.out_val = val;
  a.out_id = id;
  a.out_keys = keys;
  a.seedhash = c->seedhash;
  a.m = c->m;
  a.imax = c->imax;
  a.t = c->t;
  a.c0 = c->tune.c0;
  a.grow = c->tune.grow;
  a.chain_expect = c->tune.chain_expect;
  a.mini_expect = c->tune.mini_expect;
  a.max_rounds = c->tune.max_rounds;
  a.lane_budget = c->tune.lane_budget;
  a.kmax_refresh = c->tune.kmax_refresh;
  a.status = c->status;
  if (wb) {
    const WorkArgs wa = wb->args();
    a.order = wa.order;
    a.counter = wa.counter;
    a.meta = wa.meta;
    a.big_prefix = wa.big_prefix;
    a.big_state = wa.big_state;
  }
  // A split set merges its chunks' keys in one of its own m-entry 64-bit
  // output rows (overwritten by the signature at the end); without such an
  // output no set is split.
  a.big_keys = keys ? keys : val ? reinterpret_cast<uint64_t*>(val) : id;
  a.split_log2 = a.big_keys ? (uint32_t)c->tune.split_log2 : 0u;
  a.c0_split = c->tune.c0_split;
  a.num_items = (uint32_t)num_sets;
  a.points = c->stats;
  return a;
}

int enqueue_batched(pmh_ctx* c, const HashArgs& a, WorkBuf* wb, hipStream_t s, int per_cu, int waves,
                    hipEvent_t ev0, hipEvent_t ev1) {
  if (a.num_sets == 0) return PMH_OK;
  if (waves <= 0) waves = effective_waves(c);
  HashArgs la = a;
  const size_t lds = launch_lds(c, waves, &la.qcap);
  if (per_cu <= 0) per_cu = c->tune.blocks_per_cu;
  if (per_cu <= 0) {
    if (occupancy(c->variant, waves, lds, &per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
  }
  // a split set of at most 2^20 elements has at most 2^(21 - split_log2) chunks
  const uint64_t items = a.split_log2 ? a.num_sets << (21 - a.split_log2) : a.num_sets;
  const uint64_t grid = std::min<uint64_t>((uint64_t)c->num_cu * (uint64_t)per_cu, items);
  const WorkArgs wa = wb->args();
  if (launch_order(a.off, a.num_sets, a.split_log2, wa, c->status, s) != hipSuccess) return PMH_ERR_DEVICE;
  if (a.split_log2 && launch_big_init(wa, a.m, a.big_keys, s) != hipSuccess) return PMH_ERR_DEVICE;
  if (ev0 && hipEventRecord(ev0, s) != hipSuccess) return PMH_ERR_DEVICE;
  if (launch_hash(c->variant, la, waves, (int)grid, lds, s) != hipSuccess) return PMH_ERR_DEVICE;
  if (ev1 && hipEventRecord(ev1, s) != hipSuccess) return PMH_ERR_DEVICE;
  if (a.split_log2) {
    const uint64_t fgrid = std::min<uint64_t>((uint64_t)c->num_cu * (uint64_t)per_cu, a.num_sets);
    if (launch_big_finish(c->variant, la, waves, (int)fgrid, lds, s) != hipSuccess) return PMH_ERR_DEVICE;
  }
  return PMH_OK;
}

}  // namespace pmh

// ============================================================== C ABI
extern "C" {

const char* pmh_status_str(int st) {
  switch (st) {
    case PMH_OK: return "ok";
    case PMH_ERR_ARG: return "invalid argument";
    case PMH_ERR_M_RANGE: return "signature size m out of range";
    case PMH_ERR_VARIANT_M: return "ProbMinHash3/4 need m >= 2";
    case PMH_ERR_WEIGHT: return "negative, NaN, infinite or subnormal weight";
    case PMH_ERR_SET_TOO_LARGE: return "set with more than 2^20 elements";
    case PMH_ERR_DEVICE: return "HIP runtime error";
    case PMH_ERR_OOM: return "out of memory";
    case PMH_ERR_BUSY: return "serving queue full";
    case PMH_ERR_NOT_READY: return "request not finished";
    case PMH_ERR_SCRATCH_LIMIT: return "batch exceeds the no-allocation work buffer (at most 2^20 sets)";
    case PMH_ERR_NO_ENTRY: return "no stored tuning for this device, m and variant";
    default: return "unknown status";
  }
}

uint32_t pmh_max_m(int variant) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const size_t lim = lds_limit_bytes(dev);
  uint32_t m = kMaxM;
  while (m > 1 && lds_bytes(variant, m, 1) > lim) m -= 64;
  return m;
}

int pmh_init(uint64_t seed, uint32_t m, int variant, pmh_ctx** out) {
  if (!out) return PMH_ERR_ARG;
  *out = nullptr;
  if (variant < 1 || variant > 4) return PMH_ERR_ARG;
  if (m < 1 || m > kMaxM) return PMH_ERR_M_RANGE;
  if ((variant == 3 || variant == 4) && m < 2) return PMH_ERR_VARIANT_M;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PMH_ERR_DEVICE;
  const size_t lim = lds_limit_bytes(dev);
  if (lds_bytes(variant, m, 1) > lim) return PMH_ERR_M_RANGE;
  pmh_ctx* c = new (std::nothrow) pmh_ctx();
  if (!c) return PMH_ERR_OOM;
  c->seed = seed;
  c->seedhash = host_mix64(seed);
  c->m = m;
  c->variant = variant;
  if (variant == 3) {  // later rounds resume near the previous threshold: thinner rounds pay
    c->tune.c0 = 2.0;
    c->tune.grow = 1.35;
    c->tune.max_rounds = 8;
  }
  // A workgroup holds m 8-byte keys in LDS: past m ~ 1,536 two-wave
  // workgroups leave SIMDs with under 2 waves each, and four-wave ones keep
  // 3 or more (skewed batch at m = 4096: ProbMinHash1 17.8 -> 9.7 ms,
  // ProbMinHash3 16.3 -> 8.8 ms; at m = 1024 two waves stay ahead).
  if (m > 1536) c->tune.waves = 4;
  // ProbMinHash2/4: only the chain-capable waves (those with a label array)
  // share chain elements, so four-wave workgroups (two such waves) were never
  // the fastest; two waves up to m = 2048, eight (all with arrays) at m = 4096:
  // skewed batch at m = 4096 13.9 -> 11.5 ms (ProbMinHash2), 14.3 -> 10.8 ms
  // (ProbMinHash4) against four waves; mixed batch at m = 2048 two waves
  // 26 / 34 ms against 44 / 98 ms with four.
  // Where eight do not fit (m = 8192) four waves keep one wave per SIMD in the
  // single workgroup a CU holds.
  if (variant == 2 || variant == 4) c->tune.waves = m <= 3072 ? 2 : lds_bytes(variant, m, 8) <= lim ? 8 : 4;
  // ProbMinHash2 streams that expect more than 16 points go straight to chain
  // mode instead of restarting there after their register Fisher-Yates steps
  // (mixed batch at m = 1024: 13.0 -> 12.5 ms); ProbMinHash4's threshold is
  // 32, with a per-batch choice above 16 in its ordered lane mode (mixed
  // batch 15.6 -> 15.3 ms, unit weights 12.2 -> 10.5 ms against 16).
  if (variant == 2 || variant == 4) c->tune.chain_expect = variant == 4 ? 32.0 : 16.0;
  // A split set's chunk fills its own m keys (about m (ln m + c0_split)
  // points), so larger m takes larger chunks: sets of >= 2^16 elements in
  // chunks of 2^15 above m = 2048 (skewed batch at m = 4096: ProbMinHash1
  // 9.55 -> 9.36 ms, ProbMinHash3 7.55 -> 7.37, ProbMinHash4 9.75 -> 9.47;
  // no change at m = 1024).
  if (m > 2048) c->tune.split_log2 = 16;
  c->device = dev;
  c->lds_limit = lim;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete c;
    return PMH_ERR_DEVICE;
  }
  c->num_cu = prop.multiProcessorCount;
  plan_queues(c);
  // constant tables: 6 arrays of m+1 doubles + expm1 (19) + scalars (8) + log cells (512)
  const size_t nd = 6 * (size_t)(m + 1) + 19 + 8 + 512;
  if (hipMalloc(&c->table_mem, nd * sizeof(double)) != hipSuccess) {
    delete c;
    return PMH_ERR_OOM;
  }
  double* d = (double*)c->table_mem;
  c->t.beta = d;
  c->t.lam = d + 1 * (size_t)(m + 1);
  c->t.a = d + 2 * (size_t)(m + 1);
  c->t.c1 = d + 3 * (size_t)(m + 1);
  c->t.gam = d + 4 * (size_t)(m + 1);
  c->t.dgam = d + 5 * (size_t)(m + 1);
  c->t.expm1c = d + 6 * (size_t)(m + 1);
  c->t.scal = c->t.expm1c + 19;
  c->t.ltab = c->t.scal + 8;
  c->imax = imax_for(m);
  c->t.te_rounds = kTeRoundsMax;
  c->t.redraws = kRedrawsMax;
  c->t.lemire_floor = 0;
  int rc = PMH_OK;
  if (hipMemset(c->table_mem, 0, nd * sizeof(double)) != hipSuccess) rc = PMH_ERR_DEVICE;
  if (!rc && hipMalloc(&c->status, sizeof(uint32_t)) != hipSuccess) rc = PMH_ERR_OOM;
  if (!rc && hipMemset(c->status, 0, sizeof(uint32_t)) != hipSuccess) rc = PMH_ERR_DEVICE;
#ifdef PMH_STATS
  if (!rc && hipMalloc(&c->stats, 24 * sizeof(uint64_t)) != hipSuccess) rc = PMH_ERR_OOM;
  if (!rc && hipMemset(c->stats, 0, 24 * sizeof(uint64_t)) != hipSuccess) rc = PMH_ERR_DEVICE;
#endif
  if (!rc && scratch_work(dev, &c->scratch, &c->scratch_cap) != hipSuccess) rc = PMH_ERR_DEVICE;
  if (!rc && launch_init_tables(variant, m, c->t, nullptr) != hipSuccess) rc = PMH_ERR_DEVICE;
  if (!rc && hipDeviceSynchronize() != hipSuccess) rc = PMH_ERR_DEVICE;
  double sc[8];
  if (!rc && hipMemcpy(sc, c->t.scal, sizeof(sc), hipMemcpyDeviceToHost) != hipSuccess) rc = PMH_ERR_DEVICE;
  if (!rc) {
    c->t.te_lam = sc[0];
    c->t.te_a = sc[1];
    c->t.te_c1 = sc[2];
    c->t.delta = sc[4];
  }
  if (!rc && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) rc = PMH_ERR_DEVICE;
  if (rc) {
    pmh_destroy(c);
    return rc;
  }
  *out = c;
  return PMH_OK;
}

void pmh_destroy(pmh_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  free_work(&c->work);
  free_work(&c->gwork);
  for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
  if (c->table_mem) (void)hipFree(c->table_mem);
  if (c->status) (void)hipFree(c->status);
  if (c->stats) (void)hipFree(c->stats);
  delete c;
}

static int check_hash_args(const pmh_ctx* c, const uint64_t* ids, const double* w, const uint64_t* off,
                           uint64_t num_sets) {
  if (!c) return PMH_ERR_ARG;
  if (num_sets == 0) return PMH_OK;
  if (!off || !ids || !w) return PMH_ERR_ARG;
  if (num_sets >= 0xFFFFFFFFull) return PMH_ERR_ARG;
  return PMH_OK;
}

int pmh_pminhash_sets(pmh_ctx* c, const uint64_t* ids, const double* w, const uint64_t* off, uint64_t num_sets,
                      uint32_t* idx, double* val, uint64_t* id, uint64_t* keys, void* stream) {
  int rc = check_hash_args(c, ids, w, off, num_sets);
  if (rc || num_sets == 0) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  rc = ensure_work(c, &c->work, num_sets);
  if (rc) return rc;
  HashArgs a = make_args(c, ids, w, off, num_sets, idx, val, id, keys, &c->work);
  a.split_log2 = a.big_keys ? pmin_split_log2() : 0u;
  hipStream_t s = (hipStream_t)stream;
  int per_cu = 0;
  if (occupancy_pmin(&per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
  const uint64_t items = a.split_log2 ? num_sets << (21 - a.split_log2) : num_sets;
  const uint64_t grid = std::min<uint64_t>((uint64_t)c->num_cu * (uint64_t)per_cu, items);
  const WorkArgs wa = c->work.args();
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (c->tnext < c->tcount) {
    ev0 = c->tev[2 * c->tnext];
    ev1 = c->tev[2 * c->tnext + 1];
    c->tnext++;
  }
  if (launch_order(a.off, num_sets, a.split_log2, wa, c->status, s) != hipSuccess) return PMH_ERR_DEVICE;
  if (a.split_log2 && launch_big_init(wa, a.m, a.big_keys, s) != hipSuccess) return PMH_ERR_DEVICE;
  if (ev0 && hipEventRecord(ev0, s) != hipSuccess) return PMH_ERR_DEVICE;
  if (launch_pmin(a, (int)grid, s) != hipSuccess) return PMH_ERR_DEVICE;
  if (ev1 && hipEventRecord(ev1, s) != hipSuccess) return PMH_ERR_DEVICE;
  if (a.split_log2) {
    const uint64_t fgrid = std::min<uint64_t>((uint64_t)c->num_cu * (uint64_t)per_cu, num_sets);
    if (launch_pmin_finish(a, (int)fgrid, s) != hipSuccess) return PMH_ERR_DEVICE;
  }
  return PMH_OK;
}

int pmh_hash_sets(pmh_ctx* c, const uint64_t* ids, const double* w, const uint64_t* off, uint64_t num_sets,
                  uint32_t* idx, double* val, uint64_t* id, uint64_t* keys, void* stream) {
  int rc = check_hash_args(c, ids, w, off, num_sets);
  if (rc || num_sets == 0) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  rc = ensure_work(c, &c->work, num_sets);
  if (rc) return rc;
  HashArgs a = make_args(c, ids, w, off, num_sets, idx, val, id, keys, &c->work);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (c->tnext < c->tcount) {
    ev0 = c->tev[2 * c->tnext];
    ev1 = c->tev[2 * c->tnext + 1];
    c->tnext++;
  }
  return enqueue_batched(c, a, &c->work, (hipStream_t)stream, 0, 0, ev0, ev1);
}

int pmh_hash_sets_noalloc(pmh_ctx* c, const uint64_t* ids, const double* w, const uint64_t* off,
                          uint64_t num_sets, uint32_t* idx, double* val, uint64_t* id, uint64_t* keys,
                          void* stream) {
  int rc = check_hash_args(c, ids, w, off, num_sets);
  if (rc || num_sets == 0) return rc;
  if (num_sets > c->scratch_cap) return PMH_ERR_SCRATCH_LIMIT;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  // a view of the device's static array, found at pmh_init; never freed
  WorkBuf wb;
  wb.order = c->scratch.order;
  wb.small = c->scratch.counter;
  wb.big_prefix = c->scratch.big_prefix;
  wb.big_state = c->scratch.big_state;
  wb.cap = c->scratch_cap;
  HashArgs a = make_args(c, ids, w, off, num_sets, idx, val, id, keys, &wb);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (c->tnext < c->tcount) {
    ev0 = c->tev[2 * c->tnext];
    ev1 = c->tev[2 * c->tnext + 1];
    c->tnext++;
  }
  return enqueue_batched(c, a, &wb, (hipStream_t)stream, 0, 0, ev0, ev1);
}

int pmh_hash_sets_bbit(pmh_ctx* c, const uint64_t* ids, const double* w, const uint64_t* off, uint64_t num_sets,
                       uint32_t b, uint64_t* out_bbit, uint32_t* idx, double* val, uint64_t* id, uint64_t* keys,
                       void* stream) {
  int rc = check_hash_args(c, ids, w, off, num_sets);
  if (rc || num_sets == 0) return rc;
  if (!out_bbit || !(b == 1 || b == 2 || b == 4 || b == 8 || b == 16)) return PMH_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  rc = ensure_work(c, &c->work, num_sets);
  if (rc) return rc;
  HashArgs a = make_args(c, ids, w, off, num_sets, idx, val, id, keys, &c->work);
  a.out_bbit = out_bbit;
  a.bbit_b = b;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (c->tnext < c->tcount) {
    ev0 = c->tev[2 * c->tnext];
    ev1 = c->tev[2 * c->tnext + 1];
    c->tnext++;
  }
  return enqueue_batched(c, a, &c->work, (hipStream_t)stream, 0, 0, ev0, ev1);
}

int pmh_hash_sets_binary(pmh_ctx* c, const uint64_t* ids, const uint64_t* off, uint64_t num_sets, uint32_t* idx,
                         double* val, uint64_t* id, uint64_t* keys, void* stream) {
  if (!c) return PMH_ERR_ARG;
  if (num_sets == 0) return PMH_OK;
  if (!off || !ids || num_sets >= 0xFFFFFFFFull) return PMH_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  int rc = ensure_work(c, &c->work, num_sets);
  if (rc) return rc;
  HashArgs a = make_args(c, ids, nullptr, off, num_sets, idx, val, id, keys, &c->work);
  a.binary = 1;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (c->tnext < c->tcount) {
    ev0 = c->tev[2 * c->tnext];
    ev1 = c->tev[2 * c->tnext + 1];
    c->tnext++;
  }
  return enqueue_batched(c, a, &c->work, (hipStream_t)stream, 0, 0, ev0, ev1);
}

int pmh_update_sets(pmh_ctx* c, const uint64_t* ids, const double* w, const uint64_t* off, uint64_t num_sets,
                    uint32_t* counts, uint64_t* keys, uint32_t* idx, double* val, uint64_t* id, void* stream) {
  if (!c) return PMH_ERR_ARG;
  if (num_sets == 0) return PMH_OK;
  if (!off || !ids || !counts || !keys || num_sets >= 0xFFFFFFFFull) return PMH_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  int rc = ensure_work(c, &c->work, num_sets);
  if (rc) return rc;
  HashArgs a = make_args(c, ids, w, off, num_sets, idx, val, id, keys, &c->work);
  a.binary = w ? 0u : 1u;
  a.counts = counts;
  a.split_log2 = 0;  // every set in one workgroup: its previous keys seed the minima in LDS
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (c->tnext < c->tcount) {
    ev0 = c->tev[2 * c->tnext];
    ev1 = c->tev[2 * c->tnext + 1];
    c->tnext++;
  }
  return enqueue_batched(c, a, &c->work, (hipStream_t)stream, 0, 0, ev0, ev1);
}

int pmh_timing_begin(pmh_ctx* c, int n) {
  if (!c || n < 0 || n > 1 << 16) return PMH_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  while ((int)c->tev.size() < 2 * n) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return PMH_ERR_DEVICE;
    c->tev.push_back(e);
  }
  c->tnext = 0;
  c->tcount = n;
  return PMH_OK;
}

int pmh_timing_read(pmh_ctx* c, float* ms, int n) {
  if (!c || !ms || n < 0) return PMH_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  if (n > c->tnext) return PMH_ERR_NOT_READY;
  for (int k = 0; k < n; ++k) {
    if (hipEventSynchronize(c->tev[2 * k + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms[k], c->tev[2 * k], c->tev[2 * k + 1]) != hipSuccess)
      return PMH_ERR_DEVICE;
  }
  c->tcount = 0;
  return PMH_OK;
}

int pmh_hash_sets_plain(pmh_ctx* c, const uint64_t* ids, const double* w, const uint64_t* off,
                        uint64_t num_sets, uint32_t* idx, double* val, uint64_t* id, uint64_t* keys,
                        void* stream) {
  int rc = check_hash_args(c, ids, w, off, num_sets);
  if (rc || num_sets == 0) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  HashArgs a = make_args(c, ids, w, off, num_sets, idx, val, id, keys, nullptr);
  const int waves = effective_waves(c);
  const size_t lds = launch_lds(c, waves, &a.qcap);
  for (uint64_t s = 0; s < num_sets; ++s)
    if (launch_hash_one(c->variant, a, s, waves, lds, (hipStream_t)stream) != hipSuccess) return PMH_ERR_DEVICE;
  return PMH_OK;
}

int pmh_hash_sets_graph(pmh_ctx* c, const uint64_t* ids, const double* w, const uint64_t* off,
                        uint64_t num_sets, uint32_t* idx, double* val, uint64_t* id, uint64_t* keys,
                        void* stream) {
  int rc = check_hash_args(c, ids, w, off, num_sets);
  if (rc || num_sets == 0) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  const GraphKey key{ids, w, off, num_sets, idx, val, id, keys, c->tune_version};
  if (!c->gexec || !(key == c->gkey)) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    // The graph keeps the device addresses of its work buffer: it owns one
    // that no other call reallocates (the shared one grows with later calls).
    rc = ensure_work(c, &c->gwork, num_sets);
    if (rc) return rc;
    HashArgs a = make_args(c, ids, w, off, num_sets, idx, val, id, keys, &c->gwork);
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return PMH_ERR_DEVICE;
    rc = enqueue_batched(c, a, &c->gwork, c->cap_stream);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &gr);
    if (rc) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    if (e != hipSuccess || !gr) return PMH_ERR_DEVICE;
    if (hipGraphInstantiate(&c->gexec, gr, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(gr);
      return PMH_ERR_DEVICE;
    }
    c->graph = gr;
    c->gkey = key;
  }
  return hipGraphLaunch(c->gexec, (hipStream_t)stream) == hipSuccess ? PMH_OK : PMH_ERR_DEVICE;
}

int pmh_get_status(pmh_ctx* c, void* stream) {
  if (!c) return PMH_ERR_ARG;
  DeviceGuard g(c->device);
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PMH_ERR_DEVICE;
  uint32_t st = 0;
  if (hipMemcpy(&st, c->status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return PMH_ERR_DEVICE;
  if (st && hipMemset(c->status, 0, sizeof(uint32_t)) != hipSuccess) return PMH_ERR_DEVICE;
  if (st & kStatusWeight) return PMH_ERR_WEIGHT;
  if (st & kStatusSetTooLarge) return PMH_ERR_SET_TOO_LARGE;
  return PMH_OK;
}

int pmh_set_tuning(pmh_ctx* c, const pmh_tuning* t) {
  if (!c || !t) return PMH_ERR_ARG;
  if (!(t->grow > 1.0) || t->max_rounds < 1 || t->lane_budget < 1 || t->kmax_refresh < 1 ||
      (t->waves != 1 && t->waves != 2 && t->waves != 4 && t->waves != 8) || t->blocks_per_cu < 0 ||
      !(t->c0 > -100.0) ||
      !(t->chain_expect >= 0.0) || !(t->mini_expect >= 0.0) || t->split_log2 < 0 || t->split_log2 == 1 ||
      t->split_log2 > 21 || !(t->c0_split > -100.0) || !(t->c0_split < 1e6))
    return PMH_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->tune.c0 = t->c0;
  c->tune.grow = t->grow;
  c->tune.max_rounds = t->max_rounds;
  c->tune.chain_expect = t->chain_expect;
  c->tune.lane_budget = t->lane_budget;
  c->tune.waves = t->waves;
  c->tune.kmax_refresh = t->kmax_refresh;
  c->tune.blocks_per_cu = t->blocks_per_cu;
  c->tune.mini_expect = t->mini_expect;
  c->tune.split_log2 = t->split_log2;
  c->tune.c0_split = t->c0_split;
  c->tune_version++;
  return PMH_OK;
}

int pmh_set_caps(pmh_ctx* c, uint32_t imax, uint32_t te_rounds, uint32_t redraws, uint32_t lemire_floor) {
  if (!c || imax > kImaxMax || te_rounds < 1 || te_rounds > kTeRoundsMax || redraws > kRedrawsMax ||
      (lemire_floor & 15u))
    return PMH_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->imax = imax ? imax : imax_for(c->m);
  c->t.te_rounds = te_rounds;
  c->t.redraws = redraws;
  c->t.lemire_floor = lemire_floor;
  c->tune_version++;  // a cached graph holds the previous caps
  return PMH_OK;
}

int pmh_get_tuning(const pmh_ctx* c, pmh_tuning* t) {
  if (!c || !t) return PMH_ERR_ARG;
  t->c0 = c->tune.c0;
  t->grow = c->tune.grow;
  t->max_rounds = c->tune.max_rounds;
  t->chain_expect = c->tune.chain_expect;
  t->lane_budget = c->tune.lane_budget;
  t->waves = c->tune.waves;
  t->kmax_refresh = c->tune.kmax_refresh;
  t->blocks_per_cu = c->tune.blocks_per_cu;
  t->mini_expect = c->tune.mini_expect;
  t->split_log2 = c->tune.split_log2;
  t->c0_split = c->tune.c0_split;
  return PMH_OK;
}

int pmh_estimate(const uint64_t* idA, const uint32_t* idxA, const uint64_t* idB, const uint32_t* idxB,
                 uint32_t m, double* out) {
  if (!idA || !idxA || !idB || !idxB || !out || m == 0) return PMH_ERR_ARG;
  uint64_t eq = 0;
  for (uint32_t k = 0; k < m; ++k)
    eq += (idA[k] == idB[k] && idxA[k] != 0xFFFFFFFFu && idxB[k] != 0xFFFFFFFFu) ? 1u : 0u;
  *out = (double)eq / (double)m;
  return PMH_OK;
}

int pmh_estimate_pairs(const uint64_t* idA, const uint32_t* idxA, const uint64_t* idB, const uint32_t* idxB,
                       uint32_t m, uint64_t pairs, uint32_t* counts, void* stream) {
  if (pairs == 0) return PMH_OK;
  if (!idA || !idxA || !idB || !idxB || !counts || m == 0 || pairs > 0x7FFFFFFFull) return PMH_ERR_ARG;
  return launch_estimate(idA, idxA, idB, idxB, m, pairs, counts, (hipStream_t)stream) == hipSuccess
             ? PMH_OK
             : PMH_ERR_DEVICE;
}

int pmh_allpairs_counts(const uint32_t* fp, uint32_t k, uint32_t m, uint16_t* counts, void* stream) {
  if (k == 0) return PMH_OK;
  if (!fp || !counts || m == 0) return PMH_ERR_ARG;
  return launch_allpairs(fp, k, m, counts, (hipStream_t)stream) == hipSuccess ? PMH_OK : PMH_ERR_DEVICE;
}

static bool bbit_ok(uint32_t b) { return b == 1 || b == 2 || b == 4 || b == 8 || b == 16; }

int pmh_bbit_pack(const uint64_t* id, uint64_t num_sigs, uint32_t m, uint32_t b, uint64_t* out, void* stream) {
  if (num_sigs == 0) return PMH_OK;
  if (!id || !out || m == 0 || m > kMaxM || !bbit_ok(b)) return PMH_ERR_ARG;
  return launch_bbit_pack(id, num_sigs, m, b, out, (hipStream_t)stream) == hipSuccess ? PMH_OK : PMH_ERR_DEVICE;
}

int pmh_bbit_allpairs(const uint64_t* sig, uint32_t k, uint32_t m, uint32_t b, uint16_t* counts, void* stream) {
  if (k == 0) return PMH_OK;
  if (!sig || !counts || m == 0 || m > kMaxM || !bbit_ok(b)) return PMH_ERR_ARG;
  return launch_bbit_allpairs(sig, k, m, b, counts, (hipStream_t)stream) == hipSuccess ? PMH_OK : PMH_ERR_DEVICE;
}

int pmh_get_table(pmh_ctx* c, int which, double* out, uint32_t count) {
  if (!c || !out) return PMH_ERR_ARG;
  DeviceGuard g(c->device);
  const double* src = nullptr;
  size_t avail = 0;
  switch (which) {
    case 0: src = c->t.beta; avail = c->m + 1; break;
    case 1: src = c->t.lam; avail = c->m; break;
    case 2: src = c->t.a; avail = c->m; break;
    case 3: src = c->t.c1; avail = c->m; break;
    case 5: src = c->t.gam; avail = c->m; break;
    case 6: src = c->t.dgam; avail = c->m; break;
    case 7: src = c->t.scal; avail = 8; break;
    case 8: src = c->t.expm1c; avail = 19; break;
    case 9: src = c->t.ltab; avail = 512; break;
    default: return PMH_ERR_ARG;
  }
  if (count > avail) return PMH_ERR_ARG;
  if (hipDeviceSynchronize() != hipSuccess) return PMH_ERR_DEVICE;
  return hipMemcpy(out, src, count * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess ? PMH_OK : PMH_ERR_DEVICE;
}

int pmh_debug_eval(pmh_ctx* c, int what, const double* in, const uint64_t* in_u, double* out, uint64_t* out_u,
                   uint64_t n, void* stream) {
  if (!c || what < 0 || what > 12) return PMH_ERR_ARG;
  const bool uses_u = (what >= 3 && what <= 7) || what >= 9;
  const bool out_is_u = what == 4 || what == 6 || what == 7 || what >= 9;
  if ((uses_u && !in_u) || (!uses_u && !in) || (out_is_u && !out_u) || (!out_is_u && !out)) return PMH_ERR_ARG;
  if (what == 5 && c->variant != 3) return PMH_ERR_ARG;
  DeviceGuard g(c->device);
  return launch_debug_eval(what, in, in_u, out, out_u, n, c->m, c->variant, c->t, (hipStream_t)stream) == hipSuccess
             ? PMH_OK
             : PMH_ERR_DEVICE;
}

#ifdef PMH_STATS
// Statistics build only (not part of the product ABI): read and optionally
// reset the 24 event and cycle counters accumulated by the kernels.
int pmh_stats_read(pmh_ctx* c, uint64_t* out24, int reset) {
  if (!c || !out24 || !c->stats) return PMH_ERR_ARG;
  DeviceGuard g(c->device);
  if (hipDeviceSynchronize() != hipSuccess) return PMH_ERR_DEVICE;
  if (hipMemcpy(out24, c->stats, 24 * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess) return PMH_ERR_DEVICE;
  if (reset && hipMemset(c->stats, 0, 24 * sizeof(uint64_t)) != hipSuccess) return PMH_ERR_DEVICE;
  return PMH_OK;
}
#endif

}  // extern "C"
