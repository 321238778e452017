// Schedule autotuner: coordinate descent over the per-set schedule knobs,
// timing the batched launch with HIP events on the caller's batch.  None of
// the knobs changes a result; they trade points generated against launch
// shape and occupancy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pmh.h"
#include "pmh_runtime.h"

using namespace pmh;

namespace {

double time_once(pmh_ctx* c, const HashArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int* rc) {
  (void)hipEventRecord(e0, s);
  *rc = enqueue_batched(c, a, &c->work, s);
  (void)hipEventRecord(e1, s);
  if (*rc) return 1e30;
  if (hipEventSynchronize(e1) != hipSuccess) {
    *rc = PMH_ERR_DEVICE;
    return 1e30;
  }
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  return ms;
}

double measure(pmh_ctx* c, const HashArgs& base, int trials, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int* rc) {
  HashArgs a = make_args(c, base.ids, base.w, base.off, base.num_sets, nullptr, nullptr, nullptr, base.out_keys,
                         &c->work);
  time_once(c, a, s, e0, e1, rc);  // warm-up
  if (*rc) return 1e30;
  std::vector<double> v;
  for (int t = 0; t < trials; ++t) {
    v.push_back(time_once(c, a, s, e0, e1, rc));
    if (*rc) return 1e30;
  }
  std::sort(v.begin(), v.end());
  return v[v.size() / 2];
}

}  // namespace

// Key of a stored tuning: the device architecture and compute-unit count,
// m and the variant (the schedule's best knobs depend on all four).
static int tuning_key(const pmh_ctx* c, std::string* key) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, c->device) != hipSuccess) return PMH_ERR_DEVICE;
  std::ostringstream os;
  os << p.gcnArchName << ' ' << p.multiProcessorCount << ' ' << c->m << ' ' << c->variant;
  *key = os.str();
  return PMH_OK;
}

// Tunings are stored one per line: "<arch> <CUs> <m> <variant>" and the 11
// knobs in pmh_tuning order.
extern "C" int pmh_tuning_save(const pmh_ctx* c, const char* path) {
  if (!c || !path) return PMH_ERR_ARG;
  std::string key;
  int rc = tuning_key(c, &key);
  if (rc) return rc;
  std::vector<std::string> keep;
  {
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line))
      if (!line.empty() && line.compare(0, key.size() + 1, key + " ") != 0) keep.push_back(line);
  }
  char buf[512];
  const Tuning& t = c->tune;
  snprintf(buf, sizeof buf, "%s %.17g %.17g %d %.17g %d %d %d %d %.17g %d %.17g", key.c_str(), t.c0, t.grow,
           t.max_rounds, t.chain_expect, t.lane_budget, t.waves, t.kmax_refresh, t.blocks_per_cu, t.mini_expect,
           t.split_log2, t.c0_split);
  keep.push_back(buf);
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return PMH_ERR_ARG;
    for (const std::string& l : keep) out << l << '\n';
    if (!out) return PMH_ERR_ARG;
  }
  return std::rename(tmp.c_str(), path) == 0 ? PMH_OK : PMH_ERR_ARG;
}

extern "C" int pmh_tuning_load(pmh_ctx* c, const char* path) {
  if (!c || !path) return PMH_ERR_ARG;
  std::string key;
  int rc = tuning_key(c, &key);
  if (rc) return rc;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    if (line.compare(0, key.size() + 1, key + " ") != 0) continue;
    std::istringstream is(line.substr(key.size() + 1));
    pmh_tuning t;
    if (!(is >> t.c0 >> t.grow >> t.max_rounds >> t.chain_expect >> t.lane_budget >> t.waves >> t.kmax_refresh >>
          t.blocks_per_cu >> t.mini_expect >> t.split_log2 >> t.c0_split))
      return PMH_ERR_ARG;
    return pmh_set_tuning(c, &t);
  }
  return PMH_ERR_NO_ENTRY;
}

extern "C" int pmh_autotune(pmh_ctx* c, const uint64_t* ids, const double* w, const uint64_t* off, uint64_t num_sets,
                            int trials, void* stream, pmh_tuning* best_out) {
  if (!c || !ids || !w || !off || num_sets == 0 || num_sets >= 0xFFFFFFFFull) return PMH_ERR_ARG;
  if (trials < 1) trials = 1;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  int rc = ensure_work(c, &c->work, num_sets);
  if (rc) return rc;
  // key rows of the timed launches (also the merge rows of split sets)
  uint64_t* kbuf = nullptr;
  if (hipMalloc(&kbuf, num_sets * (uint64_t)c->m * sizeof(uint64_t)) != hipSuccess) return PMH_ERR_OOM;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipFree(kbuf);
    return PMH_ERR_DEVICE;
  }
  HashArgs base = make_args(c, ids, w, off, num_sets, nullptr, nullptr, nullptr, kbuf, &c->work);
  Tuning best = c->tune;
  double best_ms = measure(c, base, trials, s, e0, e1, &rc);
  // coordinate descent, one knob at a time, two sweeps
  for (int sweep = 0; sweep < 2 && !rc; ++sweep) {
    for (int knob = 0; knob < 7 && !rc; ++knob) {
      std::vector<Tuning> cands;
      auto add = [&](auto setter) {
        Tuning t = best;
        setter(t);
        cands.push_back(t);
      };
      switch (knob) {
        case 0:
          for (int wv : {1, 2, 4, 8})
            if (wv <= max_waves(c->variant) && lds_bytes(c->variant, c->m, wv) <= c->lds_limit)
              add([&](Tuning& t) { t.waves = wv; });
          break;
        case 1:
          for (double c0 : {1.0, 2.0, 3.0, 4.0, 6.0})
            for (double g : {1.35, 2.0})
              add([&](Tuning& t) {
                t.c0 = c0;
                t.grow = g;
                t.max_rounds = g < 1.5 ? 8 : 4;
              });
          break;
        case 2:
          for (double ce : {16.0, 32.0, 48.0, 96.0, 192.0}) add([&](Tuning& t) { t.chain_expect = ce; });
          for (double me : {3.0, 12.0, 24.0, 48.0, 96.0}) add([&](Tuning& t) { t.mini_expect = me; });
          break;
        case 3:
          for (int lb : {2, 4, 8, 16}) add([&](Tuning& t) { t.lane_budget = lb; });
          break;
        case 4:
          for (int kr : {1, 4, 16}) add([&](Tuning& t) { t.kmax_refresh = kr; });
          break;
        case 5:
          for (int bp : {0, 1, 2, 4, 8}) add([&](Tuning& t) { t.blocks_per_cu = bp; });
          break;
        case 6:
          for (int sl : {0, 12, 13, 14, 15, 16, 17}) add([&](Tuning& t) { t.split_log2 = sl; });
          break;
      }
      for (const Tuning& t : cands) {
        c->tune = t;
        base = make_args(c, ids, w, off, num_sets, nullptr, nullptr, nullptr, kbuf, &c->work);
        const double ms = measure(c, base, trials, s, e0, e1, &rc);
        if (rc) break;
        if (ms < best_ms * 0.98) {
          best_ms = ms;
          best = t;
        }
      }
    }
  }
  c->tune = best;
  c->tune_version++;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(kbuf);
  if (best_out) {
    best_out->c0 = best.c0;
    best_out->grow = best.grow;
    best_out->max_rounds = best.max_rounds;
    best_out->chain_expect = best.chain_expect;
    best_out->lane_budget = best.lane_budget;
    best_out->waves = best.waves;
    best_out->kmax_refresh = best.kmax_refresh;
    best_out->blocks_per_cu = best.blocks_per_cu;
    best_out->mini_expect = best.mini_expect;
    best_out->split_log2 = best.split_log2;
    best_out->c0_split = best.c0_split;
  }
  return rc;
}
