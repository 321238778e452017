// Host-side runtime structures shared by pmh_runtime.cpp, pmh_autotune.cpp and
// pmh_server.cpp.  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "pmh_internal.h"

namespace pmh {

// Per-call device scratch: the heavy-first work list, the persistent grid's
// work counter and the split sets' chunk prefix and completion state.
struct WorkBuf {
  uint32_t* order = nullptr;
  uint32_t* small = nullptr;  // [0]: work counter, [4..7]: meta
  uint32_t* big_prefix = nullptr;
  uint64_t* big_state = nullptr;
  uint64_t cap = 0;
  WorkArgs args() const { return WorkArgs{order, small, small + 4, big_prefix, big_state}; }
};
void free_work(WorkBuf* wb);

struct GraphKey {
  const void* ids;
  const void* w;
  const void* off;
  uint64_t num_sets;
  const void* idx;
  const void* val;
  const void* id;
  const void* keys;
  uint64_t tune_version;
  bool operator==(const GraphKey& o) const {
    return ids == o.ids && w == o.w && off == o.off && num_sets == o.num_sets && idx == o.idx && val == o.val &&
           id == o.id && keys == o.keys && tune_version == o.tune_version;
  }
};

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev);
  ~DeviceGuard();

 private:
  int prev_ = 0, dev_ = 0;
};

uint64_t host_mix64(uint64_t z);
uint32_t imax_for(uint32_t m);
size_t lds_limit_bytes(int device);

}  // namespace pmh

struct pmh_ctx {
  uint64_t seed = 0, seedhash = 0;
  uint32_t m = 0;
  int variant = 1;
  int device = 0;
  int num_cu = 1;
  size_t lds_limit = 65536;
  uint32_t qcap[4] = {256, 512, 1024, 2048};  // chain queue entries for 1, 2, 4, 8 waves per workgroup
  void* table_mem = nullptr;
  pmh::Tables t{};
  uint32_t* status = nullptr;
  uint64_t* stats = nullptr;  // event counters of the statistics build
  pmh::WorkBuf work;
  pmh::WorkBuf gwork;  // the cached graph's own work buffer
  pmh::WorkArgs scratch{};  // the device's static work buffer (not owned; pmh_hash_sets_noalloc)
  uint64_t scratch_cap = 0;
  uint32_t imax = 0;   // ProbMinHash1/3 stream cap
  pmh::Tuning tune;
  uint64_t tune_version = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  pmh::GraphKey gkey{};
  std::vector<hipEvent_t> tev;  // kernel timing: event pairs (start, stop) per recorded call
  int tnext = 0, tcount = 0;
  std::mutex mu;
};

namespace pmh {
int max_waves(int variant);  // 8 for ProbMinHash2/4, 4 for ProbMinHash1/3
int effective_waves(const pmh_ctx* c);
// Dynamic LDS of a hash launch with `waves` per workgroup; *qcap receives the
// chain queue capacity to pass in HashArgs.
size_t launch_lds(const pmh_ctx* c, int waves, uint32_t* qcap);
void plan_queues(pmh_ctx* c);
int ensure_work(pmh_ctx* c, WorkBuf* wb, uint64_t num_sets);
HashArgs make_args(const pmh_ctx* c, const uint64_t* ids, const double* w, const uint64_t* off, uint64_t num_sets,
                   uint32_t* idx, double* val, uint64_t* id, uint64_t* keys, const WorkBuf* wb);
// Order kernel, split-set init and the persistent grid (per_cu workgroups per
// CU and waves per workgroup from the tuning when 0); ev0/ev1, when given, are
// recorded right before and after the persistent hash kernel.
int enqueue_batched(pmh_ctx* c, const HashArgs& a, WorkBuf* wb, hipStream_t s, int per_cu = 0, int waves = 0,
                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
}  // namespace pmh
