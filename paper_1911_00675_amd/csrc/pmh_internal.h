// Internal interface between the HIP kernels (pmh_kernels.hip) and the host
// runtime (pmh_runtime.cpp).  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmh {

constexpr uint64_t kPhi = 0x9E3779B97F4A7C15ull;   // SplitMix64 increment
constexpr uint64_t kEmptyKey = 0xFFFFFFFFFFFFFFFFull;
constexpr uint64_t kPosMask = 0xFFFFFull;          // 20 position bits
constexpr uint64_t kMaxSet = 1ull << 20;
constexpr uint32_t kMaxM = 16384;

// device status bits (sticky until read)
constexpr uint32_t kStatusWeight = 1u;      // a negative/NaN/inf/subnormal weight was skipped
constexpr uint32_t kStatusSetTooLarge = 2u; // a set above 2^20 elements was left empty

// Per-(variant, m) constant tables in device memory, computed on the device by
// the table-init kernel from the spec formulas.
struct Tables {
  double* beta;   // PMH2: [m+1], beta[i] = m/(m-i+1)
  double* lam;    // PMH4: [m], lambda_i = log(1 + 1/(m-i)), i = 1..m-1
  double* a;      // PMH4: [m], a_i = e^lambda_i - 1 = 1/(m-i)
  double* c1;     // PMH4: [m], c1_i = a_i / lambda_i
  double* gam;    // PMH4: [m], gamma_0 = 0, gamma_i = log(1 + i/(m-i))/lambda_1
  double* dgam;   // PMH4: [m], gamma_i - gamma_{i-1}
  double* expm1c; // [19] Taylor coefficients 1/k! built by repeated division
  double* scal;   // [8]: lambda, a, c1 (PMH3), -, delta (PMH4)
  double* ltab;   // [512]: stream-logarithm cells (inv_j, -log inv_j), then (inv_j, -log 2 inv_j)
  // Loop caps (Sec. 3 advises bounding the generators' loops; part of the
  // result's definition): proposals of the truncated-exponential sampler
  // (1..32), Lemire redraws (0..8) and a validation-only floor (a multiple of
  // 16) that forces redraws of draws whose low product half lies below it
  // (0: off).
  uint32_t te_rounds;
  uint32_t redraws;
  uint32_t lemire_floor;
  // scal[0..2] and scal[4] by value, read back once the tables are built:
  // kernels take them from their arguments (scalar constant loads), not
  // through the pointer, which a call in a loop would force them to reload.
  double te_lam, te_a, te_c1;  // ProbMinHash3's truncated-exponential lambda, a, c1
  double delta;                // ProbMinHash4's last-point scale
};
constexpr uint32_t kTeRoundsMax = 32;  // word slots 16..79
constexpr uint32_t kRedrawsMax = 8;    // word slots 1..8
// Largest stream cap: word counters address point i as i << 8 in 32 bits.
constexpr uint32_t kImaxMax = (1u << 24) - 1;

// Tunables of the per-set algorithm (chosen by the autotuner or defaults).
struct Tuning {
  double c0 = 3.0;          // first threshold T0 = m (ln m + c0) / sum(w)
  double grow = 2.0;        // T_{r+1} = grow * T_r
  int max_rounds = 4;       // the last round runs with T = +inf
  double chain_expect = 48; // elements expecting more points than this run as 64-lane chains
  int lane_budget = 4;      // lane-mode steps before an element moves to chain mode
  int waves = 2;            // waves per workgroup
  int kmax_refresh = 8;     // element batches between stop-limit refreshes
  int blocks_per_cu = 0;    // persistent grid = CUs * this (0: occupancy limit)
  double mini_expect = 48;  // ProbMinHash1/3: elements expecting more points go straight to 4-lane mini-chains
                            // (at the default = chain_expect, minis take only lane-budget overflows)
  int split_log2 = 15;      // sets of >= 2^this elements run as chunks of 2^(this-1) (0: never split)
  double c0_split = 6.0;    // extra threshold margin of chunks (keeps the completion repair rare)
};

// Device scratch of one batched launch (allocated by the runtime).
struct WorkArgs {
  uint32_t* order;       // [num_sets] heavy-first set order
  uint32_t* counter;     // [2]: work counters of the persistent and the finish grid
  uint32_t* meta;        // [4]: split sets, chunk items, all items
  uint32_t* big_prefix;  // [num_sets + 1] chunk prefix of the split sets
  uint64_t* big_state;   // [num_sets] per split set: smallest chunk threshold (bits)
};

struct HashArgs {
  const uint64_t* ids;
  const double* w;
  const uint64_t* off;       // [num_sets + 1]
  uint64_t num_sets;
  uint32_t* out_idx;         // [num_sets * m] or null
  double* out_val;           // [num_sets * m] or null
  uint64_t* out_id;          // [num_sets * m] or null
  uint64_t* out_keys;        // [num_sets * m] or null
  uint64_t* out_bbit;        // [num_sets * ceil(m b / 64)] b-bit reduction (Sec. 1.3) or null
  uint32_t bbit_b;           // its field width b (1, 2, 4, 8 or 16)
  uint64_t seedhash;
  uint32_t m;
  uint32_t imax;
  Tables t;
  double c0, grow, chain_expect, mini_expect;
  int max_rounds, lane_budget, kmax_refresh;
  uint32_t qcap;             // chain queue entries in LDS (>= one batch)
  uint32_t binary;           // binary weights: no weight array, every weight 1 (Sec. 2.9 values for PMH3/4)
  uint32_t* counts;          // update mode: elements each set has absorbed (in/out); null otherwise
  uint32_t* status;          // device status word
  const uint32_t* order;     // work list (set indices), heavy first
  uint32_t* counter;         // work counters (zeroed by the order kernel)
  const uint32_t* meta;      // split sets, chunk items, all items (written by the order kernel)
  const uint32_t* big_prefix;
  uint64_t* big_state;
  uint64_t* big_keys;        // global keys of split set s at big_keys + s*m
  uint32_t split_log2;
  double c0_split;
  uint32_t num_items;
  uint64_t* points;          // optional: points generated (profiling), or null
};

// The static work buffer of the no-allocation entry point: at most
// kScratchSets sets per call; scratch_work fills *out with its parts on
// `device` (which must be current) and *cap with kScratchSets.
constexpr uint32_t kScratchSets = 1u << 20;
constexpr int kMaxDevices = 64;
hipError_t scratch_work(int device, WorkArgs* out, uint64_t* cap);

// launchers (pmh_kernels.hip)
hipError_t launch_init_tables(int variant, uint32_t m, Tables t, hipStream_t s);
hipError_t launch_order(const uint64_t* off, uint64_t num_sets, uint32_t split_log2, const WorkArgs& w,
                        uint32_t* status, hipStream_t s);
hipError_t launch_big_init(const WorkArgs& w, uint32_t m, uint64_t* big_keys, hipStream_t s);
// Up to three copies of n[g] 32-bit words (n = 0: unused), between device
// memory and device-mapped pinned host memory.
struct CopySegs {
  const uint32_t* src[3];
  uint32_t* dst[3];
  uint64_t n[3];
};
hipError_t launch_copy_words(const CopySegs& c, hipStream_t s);
hipError_t launch_big_finish(int variant, const HashArgs& a, int waves, int grid, size_t lds, hipStream_t s);
hipError_t launch_hash(int variant, const HashArgs& a, int waves, int grid, size_t lds,
                       hipStream_t s);
hipError_t launch_hash_one(int variant, const HashArgs& a, uint64_t set, int waves, size_t lds,
                           hipStream_t s);
hipError_t occupancy(int variant, int waves, size_t lds, int* blocks_per_cu);
// P-MinHash kernels (persistent chunk/set kernel, split-set finish)
hipError_t launch_pmin(const HashArgs& a, int grid, hipStream_t s);
hipError_t launch_pmin_finish(const HashArgs& a, int grid, hipStream_t s);
hipError_t occupancy_pmin(int* blocks_per_cu);
uint32_t pmin_split_log2();
// A workgroup reads its set in batches of batch_size(waves) elements; its
// chain queue holds qcap >= one batch of entries (launches size it to the LDS
// left at the register-limited occupancy, up to 8 batches).
uint32_t batch_size(int waves);
size_t lds_bytes_q(int variant, uint32_t m, int waves, uint32_t qcap);  // dynamic LDS of k_hash_*
size_t lds_bytes(int variant, uint32_t m, int waves);   // the same with a queue of 2 batches (m range check)
size_t lds_static_bytes();                                // its static LDS
hipError_t launch_estimate(const uint64_t* idA, const uint32_t* idxA, const uint64_t* idB,
                           const uint32_t* idxB, uint32_t m, uint64_t pairs, uint32_t* counts,
                           hipStream_t s);
hipError_t launch_allpairs(const uint32_t* fp, uint32_t k, uint32_t m, uint16_t* counts,
                           hipStream_t s);
hipError_t launch_bbit_pack(const uint64_t* id, uint64_t num_sigs, uint32_t m, uint32_t b, uint64_t* out,
                            hipStream_t s);
hipError_t launch_bbit_allpairs(const uint64_t* sig, uint32_t k, uint32_t m, uint32_t b, uint16_t* counts,
                                hipStream_t s);
hipError_t launch_debug_eval(int what, const double* in, const uint64_t* in_u, double* out,
                             uint64_t* out_u, uint64_t n, uint32_t m, int variant, Tables t,
                             hipStream_t s);

}  // namespace pmh
