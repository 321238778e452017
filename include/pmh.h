/*
 * pmh.h -- C ABI of the MI355X ProbMinHash signature library (libpmh.so).
 *
 * Computes ProbMinHash signatures of weighted sets as defined in
 *   O. Ertl, "ProbMinHash -- A Class of Locality-Sensitive Hash Algorithms for
 *   the (Probability) Jaccard Similarity", IEEE TKDE 2020 (arXiv 1911.00675).
 *
 * Problem statement (Sec. 1, eq. (1) and eq. (6)): a weighted set is a map
 * w: D -> [0, inf) over 64-bit element ids; its signature z_1..z_m holds, for
 * every component k, the element whose hash h_k(d) ~ Exp(lambda w(d)) is
 * smallest.  The hashes come from per-element point streams (Sec. 2.1) of the
 * four variants ProbMinHash1-4 (Sec. 2.3-2.6).  Two signatures estimate the
 * probability Jaccard similarity J_P by the fraction of equal components
 * (eq. (3)).
 *
 * Conventions for every entry point:
 *   * Pointers marked [device] are device memory of the current HIP device,
 *     owned by the caller (e.g. a torch tensor's data_ptr); the library never
 *     frees them.  Pointers marked [host] are host memory.
 *   * `stream` is a hipStream_t (NULL = the legacy default stream).  Device
 *     work is enqueued asynchronously on it and ordered with the caller's
 *     other work on that stream.
 *   * Return value: PMH_OK or a pmh_status code; argument errors are reported
 *     synchronously, before anything is enqueued.  Errors found by kernels
 *     (invalid weights, oversize sets) are sticky in the context and returned
 *     by pmh_get_status().
 *   * A context may be used by one stream at a time (its work list and counter
 *     are shared by its calls); use one context per concurrent stream.
 *
 * Input layout (CSR): set s owns elements offsets[s] .. offsets[s+1]-1 of the
 * arrays ids (uint64) and weights (float64); offsets has num_sets+1 entries
 * with offsets[0] = 0.  A weight of 0 removes the element (Sec. 1.1); a
 * negative, NaN, infinite or subnormal weight is skipped and reported as
 * PMH_ERR_WEIGHT.  At most 2^20 elements per set (PMH_ERR_SET_TOO_LARGE; such
 * a set's signature is left empty).  Duplicate ids within a set are not
 * checked.
 *
 * Output layout (SoA, row-major [num_sets][m]); each output pointer may be
 * NULL to skip it:
 *   out_idx[s*m+k]  uint32  position of z_k within set s (0xFFFFFFFF: empty)
 *   out_val[s*m+k]  float64 the winning point value, truncated to 32 fraction
 *                           bits (+inf: empty)
 *   out_id[s*m+k]   uint64  ids[offsets[s] + out_idx] (0: empty)
 *   out_keys[s*m+k] uint64  packed key (value bits | position), all ones: empty
 *
 * Determinism: the signature is a pure function of (seed, m, variant, set);
 * it does not depend on element order, batch composition, launch shape or
 * tuning, and matches the CPU reference bit for bit.
 */
#ifndef PMH_H
#define PMH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pmh_ctx pmh_ctx;
typedef struct pmh_server pmh_server;

enum {
  PMH_OK = 0,
  PMH_ERR_ARG = 1,            /* null pointer, bad count or bad enum */
  PMH_ERR_M_RANGE = 2,        /* m outside [1, pmh_max_m()] */
  PMH_ERR_VARIANT_M = 3,      /* m = 1 with ProbMinHash3/4 (Sec. 2.5, 2.6 need m >= 2) */
  PMH_ERR_WEIGHT = 4,         /* invalid weight seen by a kernel */
  PMH_ERR_SET_TOO_LARGE = 5,  /* set above 2^20 elements seen by a kernel */
  PMH_ERR_DEVICE = 6,         /* HIP runtime error */
  PMH_ERR_OOM = 7,            /* device or host allocation failed */
  PMH_ERR_BUSY = 8,           /* serving queue full */
  PMH_ERR_NOT_READY = 9,      /* serving request still in flight */
  PMH_ERR_SCRATCH_LIMIT = 10, /* pmh_hash_sets_noalloc: more sets than its static work buffer holds */
  PMH_ERR_NO_ENTRY = 11       /* pmh_tuning_load: no stored tuning for this device, m and variant */
};

/* Tunables of the per-set schedule.  None of them changes any result.
 * pmh_init sets defaults per variant and m (pmh_get_tuning reads them). */
typedef struct {
  double c0;          /* first value threshold T0 = m (ln m + c0) / sum(w) (default 3; 2 for
                         ProbMinHash3) */
  double grow;        /* threshold growth per extra round (> 1) */
  int max_rounds;     /* rounds before the unbounded final round (>= 1) */
  double chain_expect;/* elements expecting more points go to wave-chain mode (default 48;
                         ProbMinHash2 16; ProbMinHash4 32, keeping streams of 16-32 points in
                         lane mode only where a batch holds a wave of them) */
  int lane_budget;    /* ProbMinHash1/3: lane-mode points before an element moves on */
  int waves;          /* wavefronts per workgroup: 1, 2, 4, or 8 for ProbMinHash2/4 (default 2;
                         above m = 1536 4 for ProbMinHash1/3; above m = 3072 8 for
                         ProbMinHash2/4, 4 where eight do not fit; fewer where the LDS does
                         not fit) */
  int kmax_refresh;   /* element batches between stop-limit refreshes (>= 1) */
  int blocks_per_cu;  /* persistent grid = CUs * this (0: occupancy limit) */
  double mini_expect; /* ProbMinHash1/3 elements expecting more points run as 4-lane mini-chains */
  int split_log2;     /* batched forms: sets of >= 2^split_log2 elements are split into chunks of
                         2^(split_log2-1) elements on separate workgroups (0: never; else 2..21;
                         default 15, 16 above m = 2048).
                         Needs out_keys, out_val or out_id, whose rows hold the merged keys. */
  double c0_split;    /* extra margin added to c0 in the chunks' threshold */
} pmh_tuning;

/* Create a context for (seed, m, variant) on the current device.  variant is
 * 1..4 for ProbMinHash1..4.  Builds the per-m constant tables on the device
 * (beta_i of Sec. 2.4; lambda, a = e^lambda - 1 and c1 = a/lambda of the
 * truncated-exponential sampler of Sec. 2.8; lambda_i, a_i, c1_i, gamma_i,
 * delta of Sec. 2.6) and sets the default loop caps (see pmh_set_caps).
 * Synchronous.  *out receives the context. */
int pmh_init(uint64_t seed, uint32_t m, int variant, pmh_ctx** out);

/* Free the context and its device memory (synchronizes the device). */
void pmh_destroy(pmh_ctx* ctx);

/* Largest supported m on the current device (LDS-limited, <= 16384). */
uint32_t pmh_max_m(int variant);

/* Human-readable text for a status code (static storage). */
const char* pmh_status_str(int status);

/* ProbMinHash signatures (eq. (1): component k holds the element whose
 * point labelled k has the smallest value; the points are the per-element
 * streams of Sec. 2.1 with the variant's value and label laws of Sec. 2.3
 * (ProbMinHash1), 2.4 (ProbMinHash2), 2.5 (ProbMinHash3) or 2.6
 * (ProbMinHash4); the stop rule of Sec. 2 only prunes) of num_sets weighted
 * sets in one persistent launch (plus one ordering kernel): sets are taken
 * heavy-first from a device work list.  ids, weights, offsets [device];
 * outputs [device] or NULL. */
int pmh_hash_sets(pmh_ctx* ctx, const uint64_t* ids, const double* weights, const uint64_t* offsets,
                  uint64_t num_sets, uint32_t* out_idx, double* out_val, uint64_t* out_id,
                  uint64_t* out_keys, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same result
 * as pmh_hash_sets, with its work list, counters and split-set state taken
 * from a static device array of the library (one per GPU, 16 MiB, held until
 * the process ends) instead of context buffers that grow on demand.  The
 * call itself allocates nothing; inputs and outputs are the caller's as for
 * pmh_hash_sets.  At most 2^20 sets per call (PMH_ERR_SCRATCH_LIMIT, nothing
 * enqueued).  Every call of this entry point on one GPU, from any context,
 * uses the same array, and each call's ordering kernel rewrites it: calls
 * whose device work overlaps on one GPU (different streams, threads or
 * contexts) race; serialize them, e.g. on one stream. */
int pmh_hash_sets_noalloc(pmh_ctx* ctx, const uint64_t* ids, const double* weights, const uint64_t* offsets,
                          uint64_t num_sets, uint32_t* out_idx, double* out_val, uint64_t* out_id,
                          uint64_t* out_keys, void* stream);

/* pmh_hash_sets with the b-bit reduction of Sec. 1.3 (algorithm "Reduction
 * to a b-bit signature") computed in the same kernel, as each signature is
 * finished: out_bbit[num_sets][ceil(m b / 64)] uint64 [device] receives
 * exactly what pmh_bbit_pack writes for the signatures' ids (component k,
 * 1-based, keeps the b low bits of mix64(mix64(id) + k * 0x9E3779B97F4A7C15),
 * id 0 for an empty component; component k-1 at bit (k-1) b, padding zero),
 * without a second pass over the ids.  b in {1, 2, 4, 8, 16}.  The other
 * outputs are optional as for pmh_hash_sets (sets are split across
 * workgroups only when out_keys, out_val or out_id is given). */
int pmh_hash_sets_bbit(pmh_ctx* ctx, const uint64_t* ids, const double* weights, const uint64_t* offsets,
                       uint64_t num_sets, uint32_t b, uint64_t* out_bbit, uint32_t* out_idx, double* out_val,
                       uint64_t* out_id, uint64_t* out_keys, void* stream);

/* Same result with one kernel launch per set (the plain form). */
int pmh_hash_sets_plain(pmh_ctx* ctx, const uint64_t* ids, const double* weights,
                        const uint64_t* offsets, uint64_t num_sets, uint32_t* out_idx,
                        double* out_val, uint64_t* out_id, uint64_t* out_keys, void* stream);

/* Same result as pmh_hash_sets, replayed from a HIP graph captured on the
 * first call with this exact argument tuple (re-captured when it changes). */
int pmh_hash_sets_graph(pmh_ctx* ctx, const uint64_t* ids, const double* weights,
                        const uint64_t* offsets, uint64_t num_sets, uint32_t* out_idx,
                        double* out_val, uint64_t* out_id, uint64_t* out_keys, void* stream);

/* P-MinHash signatures (Sec. 1.1, algorithm P-MinHash: the paper's O(n m)
 * baseline) of num_sets weighted sets with the context's seed and m (its
 * variant is not used): component k is the smallest key over the elements of
 * positive weight of fl((1/w) * Exp(1)), the Exp(1) taken from word slot 128
 * of point k of the element's counter stream with the stream logarithm.  Same
 * inputs, outputs, keys, ties, empty-set and error conventions as
 * pmh_hash_sets.  One ordering kernel, a persistent kernel over sets and
 * 1,024-element chunks of sets of >= 2^11 elements (when out_keys, out_val or
 * out_id is given to hold the merge rows), and a finishing kernel for those
 * sets.  Timed by pmh_timing_begin like pmh_hash_sets (the persistent
 * kernel). */
int pmh_pminhash_sets(pmh_ctx* ctx, const uint64_t* ids, const double* weights, const uint64_t* offsets,
                      uint64_t num_sets, uint32_t* out_idx, double* out_val, uint64_t* out_id,
                      uint64_t* out_keys, void* stream);

/* Signatures of num_sets plain sets (every element weight 1, no weight array):
 * the binary specialisations of Sec. 2.9.  ProbMinHash1/2 give exactly what
 * pmh_hash_sets gives with unit weights.  ProbMinHash3 draws point i of an
 * element as (i - 1) + U with U uniform in [0,1) (no truncated exponential),
 * and ProbMinHash4 takes gamma_i = i with the same U for its points, which
 * makes it SuperMinHash.  U is the high 32 bits of the point's stream word
 * times 2^-32.  ids, offsets [device]; outputs [device] or NULL; same keys,
 * ties, empty-set, split and error conventions as pmh_hash_sets (no weight
 * can be invalid).  Timed by pmh_timing_begin like pmh_hash_sets. */
int pmh_hash_sets_binary(pmh_ctx* ctx, const uint64_t* ids, const uint64_t* offsets, uint64_t num_sets,
                         uint32_t* out_idx, double* out_val, uint64_t* out_id, uint64_t* out_keys,
                         void* stream);

/* Incremental signatures: adds a batch of new elements to num_sets sets
 * whose signatures are kept across calls.  The signature is a componentwise
 * minimum over the points of every element (eq. (1) and the structure of
 * Sec. 2), so a set's elements can arrive in several calls: the result after
 * any number of calls is, bit for bit, the pmh_hash_sets signature of the
 * concatenation of all the batches in call order (element positions count
 * from the set's first element ever).  keys [device, in/out]: num_sets x m
 * keys, all-ones (empty) for a new set; counts [device, in/out]: elements
 * each set has absorbed (0 for a new set), advanced by the batch's size.
 * weights [device] or NULL for the binary specialisations (as
 * pmh_hash_sets_binary).  out_idx, out_val [device] or NULL: position and
 * value of the updated signature; out_id [device, in/out] or NULL: the ids
 * from the previous call on the same rows (components that keep their
 * element keep their id), so pass it on every call of a set or never.  Sets
 * are not split across workgroups.  A set whose total would exceed 2^20
 * elements (the position field) is left unchanged and reported as
 * PMH_ERR_SET_TOO_LARGE by pmh_get_status.  Timed by pmh_timing_begin. */
int pmh_update_sets(pmh_ctx* ctx, const uint64_t* ids, const double* weights, const uint64_t* offsets,
                    uint64_t num_sets, uint32_t* counts, uint64_t* keys, uint32_t* out_idx, double* out_val,
                    uint64_t* out_id, void* stream);

/* Kernel timing for benchmarks.  After pmh_timing_begin(ctx, n) the next n
 * pmh_hash_sets (pmh_hash_sets_binary, pmh_update_sets, pmh_pminhash_sets)
 * calls record a HIP event pair right around their persistent hash kernel, on
 * the call's stream (the ordering and split-set kernels stay outside).
 * pmh_timing_read waits for the n pairs and writes their durations in
 * milliseconds to [host] ms[0..n); PMH_ERR_NOT_READY if fewer than n calls
 * were recorded.  The events are owned by the context. */
int pmh_timing_begin(pmh_ctx* ctx, int n);
int pmh_timing_read(pmh_ctx* ctx, float* ms, int n);

/* Synchronize `stream`, then return and clear the context's sticky kernel
 * errors (PMH_ERR_WEIGHT, PMH_ERR_SET_TOO_LARGE) or PMH_OK. */
int pmh_get_status(pmh_ctx* ctx, void* stream);

int pmh_set_tuning(pmh_ctx* ctx, const pmh_tuning* t);
int pmh_get_tuning(const pmh_ctx* ctx, pmh_tuning* t);

/* Loop caps of the random streams (Sec. 3 advises bounding every loop of the
 * generators).  Unlike the tuning they are part of the result's definition,
 * and the CPU reference takes the same four values:
 *   imax          points per element of the with-replacement streams
 *                 (ProbMinHash1/3; 0: the default 6 m bitlen(m) + 64, at most
 *                 2^24 - 1), the stream ends after point imax;
 *   te_rounds     proposals of the truncated-exponential sampler's second
 *                 branch (Sec. 2.8; 1..32, default 32), the last proposal is
 *                 returned when all are rejected;
 *   redraws       redraws of Lemire's bounded integers (0..8, default 8);
 *   lemire_floor  validation only: draws whose low product half lies below it
 *                 are redrawn as well, which forces the redraw path (labels
 *                 are then no longer uniform); a multiple of 16, 0 in normal
 *                 use.
 * Applies to later calls of every hashing entry point of the context
 * (P-MinHash has no such loops).  Returns PMH_ERR_ARG for values out of
 * range. */
int pmh_set_caps(pmh_ctx* ctx, uint32_t imax, uint32_t te_rounds, uint32_t redraws, uint32_t lemire_floor);

/* Time candidate schedules on the given batch ([device] inputs, the batch is
 * hashed trials times per candidate) and keep the fastest in the context;
 * *best (host, may be NULL) receives it.  Synchronous. */
int pmh_autotune(pmh_ctx* ctx, const uint64_t* ids, const double* weights, const uint64_t* offsets,
                 uint64_t num_sets, int trials, void* stream, pmh_tuning* best);

/* Stored tunings (text file at [host] path, one line per key): the key is the
 * context's device architecture (gcnArchName) and compute-unit count, m and
 * variant.  pmh_tuning_save writes the context's current tuning under its key
 * (replacing an older line; the file is rewritten through a temporary file
 * and renamed).  pmh_tuning_load applies the stored tuning for the context's
 * key (validated as pmh_set_tuning does), or returns PMH_ERR_NO_ENTRY. */
int pmh_tuning_save(const pmh_ctx* ctx, const char* path);
int pmh_tuning_load(pmh_ctx* ctx, const char* path);

/* Estimator of eq. (3) for one pair of signatures of size m, [host] inputs:
 * fraction of components k with idA[k] == idB[k], empty components (idx
 * 0xFFFFFFFF) never counting as equal.  *out [host]. */
int pmh_estimate(const uint64_t* idA, const uint32_t* idxA, const uint64_t* idB, const uint32_t* idxB,
                 uint32_t m, double* out);

/* Equal-component counts for `pairs` signature pairs, [device] inputs laid out
 * [pairs][m] (pair r compares row r of A with row r of B; empty components,
 * idx 0xFFFFFFFF, never count); counts[pairs] uint32 [device].  Divide by m
 * for eq. (3).  pairs <= 2^31 - 1. */
int pmh_estimate_pairs(const uint64_t* idA, const uint32_t* idxA, const uint64_t* idB,
                       const uint32_t* idxB, uint32_t m, uint64_t pairs, uint32_t* counts,
                       void* stream);

/* The numerators of eq. (3) for all pairs of k signatures: equal-component
 * counts over k signatures of m 32-bit fingerprints fp[k][m] [device] (0 =
 * empty component, never equal); counts[k][k] uint16 [device], saturating at
 * 65535. */
int pmh_allpairs_counts(const uint32_t* fp, uint32_t k, uint32_t m, uint16_t* counts, void* stream);

/* b-bit reduction (Sec. 1.3, algorithm "Reduction to a b-bit signature") of
 * num_sigs signatures given by their element ids id[num_sigs][m] [device]
 * (the out_id output; 0 = empty component): component k (1-based) keeps the
 * b low bits of mix64(mix64(id) + k * 0x9E3779B97F4A7C15), b in {1, 2, 4, 8,
 * 16}; packed into out[num_sigs][ceil(m b / 64)] uint64 [device], component
 * k-1 at bit (k-1) b of the signature's bit string, padding bits zero.
 * Different elements agree in a component with probability 2^-b, so
 * (equal/m - 2^-b) / (1 - 2^-b) estimates J_P.  1 <= m <= 16384. */
int pmh_bbit_pack(const uint64_t* id, uint64_t num_sigs, uint32_t m, uint32_t b, uint64_t* out, void* stream);

/* All-pairs equal-field counts of k packed b-bit signatures sig[k][ceil(m b
 * / 64)] [device]: counts[k][k] uint16 [device]. */
int pmh_bbit_allpairs(const uint64_t* sig, uint32_t k, uint32_t m, uint32_t b, uint16_t* counts, void* stream);

/* Copy a constant table to [host] out (count doubles).  which: 0 beta (PMH2,
 * m+1), 1 lambda_i, 2 a_i = e^lambda_i - 1, 3 c1_i = a_i/lambda_i,
 * 5 gamma_i, 6 dgamma_i (PMH4, m each), 7 scalars {lambda, a, c1 (PMH3), 0,
 * delta (PMH4), 0, 0, 0} (8), 8 expm1 coefficients (19), 9 stream-logarithm
 * cells (512: 256 pairs (1/c_j, L_j)); 4 is not used (PMH_ERR_ARG).
 * Synchronous. */
int pmh_get_table(pmh_ctx* ctx, int which, double* out, uint32_t count);

/* Evaluate one primitive of the random streams elementwise on [device]
 * arrays (for validation): what 0 log(in), 1 log1p(in), 2 expm1(in),
 * 3 Exp(1) from word in_u, 4 mix64(in_u), 5 truncated exponential of element
 * key in_u[k] at point k+1 (PMH3 constants), 6 Lemire(m) label of that point,
 * 7 ProbMinHash1 fixed-point spacing of that point, 8 stream logarithm(in),
 * 9 inclusive prefix sum of in_u over each aligned group of 64 entries (the
 * chain-mode spacing scan; entries < 2^51), 10, 11, 12 the same over groups
 * of 8, 4, 2 (the mini-chain scans). */
int pmh_debug_eval(pmh_ctx* ctx, int what, const double* in, const uint64_t* in_u, double* out,
                   uint64_t* out_u, uint64_t n, void* stream);

/* ---- serving: continuous batching of single-set requests ----------------
 * The server owns `slots` execution slots (stream, pinned staging, device
 * buffers).  One slot is open at a time: a submission copies its set into the
 * open slot's pinned staging; a dispatcher thread launches the open slot as
 * soon as it holds a request (copy in, heavy-first persistent kernel, copy the
 * signatures out) and the next free slot opens, so requests that arrive while
 * other batches are on the GPU form the next batch and run concurrently on
 * their own stream.  Admission: at most slot_elems elements (never below
 * 2^20, so any set fits) and slot_sets requests per slot; with a non-zero
 * hbm_budget_bytes the slots' device buffers are sized to fit it; each
 * slot's persistent grid is its share of the CUs' workgroup (LDS) capacity.
 * A batch finishes with its slowest set, so requests of >= 2^11 elements run
 * as 1,024-element chunks on separate workgroups (unless the context's
 * split_log2 is 0).  Creation runs one set through every slot (first use of a
 * stream costs milliseconds).  When every slot is in flight a submission
 * waits (back-pressure).  Results are identical to pmh_hash_sets on the same
 * set. */
int pmh_server_create(pmh_ctx* ctx, int slots, uint64_t slot_elems, uint32_t slot_sets,
                      uint64_t hbm_budget_bytes, pmh_server** out);
/* Copy a request in ([host] ids, weights of n <= 2^20 elements); *ticket
 * receives its handle.  Waits while every slot is in flight. */
int pmh_server_submit(pmh_server* s, const uint64_t* ids, const double* weights, uint32_t n,
                      uint64_t* ticket);
/* PMH_OK and the signature ([host] outputs of m entries, any may be NULL) when
 * the request is done, PMH_ERR_NOT_READY otherwise.  Results stay available
 * until fetched once. */
int pmh_server_fetch(pmh_server* s, uint64_t ticket, uint32_t* idx, double* val, uint64_t* id);
/* Open-loop replay: submits request r at arrival[r] seconds after the start
 * (busy-waiting for the scheduled time), then waits for all results.
 * latency[r] (host, seconds) = completion time - scheduled arrival.  Requests
 * are given in CSR form on the host; before the clock starts they are staged
 * once in pinned host memory (owned by the call, freed on return), from which
 * each batch is copied to the device directly.  Signatures are written to
 * [host] out_idx/out_id ([num][m], may be NULL).  *wall receives the elapsed
 * time. */
int pmh_server_replay(pmh_server* s, const uint64_t* ids, const double* weights, const uint64_t* offsets,
                      uint64_t num, const double* arrival, double* latency, uint32_t* out_idx,
                      uint64_t* out_id, double* wall);
/* Open-loop replay of num requests drawn from a pool of `pool` distinct
 * requests (CSR [host] ids, weights, offsets[pool+1]): request r is pool
 * entry order[r] (order [host] or NULL for r, num <= pool), submitted at
 * arrival[r] seconds; the pool is staged once in pinned host memory.  Same
 * outputs and timing as pmh_server_replay, which is this call with the
 * identity order. */
int pmh_server_replay_indexed(pmh_server* s, const uint64_t* ids, const double* weights, const uint64_t* offsets,
                              uint64_t pool, const uint64_t* order, uint64_t num, const double* arrival,
                              double* latency, uint32_t* out_idx, uint64_t* out_id, double* wall);
/* Counters into out8[8]: [0] batches launched, [1] requests done, [2] max
 * requests in one batch, [3] max concurrent slots busy, [4] requests that
 * waited for a slot; dispatcher timing in microseconds: [5] longest launch
 * (copies and kernels enqueued), [6] longest finish (results handed out),
 * [7] longest dispatcher loop iteration. */
int pmh_server_stats(pmh_server* s, uint64_t* out8);
void pmh_server_destroy(pmh_server* s);

#ifdef __cplusplus
}
#endif

#endif /* PMH_H */
