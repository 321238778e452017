// HIP kernels for ProbMinHash signatures on gfx950 (MI355X).
//
// O. Ertl, "ProbMinHash -- A Class of Locality-Sensitive Hash Algorithms for the
// (Probability) Jaccard Similarity", IEEE TKDE 2020.
//
// One workgroup computes the signature of one weighted set; a persistent grid
// pulls sets from a heavy-first work list.  Per set:
//
//   * keys[m] (u64, LDS) hold the running minimum of Key(x, p) per label, where
//     Key packs the point value's top bits and the element position, so a
//     single 64-bit atomic min on LDS performs "if h < q_k then q_k = h,
//     z_k = d" of the paper's algorithms (Sec. 2, basic structure).
//   * Points are generated in rounds of increasing value threshold T (a
//     schedule in the spirit of the interleaved processing of Sec. 2.7): round r
//     generates every point below T_r of every element and applies those below
//     the running stop limit max_k q_k (Sec. 2, "stop limit").  Once the stop
//     limit falls below T_r all keys are final.  The result is the exact
//     minimum over all points, independent of the processing order.
//   * Elements with short expected streams run one per lane ("lane mode");
//     long streams are handed to a queue and run 64 consecutive points per
//     wavefront ("chain mode"): ProbMinHash1/2 spacings are 64-bit fixed point
//     so a wave prefix sum reproduces the sequential accumulation exactly;
//     ProbMinHash3/4 points are independent per index; ProbMinHash2/4 resolve
//     64 Fisher-Yates steps (Sec. 2.4) per wave with in-register dependency
//     chasing.
//   * Random words are counter-based (SplitMix64 addressed by element key and
//     point index) so any lane can generate any point.
//
// All floating-point arithmetic is IEEE binary64 without contraction; fma is
// used only where the stream definitions say so.

#include <float.h>

#include <mutex>

#include "pmh_internal.h"

namespace pmh {
namespace {

constexpr double kLn2Hi = 0x1.62e42fefa0000p-1;  // ln 2 rounded to 36 bits
constexpr double kLn2Lo = 0x1.cf79abc9e3b3ap-40; // ln 2 - kLn2Hi
// Lane-mode Fisher-Yates steps kept in registers: ProbMinHash2 16 (3 waves
// per SIMD).  ProbMinHash4 32 in one- and two-wave workgroups, as a rolled
// loop (the step index is wave-uniform, so the register array is indexed in
// place; 2 waves per SIMD either way), but 4 unrolled steps in four-wave
// workgroups, where the m keys in LDS (m > 1536) bound the occupancy anyway
// and elements need hundreds of points.  Measured (mixed batch, m = 1024):
// unit weights ProbMinHash4 25.0 -> 14.0 ms with 16 steps instead of 4; 32
// steps let streams of up to 32 points stay in lane mode (unit weights 12.5
// -> 10.5 ms with a chain threshold of 32; the default threshold of 16 is
// kept for the Pareto-weighted batch, 15.8 -> 15.6 ms).
template <int V, int NW>
constexpr uint32_t kFyLaneSteps = V == 4 && NW >= 4 ? 4 : V == 4 ? 32 : 16;
template <int V, int NW>
constexpr bool kFyLaneRolled = V == 4 && NW < 4;
constexpr uint32_t kEpt = 2;                     // elements per thread per batch
// Per-wave tables that resolve the dependencies of a chain-mode tile of 64
// Fisher-Yates steps (ProbMinHash2/4): win[r] = 1 + the latest step of the
// tile that drew slot P0 + r of its position window, bkt[h] = the steps whose
// slot hashes to h.  All zero between tiles.
constexpr int kFyBuckets = 128;
// Waves of a workgroup that run ProbMinHash2/4 chain elements, each with its
// own label array u16[m] and tables; the others skip the chain pass.  At
// m = 4096 four arrays took a four-wave workgroup to 81 KB of LDS (one per
// CU); two leave room for two.  Eight-wave workgroups (ProbMinHash2/4 only)
// give every wave an array: one workgroup of 126 KB per CU at m = 4096, with
// twice the chain waves of two four-wave workgroups.
__host__ __device__ constexpr int fy_waves(int nw) { return nw == 8 ? 8 : nw < 2 ? nw : 2; }
struct FyScratch {
  uint64_t bkt[kFyBuckets];
  uint32_t win[64];
};
// ProbMinHash4 lane-mode elements are sorted per batch by expected points
// (kSortClasses classes, longest first) so the 64 lanes of a wave get streams
// of similar length: a wave runs as many steps as its longest stream.  LDS
// after the label arrays: counts[kSortClasses], offsets[kSortClasses], then
// one u16 batch index per element.
constexpr int kSortClasses = 32;
// Streams expecting more than kLaneSure points (up to chain_expect) stay in
// lane mode only where an ordered batch holds at least a wave of them;
// otherwise a few long streams would hold a whole wave, and they go to chain
// mode instead.
constexpr int kLaneSure = 16;
constexpr uint32_t kNoLane = 0xFFFFFFFFu;
__host__ __device__ constexpr size_t sort_region_offset(int nf, uint32_t m) {
  return ((size_t)nf * (sizeof(FyScratch) + (size_t)m * 2) + 15) & ~(size_t)15;
}
// Lane mode reads the per-index tables at indices 0..32 only (at most 32
// register Fisher-Yates steps): a copy of that slice sits in LDS after the
// sort region, kLaneTab entries per table (ProbMinHash2: beta; ProbMinHash4:
// gamma, gamma differences, lambda, a, c1), so a step reads LDS instead of
// waiting on global loads.
constexpr uint32_t kLaneTab = 33;
constexpr uint32_t kLogCells = 256;  // stream-logarithm cells at the start of the dynamic LDS
constexpr uint32_t kLaneTabs = 5;
__host__ __device__ constexpr size_t lane_tab_offset(int nf, uint32_t m, uint32_t batch) {
  return (sort_region_offset(nf, m) + 2 * kSortClasses * 4 + (size_t)batch * 2 + 15) & ~(size_t)15;
}

// Optional event counters (statistics build only, -DPMH_STATS): accumulated in
// LDS per workgroup and added to HashArgs::points[0..15] when a set ends.
#ifdef PMH_STATS
#define PMH_STAT(sm, i, v) atomicAdd(&(sm).st[i], (uint32_t)(v))
// shader-clock cycles of a phase, summed over waves (lane 0 of each wave)
#define PMH_TIC(t) const uint64_t t = clock64()
#define PMH_TOC(sm, i, t) \
  if ((threadIdx.x & 63) == 0) atomicAdd(&(sm).st[i], (uint32_t)(clock64() - (t)))
#else
#define PMH_STAT(sm, i, v) ((void)0)
#define PMH_TIC(t) ((void)0)
#define PMH_TOC(sm, i, t) ((void)0)
#endif
enum { kStSets, kStRounds, kStElems, kStLanePts, kStLaneIters, kStLaneApply, kStMiniSteps, kStMiniPts,
       kStMiniElems, kStChainTiles, kStChainPts, kStChainElems, kStFlush, kStBlockMax, kStApply, kStRepairs,
       kStCycBatch, kStCycBarrier, kStCycChain, kStCycMini, kStCycBlockMax, kStCycSet, kStCount };

// ---------------------------------------------------------------- randomness
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Word slot t of point i of element K is mix64(K + ((i << 8) + t + 1) * phi);
// pbase folds the point-independent part so slot t costs one add, and point
// i+1's base is point i's plus kPointStep.  Word 0 of a point serves twice:
// high 32 bits -> the uniform behind the value, low 32 bits -> the label draw.
constexpr uint64_t kPointStep = 256ull * kPhi;
__device__ __forceinline__ uint64_t pbase(uint64_t K, uint32_t i) {
  return K + (uint64_t)((i << 8) + 1u) * kPhi;
}
__device__ __forceinline__ uint64_t word(uint64_t pb, uint32_t t) { return mix64(pb + (uint64_t)t * kPhi); }
// The high half of w as an opaque 32-bit register value: the compiler would
// otherwise widen the u32 -> f64 conversions below to 64-bit ones that add a
// zero high part (an extra fp64 add each, kept under strict IEEE semantics).
__device__ __forceinline__ uint32_t hi32(uint64_t w) {
  uint32_t h = (uint32_t)(w >> 32);
  asm("" : "+v"(h));
  return h;
}
__device__ __forceinline__ double u32v(uint64_t w) { return (double)hi32(w) * 0x1p-32; }
// ((w >> 32) + 1) 2^-32, exact (the sum is at most 2^32)
__device__ __forceinline__ double upos32(uint64_t w) { return ((double)hi32(w) + 1.0) * 0x1p-32; }
// floor(s 2^32) of a spacing 0 <= s < 2^20, exact: the integral value t < 2^52
// is the low 52 bits of t + 2^52
__device__ __forceinline__ uint64_t spacing_fixed(double s) {
  const double t = trunc(s * 0x1p32);
  return (uint64_t)__double_as_longlong(t + 0x1p52) & 0xFFFFFFFFFFFFFull;
}
// T 2^-32 of the fixed-point accumulator as the nearest double: the fma
// rounds hi + lo 2^-32 once (exact below 2^53)
__device__ __forceinline__ double fixed_value(uint64_t T) {
  return fma((double)(uint32_t)T, 0x1p-32, (double)hi32(T));
}
__device__ __forceinline__ double u53(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }

// ln x = e ln 2 + 2 atanh(s), x = 2^e f, f in [sqrt(1/2), sqrt(2)), s = (f-1)/(f+1).
__device__ __forceinline__ double spec_log(double x) {
  uint64_t b = (uint64_t)__double_as_longlong(x);
  int e = (int)((b >> 52) & 0x7FF) - 1023;
  uint64_t mant = b & 0xFFFFFFFFFFFFFull;
  const bool halve = mant >= 0x6A09E667F3BCDull;
  e += halve ? 1 : 0;
  double f = __longlong_as_double((long long)(mant | (halve ? (1022ull << 52) : (1023ull << 52))));
  double s = (f - 1.0) / (f + 1.0);
  double t = s * s;
  double q = 2.0 / 21.0;
  q = __builtin_fma(q, t, 2.0 / 19.0);
  q = __builtin_fma(q, t, 2.0 / 17.0);
  q = __builtin_fma(q, t, 2.0 / 15.0);
  q = __builtin_fma(q, t, 2.0 / 13.0);
  q = __builtin_fma(q, t, 2.0 / 11.0);
  q = __builtin_fma(q, t, 2.0 / 9.0);
  q = __builtin_fma(q, t, 2.0 / 7.0);
  q = __builtin_fma(q, t, 2.0 / 5.0);
  q = __builtin_fma(q, t, 2.0 / 3.0);
  double lf = 2.0 * s + (s * t) * q;
  double de = (double)e;
  return de * kLn2Hi + (de * kLn2Lo + lf);
}

// log(1 + u), u > 0; per-m constants only.
__device__ double spec_log1p(double u) {
  if (u > 1.0) return spec_log(1.0 + u);
  double s = u / (2.0 + u);
  double t = s * s;
  double q = 2.0 / 49.0;
  for (int j = 23; j >= 1; --j) q = __builtin_fma(q, t, 2.0 / (double)(2 * j + 1));
  return 2.0 * s + (s * t) * q;
}

__device__ __forceinline__ double spec_expm1(double t, const double* c) {
  double p = c[18];
  for (int k = 17; k >= 1; --k) p = __builtin_fma(p, t, c[k]);
  return p * t;
}

// Table-driven logarithm of the streams: x = 2^e y, cell j = top 7 mantissa
// bits, r = fma(y, inv_j, -1), log1p by a degree-8 polynomial;
// tab[j + 128 h] = (inv_j, -log(inv_j)) with h = 0, or (inv_j, -log(2 inv_j))
// with h = 1 when y >= sqrt(2) (exponent e+1).
struct LogCell {
  double inv, L;
};
// a*b + c as the three-address VOP3 fma when kAsm: with a constant addend the
// compiler otherwise picks the two-address fmac and copies the constant every
// time (the hot ProbMinHash1/2 streams use it; elsewhere the plain builtin
// schedules better).
template <bool kAsm>
__device__ __forceinline__ double fma3(double a, double b, double c) {
  if constexpr (!kAsm) return __builtin_fma(a, b, c);
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}
template <bool kAsm = true>
__device__ __forceinline__ double stream_log(double x, const LogCell* tab) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  int e = (int)((b >> 52) & 0x7FF) - 1023;
  const uint64_t mant = b & 0xFFFFFFFFFFFFFull;
  const uint32_t j = (uint32_t)(mant >> 45);
  const bool halve = mant >= 0x6A09E667F3BCDull;
  e += halve ? 1 : 0;
  const LogCell c = tab[j + (halve ? 128u : 0u)];
  const double y = __longlong_as_double((long long)(mant | (1023ull << 52)));
  const double r = __builtin_fma(y, c.inv, -1.0);
  double q = 1.0 / 8.0;
  q = fma3<kAsm>(q, r, -1.0 / 7.0);
  q = fma3<kAsm>(q, r, 1.0 / 6.0);
  q = fma3<kAsm>(q, r, -1.0 / 5.0);
  q = __builtin_fma(q, r, 1.0 / 4.0);
  q = fma3<kAsm>(q, r, -1.0 / 3.0);
  q = __builtin_fma(q, r, 1.0 / 2.0);
  const double l1p = __builtin_fma(-(r * r), q, r);
  const double de = (double)e;
  return de * kLn2Hi + (de * kLn2Lo + (c.L + l1p));
}
template <bool kAsm = true>
__device__ __forceinline__ double exp1(uint64_t w, const LogCell* tab) {
  return 0.0 - stream_log<kAsm>(upos32(w), tab);
}

// Truncated exponential Exp(lam; 0, 1) of Sec. 2.8, density
// f(x) = lam e^(-lam x) / (1 - e^(-lam)) on [0, 1), with a = e^lam - 1 and
// c1 = a / lam.  f never falls below 1/c1 (its value at x -> 1), so f is a
// mixture: the uniform law with weight 1/c1, and a remainder proportional to
// e^(-lam x) - e^(-lam) = e^(-lam) expm1(lam (1 - x)).
//   Fast path: x = c1 U from the high half of the point's word 0 is below 1
//   with probability 1/c1 and then uniform.
//   Otherwise (te_slow): the remainder by proposals (x, v) uniform on
//   [0,1)^2 from the 53-bit slot pairs (16 + 2r, 17 + 2r), accepted when
//   v a <= expm1(lam t), t = 1 - x.  expm1(lam t) lies between lam t (its
//   tangent at 0) and a t (its chord on [0, 1]), so v c1 <= t accepts and
//   v >= t rejects without the series; at most `rounds` proposals, the last
//   one's x is returned.
__device__ __attribute__((noinline)) double te_slow(uint64_t pb, double lam, double a, double c1, uint32_t rounds,
                                                    const double* em) {
  double x = 0.0;
  for (uint32_t r = 0; r < rounds; ++r) {
    x = u53(word(pb, 16u + 2u * r));
    const double v = u53(word(pb, 17u + 2u * r));
    const double t = 1.0 - x;  // exact: x is a multiple of 2^-53 in [0, 1)
    if (v * c1 <= t) return x;
    if (v < t && v * a <= spec_expm1(lam * t, em)) return x;
  }
  return x;
}
// w0 = the point's word 0, pb its counter base.
__device__ __forceinline__ double trunc_exp(uint64_t w0, uint64_t pb, double lam, double a, double c1,
                                            const Tables& t) {
  const double x = c1 * u32v(w0);
  if (x < 1.0) return x;
  return te_slow(pb, lam, a, c1, t.te_rounds, t.expm1c);
}

// Redraws of Lemire's method: a draw whose low product half lies below
// (2^32 - s) mod s (or below the validation floor) is biased and takes the
// low half of the next word of slots 1..redraws.  capw = floor | redraws
// (the floor is a multiple of 16, redraws <= 8): one argument of the call,
// which keeps ProbMinHash4 within 168 VGPRs (3 waves per SIMD).
__device__ __attribute__((noinline)) uint64_t lemire_redraw(uint64_t pb, uint32_t s, uint64_t prod, uint32_t capw) {
  const uint32_t floor = capw & ~15u, redraws = capw & 15u;
  uint32_t thr = (0u - s) % s;
  thr = thr < floor ? floor : thr;
  uint32_t lo = (uint32_t)prod;
  for (uint32_t r = 1; lo < thr && r <= redraws; ++r) {
    const uint64_t x = word(pb, r) & 0xFFFFFFFFull;
    prod = x * (uint64_t)s;
    lo = (uint32_t)prod;
  }
  return prod;
}
// Uniform integer in [0, s) (Lemire's multiply-shift with rejection) from the
// low half of the point's word 0.  The threshold is below s and below the
// floor, so a low half of at least s | floor (>= both) needs no redraw.
__device__ __forceinline__ uint32_t lemire(uint64_t w0, uint64_t pb, uint32_t s, const Tables& t) {
  const uint64_t x = w0 & 0xFFFFFFFFull;
  uint64_t prod = x * (uint64_t)s;
  if ((uint32_t)prod < (s | t.lemire_floor)) prod = lemire_redraw(pb, s, prod, t.lemire_floor | t.redraws);
  return (uint32_t)(prod >> 32);
}

__device__ __forceinline__ uint64_t make_key(double x, uint32_t p) {
  return ((uint64_t)__double_as_longlong(x) & ~kPosMask) | (uint64_t)p;
}
__device__ __forceinline__ bool weight_ok(double w) { return w >= 0x1p-1022 && w <= DBL_MAX; }

// --------------------------------------------------------------- wave utils
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
  uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
  uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, mask);
  uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), mask);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) {
    uint64_t o = shfl_xor_u64(v, d);
    v = o > v ? o : v;
  }
  return v;
}
__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  return v;
}
// DPP lane moves (gfx9 row operations).  update_dpp(old = 0, ...) writes 0
// where the source lane is outside the row or the row is masked off.
constexpr int kDppRowShr = 0x110;     // + n: lane i takes lane i - n of its row of 16
constexpr int kDppRowBcast15 = 0x142; // lane 15 of each row to the next row
constexpr int kDppRowBcast31 = 0x143; // lane 31 to rows 2 and 3
template <int N>
__device__ __forceinline__ uint32_t dpp_shr(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr + N, 0xf, 0xf, true);
}
// Inclusive prefix sum over the 64 lanes of u32 values whose total fits 32 bits.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
  x += dpp_shr<1>(x);
  x += dpp_shr<2>(x);
  x += dpp_shr<4>(x);
  x += dpp_shr<8>(x);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowBcast15, 0xa, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowBcast31, 0xc, 0xf, false);
  return x;
}
// Inclusive prefix sum over the 64 lanes of fixed-point spacings v < 2^51:
// scanned as 26-bit low and 25-bit high limbs (64 of each fit 32 bits) with
// DPP row moves instead of LDS-crossbar shuffles.
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v, int lane) {
  (void)lane;
  const uint32_t lo = wave_incl_scan_u32((uint32_t)v & 0x3FFFFFFu);
  const uint32_t hi = wave_incl_scan_u32((uint32_t)(v >> 26));
  return ((uint64_t)hi << 26) + lo;
}
// The same within aligned groups of G = 2, 4 or 8 lanes (j = lane & (G-1)).
template <int G>
__device__ __forceinline__ uint32_t group_incl_scan_u32(uint32_t x, int j) {
  uint32_t o = dpp_shr<1>(x);
  x += j >= 1 ? o : 0u;
  if constexpr (G >= 4) {
    o = dpp_shr<2>(x);
    x += j >= 2 ? o : 0u;
  }
  if constexpr (G == 8) {
    o = dpp_shr<4>(x);
    x += j >= 4 ? o : 0u;
  }
  return x;
}
template <int G>
__device__ __forceinline__ uint64_t group_incl_scan_u64(uint64_t v, int j) {
  const uint32_t lo = group_incl_scan_u32<G>((uint32_t)v & 0x3FFFFFFu, j);
  const uint32_t hi = group_incl_scan_u32<G>((uint32_t)(v >> 26), j);
  return ((uint64_t)hi << 26) + lo;
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t lds_load_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// The atomic returns nothing, so the wave does not wait on it; reading the
// slot first to skip atomics that cannot lower it put that read's latency
// on every point.
__device__ __forceinline__ void lds_min(uint64_t* keys, uint32_t l, uint64_t key) {
  atomicMin((unsigned long long*)&keys[l], (unsigned long long)key);
}

// ---------------------------------------------------------------- set state
struct ChainEntry {
  uint32_t p;
  uint32_t i;     // next point index
  uint64_t tacc;  // ProbMinHash1: fixed-point accumulator through point i-1;
                  // ProbMinHash2/3/4 (no accumulator carried: 2/4 restart at
                  // point 1): the element key K, so a refill needs neither
                  // the id nor its hash
};

struct Shared {
  uint64_t red_u[16];
  double red_d[16];
  uint64_t kmax;          // stop-limit estimate, always >= max_k keys[k]
  uint32_t qhead, qtail;  // long-chain queue: front of the queue array
  uint32_t mhead, mtail;  // mini-chain queue: back of the queue array
  uint32_t item;
#ifdef PMH_STATS
  uint32_t st[24];
#endif
};

// Per-round view of one set, kept in registers.
struct Round {
  const uint64_t* ids;
  const double* w;
  uint32_t n, m, imax;
  uint32_t qcap;
  uint64_t K0;     // seed hash
  double T, Tprev; // generate points below T; points below Tprev were handled
  const LogCell* lt;  // logarithm table (LDS copy)
};

// Weight of element p; binary sets (no weight array) have every weight 1.
__device__ __forceinline__ double elem_w(const Round& R, uint32_t p) { return R.w ? R.w[p] : 1.0; }

__device__ __forceinline__ uint64_t shared_kmax(Shared& sm) {
  return __hip_atomic_load(&sm.kmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int NW>
__device__ uint64_t block_max_keys(const uint64_t* keys, uint32_t m, Shared& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  PMH_TIC(t_bm);
  uint64_t v = 0;
  for (uint32_t k = tid; k < m; k += NW * 64) {
    uint64_t x = keys[k];
    v = x > v ? x : v;
  }
  v = wave_max_u64(v);
  if (lane == 0) sm.red_u[wv] = v;
  __syncthreads();
  if (tid == 0) {
    PMH_STAT(sm, kStBlockMax, 1);
    uint64_t r = sm.red_u[0];
    for (int i = 1; i < NW; ++i) r = sm.red_u[i] > r ? sm.red_u[i] : r;
    sm.kmax = r;
  }
  __syncthreads();
  PMH_TOC(sm, kStCycBlockMax, t_bm);
  return sm.kmax;
}

__device__ __forceinline__ uint64_t wave_max_keys(const uint64_t* keys, uint32_t m, int lane) {
  uint64_t v = 0;
  for (uint32_t k = lane; k < m; k += 64) {
    uint64_t x = lds_load_u64(&keys[k]);
    v = x > v ? x : v;
  }
  return wave_max_u64(v);
}

// Long streams go to the front of the queue array, medium streams to the back.
__device__ __forceinline__ void push_long(Shared& sm, ChainEntry* q, uint32_t p, uint32_t i, uint64_t tacc) {
  const uint32_t slot = atomicAdd(&sm.qtail, 1u);
  q[slot] = ChainEntry{p, i, tacc};
}
__device__ __forceinline__ void push_mini(Shared& sm, ChainEntry* q, uint32_t qcap, uint32_t p, uint32_t i,
                                          uint64_t tacc) {
  const uint32_t slot = atomicAdd(&sm.mtail, 1u);
  q[qcap - 1 - slot] = ChainEntry{p, i, tacc};
}

// ProbMinHash3 (Sec. 2.5): point i of an element of weight w lies in
// [(i-1)/w, i/w), so a later round need not regenerate the points below Tprev.
// Points 1..f with f = floor(w Tprev (1 - 2^-40)) end below Tprev by a relative
// margin far above the rounding of their computed values (a few units of
// 2^-53), so they are skipped and the round starts at point f + 1.  Returns
// imax + 1 when every point of the stream lies below Tprev.
template <int V>
__device__ __forceinline__ uint32_t first_index(double w, double Tprev, uint32_t imax) {
  if (V != 3 || !(Tprev > 0.0)) return 1;
  const double f = floor(w * Tprev * (1.0 - 0x1p-40));
  if (!(f >= 1.0)) return 1;
  return f >= (double)imax ? imax + 1 : (uint32_t)f + 1;
}

// ------------------------------------------------------------- lane mode
// Returns after the element's points below R.T are applied, or after pushing
// the element to a chain queue.
template <int V, int NW>
__device__ __forceinline__ int lane_elem(const HashArgs& A, const Round& R, uint32_t p, double winv,
                                          uint64_t K, uint64_t kmax, uint64_t* keys, Shared& sm,
                                          ChainEntry* q, int budget, uint32_t i0) {
  const Tables& t = A.t;
  const uint32_t m = R.m;
  const LogCell* lt = R.lt;
  if constexpr (V == 1) {
    uint64_t tacc = 0;
    uint32_t i = 1;
    uint64_t pb = pbase(K, 1);
    for (int step = 0;; ++step, pb += kPointStep) {
      if (step == budget) {
        push_mini(sm, q, R.qcap, p, i, tacc);
        return step;
      }
      const uint64_t w0 = mix64(pb);
      tacc += spacing_fixed(exp1(w0, lt));
      const double x = winv * fixed_value(tacc);
      PMH_STAT(sm, kStLanePts, 1);
      if (!(x < R.T)) return step + 1;
      const uint64_t key = make_key(x, p);
      if (key >= kmax) return step + 1;
      if (x >= R.Tprev) {
        PMH_STAT(sm, kStLaneApply, 1);
        lds_min(keys, lemire(w0, pb, m, t), key);
      }
      if (i == R.imax) return step + 1;
      ++i;
    }
  } else if constexpr (V == 3) {
    const double lam = t.te_lam, a3 = t.te_a, c13 = t.te_c1;
    uint32_t i = i0;
    uint64_t pb = pbase(K, i0);
    for (int step = 0;; ++step, pb += kPointStep) {
      const double lb = winv * (double)(i - 1);
      if (!(lb < R.T)) return step;
      if (make_key(lb, p) >= kmax) return step;
      if (step == budget) {
        push_mini(sm, q, R.qcap, p, i, K);
        return step;
      }
      const uint64_t w0 = mix64(pb);
      const double x = A.binary ? lb + u32v(w0) : lb + winv * trunc_exp(w0, pb, lam, a3, c13, t);
      const uint64_t key = make_key(x, p);
      PMH_STAT(sm, kStLanePts, 1);
      if (x >= R.Tprev && key < kmax) {
        PMH_STAT(sm, kStLaneApply, 1);
        lds_min(keys, lemire(w0, pb, m, t), key);
      }
      if (i == R.imax) return step + 1;
      ++i;
    }
  } else {
    // ProbMinHash2/4: the first kFyLaneSteps Fisher-Yates steps with the
    // touched slots kept in registers (step s wrote value tr[s] >> 16 into
    // slot tr[s] & 0xFFFF; m <= 2^14); longer streams restart in chain mode,
    // whose 64-step tiles cost far more per point for short streams.
    constexpr uint32_t kSteps = kFyLaneSteps<V, NW>;
    static_assert(kSteps < kLaneTab, "lane-mode table slice too short");
    constexpr int kUnroll = kFyLaneRolled<V, NW> ? 1 : (int)kSteps;
    extern __shared__ __align__(16) unsigned char dyn[];
    const double* L = reinterpret_cast<const double*>(dyn + kLogCells * sizeof(LogCell) + (size_t)m * 8 +
                                                      (size_t)R.qcap * sizeof(ChainEntry) +
                                                      lane_tab_offset(fy_waves(NW), m, kEpt * NW * 64));
    uint32_t tr[kSteps];
    uint64_t tacc = 0;
    // ProbMinHash4's rolled loop loads the next step's gamma_{i-1},
    // gamma_i - gamma_{i-1} and c1_i one step ahead (index clamped to the
    // slice): at two waves per SIMD the LDS latency was exposed every step.
    constexpr bool kAhead = V == 4 && kFyLaneRolled<V, NW>;
    double gp_n = 0.0, dg_n = 0.0, c1_n = 0.0;
    if constexpr (kAhead) {
      gp_n = L[0];
      dg_n = L[kLaneTab + 1];
      c1_n = L[4 * kLaneTab + 1];
    }
#pragma unroll kUnroll
    for (uint32_t step = 0; step < kSteps; ++step) {
      const uint32_t i = step + 1;
      if (i > m) return (int)step;
      const uint64_t pb = pbase(K, i);
      const uint64_t w0 = mix64(pb);
      double x;
      if constexpr (V == 2) {
        tacc += spacing_fixed(L[i] * exp1(w0, lt));  // beta_i
        x = winv * fixed_value(tacc);
        if (!(x < R.T)) return (int)step + 1;
        if (make_key(x, p) >= kmax) return (int)step + 1;
      } else {
        double gp, dg, c1v;  // gamma_{i-1}, gamma_i - gamma_{i-1}, c1_i
        if constexpr (kAhead) {
          gp = gp_n;
          dg = dg_n;
          c1v = c1_n;
          const uint32_t in = i < kSteps ? i + 1u : i;
          gp_n = L[in - 1];
          dg_n = L[kLaneTab + in];
          c1_n = L[4 * kLaneTab + in];
        } else {
          gp = L[i - 1];
          dg = L[kLaneTab + i];
          c1v = L[4 * kLaneTab + i];
        }
        const double lb = A.binary ? (double)(i - 1) : winv * gp;
        if (!(lb < R.T)) return (int)step;
        if (make_key(lb, p) >= kmax) return (int)step;
        if (A.binary) {
          x = lb + u32v(w0);
        } else if (i < m) {
          x = winv * (gp + dg * trunc_exp(w0, pb, L[2 * kLaneTab + i], L[3 * kLaneTab + i], c1v, t));
        } else {
          x = winv * (gp + t.delta * exp1<false>(w0, lt));
        }
      }
      PMH_STAT(sm, kStLanePts, 1);
      // Fisher-Yates step i: slot j = (i-1) + U{0..m-i}; label = g[j]; g[j] = g[i-1]
      const uint32_t j = (i - 1) + lemire(w0, pb, m - i + 1, t);
      uint32_t l = j, v = i - 1;
#pragma unroll kUnroll
      for (uint32_t s = 0; s < step; ++s) {
        const uint32_t sj = tr[s] & 0xFFFFu, sv = tr[s] >> 16;
        if (sj == j) l = sv;
        if (sj == i - 1) v = sv;
      }
      tr[step] = j | (v << 16);
      const uint64_t key = make_key(x, p);
      if (x >= R.Tprev && key < kmax) lds_min(keys, l, key);
      if (i == m) return (int)step + 1;
    }
    push_long(sm, q, p, 1, K);
    return (int)kSteps;
  }
}

// ------------------------------------------------------------ chain mode
// One wavefront runs one element's stream, 64 consecutive points per step,
// until a point reaches R.T or the stop limit.
template <int V>
__device__ void chain_elem(const HashArgs& A, const Round& R, ChainEntry e, double winv, uint64_t K,
                           uint64_t* keys, uint16_t* g, FyScratch* fs, Shared& sm) {
  const Tables& t = A.t;
  const int lane = threadIdx.x & 63;
  const uint32_t m = R.m;
  const LogCell* lt = R.lt;
  const uint32_t p = e.p;
  const uint32_t end = (V == 2 || V == 4) ? m : R.imax;
  uint64_t kmax = shared_kmax(sm);
  uint32_t i0 = e.i;
  uint64_t tacc = e.tacc;
  if (lane == 0) PMH_STAT(sm, kStChainElems, 1);
  if constexpr (V == 2 || V == 4) {
    i0 = 1;
    tacc = 0;
    {
      // 8 labels per 16-byte store where 8 | m (the array is then 16-byte aligned)
      const uint32_t n8 = (m & 7u) == 0 ? m >> 3 : 0u;
      uint4* g8 = reinterpret_cast<uint4*>(g);
      for (uint32_t c = lane; c < n8; c += 64) {
        uint32_t a = c << 3;
        asm volatile("" : "+v"(a));
        a |= (a + 1u) << 16;
        g8[c] = make_uint4(a, a + 0x00020002u, a + 0x00040004u, a + 0x00060006u);
      }
      for (uint32_t k = (n8 << 3) + lane; k < m; k += 64) g[k] = (uint16_t)k;
    }
    __builtin_amdgcn_wave_barrier();
  }
  uint64_t pb = pbase(K, i0) + (uint64_t)lane * kPointStep;
  // ProbMinHash4: the interval tables of a tile's points (gamma_{i-1},
  // gamma_i - gamma_{i-1}, c1_i) are loaded one tile ahead, so their latency
  // overlaps the previous tile's Fisher-Yates work (indices clamped to the
  // tables; the values of points past m are never used).
  double gp_n = 0.0, dg_n = 0.0, c1_n = 0.0;
  auto tload = [&](uint32_t ii) {
    if constexpr (V == 4) {
      const uint32_t k = ii < m ? ii : m - 1u;
      gp_n = t.gam[(ii <= m ? ii : m) - 1u];
      dg_n = t.dgam[k];
      c1_n = t.c1[k];
    }
  };
  tload(i0 + (uint32_t)lane);
  for (uint32_t tile = 1;; ++tile, pb += 64ull * kPointStep) {
    const uint32_t i = i0 + (uint32_t)lane;
    const bool valid = i <= end;
    const double gp = gp_n, dg = dg_n, c1v = c1_n;
    tload(i + 64u);
    const uint64_t w0 = mix64(pb);
    double x = 0.0;
    uint64_t key = kEmptyKey;
    bool stop;
    uint64_t tl = 0;
    if constexpr (V == 1 || V == 2) {
      uint64_t d = 0;
      if (valid) {
        double E = exp1(w0, lt);
        if constexpr (V == 2) E = t.beta[i] * E;
        d = spacing_fixed(E);
      }
      tl = tacc + wave_incl_scan_u64(d, lane);
      x = winv * fixed_value(tl);
      key = make_key(x, p);
      stop = !valid || !(x < R.T) || key >= kmax;
    } else if constexpr (V == 3) {
      const double lb = winv * (double)(i - 1);
      stop = !valid || !(lb < R.T) || make_key(lb, p) >= kmax;
      if (!stop) {
        x = A.binary ? lb + u32v(w0) : lb + winv * trunc_exp(w0, pb, t.te_lam, t.te_a, t.te_c1, t);
        key = make_key(x, p);
      }
    } else {
      stop = !valid;
      if (valid) {
        const double lb = A.binary ? (double)(i - 1) : winv * gp;
        stop = !(lb < R.T) || make_key(lb, p) >= kmax;
      }
      if (!stop) {
        if (A.binary) {
          x = (double)(i - 1) + u32v(w0);
        } else if (i < m) {
          // the sampler's fast path needs c1 only; lambda_i and a_i are read
          // when it falls through
          double e = c1v * u32v(w0);
          if (!(e < 1.0)) e = te_slow(pb, t.lam[i], t.a[i], c1v, t.te_rounds, t.expm1c);
          x = winv * (gp + dg * e);
        } else {
          x = winv * (gp + t.delta * exp1<false>(w0, lt));
        }
        key = make_key(x, p);
      }
    }
    const uint64_t stopmask = __builtin_amdgcn_ballot_w64(stop);
    const int first = stopmask ? __builtin_ctzll(stopmask) : 64;
    const bool active = lane < first;
    const bool apply = active && x >= R.Tprev && key < kmax;
    if (lane == 0) {
      PMH_STAT(sm, kStChainTiles, 1);
      PMH_STAT(sm, kStChainPts, first);
    }
    uint32_t label = 0;
    if constexpr (V == 1 || V == 3) {
      if (apply) label = lemire(w0, pb, m, t);
    } else {
      // 64 Fisher-Yates steps at once.  Step L (point i0+L) consumes position
      // P = i-1 and draws slot j >= P; its label is g[j] as the latest earlier
      // step drawing slot j left it (else the tile's initial g[j]), and it
      // writes into slot j the value g[P] held before it: the value the latest
      // earlier step drawing slot P wrote (else the initial g[P]).  No later
      // step draws slot P (its slots lie at or above its own position > P),
      // and a step drawing its own position (j = P) changes nothing later
      // steps see, so only j > P enters the window table.  The tables find
      // those latest steps; chains of steps writing each other's positions
      // are resolved by pointer jumping.
      const int P = (int)i - 1;
      const int j = active ? P + (int)lemire(w0, pb, m - i + 1, t) : -1;
      const int r = j - ((int)i0 - 1);  // window index of slot j (>= lane)
      const int h = j & (kFyBuckets - 1);
      const bool inwin = active && j != P && r < 64;
      // the lane's bit and table address are rebuilt per tile: hoisted out of
      // the loop they stay live through the point generation (+8 VGPRs)
      int ln = lane;
      asm volatile("" : "+v"(ln));
      const uint64_t bit = 1ull << ln;
      if (inwin)
        __hip_atomic_fetch_max(&fs->win[r], (uint32_t)ln + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (active) __hip_atomic_fetch_or(&fs->bkt[h], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __builtin_amdgcn_wave_barrier();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const int lastP = active ? (int)fs->win[ln] - 1 : -1;  // an earlier step (j > P above)
      uint64_t mates = active ? fs->bkt[h] & ~bit : 0ull;
      __builtin_amdgcn_wave_barrier();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (inwin) fs->win[r] = 0u;
      if (active) fs->bkt[h] = 0ull;
      // Among the bucket mates (highest lane first): a later step with the
      // same slot (bit 8 of jl), and the latest earlier one (jl & 0xFF, 0xFF:
      // none).
      int jl = 0xFF;
      while (__builtin_amdgcn_ballot_w64(mates != 0ull)) {
        const int c = mates ? 63 - __builtin_clzll(mates) : lane;
        const int jc = __shfl(j, c);
        if (mates) {
          mates &= ~(1ull << c);
          if (jc == j) {
            if (c > lane) {
              jl |= 0x100;
            } else {
              jl = (jl & 0x100) | c;
              mates = 0ull;
            }
          }
        }
      }
      const int lastJ = (jl & 0xFF) == 0xFF ? -1 : (jl & 0xFF);
      const bool later = (jl & 0x100) != 0;
      const int gj = active ? (int)g[j] : 0;
      const int gp = active ? (int)g[P] : 0;
      int v = gp, ptr = lastP;  // value step L writes = g[P] at step L
      while (__builtin_amdgcn_ballot_w64(ptr >= 0)) {
        const int src = ptr >= 0 ? ptr : lane;
        const int vv = __shfl(v, src);
        const int pp = __shfl(ptr, src);
        if (ptr >= 0) {
          v = vv;
          ptr = pp;
        }
      }
      const int fromJ = __shfl(v, lastJ >= 0 ? lastJ : lane);
      label = (uint32_t)(lastJ >= 0 ? fromJ : gj);
      __builtin_amdgcn_wave_barrier();
      if (first == 64 && active && !later) g[j] = (uint16_t)v;
      __builtin_amdgcn_wave_barrier();
    }
    if (apply) {
      PMH_STAT(sm, kStApply, 1);
      lds_min(keys, label, key);
    }
    if (first < 64) break;
    if constexpr (V == 1 || V == 2) tacc = readlane_u64(tl, 63);
    i0 += 64;
    if ((tile & 15) == 0) {  // tighten the shared stop limit now and then
      const uint64_t km = wave_max_keys(keys, m, lane);
      if (lane == 0 && km < shared_kmax(sm)) atomicMin((unsigned long long*)&sm.kmax, (unsigned long long)km);
    }
    const uint64_t ks = shared_kmax(sm);
    kmax = ks < kmax ? ks : kmax;
  }
}

// Mini-chain mode (ProbMinHash1/3): the wave is split into groups of G lanes,
// each running one medium-length stream G consecutive points per step and
// taking the next queued stream as soon as its own ends.  Streams reach this
// mode after the lane budget with a few points left, so narrow groups waste
// fewer lanes on a stream's last step (4 lanes measured faster than 2 or 8).
constexpr int kMiniLanes = 4;
template <int V, int G>
__device__ void mini_pass(const HashArgs& A, const Round& R, uint64_t* keys, ChainEntry* q, Shared& sm) {
  const Tables& t = A.t;
  const int lane = threadIdx.x & 63;
  const int j = lane & (G - 1), leader = lane & ~(G - 1), grp = lane / G;
  const uint32_t m = R.m, end = R.imax;
  const LogCell* lt = R.lt;
  const uint32_t mtail = sm.mtail;
  bool have = false;
  uint32_t p = 0, i0 = 1;
  uint64_t tacc = 0, K = 0, pb = 0;
  double winv = 0.0;
  uint64_t kmax = shared_kmax(sm);
  for (uint32_t step = 0;; ++step) {
    if (!have) {  // group-uniform
      uint32_t e = 0;
      if (j == 0) e = atomicAdd(&sm.mhead, 1u);
      e = (uint32_t)__shfl((int)e, leader);
      if (e < mtail) {
        const ChainEntry ce = q[R.qcap - 1 - e];
        p = ce.p;
        i0 = ce.i;
        tacc = V == 3 ? 0 : ce.tacc;
        winv = 1.0 / elem_w(R, p);
        K = V == 3 ? ce.tacc : mix64(R.ids[p] ^ R.K0);
        pb = pbase(K, i0) + (uint64_t)j * kPointStep;
        have = true;
        if (j == 0) PMH_STAT(sm, kStMiniElems, 1);
      }
    }
    if (__builtin_amdgcn_ballot_w64(have) == 0) break;
    const uint32_t i = i0 + (uint32_t)j;
    const bool valid = have && i <= end;
    const uint64_t w0 = mix64(pb);
    double x = 0.0;
    uint64_t key = kEmptyKey, tl = 0;
    bool stop;
    if constexpr (V == 1) {
      const uint64_t d = group_incl_scan_u64<G>(valid ? spacing_fixed(exp1(w0, lt)) : 0, j);
      tl = tacc + d;
      x = winv * fixed_value(tl);
      key = make_key(x, p);
      stop = !valid || !(x < R.T) || key >= kmax;
    } else {
      const double lb = winv * (double)(i - 1);
      stop = !valid || !(lb < R.T) || make_key(lb, p) >= kmax;
      if (!stop) {
        x = A.binary ? lb + u32v(w0) : lb + winv * trunc_exp(w0, pb, t.te_lam, t.te_a, t.te_c1, t);
        key = make_key(x, p);
      }
    }
    const uint64_t smask = __builtin_amdgcn_ballot_w64(stop);
    const uint32_t bits = (uint32_t)(smask >> (grp * G)) & ((1u << G) - 1u);
    const int first = __builtin_ctz(bits | (1u << G));
    const bool apply = have && j < first && x >= R.Tprev && key < kmax;
    if (lane == 0) PMH_STAT(sm, kStMiniSteps, 1);
    if (have && j == 0) PMH_STAT(sm, kStMiniPts, first);
    if (apply) {
      PMH_STAT(sm, kStApply, 1);
      lds_min(keys, lemire(w0, pb, m, t), key);
    }
    const uint64_t tlast = shfl_u64(tl, leader + G - 1);
    if (have) {
      if (first < G) {
        have = false;
      } else {
        i0 += G;
        pb += (uint64_t)G * kPointStep;
        tacc = tlast;
      }
    }
    if ((step & 3) == 3) {
      const uint64_t ks = shared_kmax(sm);
      kmax = ks < kmax ? ks : kmax;
    }
  }
}

template <int V, int NW>
__device__ void chain_pass(const HashArgs& A, const Round& R, uint64_t* keys, ChainEntry* q, uint16_t* fy,
                           Shared& sm) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // fy: fy_waves(NW) FyScratch tables, then as many label arrays of m
  constexpr int NF = fy_waves(NW);
  FyScratch* fs = (V == 2 || V == 4) ? reinterpret_cast<FyScratch*>(fy) + wv : nullptr;
  uint16_t* g = (V == 2 || V == 4) ? reinterpret_cast<uint16_t*>(reinterpret_cast<FyScratch*>(fy) + NF) + (size_t)wv * R.m
                                   : nullptr;
  const uint32_t qtail = sm.qtail;
  PMH_TIC(t_chain);
  // waves without a label array take no chain element (wave-uniform)
  for (; !((V == 2 || V == 4) && wv >= NF);) {  // long streams first
    uint32_t e = 0;
    if (lane == 0) e = atomicAdd(&sm.qhead, 1u);
    e = (uint32_t)__shfl((int)e, 0);
    if (e >= qtail) break;
    const ChainEntry ce = q[e];
    chain_elem<V>(A, R, ce, 1.0 / elem_w(R, ce.p), V != 1 ? ce.tacc : mix64(R.ids[ce.p] ^ R.K0), keys, g, fs,
                  sm);
  }
  PMH_TOC(sm, kStCycChain, t_chain);
  PMH_TIC(t_mini);
  if constexpr (V == 1 || V == 3) mini_pass<V, kMiniLanes>(A, R, keys, q, sm);
  PMH_TOC(sm, kStCycMini, t_mini);
  PMH_TIC(t_bar);
  __syncthreads();
  if (threadIdx.x == 0) {
    sm.qhead = sm.qtail = 0;
    sm.mhead = sm.mtail = 0;
  }
  __syncthreads();
  PMH_TOC(sm, kStCycBarrier, t_bar);
}

// ------------------------------------------------------------- one set
// Per-set registers and LDS initialisation shared by whole sets and chunks.
template <int NW>
__device__ __forceinline__ Round set_round(const HashArgs& A, uint64_t set, uint32_t qcap, const LogCell* lt,
                                           Shared& sm) {
  const int tid = threadIdx.x;
  const uint64_t a = A.off[set], b = A.off[set + 1];
  const uint64_t n64 = b - a;
  Round R;
  R.ids = A.ids + a;
  R.w = A.w ? A.w + a : nullptr;
  R.n = (uint32_t)(n64 > kMaxSet ? 0 : n64);
  R.m = A.m;
  R.imax = A.imax;
  R.qcap = qcap;
  R.K0 = A.seedhash;
  R.lt = lt;
  R.T = R.Tprev = 0.0;
  if (n64 > kMaxSet && tid == 0) atomicOr(A.status, kStatusSetTooLarge);
#ifdef PMH_STATS
  if (tid < 24) sm.st[tid] = 0;
  __syncthreads();
  if (tid == 0) PMH_STAT(sm, kStSets, 1);
#endif
  return R;
}

// Sum of the valid weights of elements [p0, p1); flags invalid weights.
template <int NW>
__device__ double block_weight_sum(const HashArgs& A, const Round& R, uint32_t p0, uint32_t p1, Shared& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double ws = 0.0;
  bool bad = false;
  for (uint32_t p = p0 + tid; p < p1; p += NW * 64) {
    const double w = elem_w(R, p);
    if (weight_ok(w)) ws += w;
    else if (w != 0.0) bad = true;
  }
  ws = wave_sum_f64(ws);
  __syncthreads();  // red_d may still be read by an earlier reduction
  if (lane == 0) sm.red_d[wv] = ws;
  if (bad) atomicOr(A.status, kStatusWeight);
  __syncthreads();
  double W = 0.0;
  for (int i = 0; i < NW; ++i) W += sm.red_d[i];
  return W;
}

// ProbMinHash4 lane mode over one batch: streams expecting more than
// chain_expect points go to the chain queue, the others run one per lane.  In
// sets whose elements expect more than a point each (`sort`, block-uniform)
// they are first counted into classes by expected points and dealt to the
// lanes longest first through LDS (weights and ids then read again, from
// cache), so the 64 lanes of a wave get streams of similar length: a wave
// runs as many steps as its longest stream; streams expecting more than
// kLaneSure points stay only if the batch holds a wave of them.  Otherwise
// each thread keeps its own prefetched ones, and streams expecting more than
// kLaneSure points go to the chain queue.
template <int V, int NW>
__device__ __forceinline__ void lane_batch(const HashArgs& A, const Round& R, uint32_t base, uint32_t p1,
                                           const double* wc, const uint64_t* idc, double Teff, uint64_t kmax,
                                           uint64_t* keys, ChainEntry* q, uint16_t* fy, Shared& sm, bool sort) {
  constexpr int BS = NW * 64;
  const int tid = threadIdx.x;
  uint32_t pk[kEpt];
  double wk[kEpt];
  uint64_t idk[kEpt];
  int cls[kEpt];
#pragma unroll
  for (uint32_t k = 0; k < kEpt; ++k) {
    cls[k] = -1;
    pk[k] = base + k * BS + tid;
    wk[k] = wc[k];
    idk[k] = idc[k];
    if (pk[k] >= p1) continue;
    const double w = wc[k];
    if (!weight_ok(w)) continue;
    PMH_STAT(sm, kStElems, 1);
    const double lam = w * Teff;  // expected points generated
    if (lam > A.chain_expect || (!sort && lam > (double)kLaneSure)) {
      push_long(sm, q, pk[k], 1, mix64(idc[k] ^ R.K0));
      continue;
    }
    cls[k] = lam < (double)(kSortClasses - 1) ? (int)lam : kSortClasses - 1;
  }
  if (sort) {  // block-uniform
    uint32_t* cnt = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(fy) +
                                                sort_region_offset(fy_waves(NW), R.m));
    uint32_t* off = cnt + kSortClasses;
    uint16_t* idx = reinterpret_cast<uint16_t*>(off + kSortClasses);
    uint32_t pos[kEpt];
#pragma unroll
    for (uint32_t k = 0; k < kEpt; ++k) pos[k] = cls[k] >= 0 ? atomicAdd(&cnt[cls[k]], 1u) : 0u;
    __syncthreads();
    if (tid < 64) {  // offsets, longest class first
      constexpr int kHi = kSortClasses - kLaneSure;  // classes >= kLaneSure come first
      const uint32_t c = tid < kSortClasses ? cnt[kSortClasses - 1 - tid] : 0u;
      const uint32_t incl = wave_incl_scan_u32(c);
      const uint32_t hi = (uint32_t)__shfl((int)incl, kHi - 1);
      if (tid < kSortClasses) {
        // fewer than a wave of long streams: they go to chain mode
        const bool drop = hi < 64u && tid < kHi;
        off[kSortClasses - 1 - tid] = drop ? kNoLane : incl - c - (hi < 64u ? hi : 0u);
      }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kEpt; ++k) {
      if (cls[k] < 0) continue;
      const uint32_t o = off[cls[k]];
      if (o == kNoLane) {
        push_long(sm, q, base + k * BS + tid, 1, mix64(idc[k] ^ R.K0));
        cls[k] = -1;
      } else {
        idx[o + pos[k]] = (uint16_t)(k * BS + tid);
      }
    }
    const uint32_t total = off[0] + cnt[0];  // class 0 comes last
    // one class only (equal weights): nothing to reorder (every wave reads
    // the same counts, so this is block-uniform)
    const int lane = tid & 63;
    const bool one = __builtin_popcountll(__ballot(lane < kSortClasses && cnt[lane & (kSortClasses - 1)] != 0u &&
                                                   off[lane & (kSortClasses - 1)] != kNoLane)) <= 1;
    __syncthreads();
    if (tid < kSortClasses) cnt[tid] = 0u;  // read above; the next batch counts after two more barriers
    if (!one) {
#pragma unroll
      for (uint32_t k = 0; k < kEpt; ++k) {
        const uint32_t s = k * BS + tid;
        cls[k] = s < total ? 0 : -1;
        if (s < total) {
          pk[k] = base + idx[s];
          wk[k] = elem_w(R, pk[k]);
          idk[k] = R.ids[pk[k]];
        }
      }
    }
  }
#pragma unroll
  for (uint32_t k = 0; k < kEpt; ++k) {
    if (cls[k] < 0) continue;
    const int steps = lane_elem<V, NW>(A, R, pk[k], 1.0 / wk[k], mix64(idk[k] ^ R.K0), kmax, keys, sm, q,
                                       A.lane_budget, 1);
#ifdef PMH_STATS
    int mx = steps;
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d));
    if ((threadIdx.x & 63) == __builtin_ctzll(__ballot(true))) PMH_STAT(sm, kStLaneIters, mx);
#else
    (void)steps;
#endif
  }
}

// One round over elements [p0, p1): every point below R.T is generated and
// the ones that can still lower a key are applied (stop limit kmax_start at
// entry, refreshed as keys fall).  Returns the block max of the keys.
template <int V, int NW, bool kPf = false>
__device__ uint64_t round_pass(const HashArgs& A, const Round& R, uint32_t p0, uint32_t p1, uint64_t kmax_start,
                               uint64_t* keys, ChainEntry* q, uint16_t* fy, Shared& sm) {
  constexpr int BS = NW * 64;
  const int tid = threadIdx.x;
  const uint32_t m = R.m, qcap = R.qcap;
  if (tid == 0) {
    sm.kmax = kmax_start;
    sm.qhead = sm.qtail = 0;
    sm.mhead = sm.mtail = 0;
    PMH_STAT(sm, kStRounds, 1);
  }
  __syncthreads();
  const uint32_t batch = kEpt * BS;
  // ProbMinHash2/4: ordering lane-mode streams pays where an element expects
  // more than one point on average (T0 W = m (ln m + c0) points over n
  // elements); sets of mostly one-point elements keep the prefetched order.
  bool sort = false;
  if constexpr (V == 4) sort = (double)R.n < (double)m * (log((double)m) + A.c0);
  // The weights and ids of the next batch are loaded while this one runs
  // (ProbMinHash3 only in its kPf instantiation: the extra registers, 124 ->
  // 148 in four-wave workgroups, cost a wave per SIMD wherever the keys in LDS
  // do not already bound the occupancy, and there the loads are better issued
  // on demand).
  constexpr bool kPrefetch = V != 3 || kPf;
  double wn[kEpt];
  uint64_t idn[kEpt];
#pragma unroll
  for (uint32_t k = 0; k < kEpt; ++k) {
    const uint32_t p = p0 + k * BS + tid;
    wn[k] = kPrefetch && p < p1 ? elem_w(R, p) : 0.0;
    idn[k] = kPrefetch && p < p1 ? R.ids[p] : 0;
  }
  for (uint32_t base = p0, nb = 0; base < p1; base += batch, ++nb) {
    double wc[kEpt];
    uint64_t idc[kEpt];
#pragma unroll
    for (uint32_t k = 0; k < kEpt; ++k) {
      if constexpr (kPrefetch) {
        wc[k] = wn[k];
        idc[k] = idn[k];
        const uint32_t p = base + batch + k * BS + tid;
        if (p < p1) {
          wn[k] = elem_w(R, p);
          idn[k] = R.ids[p];
        }
      } else {
        const uint32_t p = base + k * BS + tid;
        wc[k] = p < p1 ? elem_w(R, p) : 0.0;
        idc[k] = 0;
      }
    }
    PMH_TIC(t_batch);
    const uint64_t kmax = shared_kmax(sm);
    // points above the stop limit's value are never generated: the expected
    // count of an element is its weight times the smaller of T and that value
    const double Tk = kmax == kEmptyKey ? R.T : __longlong_as_double((long long)(kmax & ~kPosMask));
    const double Teff = Tk < R.T ? Tk : R.T;
    if constexpr (V == 4) {
      lane_batch<V, NW>(A, R, base, p1, wc, idc, Teff, kmax, keys, q, fy, sm, sort);
    } else {
#pragma unroll
    for (uint32_t k = 0; k < kEpt; ++k) {
      const uint32_t p = base + k * BS + tid;
      if (p >= p1) break;
      const double w = wc[k];
      if (!weight_ok(w)) continue;
      PMH_STAT(sm, kStElems, 1);
      const uint32_t i0 = first_index<V>(w, R.Tprev, R.imax);
      if (i0 > R.imax) continue;
      const double lam = w * (V == 3 ? Teff - R.Tprev : Teff);  // expected points generated
      // ProbMinHash2/3 queue entries carry K (see ChainEntry)
      uint64_t K = 0;
      if constexpr (V != 1) K = mix64((kPrefetch ? idc[k] : R.ids[p]) ^ R.K0);
      if (lam > A.chain_expect) {
        push_long(sm, q, p, i0, K);
        continue;
      }
      if ((V == 1 || V == 3) && lam > A.mini_expect) {
        push_mini(sm, q, qcap, p, i0, K);
        continue;
      }
      if constexpr (V == 1) K = mix64((kPrefetch ? idc[k] : R.ids[p]) ^ R.K0);
      const double winv = 1.0 / w;
      const int steps = lane_elem<V, NW>(A, R, p, winv, K, kmax, keys, sm, q, A.lane_budget, i0);
#ifdef PMH_STATS
      // wave-level cost of this element slot: the longest lane
      int mx = steps;
      for (int d = 32; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d));
      if ((threadIdx.x & 63) == __builtin_ctzll(__ballot(true))) PMH_STAT(sm, kStLaneIters, mx);
#else
      (void)steps;
#endif
    }
    }
    PMH_TOC(sm, kStCycBatch, t_batch);
    PMH_TIC(t_bar);
    __syncthreads();
    const uint32_t qt = sm.qtail + sm.mtail;  // read by every thread before anyone pushes again
    __syncthreads();
    PMH_TOC(sm, kStCycBarrier, t_bar);
    const bool flush = qt + batch > qcap;
    if (flush && tid == 0) PMH_STAT(sm, kStFlush, 1);
    if (flush) chain_pass<V, NW>(A, R, keys, q, fy, sm);
    if (flush || (nb % (uint32_t)A.kmax_refresh) == (uint32_t)A.kmax_refresh - 1) block_max_keys<NW>(keys, m, sm);
  }
  __syncthreads();
  chain_pass<V, NW>(A, R, keys, q, fy, sm);
  return block_max_keys<NW>(keys, m, sm);
}

// Rounds of growing thresholds over the whole set until every key is final
// (keys must hold the set's current minima on entry, with every point below
// Tprev applied).
template <int V, int NW, bool kPf = false>
__device__ void set_rounds(const HashArgs& A, Round& R, double T, double Tprev, uint64_t kmax_round,
                           uint64_t* keys, ChainEntry* q, uint16_t* fy, Shared& sm) {
  for (int round = 0;; ++round) {
    const bool last = round + 1 >= A.max_rounds || !(T < DBL_MAX) || !(T > 0.0);
    R.T = last ? __longlong_as_double(0x7FF0000000000000ll) : T;
    R.Tprev = Tprev;
    const uint64_t K = round_pass<V, NW, kPf>(A, R, 0, R.n, kmax_round, keys, q, fy, sm);
    if (last || K < make_key(R.T, 0)) break;
    Tprev = R.T;
    T = R.T * A.grow;
    kmax_round = K;
  }
}

// An update call's previous key as it seeds the LDS minima: position bits
// cleared, so that on equal truncated values it stays ahead of every new
// element (all of which come later in the set's element sequence).
__device__ __forceinline__ uint64_t seed_key(uint64_t old) { return old == kEmptyKey ? old : old & ~kPosMask; }

// keys (LDS) -> (position, value, id) of the set's signature.  Update mode
// (A.counts): a component whose LDS key still equals its seed keeps the
// previous key and id; one a new element won takes position base + p.
template <int NW, bool kBbit = false>
__device__ void epilogue(const HashArgs& A, const Round& R, uint64_t set, const uint64_t* keys, Shared& sm) {
  constexpr int BS = NW * 64;
  const int tid = threadIdx.x;
  const uint32_t m = R.m;
  __syncthreads();
  const uint64_t o = set * (uint64_t)m;
  const uint32_t base = A.counts ? A.counts[set] : 0u;  // re-read: not kept live through the rounds
  for (uint32_t k = tid; k < m; k += BS) {
    uint64_t key = keys[k];
    bool fresh = true;
    if (A.counts) {
      const uint64_t old = A.out_keys[o + k];
      if (key == seed_key(old)) {
        key = old;
        fresh = false;
      } else {
        key = (key & ~kPosMask) | (uint64_t)(base + (uint32_t)(key & kPosMask));
      }
    }
    if (A.out_keys) A.out_keys[o + k] = key;
    const bool empty = key == kEmptyKey;
    const uint32_t pos = (uint32_t)(key & kPosMask);
    if (A.out_idx) A.out_idx[o + k] = empty ? 0xFFFFFFFFu : pos;
    if (A.out_val) A.out_val[o + k] = empty ? __longlong_as_double(0x7FF0000000000000ll)
                                            : __longlong_as_double((long long)(key & ~kPosMask));
    if (A.out_id && fresh) A.out_id[o + k] = empty ? 0ull : R.ids[pos - base];
  }
  if (A.counts && tid == 0) A.counts[set] = base + R.n;
  if constexpr (kBbit) {
    // b-bit reduction (Sec. 1.3) of the finished signature: component k
    // (0-based) keeps the b low bits of mix64(mix64(z) + (k + 1) phi), z its
    // element id (0: empty).  A wave's lanes hold consecutive components, so
    // an OR over aligned groups of 64/b lanes assembles each packed word.
    // Its own kernel instantiations: inlined into the others it raised
    // ProbMinHash2's and ProbMinHash4's registers past 3 waves per SIMD.
    const uint32_t lb = (uint32_t)__builtin_ctz(A.bbit_b);  // log2 b
    const uint32_t per = 64u >> lb;
    const uint64_t mask = (1ull << A.bbit_b) - 1ull;
    const uint64_t words = (((uint64_t)m << lb) + 63) >> 6;
    for (uint32_t k0 = 0; k0 < m; k0 += BS) {
      const uint32_t k = k0 + (uint32_t)tid;
      uint64_t f = 0;
      if (k < m) {
        const uint64_t key = keys[k];
        const uint64_t z = key == kEmptyKey ? 0ull : R.ids[(uint32_t)(key & kPosMask)];
        f = (mix64(mix64(z) + (uint64_t)(k + 1) * kPhi) & mask) << ((k & (per - 1)) << lb);
      }
      for (uint32_t d = 1; d < per; d <<= 1) f |= shfl_xor_u64(f, (int)d);
      if (k < m && (k & (per - 1)) == 0) A.out_bbit[set * words + (k >> (6 - lb))] = f;
    }
  }
  __syncthreads();
#ifdef PMH_STATS
  if (tid < kStCount && A.points) atomicAdd((unsigned long long*)&A.points[tid], (unsigned long long)sm.st[tid]);
#endif
}

template <int V, int NW, bool kBbit = false, bool kPf = false>
__device__ void process_set(const HashArgs& A, uint64_t set, uint64_t* keys, ChainEntry* q, uint32_t qcap,
                            uint16_t* fy, const LogCell* lt, Shared& sm) {
  Round R = set_round<NW>(A, set, qcap, lt, sm);
  PMH_TIC(t_set);
  uint64_t kmax0 = kEmptyKey;
  if (A.counts) {
    // Update: the new elements extend the set's element sequence after the
    // elements it has absorbed; the previous keys seed the minima and the
    // stop limit.  A sequence beyond the position field takes no element:
    // the epilogue writes the set back as it was.
    const uint64_t n64 = A.off[set + 1] - A.off[set];
    if ((uint64_t)A.counts[set] + n64 > kMaxSet) {
      if (threadIdx.x == 0) atomicOr(A.status, kStatusSetTooLarge);
      R.n = 0;
    }
    const uint64_t o = set * (uint64_t)R.m;
    for (uint32_t k = threadIdx.x; k < R.m; k += NW * 64) keys[k] = seed_key(A.out_keys[o + k]);
    kmax0 = block_max_keys<NW>(keys, R.m, sm);
  } else {
    for (uint32_t k = threadIdx.x; k < R.m; k += NW * 64) keys[k] = kEmptyKey;
  }
  const double W = block_weight_sum<NW>(A, R, 0, R.n, sm);
  if (W > 0.0) set_rounds<V, NW, kPf>(A, R, (double)R.m * (log((double)R.m) + A.c0) / W, 0.0, kmax0, keys, q, fy, sm);
  PMH_TOC(sm, kStCycSet, t_set);
  epilogue<NW, kBbit>(A, R, set, keys, sm);
}

// One chunk of a set split across workgroups.  The chunk generates every
// point below its own threshold T_c (from its weight sum scaled to the whole
// set), merges its keys into the set's merge row with a 64-bit atomic min and
// lowers the set's smallest threshold.  Finishing the set is left to
// k_big_finish, after the kernel boundary has made every merge visible.
template <int V, int NW, bool kPf = false>
__device__ void process_chunk(const HashArgs& A, uint64_t set, uint32_t big, uint32_t chunk, uint64_t* keys,
                              ChainEntry* q, uint32_t qcap, uint16_t* fy, const LogCell* lt, Shared& sm) {
  constexpr int BS = NW * 64;
  const int tid = threadIdx.x;
  Round R = set_round<NW>(A, set, qcap, lt, sm);
  const uint32_t m = R.m;
  const uint32_t csize = 1u << (A.split_log2 - 1);
  const uint32_t p0 = chunk * csize, p1 = p0 + csize < R.n ? p0 + csize : R.n;
  uint64_t* gk = A.big_keys + set * (uint64_t)m;
  for (uint32_t k = tid; k < m; k += BS) keys[k] = kEmptyKey;
  const double Wc = block_weight_sum<NW>(A, R, p0, p1, sm);
  if (Wc > 0.0) {
    const double West = Wc * ((double)R.n / (double)(p1 - p0));
    const double T = (double)m * (log((double)m) + A.c0 + A.c0_split) / West;
    R.T = T > 0.0 ? T : __longlong_as_double(0x7FF0000000000000ll);
    R.Tprev = 0.0;
    round_pass<V, NW, kPf>(A, R, p0, p1, kEmptyKey, keys, q, fy, sm);
    for (uint32_t k = tid; k < m; k += BS)
      if (keys[k] != kEmptyKey) atomicMin((unsigned long long*)&gk[k], (unsigned long long)keys[k]);
    if (tid == 0) atomicMin((unsigned long long*)&A.big_state[big], (unsigned long long)__double_as_longlong(R.T));
  }
  __syncthreads();
#ifdef PMH_STATS
  if (tid < kStCount && A.points) atomicAdd((unsigned long long*)&A.points[tid], (unsigned long long)sm.st[tid]);
#endif
}

// Completion of a split set: every merged key below the smallest chunk
// threshold Tmin is final (all points below Tmin were applied); otherwise one
// unbounded round over the whole set finishes it.  Then the epilogue.
template <int V, int NW, bool kBbit = false>
__device__ void finish_set(const HashArgs& A, uint64_t set, uint32_t big, uint64_t* keys, ChainEntry* q,
                           uint32_t qcap, uint16_t* fy, const LogCell* lt, Shared& sm) {
  const int tid = threadIdx.x;
  Round R = set_round<NW>(A, set, qcap, lt, sm);
  const uint32_t m = R.m;
  const uint64_t* gk = A.big_keys + set * (uint64_t)m;
  for (uint32_t k = tid; k < m; k += NW * 64) keys[k] = gk[k];
  const double Tmin = __longlong_as_double((long long)A.big_state[big]);
  __syncthreads();
  const uint64_t K = block_max_keys<NW>(keys, m, sm);
  if (!(K < make_key(Tmin, 0))) {  // some label not covered below the smallest threshold:
    if (tid == 0) PMH_STAT(sm, kStRepairs, 1);  // more rounds over the whole set, above Tmin
    set_rounds<V, NW>(A, R, Tmin * A.grow, Tmin, K, keys, q, fy, sm);
  }
  epilogue<NW, kBbit>(A, R, set, keys, sm);
}

// Dynamic LDS: log table (kLogCells cells) | keys[m] | chain queue |
// Fisher-Yates arrays, sort region and lane-mode tables (ProbMinHash2/4).
template <int V, int NW>
__device__ __forceinline__ void carve(const HashArgs& A, LogCell*& lt, uint64_t*& keys, ChainEntry*& q,
                                      uint32_t& qcap, uint16_t*& fy) {
  extern __shared__ __align__(16) unsigned char dyn[];
  const uint32_t m = A.m;
  lt = reinterpret_cast<LogCell*>(dyn);
  unsigned char* base = dyn + kLogCells * sizeof(LogCell);
  keys = reinterpret_cast<uint64_t*>(base);
  q = reinterpret_cast<ChainEntry*>(base + (size_t)m * 8);
  qcap = A.qcap;
  fy = (V == 2 || V == 4) ? reinterpret_cast<uint16_t*>(base + (size_t)m * 8 + (size_t)qcap * sizeof(ChainEntry))
                          : nullptr;
  const LogCell* src = reinterpret_cast<const LogCell*>(A.t.ltab);
  for (uint32_t k = threadIdx.x; k < kLogCells; k += NW * 64) lt[k] = src[k];
  if constexpr (V == 2 || V == 4) {
    uint64_t* z = reinterpret_cast<uint64_t*>(fy);
    for (uint32_t k = threadIdx.x; k < fy_waves(NW) * sizeof(FyScratch) / 8; k += NW * 64) z[k] = 0ull;
    uint32_t* cnt = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(fy) + sort_region_offset(fy_waves(NW), m));
    if (threadIdx.x < kSortClasses) cnt[threadIdx.x] = 0u;
    double* ltab = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(fy) +
                                             lane_tab_offset(fy_waves(NW), m, kEpt * NW * 64));
    const uint32_t ix = threadIdx.x;  // kLaneTab <= 64 threads
    if (ix < kLaneTab) {
      if constexpr (V == 2) {
        ltab[ix] = ix <= m ? A.t.beta[ix] : 0.0;
      } else {
        const bool in = ix < m;
        ltab[ix] = in ? A.t.gam[ix] : 0.0;
        ltab[kLaneTab + ix] = in ? A.t.dgam[ix] : 0.0;
        ltab[2 * kLaneTab + ix] = in ? A.t.lam[ix] : 0.0;
        ltab[3 * kLaneTab + ix] = in ? A.t.a[ix] : 0.0;
        ltab[4 * kLaneTab + ix] = in ? A.t.c1[ix] : 0.0;
      }
    }
  }
  __syncthreads();
}

// Persistent grid.  Work items: first the chunks of the split sets (heavy
// first), then one item per remaining set.  meta = {split sets, chunk items,
// total items}, written by k_order.
template <int V, int NW, bool kBbit = false, bool kPf = false>
__global__ __launch_bounds__(NW * 64) void k_hash_persistent(HashArgs A) {
  __shared__ Shared sm;
  __shared__ uint32_t job[3];
  LogCell* lt;
  uint64_t* keys;
  ChainEntry* q;
  uint32_t qcap;
  uint16_t* fy;
  carve<V, NW>(A, lt, keys, q, qcap, fy);
  const uint32_t num_big = A.meta[0], vbig = A.meta[1], total = A.meta[2];
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t v = atomicAdd(&A.counter[0], 1u);
      job[0] = v;
      if (v < vbig) {  // chunk of a split set: find b with prefix[b] <= v < prefix[b+1]
        uint32_t lo = 0, hi = num_big;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (A.big_prefix[mid] <= v) lo = mid;
          else hi = mid;
        }
        job[1] = lo;
        job[2] = v - A.big_prefix[lo];
      } else if (v < total) {
        job[1] = num_big + (v - vbig);
      }
    }
    __syncthreads();
    const uint32_t v = job[0], j1 = job[1], j2 = job[2];
    __syncthreads();
    if (v >= total) break;
    if (v < vbig) process_chunk<V, NW, kPf>(A, A.order[j1], j1, j2, keys, q, qcap, fy, lt, sm);
    else process_set<V, NW, kBbit, kPf>(A, A.order[j1], keys, q, qcap, fy, lt, sm);
  }
}

// Persistent grid over the split sets (order[0 .. meta[0])), after the
// chunk kernel.
template <int V, int NW, bool kBbit = false>
__global__ __launch_bounds__(NW * 64) void k_big_finish(HashArgs A) {
  __shared__ Shared sm;
  __shared__ uint32_t job;
  LogCell* lt;
  uint64_t* keys;
  ChainEntry* q;
  uint32_t qcap;
  uint16_t* fy;
  const uint32_t num_big = A.meta[0];
  if (num_big == 0) return;
  carve<V, NW>(A, lt, keys, q, qcap, fy);
  for (;;) {
    if (threadIdx.x == 0) job = atomicAdd(&A.counter[1], 1u);
    __syncthreads();
    const uint32_t b = job;
    __syncthreads();
    if (b >= num_big) break;
    finish_set<V, NW, kBbit>(A, A.order[b], b, keys, q, qcap, fy, lt, sm);
  }
}

template <int V, int NW>
__global__ __launch_bounds__(NW * 64) void k_hash_one(HashArgs A, uint64_t set) {
  __shared__ Shared sm;
  LogCell* lt;
  uint64_t* keys;
  ChainEntry* q;
  uint32_t qcap;
  uint16_t* fy;
  carve<V, NW>(A, lt, keys, q, qcap, fy);
  process_set<V, NW>(A, set, keys, q, qcap, fy, lt, sm);
}

// --------------------------------------------------------------- P-MinHash
// Sec. 1.1, algorithm P-MinHash: every element of positive weight draws one
// exponential value per component, scaled by 1/w; each component keeps the
// smallest key.  The k-th value of element K uses word slot 128 of point k
// of the element's counter stream (no ProbMinHash stream uses that slot),
// Exp(1) by the stream logarithm, value fl(winv * Exp(1)), the same key.
// A workgroup of kPminThreads owns one work item (a whole set or a chunk of
// a split set).  Its threads own components k = tid + j*kPminThreads,
// kPminComps of them per pass, with their minima in registers; the item's
// elements are staged in LDS (key hash and 1/w computed once per pass) and
// every thread runs through all of them.  Work is n*m points, so the split
// threshold is low: sets of >= 2^11 elements run as 1,024-element chunks
// merged by 64-bit atomic min (exact: min is associative).
constexpr int kPminThreads = 256;
constexpr int kPminComps = 4;
constexpr uint32_t kPminSlot = 128;
constexpr uint32_t kPminSplitLog2 = 11;

struct PminElem {
  uint64_t K;
  double winv;  // 0: skipped element (zero or invalid weight)
};

__device__ void pmin_item(const HashArgs& A, uint64_t set, uint32_t p0, uint32_t p1, uint64_t* gk,
                          const LogCell* lt, PminElem* st) {
  const int tid = threadIdx.x;
  const uint64_t a = A.off[set];
  const uint64_t* ids = A.ids + a;
  const double* w = A.w + a;
  const uint32_t m = A.m;
  const uint64_t o = set * (uint64_t)m;
  for (uint32_t k0 = 0; k0 < m; k0 += kPminThreads * kPminComps) {
    uint64_t kmin[kPminComps], koff[kPminComps];
#pragma unroll
    for (int j = 0; j < kPminComps; ++j) {
      const uint64_t k = k0 + (uint32_t)(j * kPminThreads + tid);  // component k+1 of the paper
      kmin[j] = kEmptyKey;
      koff[j] = ((((k + 1) << 8) | kPminSlot) + 1) * kPhi;  // word (k+1, slot) = mix64(K + koff)
    }
    for (uint32_t b = p0; b < p1; b += kPminThreads) {
      __syncthreads();  // the previous batch is consumed
      const uint32_t p = b + (uint32_t)tid;
      if (p < p1) {
        const double wt = w[p];
        const bool ok = weight_ok(wt);
        if (!ok && wt != 0.0) atomicOr(A.status, kStatusWeight);
        st[tid] = PminElem{ok ? mix64(ids[p] ^ A.seedhash) : 0ull, ok ? 1.0 / wt : 0.0};
      }
      __syncthreads();
      const uint32_t cnt = p1 - b < (uint32_t)kPminThreads ? p1 - b : (uint32_t)kPminThreads;
      for (uint32_t e = 0; e < cnt; ++e) {
        const PminElem el = st[e];
        if (el.winv == 0.0) continue;  // uniform across the workgroup
#pragma unroll
        for (int j = 0; j < kPminComps; ++j) {
          const uint64_t key = make_key(el.winv * exp1(mix64(el.K + koff[j]), lt), b + e);
          kmin[j] = key < kmin[j] ? key : kmin[j];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kPminComps; ++j) {
      const uint32_t k = k0 + (uint32_t)(j * kPminThreads + tid);
      if (k >= m) continue;
      const uint64_t key = kmin[j];
      if (gk) {
        if (key != kEmptyKey) atomicMin((unsigned long long*)&gk[k], (unsigned long long)key);
        continue;
      }
      const bool empty = key == kEmptyKey;
      const uint32_t pos = (uint32_t)(key & kPosMask);
      if (A.out_keys) A.out_keys[o + k] = key;
      if (A.out_idx) A.out_idx[o + k] = empty ? 0xFFFFFFFFu : pos;
      if (A.out_val) A.out_val[o + k] = empty ? __longlong_as_double(0x7FF0000000000000ll)
                                              : __longlong_as_double((long long)(key & ~kPosMask));
      if (A.out_id) A.out_id[o + k] = empty ? 0ull : ids[pos];
    }
  }
}

__device__ __forceinline__ void pmin_load_table(const HashArgs& A, LogCell* lt) {
  const LogCell* src = reinterpret_cast<const LogCell*>(A.t.ltab);
  for (uint32_t k = threadIdx.x; k < kLogCells; k += kPminThreads) lt[k] = src[k];
  __syncthreads();
}

// Persistent grid over the items of k_order's work list (split_log2 =
// kPminSplitLog2 when a merge row exists): chunks of the split sets first,
// then one item per remaining set, heavy first.
__global__ __launch_bounds__(kPminThreads) void k_pmin(HashArgs A) {
  __shared__ LogCell lt[kLogCells];
  __shared__ PminElem st[kPminThreads];
  __shared__ uint32_t job[3];
  pmin_load_table(A, lt);
  const uint32_t num_big = A.meta[0], vbig = A.meta[1], total = A.meta[2];
  const uint32_t csize = A.split_log2 ? 1u << (A.split_log2 - 1) : 0u;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t v = atomicAdd(&A.counter[0], 1u);
      job[0] = v;
      if (v < vbig) {
        uint32_t lo = 0, hi = num_big;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (A.big_prefix[mid] <= v) lo = mid;
          else hi = mid;
        }
        job[1] = lo;
        job[2] = v - A.big_prefix[lo];
      } else if (v < total) {
        job[1] = num_big + (v - vbig);
      }
    }
    __syncthreads();
    const uint32_t v = job[0], j1 = job[1], j2 = job[2];
    __syncthreads();
    if (v >= total) break;
    const uint64_t set = A.order[j1];
    const uint64_t n64 = A.off[set + 1] - A.off[set];
    if (n64 > kMaxSet) {  // reported by k_order; outputs stay empty
      pmin_item(A, set, 0, 0, nullptr, lt, st);
      continue;
    }
    const uint32_t n = (uint32_t)n64;
    if (v < vbig) {
      const uint32_t p0 = j2 * csize, p1 = p0 + csize < n ? p0 + csize : n;
      pmin_item(A, set, p0, p1, A.big_keys + set * (uint64_t)A.m, lt, st);
    } else {
      pmin_item(A, set, 0, n, nullptr, lt, st);
    }
  }
}

// Outputs of the split sets from their merged rows (after the chunk kernel).
__global__ __launch_bounds__(kPminThreads) void k_pmin_finish(HashArgs A) {
  const uint32_t num_big = A.meta[0];
  const uint32_t m = A.m;
  for (uint32_t b = blockIdx.x; b < num_big; b += gridDim.x) {
    const uint64_t set = A.order[b];
    const uint64_t o = set * (uint64_t)m;
    const uint64_t* ids = A.ids + A.off[set];
    for (uint32_t k = threadIdx.x; k < m; k += kPminThreads) {
      const uint64_t key = A.big_keys[o + k];  // read before any output of this entry is written
      const bool empty = key == kEmptyKey;
      const uint32_t pos = (uint32_t)(key & kPosMask);
      if (A.out_keys) A.out_keys[o + k] = key;
      if (A.out_idx) A.out_idx[o + k] = empty ? 0xFFFFFFFFu : pos;
      if (A.out_val) A.out_val[o + k] = empty ? __longlong_as_double(0x7FF0000000000000ll)
                                              : __longlong_as_double((long long)(key & ~kPosMask));
      if (A.out_id) A.out_id[o + k] = empty ? 0ull : ids[pos];
    }
  }
}

// ------------------------------------------------------ heavy-first order
// One workgroup: counting sort of the sets by size class (bit length of n),
// largest class first (oversize sets last); sets with n >= 2^split_log2 are
// split into chunks of 2^(split_log2-1) elements: their chunk counts are
// prefix-summed into big_prefix and their state reset.  Also resets the
// persistent work counter and writes meta.
__global__ __launch_bounds__(1024) void k_order(const uint64_t* off, uint64_t num_sets, uint32_t split_log2,
                                                uint32_t* order, uint32_t* counter, uint32_t* meta,
                                                uint32_t* big_prefix, uint64_t* big_state, uint32_t* status) {
  __shared__ uint32_t cnt[24];
  __shared__ uint32_t pos[24];
  __shared__ uint32_t scan[1024];
  __shared__ uint32_t carry, num_big_s;
  const int tid = threadIdx.x;
  if (tid < 24) cnt[tid] = 0;
  __syncthreads();
  for (uint64_t s = tid; s < num_sets; s += blockDim.x) {
    const uint64_t n = off[s + 1] - off[s];
    const uint32_t c = n > kMaxSet ? 23u : (n ? 64u - (uint32_t)__builtin_clzll(n) : 0u);
    atomicAdd(&cnt[c], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int c = 21; c >= 0; --c) {
      pos[c] = acc;
      acc += cnt[c];
    }
    pos[22] = acc;
    pos[23] = acc;
    uint32_t nb = 0;
    if (split_log2 > 0)
      for (uint32_t c = split_log2 + 1; c <= 21; ++c) nb += cnt[c];
    meta[0] = nb;
    num_big_s = nb;
    counter[0] = 0;
    counter[1] = 0;
    carry = 0;
    if (cnt[23]) atomicOr(status, kStatusSetTooLarge);
  }
  __syncthreads();
  for (uint64_t s = tid; s < num_sets; s += blockDim.x) {
    const uint64_t n = off[s + 1] - off[s];
    const uint32_t c = n > kMaxSet ? 23u : (n ? 64u - (uint32_t)__builtin_clzll(n) : 0u);
    order[atomicAdd(&pos[c], 1u)] = (uint32_t)s;
  }
  __syncthreads();
  // chunk counts of the split sets (they occupy order[0 .. num_big))
  const uint32_t num_big = num_big_s;
  const uint32_t csize_log2 = split_log2 > 0 ? split_log2 - 1 : 0;
  for (uint32_t b0 = 0; b0 < num_big; b0 += 1024) {
    const uint32_t b = b0 + tid;
    uint32_t c = 0;
    if (b < num_big) {
      const uint32_t s = order[b];
      const uint64_t n = off[s + 1] - off[s];
      c = (uint32_t)((n + (1ull << csize_log2) - 1) >> csize_log2);
      big_state[b] = 0x7FF0000000000000ull;  // smallest chunk threshold (+inf)
    }
    scan[tid] = c;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan
      const uint32_t x = tid >= d ? scan[tid - d] : 0u;
      __syncthreads();
      scan[tid] += x;
      __syncthreads();
    }
    if (b < num_big) big_prefix[b + 1] = carry + scan[tid];
    __syncthreads();
    if (tid == 0) carry += scan[1023];
    __syncthreads();
  }
  if (tid == 0) {
    big_prefix[0] = 0;
    meta[1] = carry;                                  // chunk items
    meta[2] = carry + (uint32_t)(num_sets - num_big);  // all items
  }
}

// Serving copies between device buffers and pinned host memory
// (device-mapped aliases): up to three segments of 32-bit words.  A kernel
// rather than asynchronous copy calls, which were seen to hold the calling
// thread for up to ~10 ms.
__global__ __launch_bounds__(256) void k_copy_words(CopySegs c) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
#pragma unroll
  for (int g = 0; g < 3; ++g)
    for (uint64_t k = t0; k < c.n[g]; k += stride) c.dst[g][k] = c.src[g][k];
}

// Global keys of the split sets start empty.
__global__ __launch_bounds__(256) void k_big_init(const uint32_t* order, const uint32_t* meta, uint32_t m,
                                                  uint64_t* big_keys) {
  const uint64_t total = (uint64_t)meta[0] * m;
  for (uint64_t e = blockIdx.x * 256ull + threadIdx.x; e < total; e += (uint64_t)gridDim.x * 256) {
    const uint64_t b = e / m, k = e % m;
    big_keys[(uint64_t)order[b] * m + k] = kEmptyKey;
  }
}

// ---------------------------------------------------------- constant tables
__global__ void k_init_tables(int variant, uint32_t m, Tables t) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    t.expm1c[0] = 1.0;
    for (int k = 1; k <= 18; ++k) t.expm1c[k] = t.expm1c[k - 1] / (double)k;
  }
  if (i < 128) {  // stream logarithm cells: centre 1 + (j + 1/2)/128, c_0 = 1, c_127 = 2
    const double c = i == 0 ? 1.0 : (i == 127 ? 2.0 : 1.0 + ((double)i + 0.5) / 128.0);
    const double inv = 1.0 / c;
    t.ltab[2 * i] = inv;
    t.ltab[2 * i + 1] = 0.0 - spec_log(inv);
    t.ltab[2 * (128 + i)] = inv;
    t.ltab[2 * (128 + i) + 1] = 0.0 - spec_log(2.0 * inv);
  }
  if (variant == 2 && i <= m) t.beta[i] = i == 0 ? 0.0 : (double)m / (double)(m - i + 1);
  if (variant == 3 && i == 0) {  // lambda = log(1 + 1/(m-1)), so e^lambda - 1 = 1/(m-1) exactly
    const double a = 1.0 / (double)(m - 1);
    const double lam = spec_log1p(a);
    t.scal[0] = lam;
    t.scal[1] = a;
    t.scal[2] = a / lam;
  }
  if (variant == 4 && i < m) {
    const double lam1 = spec_log1p(1.0 / (double)(m - 1));
    if (i == 0) {
      t.lam[0] = t.a[0] = t.c1[0] = 0.0;
      t.gam[0] = 0.0;
      t.dgam[0] = 0.0;
      t.scal[4] = 1.0 / lam1;
    } else {
      const double a = 1.0 / (double)(m - i);
      const double l = spec_log1p(a);
      t.lam[i] = l;  // e^lambda_i - 1 = 1/(m-i) exactly
      t.a[i] = a;
      t.c1[i] = a / l;
      const double gi = spec_log1p((double)i / (double)(m - i)) / lam1;
      const double gp = i == 1 ? 0.0 : spec_log1p((double)(i - 1) / (double)(m - i + 1)) / lam1;
      t.gam[i] = gi;
      t.dgam[i] = gi - gp;
    }
  }
}

// ------------------------------------------------------------- estimation
// counts[pair] = #{k : idA[k] == idB[k], both components non-empty}
__global__ __launch_bounds__(256) void k_estimate(const uint64_t* idA, const uint32_t* idxA,
                                                  const uint64_t* idB, const uint32_t* idxB, uint32_t m,
                                                  uint32_t* counts) {
  __shared__ uint32_t red[4];
  const uint64_t pr = blockIdx.x;
  const uint64_t o = pr * m;
  uint32_t c = 0;
  for (uint32_t k = threadIdx.x; k < m; k += 256)
    c += (idA[o + k] == idB[o + k] && idxA[o + k] != 0xFFFFFFFFu && idxB[o + k] != 0xFFFFFFFFu) ? 1u : 0u;
  for (int d = 32; d >= 1; d >>= 1) c += (uint32_t)__shfl_xor((int)c, d);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[pr] = red[0] + red[1] + red[2] + red[3];
}

// All-pairs equal-component counts over k signatures of m 32-bit fingerprints
// (fingerprint 0 marks an empty component and never matches).  64x64 pair
// tile per workgroup, 16 components staged in LDS per step, 4x4 pairs per
// thread.
constexpr int kApTile = 64, kApK = 16;
__global__ __launch_bounds__(256) void k_allpairs(const uint32_t* fp, uint32_t k, uint32_t m,
                                                  uint16_t* counts) {
  __shared__ uint32_t sa[kApK][kApTile + 1];
  __shared__ uint32_t sb[kApK][kApTile + 1];
  const uint32_t bi = blockIdx.y * kApTile, bj = blockIdx.x * kApTile;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  uint32_t acc[4][4] = {};
  for (uint32_t c0 = 0; c0 < m; c0 += kApK) {
    for (int e = threadIdx.x; e < kApK * kApTile; e += 256) {
      const int r = e / kApK, c = e % kApK;
      const uint32_t cc = c0 + c;
      sa[c][r] = (bi + r < k && cc < m) ? fp[(uint64_t)(bi + r) * m + cc] : 0u;
      sb[c][r] = (bj + r < k && cc < m) ? fp[(uint64_t)(bj + r) * m + cc] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kApK; ++c) {
      uint32_t av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = sa[c][ty * 4 + u];
        bv[u] = sb[c][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += (av[u] == bv[v] && av[u] != 0u) ? 1u : 0u;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t r = bi + ty * 4 + u, c = bj + tx * 4 + v;
      if (r < k && c < k) counts[(uint64_t)r * k + c] = (uint16_t)(acc[u][v] > 65535u ? 65535u : acc[u][v]);
    }
}

// ----------------------------------------------------- b-bit reduction
// Sec. 1.3, algorithm "Reduction to a b-bit signature": component k (1-based)
// of element id z (0 = empty) keeps the b low bits of mix64(mix64(z) + k phi);
// fields are packed b in {1, 2, 4, 8, 16} per 64-bit word (component k-1 at
// bit (k-1) b of the signature's bit string), ceil(m b / 64) words per
// signature, high padding bits zero.  One thread per output word.
__global__ __launch_bounds__(256) void k_bbit_pack(const uint64_t* id, uint64_t num_sigs, uint32_t m, uint32_t b,
                                                   uint64_t* out) {
  const uint64_t W = ((uint64_t)m * b + 63) / 64;
  const uint64_t word = blockIdx.x * 256ull + threadIdx.x;
  if (word >= num_sigs * W) return;
  const uint64_t s = word / W, w = word % W;
  const uint32_t per = 64u / b;
  const uint32_t k0 = (uint32_t)w * per, k1 = k0 + per < m ? k0 + per : m;
  const uint64_t mask = (1ull << b) - 1ull;
  const uint64_t* z = id + s * m;
  uint64_t acc = 0;
  for (uint32_t k = k0; k < k1; ++k)
    acc |= (mix64(mix64(z[k]) + (uint64_t)(k + 1) * kPhi) & mask) << ((k - k0) * b);
  out[word] = acc;
}

// Fields of x that are nonzero, one bit each (at the field's lowest bit).
template <int B>
__device__ __forceinline__ uint64_t bbit_nonzero(uint64_t x) {
  if constexpr (B >= 2) x |= x >> 1;
  if constexpr (B >= 4) x |= x >> 2;
  if constexpr (B >= 8) x |= x >> 4;
  if constexpr (B >= 16) x |= x >> 8;
  constexpr uint64_t low = B == 1 ? ~0ull : B == 2 ? 0x5555555555555555ull : B == 4 ? 0x1111111111111111ull
                                  : B == 8 ? 0x0101010101010101ull : 0x0001000100010001ull;
  return x & low;
}

// All-pairs equal-field counts of k packed b-bit signatures (W words each):
// 64x64 signature tiles, kApK words staged in LDS, 4x4 pairs per thread;
// equal = m - (fields that differ), padding fields being zero in both.
template <int B>
__global__ __launch_bounds__(256) void k_bbit_allpairs(const uint64_t* sig, uint32_t k, uint32_t W, uint32_t m,
                                                       uint16_t* counts) {
  __shared__ uint64_t sa[kApK][kApTile + 1];
  __shared__ uint64_t sb[kApK][kApTile + 1];
  const uint32_t bi = blockIdx.y * kApTile, bj = blockIdx.x * kApTile;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  uint32_t diff[4][4] = {};
  for (uint32_t c0 = 0; c0 < W; c0 += kApK) {
    for (int e = threadIdx.x; e < kApK * kApTile; e += 256) {
      const int r = e / kApK, c = e % kApK;
      const uint32_t cc = c0 + c;
      sa[c][r] = (bi + r < k && cc < W) ? sig[(uint64_t)(bi + r) * W + cc] : 0ull;
      sb[c][r] = (bj + r < k && cc < W) ? sig[(uint64_t)(bj + r) * W + cc] : 0ull;
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < kApK; ++c) {
      uint64_t av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = sa[c][ty * 4 + u];
        bv[u] = sb[c][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) diff[u][v] += (uint32_t)__popcll(bbit_nonzero<B>(av[u] ^ bv[v]));
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t r = bi + ty * 4 + u, c = bj + tx * 4 + v;
      const uint32_t eq = m - diff[u][v];
      if (r < k && c < k) counts[(uint64_t)r * k + c] = (uint16_t)(eq > 65535u ? 65535u : eq);
    }
}

// --------------------------------------------------------- debug primitives
// what: 0 log(x), 1 log1p(x), 2 expm1(x), 3 Exp(1) of word u, 4 mix64(u),
// 5 truncated exponential of (K = u, point k+1) with PMH3 constants,
// 6 Lemire(m) of (K = u, point k+1), 7 ProbMinHash1 spacing of (K = u, k+1)
__global__ void k_debug(int what, const double* in, const uint64_t* in_u, double* out, uint64_t* out_u,
                        uint64_t n, uint32_t m, Tables t) {
  const uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  switch (what) {
    case 0: out[k] = spec_log(in[k]); break;
    case 1: out[k] = spec_log1p(in[k]); break;
    case 2: out[k] = spec_expm1(in[k], t.expm1c); break;
    case 3: out[k] = exp1(in_u[k], (const LogCell*)t.ltab); break;
    case 4: out_u[k] = mix64(in_u[k]); break;
    case 5: {
      const uint64_t pb = pbase(in_u[k], (uint32_t)k + 1);
      out[k] = trunc_exp(mix64(pb), pb, t.scal[0], t.scal[1], t.scal[2], t);
      break;
    }
    case 6: {
      const uint64_t pb = pbase(in_u[k], (uint32_t)k + 1);
      out_u[k] = lemire(mix64(pb), pb, m, t);
      break;
    }
    case 7: out_u[k] = spacing_fixed(exp1(mix64(pbase(in_u[k], (uint32_t)k + 1)), (const LogCell*)t.ltab)); break;
    case 8: out[k] = stream_log(in[k], (const LogCell*)t.ltab); break;
    default: break;
  }
}

// Wave prefix sums of the fixed-point spacings (64-lane chains: what 9;
// mini-chain groups of 8, 4, 2 lanes: what 10, 11, 12), every lane
// participating; inputs beyond n count as 0.
__global__ void k_debug_scan(int what, const uint64_t* in_u, uint64_t* out_u, uint64_t n) {
  const uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t v = k < n ? in_u[k] : 0;
  const int lane = threadIdx.x & 63;
  const uint64_t r = what == 9    ? wave_incl_scan_u64(v, lane)
                     : what == 10 ? group_incl_scan_u64<8>(v, lane & 7)
                     : what == 11 ? group_incl_scan_u64<4>(v, lane & 3)
                                  : group_incl_scan_u64<2>(v, lane & 1);
  if (k < n) out_u[k] = r;
}

}  // namespace

// ------------------------------------------------------- static work buffer
// Work list, counters and split-set state of pmh_hash_sets_noalloc, for
// callers that cannot allocate: batches of at most kScratchSets sets.  Laid
// out as WorkBuf expects: 8 u32 (counters, meta) at offset 0, order u32[max]
// at 256, big_prefix u32[max + 1] after it, big_state u64[max] 256-aligned
// after that.  Every field a launch reads is written by k_order first.
constexpr size_t kScratchOrder = 256;
constexpr size_t kScratchPrefix = kScratchOrder + (size_t)kScratchSets * 4;
constexpr size_t kScratchState = (kScratchPrefix + ((size_t)kScratchSets + 1) * 4 + 255) & ~(size_t)255;
constexpr size_t kScratchBytes = kScratchState + (size_t)kScratchSets * 8;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// The array's device address on `device` (current when called), looked up
// once per device: every device holds its own copy at its own address, and
// the host-side name of the array is no device address.
hipError_t scratch_work(int device, WorkArgs* out, uint64_t* cap) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return e;
      if (!p) return hipErrorInvalidSymbol;
      addr[device] = p;
    }
    base = static_cast<unsigned char*>(addr[device]);
  }
  uint32_t* small = reinterpret_cast<uint32_t*>(base);
  out->order = reinterpret_cast<uint32_t*>(base + kScratchOrder);
  out->counter = small;
  out->meta = small + 4;
  out->big_prefix = reinterpret_cast<uint32_t*>(base + kScratchPrefix);
  out->big_state = reinterpret_cast<uint64_t*>(base + kScratchState);
  *cap = kScratchSets;
  return hipSuccess;
}

// ------------------------------------------------------------------ launchers
uint32_t batch_size(int waves) { return kEpt * (uint32_t)waves * 64; }

size_t lds_bytes_q(int variant, uint32_t m, int waves, uint32_t qcap) {
  size_t b = kLogCells * sizeof(LogCell) + (size_t)m * 8 + (size_t)qcap * sizeof(ChainEntry);
  if (variant == 2 || variant == 4)
    b += lane_tab_offset(fy_waves(waves), m, batch_size(waves)) + (size_t)kLaneTabs * kLaneTab * 8;
  return b;
}

size_t lds_bytes(int variant, uint32_t m, int waves) { return lds_bytes_q(variant, m, waves, 2 * batch_size(waves)); }

size_t lds_static_bytes() {
  return sizeof(Shared) + 64;  // the per-workgroup static block (k_hash_*) plus alignment slack
}

// The kernels carve the chain queue (a.qcap entries) out of the dynamic LDS and
// fill it up to one batch beyond the flush point: refuse launches whose queue
// or LDS is smaller than that layout needs.
template <int V, int NW>
static bool shape_ok(const HashArgs& a, size_t lds) {
  return a.qcap >= batch_size(NW) && lds >= lds_bytes_q(V, a.m, NW, a.qcap);
}
// Launches with an out_bbit output take the instantiations with the b-bit
// epilogue.  Four-wave ProbMinHash3 launches whose LDS already holds a CU to
// at most three workgroups (m above about 3,000) take the instantiation that
// prefetches each batch's weights and ids: its 148 VGPRs allow three as well
// (skewed batch at m = 4096: 8.70 -> 7.55 ms; 100 sets of 10^6 elements 1.65
// -> 1.37 ms), while with four workgroups per CU they cost one.
constexpr size_t kLdsPerCu = 160 * 1024;
template <int V, int NW>
static hipError_t launch_hash_t(const HashArgs& a, int grid, size_t lds, hipStream_t s) {
  if (!shape_ok<V, NW>(a, lds)) return hipErrorInvalidValue;
  if constexpr (V == 3 && NW == 4) {
    if ((lds + lds_static_bytes()) * 4 > kLdsPerCu) {
      if (a.out_bbit)
        hipLaunchKernelGGL((k_hash_persistent<V, NW, true, true>), dim3(grid), dim3(NW * 64), lds, s, a);
      else
        hipLaunchKernelGGL((k_hash_persistent<V, NW, false, true>), dim3(grid), dim3(NW * 64), lds, s, a);
      return hipGetLastError();
    }
  }
  if (a.out_bbit)
    hipLaunchKernelGGL((k_hash_persistent<V, NW, true>), dim3(grid), dim3(NW * 64), lds, s, a);
  else
    hipLaunchKernelGGL((k_hash_persistent<V, NW>), dim3(grid), dim3(NW * 64), lds, s, a);
  return hipGetLastError();
}
template <int V, int NW>
static hipError_t launch_finish_t(const HashArgs& a, int grid, size_t lds, hipStream_t s) {
  if (!shape_ok<V, NW>(a, lds)) return hipErrorInvalidValue;
  if (a.out_bbit)
    hipLaunchKernelGGL((k_big_finish<V, NW, true>), dim3(grid), dim3(NW * 64), lds, s, a);
  else
    hipLaunchKernelGGL((k_big_finish<V, NW>), dim3(grid), dim3(NW * 64), lds, s, a);
  return hipGetLastError();
}
template <int V, int NW>
static hipError_t launch_one_t(const HashArgs& a, uint64_t set, size_t lds, hipStream_t s) {
  if (!shape_ok<V, NW>(a, lds)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_hash_one<V, NW>), dim3(1), dim3(NW * 64), lds, s, a, set);
  return hipGetLastError();
}
template <int V, int NW>
static hipError_t occ_t(size_t lds, int* out) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, (const void*)k_hash_persistent<V, NW>, NW * 64, lds);
}

#define PMH_DISPATCH(FN, ...)                                       \
  switch (variant * 16 + waves) {                                   \
    case 16 + 1: return FN<1, 1>(__VA_ARGS__);                      \
    case 16 + 2: return FN<1, 2>(__VA_ARGS__);                      \
    case 16 + 4: return FN<1, 4>(__VA_ARGS__);                      \
    case 32 + 1: return FN<2, 1>(__VA_ARGS__);                      \
    case 32 + 2: return FN<2, 2>(__VA_ARGS__);                      \
    case 32 + 4: return FN<2, 4>(__VA_ARGS__);                      \
    case 48 + 1: return FN<3, 1>(__VA_ARGS__);                      \
    case 48 + 2: return FN<3, 2>(__VA_ARGS__);                      \
    case 48 + 4: return FN<3, 4>(__VA_ARGS__);                      \
    case 64 + 1: return FN<4, 1>(__VA_ARGS__);                      \
    case 64 + 2: return FN<4, 2>(__VA_ARGS__);                      \
    case 64 + 4: return FN<4, 4>(__VA_ARGS__);                      \
    case 32 + 8: return FN<2, 8>(__VA_ARGS__);                      \
    case 64 + 8: return FN<4, 8>(__VA_ARGS__);                      \
    default: return hipErrorInvalidValue;                           \
  }

hipError_t launch_hash(int variant, const HashArgs& a, int waves, int grid, size_t lds, hipStream_t s) {
  PMH_DISPATCH(launch_hash_t, a, grid, lds, s)
}
hipError_t launch_big_finish(int variant, const HashArgs& a, int waves, int grid, size_t lds, hipStream_t s) {
  PMH_DISPATCH(launch_finish_t, a, grid, lds, s)
}
hipError_t launch_hash_one(int variant, const HashArgs& a, uint64_t set, int waves, size_t lds, hipStream_t s) {
  PMH_DISPATCH(launch_one_t, a, set, lds, s)
}
hipError_t occupancy(int variant, int waves, size_t lds, int* blocks_per_cu) {
  PMH_DISPATCH(occ_t, lds, blocks_per_cu)
}

hipError_t launch_order(const uint64_t* off, uint64_t num_sets, uint32_t split_log2, const WorkArgs& w,
                        uint32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_order, dim3(1), dim3(1024), 0, s, off, num_sets, split_log2, w.order, w.counter, w.meta,
                     w.big_prefix, w.big_state, status);
  return hipGetLastError();
}

hipError_t launch_big_init(const WorkArgs& w, uint32_t m, uint64_t* big_keys, hipStream_t s) {
  hipLaunchKernelGGL(k_big_init, dim3(512), dim3(256), 0, s, w.order, w.meta, m, big_keys);
  return hipGetLastError();
}

hipError_t launch_pmin(const HashArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_pmin, dim3(grid), dim3(kPminThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_pmin_finish(const HashArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_pmin_finish, dim3(grid), dim3(kPminThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t occupancy_pmin(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)k_pmin, kPminThreads, 0);
}
uint32_t pmin_split_log2() { return kPminSplitLog2; }

hipError_t launch_copy_words(const CopySegs& c, hipStream_t s) {
  const uint64_t n = std::max(c.n[0], std::max(c.n[1], c.n[2]));
  if (n == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((n + 1023) / 1024, 2048);
  hipLaunchKernelGGL(k_copy_words, dim3((uint32_t)blocks), dim3(256), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_init_tables(int variant, uint32_t m, Tables t, hipStream_t s) {
  const uint32_t n = (m + 1) > 128 ? (m + 1) : 128;
  hipLaunchKernelGGL(k_init_tables, dim3((n + 255) / 256), dim3(256), 0, s, variant, m, t);
  return hipGetLastError();
}

hipError_t launch_estimate(const uint64_t* idA, const uint32_t* idxA, const uint64_t* idB, const uint32_t* idxB,
                           uint32_t m, uint64_t pairs, uint32_t* counts, hipStream_t s) {
  if (pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_estimate, dim3((uint32_t)pairs), dim3(256), 0, s, idA, idxA, idB, idxB, m, counts);
  return hipGetLastError();
}

hipError_t launch_allpairs(const uint32_t* fp, uint32_t k, uint32_t m, uint16_t* counts, hipStream_t s) {
  if (k == 0) return hipSuccess;
  const uint32_t tiles = (k + kApTile - 1) / kApTile;
  hipLaunchKernelGGL(k_allpairs, dim3(tiles, tiles), dim3(256), 0, s, fp, k, m, counts);
  return hipGetLastError();
}

hipError_t launch_bbit_pack(const uint64_t* id, uint64_t num_sigs, uint32_t m, uint32_t b, uint64_t* out,
                            hipStream_t s) {
  const uint64_t words = num_sigs * (((uint64_t)m * b + 63) / 64);
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bbit_pack, dim3((uint32_t)((words + 255) / 256)), dim3(256), 0, s, id, num_sigs, m, b, out);
  return hipGetLastError();
}

hipError_t launch_bbit_allpairs(const uint64_t* sig, uint32_t k, uint32_t m, uint32_t b, uint16_t* counts,
                                hipStream_t s) {
  if (k == 0) return hipSuccess;
  const uint32_t W = (uint32_t)(((uint64_t)m * b + 63) / 64);
  const uint32_t tiles = (k + kApTile - 1) / kApTile;
  const dim3 g(tiles, tiles);
  switch (b) {
    case 1: hipLaunchKernelGGL(k_bbit_allpairs<1>, g, dim3(256), 0, s, sig, k, W, m, counts); break;
    case 2: hipLaunchKernelGGL(k_bbit_allpairs<2>, g, dim3(256), 0, s, sig, k, W, m, counts); break;
    case 4: hipLaunchKernelGGL(k_bbit_allpairs<4>, g, dim3(256), 0, s, sig, k, W, m, counts); break;
    case 8: hipLaunchKernelGGL(k_bbit_allpairs<8>, g, dim3(256), 0, s, sig, k, W, m, counts); break;
    case 16: hipLaunchKernelGGL(k_bbit_allpairs<16>, g, dim3(256), 0, s, sig, k, W, m, counts); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_debug_eval(int what, const double* in, const uint64_t* in_u, double* out, uint64_t* out_u,
                             uint64_t n, uint32_t m, int variant, Tables t, hipStream_t s) {
  (void)variant;
  if (n == 0) return hipSuccess;
  if (what >= 9) {
    hipLaunchKernelGGL(k_debug_scan, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, what, in_u, out_u, n);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_debug, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, what, in, in_u, out, out_u, n,
                     m, t);
  return hipGetLastError();
}

}  // namespace pmh
