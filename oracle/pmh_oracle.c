/*
 * pmh_oracle.c -- plain, sequential CPU oracle for ProbMinHash signatures.
 *
 *   O. Ertl, "ProbMinHash -- A Class of Locality-Sensitive Hash Algorithms for
 *   the (Probability) Jaccard Similarity", IEEE TKDE 2020 (arXiv 1911.00675).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the GPU library: every primitive
 * below is written here from its definition.
 *
 * What it computes (all arithmetic IEEE binary64, round-to-nearest, no
 * contraction; fma only where written):
 *
 *   * the per-element random streams of the four ProbMinHash variants
 *     (Sec. 2.1 "Sequence Generation", Sec. 2.3-2.6), driven by a counter-based
 *     SplitMix64 word stream, an atanh-series logarithm and Lemire's bounded
 *     integers (the readings of Sec. 3's PRNG remarks listed in the design
 *     notes);
 *   * the truncated exponential Exp(lambda; 0, 1) of Sec. 2.8, sampled by a
 *     scheme derived here from its density (uniform part plus a rejection
 *     step bounded by the tangent and the chord of expm1);
 *   * ProbMinHash1-4 (Sec. 2.3-2.6): one loop consumes an element's stream
 *     point by point and stops once a lower bound of its remaining points
 *     reaches the stop limit max_k q_k (Sec. 2), the bounds being the points
 *     themselves for the exponential-spacing streams and the interval starts
 *     of Sec. 2.5/2.6; labels by Lemire's method or by the lazily initialised
 *     permutation of Sec. 2.4; everything in a 64-bit (value, position) key
 *     space;
 *   * the interleaved variants ProbMinHash1a and ProbMinHash3a (Sec. 2.7): the
 *     same step applied in passes over the live elements;
 *   * a brute-force reference that generates every point of every element's
 *     stream with no stop rule and takes the per-label minimum, i.e. the
 *     signature definition of eq. (1) with the hash values of eq. (9);
 *   * the loop caps Sec. 3 recommends (stream length, sampler proposals,
 *     Lemire redraws) as parameters, so that the capped paths can be forced.
 *
 * Pins (see tests/): the word stream against the published SplitMix64 output
 * sequence; sequential == brute force == interleaved on tiny inputs, also
 * under forced caps; logarithm/expm1/log1p against the C library within a few
 * ulp; Exp(1), truncated-exponential, Lemire and permutation distribution
 * tests; the collision law Pr(z_k(A) = z_k(B)) = J_P; the relative-MSE band of
 * Sec. 3.1; SuperMinHash's alpha(m,u) (exact closed forms) for ProbMinHash4
 * with equal weights (Sec. 2.9).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_PHI 0x9E3779B97F4A7C15ULL
#define O_EMPTY 0xFFFFFFFFFFFFFFFFULL
#define O_POS_MASK 0xFFFFFULL /* 20 position bits */
#define O_MAX_SET ((uint64_t)1 << 20)
#define O_MAX_M 16384u

enum { O_OK = 0, O_ERR_ARG = 1, O_ERR_M_RANGE = 2, O_ERR_VARIANT_M = 3, O_ERR_WEIGHT = 4,
       O_ERR_SET_TOO_LARGE = 5, O_ERR_OOM = 7 };

/* ------------------------------------------------------------------------ */
/* Randomness: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) addressed by a
 * counter.  The element key K is a hash of (seed, element id) only, so equal
 * elements of different sets draw identical streams (Sec. 2, "PRNG seeded with
 * a hash of d").  Word c of element K is the c-th SplitMix64 output for the
 * state K: mix(K + (c+1)*phi).  c = (i << 8) | t addresses slot t of point i. */
static inline uint64_t o_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t o_word(uint64_t K, uint64_t i, unsigned t) {
    uint64_t c = (i << 8) | (uint64_t)t;
    return o_mix64(K + (c + 1) * O_PHI);
}
/* Slots of point i.  Word 0 serves the point twice: its high 32 bits are the
 * uniform behind the point value, its low 32 bits the label draw.  (The
 * paper's implementation spends 53 random bits per uniform; with 32 the
 * first-point values of ProbMinHash3/4 lie on a 2^-32 grid, so equal truncated
 * values -- decided by position -- occur with probability about
 * n / (m 2^32) per component.)  Words 1..8 hold Lemire redraws (low 32 bits);
 * words 16..79 the proposal pairs of the truncated-exponential sampler (53-bit
 * uniforms). */
#define O_SLOT_POINT 0u
#define O_SLOT_REDRAW 1u
#define O_SLOT_REJ 16u

static inline double o_u32(uint64_t w) { return (double)(w >> 32) * 0x1p-32; }        /* [0,1) */
static inline double o_upos(uint64_t w) { return (double)((w >> 32) + 1) * 0x1p-32; } /* (0,1] */
static inline double o_u53(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }        /* [0,1) */

/* ------------------------------------------------------------------------ */
/* Logarithm written from ln x = e ln 2 + 2 atanh((f-1)/(f+1)), x = 2^e f with
 * f in [sqrt(1/2), sqrt(2)); atanh(s) = s + s^3/3 + s^5/5 + ...  For |s| <=
 * 0.1716 the series terms up to s^21 reach below 2^-53 relative. */
static const double O_LN2_HI = 0x1.62e42fefa0000p-1; /* ln 2 rounded to 36 bits */
static const double O_LN2_LO = 0x1.cf79abc9e3b3ap-40; /* ln 2 - O_LN2_HI */

double or_log(double x) {
    uint64_t b;
    memcpy(&b, &x, 8);
    int e = (int)((b >> 52) & 0x7FF) - 1023;
    uint64_t mant = b & 0xFFFFFFFFFFFFFULL;
    uint64_t fb;
    if (mant >= 0x6A09E667F3BCDULL) { /* f >= sqrt(2): use f/2 */
        fb = mant | (1022ULL << 52);
        e += 1;
    } else {
        fb = mant | (1023ULL << 52);
    }
    double f;
    memcpy(&f, &fb, 8);
    double s = (f - 1.0) / (f + 1.0);
    double t = s * s;
    /* Q(t) = sum_{j=1..10} (2/(2j+1)) t^(j-1) */
    double q = 2.0 / 21.0;
    q = fma(q, t, 2.0 / 19.0);
    q = fma(q, t, 2.0 / 17.0);
    q = fma(q, t, 2.0 / 15.0);
    q = fma(q, t, 2.0 / 13.0);
    q = fma(q, t, 2.0 / 11.0);
    q = fma(q, t, 2.0 / 9.0);
    q = fma(q, t, 2.0 / 7.0);
    q = fma(q, t, 2.0 / 5.0);
    q = fma(q, t, 2.0 / 3.0);
    double lf = 2.0 * s + (s * t) * q;
    double de = (double)e;
    return de * O_LN2_HI + (de * O_LN2_LO + lf);
}

/* log(1+u) for u > 0; used only for the per-m constants. */
double or_log1p(double u) {
    if (u > 1.0) return or_log(1.0 + u);
    double s = u / (2.0 + u); /* log1p(u) = 2 atanh(u/(2+u)), |s| <= 1/3 */
    double t = s * s;
    double q = 2.0 / 49.0; /* j = 24 */
    for (int j = 23; j >= 1; --j) q = fma(q, t, 2.0 / (double)(2 * j + 1));
    return 2.0 * s + (s * t) * q;
}

/* exp(t) - 1 for t in [0, ln 2]: Taylor series to degree 18, coefficients
 * e_k = e_{k-1} / k, e_0 = 1, evaluated by Horner with fma. */
double or_expm1(double t) {
    double e[19];
    e[0] = 1.0;
    for (int k = 1; k <= 18; ++k) e[k] = e[k - 1] / (double)k;
    double p = e[18];
    for (int k = 17; k >= 1; --k) p = fma(p, t, e[k]);
    return p * t;
}

/* Table-driven logarithm for the streams' Exp(1) variates (the counterpart of
 * the table-based exponential sampler of Sec. 3).  x = 2^e y, y = 1.m in
 * [1,2); j = top 7 bits of m; cell centre c_j = 1 + (j + 1/2)/128, except
 * c_0 = 1.  If y >= sqrt(2) the reduction uses y/2 against c_j/2 (c_127 = 2,
 * so the cell below 1 is centred on 1) and exponent e+1.  With r =
 * fma(y, 1/c_j, -1) (the same ratio in both cases), |r| <= 2^-7:
 *   log x = e' ln2_hi + (e' ln2_lo + (L + log1p8(r))),  L = log(c'),
 * log1p8(r) = r + r^2 (-1/2 + r/3 - ... + r^6/8) by Horner with fma.  The
 * table (1/c_j, log c_j, log(c_j/2)) is built with the series logarithm. */
static double o_ltab_inv[128], o_ltab_l[128], o_ltab_lh[128];
static pthread_once_t o_ltab_once = PTHREAD_ONCE_INIT;
static void o_ltab_init(void) {
    for (int j = 0; j < 128; ++j) {
        double c = (j == 0) ? 1.0 : 1.0 + ((double)j + 0.5) / 128.0;
        if (j == 127) c = 2.0;
        o_ltab_inv[j] = 1.0 / c;
        /* log c' taken as -log of the stored reciprocal, so that
         * log y = log(y inv) - log(inv) holds for the rounded inv itself */
        o_ltab_l[j] = 0.0 - or_log(o_ltab_inv[j]);
        o_ltab_lh[j] = 0.0 - or_log(2.0 * o_ltab_inv[j]);
    }
}

double or_log_stream(double x) {
    pthread_once(&o_ltab_once, o_ltab_init);
    uint64_t b;
    memcpy(&b, &x, 8);
    int e = (int)((b >> 52) & 0x7FF) - 1023;
    uint64_t mant = b & 0xFFFFFFFFFFFFFULL;
    unsigned j = (unsigned)(mant >> 45);
    uint64_t yb = mant | (1023ULL << 52);
    double y;
    memcpy(&y, &yb, 8);
    double L = o_ltab_l[j];
    if (mant >= 0x6A09E667F3BCDULL) { /* y >= sqrt(2) */
        e += 1;
        L = o_ltab_lh[j];
    }
    double r = fma(y, o_ltab_inv[j], -1.0);
    double q = 1.0 / 8.0;
    q = fma(q, r, -1.0 / 7.0);
    q = fma(q, r, 1.0 / 6.0);
    q = fma(q, r, -1.0 / 5.0);
    q = fma(q, r, 1.0 / 4.0);
    q = fma(q, r, -1.0 / 3.0);
    q = fma(q, r, 1.0 / 2.0);
    double l1p = fma(-(r * r), q, r);
    double de = (double)e;
    return de * O_LN2_HI + (de * O_LN2_LO + (L + l1p));
}

/* The 256 (1/c, L) cells in the layout [j + 128 h] (for the tests). */
void or_log_table(double* out512) {
    pthread_once(&o_ltab_once, o_ltab_init);
    for (int j = 0; j < 128; ++j) {
        out512[2 * j] = o_ltab_inv[j];
        out512[2 * j + 1] = o_ltab_l[j];
        out512[2 * (128 + j)] = o_ltab_inv[j];
        out512[2 * (128 + j) + 1] = o_ltab_lh[j];
    }
}

/* Exp(1) by inversion; 0 - log(u) keeps the result +0 for u = 1. */
static inline double o_exp1(uint64_t w) { return 0.0 - or_log_stream(o_upos(w)); }

/* ------------------------------------------------------------------------ */
/* Loop caps.  Sec. 3 advises bounding every loop of the generators; the caps
 * are part of the definition of the result:
 *   imax          points per element for the with-replacement variants
 *                 ProbMinHash1/3 (default 6 m bitlen(m) + 64);
 *   te_rounds     proposals of the truncated-exponential sampler's second
 *                 branch (default 32, at most 32: word slots 16..79);
 *   redraws       Lemire redraws (default 8, at most 8: word slots 1..8);
 *   lemire_floor  validation only: draws whose low product half lies below
 *                 max(threshold, floor) are redrawn too, which forces the
 *                 redraw path (labels are then not uniform); default 0. */
typedef struct {
    uint64_t imax;
    unsigned te_rounds;
    unsigned redraws;
    uint32_t lemire_floor;
} o_caps;

#define O_TE_ROUNDS_MAX 32u
#define O_REDRAWS_MAX 8u

/* Uniform integer in [0, s) by Lemire's multiply-shift: the product of s and
 * the low 32 bits of the point's word; its high half is the draw, and its low
 * half decides rejection (below (2^32 - s) mod s the draw is biased and the
 * next word of slots 1..8 is tried). */
static uint32_t o_lemire(const o_caps *C, uint64_t K, uint64_t i, uint32_t s) {
    uint32_t thr = (uint32_t)(0u - s) % s;
    if (thr < C->lemire_floor) thr = C->lemire_floor;
    uint64_t prod = (o_word(K, i, O_SLOT_POINT) & 0xFFFFFFFFULL) * (uint64_t)s;
    for (unsigned r = 1; r <= C->redraws && (uint32_t)prod < thr; ++r)
        prod = (o_word(K, i, O_SLOT_REDRAW + r - 1) & 0xFFFFFFFFULL) * (uint64_t)s;
    return (uint32_t)(prod >> 32);
}

/* Truncated exponential Exp(lam; 0, 1) of Sec. 2.8: density
 * f(x) = lam e^(-lam x) / (1 - e^(-lam)) on [0, 1).  The scheme below is
 * derived from f.  Let a = e^lam - 1 and c1 = a / lam.
 *   1. f is smallest at x -> 1, where it equals lam / a = 1 / c1, so f is the
 *      mixture of the uniform law (weight 1/c1) and a remainder.  x = c1 U
 *      with U uniform in [0, 1) lies below 1 with probability 1/c1 and is then
 *      uniform on [0, 1): that draw is the uniform part.
 *   2. The remainder is proportional to e^(-lam x) - e^(-lam), i.e. to
 *      g(t) = expm1(lam t) with t = 1 - x.  g is convex with g(0) = 0 and
 *      g(1) = a, so a uniform point (x, v) of [0,1)^2 is accepted when
 *      v a <= g(t).  Two bounds decide most proposals without evaluating g:
 *      g(t) >= lam t (tangent at 0) accepts when v c1 <= t, and g(t) <= a t
 *      (chord) rejects when v >= t.
 * Step 1 uses the high 32 bits of the point's word (its low half is the label
 * draw); the proposals of step 2 use 53-bit uniforms from slot pairs
 * (16 + 2r, 17 + 2r), r < te_rounds; after the last rejected proposal its x is
 * returned. */
static double o_te(const o_caps *C, uint64_t K, uint64_t i, double lam, double a, double c1) {
    double x = c1 * o_u32(o_word(K, i, O_SLOT_POINT));
    if (x < 1.0) return x;
    for (unsigned r = 0; r < C->te_rounds; ++r) {
        x = o_u53(o_word(K, i, O_SLOT_REJ + 2 * r));
        const double v = o_u53(o_word(K, i, O_SLOT_REJ + 2 * r + 1));
        const double t = 1.0 - x;
        if (v * c1 <= t) return x;
        if (v < t && v * a <= or_expm1(lam * t)) return x;
    }
    return x;
}

/* Packed key: sign, exponent and top 32 fraction bits of the point value,
 * then the 20-bit position.  Integer order = (value truncated, position). */
static inline uint64_t o_key(double x, uint32_t p) {
    uint64_t b;
    memcpy(&b, &x, 8);
    return (b & ~O_POS_MASK) | (uint64_t)p;
}

/* ------------------------------------------------------------------------ */
/* Per-(variant, m) constants. */
typedef struct {
    int variant;
    uint32_t m;
    o_caps caps;
    double *beta;                   /* PMH2: beta[i] = m/(m-i+1), i = 1..m */
    double lam3, a3, c13;           /* PMH3: lambda, e^lambda - 1, (e^lambda - 1)/lambda */
    double *lam4, *a4, *c14;        /* PMH4, i = 1..m-1: the same for lambda_i */
    double *gam, *dgam;             /* PMH4: gamma[0..m-1], dgamma[1..m-1] */
    double delta;                   /* PMH4 */
    int binary;                     /* Sec. 2.9 specialisation (variants 5..8 = binary 1..4) */
} o_params;

static unsigned o_bitlen(uint32_t m) {
    unsigned b = 0;
    while (m) { ++b; m >>= 1; }
    return b;
}

uint64_t or_imax(uint32_t m) { return 6ULL * m * o_bitlen(m) + 64; }

static void o_params_free(o_params *P) {
    free(P->beta); free(P->lam4); free(P->a4); free(P->c14);
    free(P->gam); free(P->dgam);
    memset(P, 0, sizeof(*P));
}

/* caps4 = {imax (0: default), te_rounds, redraws, lemire_floor} or NULL. */
static int o_params_init(o_params *P, int variant, uint32_t m, const uint64_t *caps4) {
    memset(P, 0, sizeof(*P));
    /* Variants 5..8: ProbMinHash1..4 specialised to binary weights (Sec. 2.9,
     * "Conventional Jaccard Similarity"), called with unit weights.  PMH1/2
     * are unchanged (1/w = 1); PMH3 draws U[0,1) instead of the truncated
     * exponential; PMH4 takes gamma_i = i and U[0,1) for both samplers. */
    if (variant >= 5 && variant <= 8) {
        P->binary = 1;
        variant -= 4;
    }
    if (variant < 1 || variant > 4) return O_ERR_ARG;
    if (m < 1 || m > O_MAX_M) return O_ERR_M_RANGE;
    if ((variant == 3 || variant == 4) && m < 2) return O_ERR_VARIANT_M;
    P->variant = variant;
    P->m = m;
    P->caps.imax = or_imax(m);
    P->caps.te_rounds = O_TE_ROUNDS_MAX;
    P->caps.redraws = O_REDRAWS_MAX;
    P->caps.lemire_floor = 0;
    if (caps4) {
        if (caps4[1] < 1 || caps4[1] > O_TE_ROUNDS_MAX || caps4[2] > O_REDRAWS_MAX ||
            caps4[3] > 0xFFFFFFFFULL || caps4[0] > 0xFFFFFFFFULL)
            return O_ERR_ARG;
        if (caps4[0]) P->caps.imax = caps4[0];
        P->caps.te_rounds = (unsigned)caps4[1];
        P->caps.redraws = (unsigned)caps4[2];
        P->caps.lemire_floor = (uint32_t)caps4[3];
    }
    double dm = (double)m;
    if (variant == 2) {
        P->beta = malloc(sizeof(double) * (m + 1));
        if (!P->beta) return O_ERR_OOM;
        P->beta[0] = 0.0;
        for (uint32_t i = 1; i <= m; ++i) P->beta[i] = dm / (double)(m - i + 1);
    } else if (variant == 3) {
        /* lambda = log(1 + 1/(m-1)), so e^lambda - 1 = 1/(m-1) exactly */
        P->a3 = 1.0 / (double)(m - 1);
        P->lam3 = or_log1p(P->a3);
        P->c13 = P->a3 / P->lam3;
    } else if (variant == 4) {
        P->lam4 = malloc(sizeof(double) * m);
        P->a4 = malloc(sizeof(double) * m);
        P->c14 = malloc(sizeof(double) * m);
        P->gam = malloc(sizeof(double) * m);
        P->dgam = malloc(sizeof(double) * m);
        if (!P->lam4 || !P->a4 || !P->c14 || !P->gam || !P->dgam) {
            o_params_free(P);
            return O_ERR_OOM;
        }
        P->lam4[0] = P->a4[0] = P->c14[0] = 0.0;
        for (uint32_t i = 1; i < m; ++i) {
            /* lambda_i = log(1 + 1/(m-i)): e^lambda_i - 1 = 1/(m-i) */
            P->a4[i] = 1.0 / (double)(m - i);
            P->lam4[i] = or_log1p(P->a4[i]);
            P->c14[i] = P->a4[i] / P->lam4[i];
        }
        P->gam[0] = 0.0;
        for (uint32_t i = 1; i < m; ++i)
            P->gam[i] = or_log1p((double)i / (double)(m - i)) / P->lam4[1];
        P->dgam[0] = 0.0;
        if (P->binary)
            for (uint32_t i = 0; i < m; ++i) P->gam[i] = (double)i;
        for (uint32_t i = 1; i < m; ++i) P->dgam[i] = P->gam[i] - P->gam[i - 1];
        P->delta = 1.0 / P->lam4[1];
    }
    return O_OK;
}

/* ------------------------------------------------------------------------ */
/* Point streams (Sec. 2.1, 2.3-2.6).  Point i >= 1 of element K (weight
 * inverse winv).  ProbMinHash1/2 accumulate the exponential spacings in
 * 64-bit fixed point (2^-32 units) and round once:
 * x_i = winv * (T_i 2^-32), T_i = T_{i-1} + floor(s_i 2^32). */
static inline uint64_t o_spacing(const o_params *P, uint64_t K, uint64_t i) {
    double E = o_exp1(o_word(K, i, O_SLOT_POINT));
    if (P->variant == 2) E = P->beta[i] * E;
    return (uint64_t)(E * 0x1p32);
}
static inline double o_fixed_value(double winv, uint64_t T) { return winv * ((double)T * 0x1p-32); }

/* ProbMinHash3/4 place point i in an interval starting at o_lower(i) (Sec. 2.5,
 * Sec. 2.6): winv (i-1), resp. winv gamma_{i-1}; the intervals increase with i. */
static inline double o_lower(const o_params *P, double winv, uint64_t i) {
    if (P->variant == 3) return winv * (double)(i - 1);
    return winv * P->gam[i - 1];
}
static inline double o_value3(const o_params *P, uint64_t K, uint64_t i, double winv) {
    if (P->binary) return (double)(i - 1) + o_u32(o_word(K, i, O_SLOT_POINT));
    double lb = winv * (double)(i - 1);
    return lb + winv * o_te(&P->caps, K, i, P->lam3, P->a3, P->c13);
}
static inline double o_value4(const o_params *P, uint64_t K, uint64_t i, double winv) {
    uint32_t m = P->m;
    if (P->binary) return (double)(i - 1) + o_u32(o_word(K, i, O_SLOT_POINT));
    if (i < m)
        return winv * (P->gam[i - 1] + P->dgam[i] * o_te(&P->caps, K, i, P->lam4[i], P->a4[i], P->c14[i]));
    return winv * (P->gam[m - 1] + P->delta * o_exp1(o_word(K, i, O_SLOT_POINT)));
}
/* Last point of a stream: the without-replacement variants draw every label
 * once (Sec. 2.4, 2.6), the others stop at the cap. */
static inline uint64_t o_stream_end(const o_params *P) {
    return (P->variant == 2 || P->variant == 4) ? P->m : P->caps.imax;
}

/* Random permutation of the labels drawn one step at a time (Sec. 2.4: a
 * Fisher-Yates shuffle whose array is initialised lazily, so a stream that
 * stops early costs only its steps).  g[j] is valid where v[j] equals the
 * current version c; elsewhere the slot still holds j.  Step i (1-based)
 * draws slot j uniformly from i-1..m-1, yields the value of slot j and moves
 * the value of slot i-1 into slot j. */
typedef struct {
    uint32_t *g, *v;
    uint32_t c, i, m;
} o_perm;

static int o_perm_init(o_perm *F, uint32_t m) {
    F->g = malloc(sizeof(uint32_t) * m);
    F->v = calloc(m, sizeof(uint32_t));
    F->c = 0;
    F->i = 0;
    F->m = m;
    return (F->g && F->v) ? O_OK : O_ERR_OOM;
}
static void o_perm_free(o_perm *F) { free(F->g); free(F->v); }
static inline void o_perm_reset(o_perm *F) {
    if (F->c == 0xFFFFFFFFu) { /* the version counter would wrap: clear the versions */
        memset(F->v, 0, sizeof(uint32_t) * F->m);
        F->c = 0;
    }
    F->i = 0;
    F->c += 1;
}
static inline uint32_t o_perm_slot(const o_perm *F, uint32_t j) { return F->v[j] == F->c ? F->g[j] : j; }
static inline uint32_t o_perm_next(const o_caps *C, o_perm *F, uint64_t K) {
    const uint32_t i = ++F->i;
    const uint32_t j = (i - 1) + o_lemire(C, K, i, F->m - i + 1);
    const uint32_t out = o_perm_slot(F, j);
    F->g[j] = o_perm_slot(F, i - 1);
    F->v[j] = F->c;
    return out;
}

/* ------------------------------------------------------------------------ */
/* Signature under construction: keys[k] = the smallest key offered to
 * component k so far (eq. (1) in key space), and the stop limit kmax =
 * max_k keys[k] (Sec. 2: no point at or above it can change the signature).
 * kmax stays EMPTY while some component is empty and is recomputed by a scan
 * when the component holding it is lowered. */
typedef struct {
    uint64_t *keys;
    uint32_t m;
    uint32_t empty;  /* components still EMPTY */
    uint64_t kmax;
    uint64_t points; /* points generated */
    uint64_t labels; /* labels drawn */
} o_sig;

static void o_sig_reset(o_sig *S) {
    for (uint32_t k = 0; k < S->m; ++k) S->keys[k] = O_EMPTY;
    S->empty = S->m;
    S->kmax = O_EMPTY;
}
static void o_offer(o_sig *S, uint32_t k, uint64_t key) {
    const uint64_t old = S->keys[k];
    if (key >= old) return;
    S->keys[k] = key;
    if (old == O_EMPTY) {
        if (--S->empty > 0) return;
    } else if (old != S->kmax) {
        return;
    }
    uint64_t mx = 0;
    for (uint32_t j = 0; j < S->m; ++j) mx = S->keys[j] > mx ? S->keys[j] : mx;
    S->kmax = mx;
}

/* One element's stream as it is consumed point by point. */
typedef struct {
    uint32_t p;     /* position in the set (the key's tie-break) */
    double winv;
    uint64_t K;
    uint64_t i;     /* next point */
    uint64_t T;     /* ProbMinHash1/2: fixed-point sum through point i-1 */
    double x;       /* value of point i-1 */
} o_elem;

static inline o_elem o_elem_start(uint64_t seedhash, uint64_t id, double w, uint32_t p) {
    o_elem e = {p, 1.0 / w, o_mix64(id ^ seedhash), 1, 0, 0.0};
    return e;
}

/* Consumes point i of the element unless a lower bound of the values of
 * points i, i+1, ... reaches the stop limit; offers the point to its label.
 * Returns 1 while a later point may still lower a component.  Lower bounds:
 * the exponential-spacing streams (ProbMinHash1/2) increase, so the previous
 * point bounds the next ones and a point bounds itself; the interval streams
 * (ProbMinHash3/4) are bounded by the start of the point's interval.  F: the
 * element's permutation (ProbMinHash2/4). */
static int o_step(const o_params *P, o_elem *e, o_perm *F, o_sig *S) {
    const uint64_t i = e->i;
    const int expo = P->variant <= 2;
    double x;
    if (expo) {
        if (i > 1 && o_key(e->x, e->p) >= S->kmax) return 0;
        e->T += o_spacing(P, e->K, i);
        x = o_fixed_value(e->winv, e->T);
        S->points++;
        if (o_key(x, e->p) >= S->kmax) return 0;
    } else {
        if (o_key(o_lower(P, e->winv, i), e->p) >= S->kmax) return 0;
        x = P->variant == 3 ? o_value3(P, e->K, i, e->winv) : o_value4(P, e->K, i, e->winv);
        S->points++;
    }
    const uint64_t key = o_key(x, e->p);
    if (P->variant == 2 || P->variant == 4) { /* every generated point takes its permutation step */
        S->labels++;
        o_offer(S, o_perm_next(&P->caps, F, e->K), key);
    } else if (key < S->kmax) {
        S->labels++;
        o_offer(S, o_lemire(&P->caps, e->K, i, P->m), key);
    }
    e->x = x;
    e->i = i + 1;
    if (i == o_stream_end(P)) return 0;
    if (expo) return o_key(x, e->p) < S->kmax;
    return o_key(o_lower(P, e->winv, i + 1), e->p) < S->kmax;
}

/* Sequential signature (Sec. 2.3-2.6): each element's stream in turn, until
 * it can no longer lower a component. */
static void o_sign_seq(const o_params *P, uint64_t seedhash, const uint64_t *ids, const double *w,
                       uint32_t n, o_sig *S, o_perm *F) {
    o_sig_reset(S);
    for (uint32_t p = 0; p < n; ++p) {
        if (!(w[p] > 0.0)) continue;
        o_elem e = o_elem_start(seedhash, ids[p], w[p], p);
        o_perm_reset(F);
        while (o_step(P, &e, F, S)) {
        }
    }
}

/* Interleaved ProbMinHash1a / ProbMinHash3a (Sec. 2.7): one point of every
 * element, then passes over the elements that can still lower a component,
 * one point each, until none is left.  *buffer receives the number of live
 * elements after the first pass (the largest the buffer gets). */
static int o_sign_interleaved(const o_params *P, uint64_t seedhash, const uint64_t *ids,
                              const double *w, uint32_t n, o_sig *S, uint64_t *buffer) {
    o_sig_reset(S);
    o_elem *live = malloc(sizeof(o_elem) * (n ? n : 1));
    if (!live) return O_ERR_OOM;
    uint32_t s = 0;
    for (uint32_t p = 0; p < n; ++p) {
        if (!(w[p] > 0.0)) continue;
        o_elem e = o_elem_start(seedhash, ids[p], w[p], p);
        if (o_step(P, &e, NULL, S)) live[s++] = e;
    }
    *buffer = s;
    while (s > 0) {
        uint32_t t = 0;
        for (uint32_t j = 0; j < s; ++j)
            if (o_step(P, &live[j], NULL, S)) live[t++] = live[j];
        s = t;
    }
    free(live);
    return O_OK;
}

/* Brute force: every point of every element's stream (to the end of the
 * permutation for PMH2/4, to the cap for PMH1/3), then key_k = min over all
 * points labelled k.  No stop rule is involved. */
static int o_sign_brute(const o_params *P, uint64_t seedhash, const uint64_t *ids, const double *w,
                        uint32_t n, uint64_t *keys, uint64_t *points) {
    const uint32_t m = P->m;
    o_perm F;
    if (o_perm_init(&F, m) != O_OK) { o_perm_free(&F); return O_ERR_OOM; }
    for (uint32_t k = 0; k < m; ++k) keys[k] = O_EMPTY;
    const uint64_t last = o_stream_end(P);
    for (uint32_t p = 0; p < n; ++p) {
        if (!(w[p] > 0.0)) continue;
        double winv = 1.0 / w[p];
        uint64_t K = o_mix64(ids[p] ^ seedhash);
        uint64_t T = 0;
        o_perm_reset(&F);
        for (uint64_t i = 1; i <= last; ++i) {
            double x;
            uint32_t k;
            if (P->variant <= 2) {
                T += o_spacing(P, K, i);
                x = o_fixed_value(winv, T);
            } else if (P->variant == 3) {
                x = o_value3(P, K, i, winv);
            } else {
                x = o_value4(P, K, i, winv);
            }
            if (P->variant == 1 || P->variant == 3) k = o_lemire(&P->caps, K, i, m);
            else k = o_perm_next(&P->caps, &F, K);
            (*points)++;
            uint64_t key = o_key(x, p);
            if (key < keys[k]) keys[k] = key;
        }
    }
    o_perm_free(&F);
    return O_OK;
}

/* ------------------------------------------------------------------------ */
/* Exported API (ctypes).  Weights: 0 skips the element; negative, NaN,
 * infinite or subnormal weights are rejected. */
static int o_check_weights(const double *w, uint64_t n) {
    for (uint64_t p = 0; p < n; ++p) {
        double x = w[p];
        if (x == 0.0) continue;
        if (!(x > 0.0) || !(x <= 0x1.fffffffffffffp+1023) || x < 0x1p-1022) return O_ERR_WEIGHT;
    }
    return O_OK;
}

uint64_t or_seedhash(uint64_t seed) { return o_mix64(seed); }
uint64_t or_mix64(uint64_t z) { return o_mix64(z); }
uint64_t or_word(uint64_t K, uint64_t i, unsigned t) { return o_word(K, i, t); }
double or_exp1_word(uint64_t w) { return o_exp1(w); }
/* Lemire draw from [0, s) of point i with redraws <= 8 and a validation floor. */
uint32_t or_lemire(uint64_t K, uint64_t i, uint32_t s, unsigned redraws, uint32_t floor) {
    o_caps C = {0, O_TE_ROUNDS_MAX, redraws > O_REDRAWS_MAX ? O_REDRAWS_MAX : redraws, floor};
    return o_lemire(&C, K, i, s);
}
/* Truncated exponential of point i (rate lam, a = e^lam - 1, c1 = a/lam) with
 * at most rounds (1..32) proposals in the second branch. */
double or_te(uint64_t K, uint64_t i, double lam, double a, double c1, unsigned rounds) {
    o_caps C = {0, rounds < 1 ? 1 : (rounds > O_TE_ROUNDS_MAX ? O_TE_ROUNDS_MAX : rounds), O_REDRAWS_MAX, 0};
    return o_te(&C, K, i, lam, a, c1);
}
uint64_t or_key(double x, uint32_t p) { return o_key(x, p); }

/* Constants of (variant, m) for inspection by the tests.  out[] receives
 * PMH3: {lambda, a = e^lambda - 1, c1 = a/lambda}; PMH4 with index i:
 * {lambda_i, a_i, c1_i, gamma_i, dgamma_i, delta}; PMH2 with index i:
 * {beta_i}. */
int or_constants(int variant, uint32_t m, uint32_t i, double *out) {
    o_params P;
    int rc = o_params_init(&P, variant, m, NULL);
    if (rc) return rc;
    if (P.variant == 2 && i >= 1 && i <= m) out[0] = P.beta[i];
    if (P.variant == 3) { out[0] = P.lam3; out[1] = P.a3; out[2] = P.c13; }
    if (P.variant == 4 && i < m) {
        out[0] = P.lam4[i]; out[1] = P.a4[i]; out[2] = P.c14[i];
        out[3] = P.gam[i]; out[4] = P.dgam[i]; out[5] = P.delta;
    }
    o_params_free(&P);
    return O_OK;
}

/* Points 1..count of element K with weight inverse winv, for stream tests:
 * values and labels written to xs/ls (labels by Lemire for PMH1/3, by the
 * permutation steps 1..count for PMH2/4).  caps4 as for or_sign_capped. */
int or_stream(int variant, uint32_t m, uint64_t K, double winv, uint64_t count, double *xs,
              uint32_t *ls, const uint64_t *caps4) {
    o_params P;
    int rc = o_params_init(&P, variant, m, caps4);
    if (rc) return rc;
    o_perm F;
    if (o_perm_init(&F, m) != O_OK) { o_perm_free(&F); o_params_free(&P); return O_ERR_OOM; }
    o_perm_reset(&F);
    uint64_t T = 0;
    const uint64_t last = o_stream_end(&P);
    for (uint64_t i = 1; i <= count && i <= last; ++i) {
        if (P.variant <= 2) {
            T += o_spacing(&P, K, i);
            xs[i - 1] = o_fixed_value(winv, T);
        } else if (P.variant == 3) {
            xs[i - 1] = o_value3(&P, K, i, winv);
        } else {
            xs[i - 1] = o_value4(&P, K, i, winv);
        }
        ls[i - 1] = (P.variant == 1 || P.variant == 3) ? o_lemire(&P.caps, K, i, m) : o_perm_next(&P.caps, &F, K);
    }
    o_perm_free(&F);
    o_params_free(&P);
    return O_OK;
}

/* mode 0: sequential (Sec. 2.3-2.6), 1: interleaved (Sec. 2.7, PMH1/PMH3
 * only), 2: brute force.  keys[m] out; stats[3] = {points, labels, buffer
 * size after the first pass (interleaved mode, else 0)}.  caps4 = {imax (0:
 * default), te_rounds (1..32), redraws (0..8), lemire_floor} or NULL for the
 * default caps. */
int or_sign_capped(int mode, int variant, uint64_t seed, uint32_t m, const uint64_t *ids, const double *w,
                   uint64_t n, uint64_t *keys, uint64_t *stats, const uint64_t *caps4) {
    if ((!ids || !w) && n) return O_ERR_ARG;
    if (n > O_MAX_SET) return O_ERR_SET_TOO_LARGE;
    int rc = o_check_weights(w, n);
    if (rc) return rc;
    o_params P;
    rc = o_params_init(&P, variant, m, caps4);
    if (rc) return rc;
    if (mode == 1 && P.variant != 1 && P.variant != 3) { o_params_free(&P); return O_ERR_ARG; }
    const uint64_t sh = o_mix64(seed);
    uint64_t points = 0, labels = 0, buffer = 0;
    if (mode == 2) {
        rc = o_sign_brute(&P, sh, ids, w, (uint32_t)n, keys, &points);
    } else {
        o_sig S = {keys, m, 0, 0, 0, 0};
        o_perm F;
        rc = o_perm_init(&F, m);
        if (rc) rc = O_ERR_OOM;
        else if (mode == 0) o_sign_seq(&P, sh, ids, w, (uint32_t)n, &S, &F);
        else rc = o_sign_interleaved(&P, sh, ids, w, (uint32_t)n, &S, &buffer);
        o_perm_free(&F);
        points = S.points;
        labels = S.labels;
    }
    if (stats) { stats[0] = points; stats[1] = labels; stats[2] = buffer; }
    o_params_free(&P);
    return rc;
}

int or_sign(int mode, int variant, uint64_t seed, uint32_t m, const uint64_t *ids, const double *w,
            uint64_t n, uint64_t *keys, uint64_t *stats) {
    return or_sign_capped(mode, variant, seed, m, ids, w, n, keys, stats, NULL);
}

/* ------------------------------------------------------------------------ */
/* P-MinHash (Sec. 1.1, algorithm "P-MinHash"): every element of positive
 * weight draws m exponential values of rate 1 scaled by its reciprocal weight,
 * one per component, and component k keeps the smallest (eq. (2) with the
 * hash functions of Sec. 1.1).  Reading: the k-th value of element K takes
 * its uniform from slot 128 of point k of the element's counter stream (a
 * slot no ProbMinHash stream uses), Exp(1) by the same stream logarithm, and
 * the value fl(winv * Exp(1)) enters the same (value, position) key space. */
#define O_SLOT_PMIN 128u
static void o_pminhash(uint64_t sh, const uint64_t *ids, const double *w, uint32_t n, uint32_t m,
                       uint64_t *keys) {
    for (uint32_t k = 0; k < m; ++k) keys[k] = O_EMPTY;
    for (uint32_t p = 0; p < n; ++p) {
        if (w[p] == 0.0) continue;
        const double winv = 1.0 / w[p];
        const uint64_t K = o_mix64(ids[p] ^ sh);
        for (uint32_t k = 1; k <= m; ++k) {
            const uint64_t key = o_key(winv * o_exp1(o_word(K, k, O_SLOT_PMIN)), p);
            if (key < keys[k - 1]) keys[k - 1] = key;
        }
    }
}

int or_pminhash(uint64_t seed, uint32_t m, const uint64_t *ids, const double *w, uint64_t n,
                uint64_t *keys) {
    if ((!ids || !w) && n) return O_ERR_ARG;
    if (m < 1 || m > O_MAX_M) return O_ERR_M_RANGE;
    if (n > O_MAX_SET) return O_ERR_SET_TOO_LARGE;
    int rc = o_check_weights(w, n);
    if (rc) return rc;
    o_pminhash(o_mix64(seed), ids, w, (uint32_t)n, m, keys);
    return O_OK;
}

/* ------------------------------------------------------------------------ */
/* b-bit reduction (Sec. 1.3, algorithm "Reduction to a b-bit signature"):
 * component k (1-based) of value z -- the component's element id, 0 when the
 * component is empty -- becomes the b least significant bits of a hash of
 * the pair (z, k).  Reading: hash = mix64(mix64(z) + k*phi), so equal ids in
 * the same component always agree and different ids agree with probability
 * 2^-b, independently across components.  Packing: b in {1, 2, 4, 8, 16},
 * component k-1 in bits [((k-1) b) mod 64, +b) of word ((k-1) b) / 64,
 * ceil(m b / 64) words per signature, unused high bits zero. */
uint64_t or_bbit_hash(uint64_t z, uint64_t k) { return o_mix64(o_mix64(z) + k * O_PHI); }

int or_bbit_pack(const uint64_t *ids, uint64_t num_sigs, uint32_t m, uint32_t b, uint64_t *out) {
    if (m < 1 || (b != 1 && b != 2 && b != 4 && b != 8 && b != 16)) return O_ERR_ARG;
    const uint64_t W = ((uint64_t)m * b + 63) / 64;
    const uint64_t mask = ((uint64_t)1 << b) - 1;
    for (uint64_t s = 0; s < num_sigs; ++s) {
        uint64_t *o = out + s * W;
        for (uint64_t w = 0; w < W; ++w) o[w] = 0;
        for (uint32_t k = 0; k < m; ++k) {
            const uint64_t v = or_bbit_hash(ids[s * m + k], (uint64_t)k + 1) & mask;
            const uint64_t bit = (uint64_t)k * b;
            o[bit / 64] |= v << (bit % 64);
        }
    }
    return O_OK;
}

/* Number of components whose b-bit fields agree, by unpacking. */
uint32_t or_bbit_equal(const uint64_t *a, const uint64_t *c, uint32_t m, uint32_t b) {
    const uint64_t mask = ((uint64_t)1 << b) - 1;
    uint32_t eq = 0;
    for (uint32_t k = 0; k < m; ++k) {
        const uint64_t bit = (uint64_t)k * b;
        eq += ((a[bit / 64] >> (bit % 64)) & mask) == ((c[bit / 64] >> (bit % 64)) & mask);
    }
    return eq;
}

/* Decode keys into (idx, val, id): idx = position, val = truncated value,
 * id = ids[idx]; an empty component gives idx 0xFFFFFFFF, val +inf, id 0. */
void or_decode(const uint64_t *keys, uint64_t m, const uint64_t *ids, uint32_t *idx, double *val,
               uint64_t *id) {
    for (uint64_t k = 0; k < m; ++k) {
        uint64_t key = keys[k];
        if (key == O_EMPTY) {
            if (idx) idx[k] = 0xFFFFFFFFu;
            if (val) val[k] = INFINITY;
            if (id) id[k] = 0;
            continue;
        }
        uint32_t p = (uint32_t)(key & O_POS_MASK);
        uint64_t vb = key & ~O_POS_MASK;
        if (idx) idx[k] = p;
        if (val) memcpy(&val[k], &vb, 8);
        if (id) id[k] = ids[p];
    }
}

/* Batch of sets in CSR form on a pool of threads, sequential algorithm per
 * set.  keys_out: num_sets * m.  stats: {points, labels} summed. */
typedef struct {
    const o_params *P;  /* NULL: P-MinHash with m = pm */
    uint32_t pm;
    uint64_t sh;
    const uint64_t *ids;
    const double *w;
    const uint64_t *off;
    uint64_t num_sets;
    uint64_t *keys;
    volatile uint64_t next;
    pthread_mutex_t lock;
    uint64_t points, labels;
    int rc;
} o_batch;

static void *o_batch_worker(void *arg) {
    o_batch *B = arg;
    const uint32_t m = B->P ? B->P->m : B->pm;
    o_perm F;
    int rc = o_perm_init(&F, m);
    uint64_t points = 0, labels = 0;
    if (!rc) {
        for (;;) {
            uint64_t s = __atomic_fetch_add(&B->next, 1, __ATOMIC_RELAXED);
            if (s >= B->num_sets) break;
            uint64_t a = B->off[s], b = B->off[s + 1];
            if (B->P) {
                o_sig S = {B->keys + s * m, m, 0, 0, 0, 0};
                o_sign_seq(B->P, B->sh, B->ids + a, B->w + a, (uint32_t)(b - a), &S, &F);
                points += S.points;
                labels += S.labels;
            } else {
                o_pminhash(B->sh, B->ids + a, B->w + a, (uint32_t)(b - a), m, B->keys + s * m);
            }
        }
    } else {
        rc = O_ERR_OOM;
    }
    pthread_mutex_lock(&B->lock);
    B->points += points;
    B->labels += labels;
    if (rc) B->rc = rc;
    pthread_mutex_unlock(&B->lock);
    o_perm_free(&F);
    return NULL;
}

int or_sign_batch_capped(int variant, uint64_t seed, uint32_t m, const uint64_t *ids, const double *w,
                         const uint64_t *offsets, uint64_t num_sets, uint64_t *keys_out, int nthreads,
                         uint64_t *stats, const uint64_t *caps4) {
    if (!offsets || !keys_out) return O_ERR_ARG;
    if (offsets[0] != 0) return O_ERR_ARG;
    for (uint64_t s = 0; s < num_sets; ++s) {
        if (offsets[s + 1] < offsets[s]) return O_ERR_ARG;
        if (offsets[s + 1] - offsets[s] > O_MAX_SET) return O_ERR_SET_TOO_LARGE;
    }
    int rc = o_check_weights(w, offsets[num_sets]);
    if (rc) return rc;
    o_params P;
    rc = o_params_init(&P, variant, m, caps4);
    if (rc) return rc;
    o_batch B = {&P, m, o_mix64(seed), ids, w, offsets, num_sets, keys_out, 0,
                 PTHREAD_MUTEX_INITIALIZER, 0, 0, 0};
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = malloc(sizeof(pthread_t) * nthreads);
    int started = 0;
    for (int t = 0; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, o_batch_worker, &B) == 0) ++started;
    if (started == 0) o_batch_worker(&B);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    free(th);
    if (stats) { stats[0] = B.points; stats[1] = B.labels; }
    o_params_free(&P);
    return B.rc;
}

int or_sign_batch(int variant, uint64_t seed, uint32_t m, const uint64_t *ids, const double *w,
                  const uint64_t *offsets, uint64_t num_sets, uint64_t *keys_out, int nthreads,
                  uint64_t *stats) {
    return or_sign_batch_capped(variant, seed, m, ids, w, offsets, num_sets, keys_out, nthreads, stats, NULL);
}

/* P-MinHash over a batch of sets in CSR form (keys_out: num_sets * m). */
int or_pminhash_batch(uint64_t seed, uint32_t m, const uint64_t *ids, const double *w,
                      const uint64_t *offsets, uint64_t num_sets, uint64_t *keys_out, int nthreads) {
    if (!offsets || !keys_out || offsets[0] != 0) return O_ERR_ARG;
    if (m < 1 || m > O_MAX_M) return O_ERR_M_RANGE;
    for (uint64_t s = 0; s < num_sets; ++s) {
        if (offsets[s + 1] < offsets[s]) return O_ERR_ARG;
        if (offsets[s + 1] - offsets[s] > O_MAX_SET) return O_ERR_SET_TOO_LARGE;
    }
    int rc = o_check_weights(w, offsets[num_sets]);
    if (rc) return rc;
    o_batch B = {NULL, m, o_mix64(seed), ids, w, offsets, num_sets, keys_out, 0,
                 PTHREAD_MUTEX_INITIALIZER, 0, 0, 0};
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = malloc(sizeof(pthread_t) * nthreads);
    int started = 0;
    for (int t = 0; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, o_batch_worker, &B) == 0) ++started;
    if (started == 0) o_batch_worker(&B);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    free(th);
    return B.rc;
}
