"""CPU oracle for ProbMinHash signatures (Ertl, IEEE TKDE 2020, arXiv 1911.00675).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The product library never imports,
links or calls anything here, and nothing here calls the product library.

Two layers:

* ``liboracle.so`` (``pmh_oracle.c``): ProbMinHash1-4 (Sec. 2.3-2.6) as one
  stream-consuming loop with the stop rule of Sec. 2 and the per-variant lower
  bounds of Sec. 2.5/2.6, the lazily initialised random permutation of
  Sec. 2.4, the interleaved ProbMinHash1a/3a (Sec. 2.7), a brute-force
  signature (eq. (1) with the hash values of eq. (9)), P-MinHash (Sec. 1.1,
  the paper's O(nm) baseline), the b-bit reduction of Sec. 1.3 and the
  random-stream primitives, with the loop caps of Sec. 3 as parameters.
* numpy functions below: the probability Jaccard similarity J_P written out
  from its definition (Sec. 1.1, "Incorporating Weights"), an O(N log N) form
  of it, the estimator of eq. (3), SuperMinHash's variance factor alpha(m, u)
  (eq. (8)) and the MSE moments quoted in Sec. 3.1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pmh_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

EMPTY = 0xFFFFFFFFFFFFFFFF
IDX_EMPTY = 0xFFFFFFFF
POS_MASK = 0xFFFFF

OK, ERR_ARG, ERR_M_RANGE, ERR_VARIANT_M, ERR_WEIGHT, ERR_SET_TOO_LARGE = 0, 1, 2, 3, 4, 5
ERR_OOM = 7

MODE_SEQUENTIAL, MODE_INTERLEAVED, MODE_BRUTE = 0, 1, 2


CFLAGS = ["-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-fPIC"]


def build(force: bool = False) -> str:
    """Compile the oracle with strict IEEE double semantics (no contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc"] + CFLAGS + ["-shared", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u64, u32, dbl, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_int
        vp = ctypes.c_void_p
        sig = {
            "or_log": (dbl, [dbl]), "or_log1p": (dbl, [dbl]), "or_expm1": (dbl, [dbl]),
            "or_log_stream": (dbl, [dbl]), "or_log_table": (None, [vp]),
            "or_seedhash": (u64, [u64]), "or_mix64": (u64, [u64]),
            "or_word": (u64, [u64, u64, ctypes.c_uint]), "or_exp1_word": (dbl, [u64]),
            "or_lemire": (u32, [u64, u64, u32, ctypes.c_uint, u32]),
            "or_te": (dbl, [u64, u64, dbl, dbl, dbl, ctypes.c_uint]),
            "or_key": (u64, [dbl, u32]), "or_imax": (u64, [u32]),
            "or_constants": (i32, [i32, u32, u32, vp]),
            "or_stream": (i32, [i32, u32, u64, dbl, u64, vp, vp, vp]),
            "or_sign": (i32, [i32, i32, u64, u32, vp, vp, u64, vp, vp]),
            "or_sign_capped": (i32, [i32, i32, u64, u32, vp, vp, u64, vp, vp, vp]),
            "or_sign_batch_capped": (i32, [i32, u64, u32, vp, vp, vp, u64, vp, i32, vp, vp]),
            "or_decode": (None, [vp, u64, vp, vp, vp, vp]),
            "or_sign_batch": (i32, [i32, u64, u32, vp, vp, vp, u64, vp, i32, vp]),
            "or_pminhash": (i32, [u64, u32, vp, vp, u64, vp]),
            "or_bbit_hash": (u64, [u64, u64]),
            "or_bbit_pack": (i32, [vp, u64, u32, u32, vp]),
            "or_bbit_equal": (u32, [vp, vp, u32, u32]),
            "or_pminhash_batch": (i32, [u64, u32, vp, vp, vp, u64, vp, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle status {code}")
        self.code = code


# --------------------------------------------------------------------------- #
# primitives (for the distribution and accuracy pins)

def spec_log(x: float) -> float:
    return lib().or_log(float(x))


def stream_log(x: float) -> float:
    """Table-driven logarithm behind the streams' Exp(1) variates."""
    return lib().or_log_stream(float(x))


def stream_log_table() -> np.ndarray:
    out = np.zeros(512, dtype=np.float64)
    lib().or_log_table(_ptr(out))
    return out


def spec_log1p(x: float) -> float:
    return lib().or_log1p(float(x))


def spec_expm1(x: float) -> float:
    return lib().or_expm1(float(x))


def seedhash(seed: int) -> int:
    return lib().or_seedhash(seed & EMPTY)


def mix64(z: int) -> int:
    return lib().or_mix64(z & EMPTY)


def element_key(seed: int, elem_id: int) -> int:
    return mix64((elem_id & EMPTY) ^ seedhash(seed))


def word(K: int, i: int, t: int) -> int:
    return lib().or_word(K, i, t)


def exp1_of_word(w: int) -> float:
    return lib().or_exp1_word(w)


def lemire(K: int, i: int, s: int, redraws: int = 8, floor: int = 0) -> int:
    """Uniform label in [0, s) of point i (Lemire), at most `redraws` redraws;
    floor > 0 also redraws every low product half below it (validation)."""
    return lib().or_lemire(K, i, s, redraws, floor)


def trunc_exp(K: int, i: int, lam: float, a: float, c1: float, rounds: int = 32) -> float:
    """Exp(lam; 0, 1) variate of point i (Sec. 2.8), a = e^lam - 1, c1 = a/lam."""
    return lib().or_te(K, i, lam, a, c1, rounds)


def key(x: float, p: int) -> int:
    return lib().or_key(x, p)


def imax(m: int) -> int:
    return lib().or_imax(m)


def constants(variant: int, m: int, i: int = 0) -> np.ndarray:
    out = np.zeros(8, dtype=np.float64)
    rc = lib().or_constants(variant, m, i, _ptr(out))
    if rc:
        raise OracleError(rc)
    return out


class Caps:
    """Loop caps of the streams (Sec. 3 advises bounding every loop): imax
    points per ProbMinHash1/3 element (0: the default 6 m bitlen(m) + 64),
    te_rounds proposals of the truncated-exponential sampler (1..32), redraws
    of Lemire's method (0..8), and lemire_floor, a validation-only switch that
    forces redraws of every draw whose low product half lies below it."""

    def __init__(self, imax: int = 0, te_rounds: int = 32, redraws: int = 8, lemire_floor: int = 0):
        self.imax, self.te_rounds, self.redraws, self.lemire_floor = imax, te_rounds, redraws, lemire_floor

    def array(self):
        return np.array([self.imax, self.te_rounds, self.redraws, self.lemire_floor], dtype=np.uint64)


def _caps_ptr(caps):
    if caps is None:
        return None, None
    a = caps.array()
    return a, _ptr(a)


def stream(variant: int, m: int, K: int, winv: float, count: int, caps: Caps | None = None):
    """Values and labels of points 1..count of one element's stream."""
    xs = np.zeros(count, dtype=np.float64)
    ls = np.zeros(count, dtype=np.uint32)
    keep, cp = _caps_ptr(caps)
    rc = lib().or_stream(variant, m, K, winv, count, _ptr(xs), _ptr(ls), cp)
    if rc:
        raise OracleError(rc)
    return xs, ls


# --------------------------------------------------------------------------- #
# signatures

def sign(variant: int, seed: int, m: int, ids, weights, mode: int = MODE_SEQUENTIAL,
         return_stats: bool = False, caps: Caps | None = None):
    """Keys (uint64[m]) of one weighted set."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    assert ids.shape == w.shape
    keys = np.zeros(m, dtype=np.uint64)
    stats = np.zeros(3, dtype=np.uint64)  # points, labels, interleaved buffer size after pass 1
    keep, cp = _caps_ptr(caps)
    rc = lib().or_sign_capped(mode, variant, seed & EMPTY, m, _ptr(ids), _ptr(w), ids.size, _ptr(keys),
                              _ptr(stats), cp)
    if rc:
        raise OracleError(rc)
    return (keys, stats) if return_stats else keys


def sign_batch(variant: int, seed: int, m: int, ids, weights, offsets, nthreads: int = 1,
               return_stats: bool = False, caps: Caps | None = None):
    """Keys (uint64[num_sets, m]) of a CSR batch, sequential algorithm per set."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    S = off.size - 1
    keys = np.zeros((S, m), dtype=np.uint64)
    stats = np.zeros(2, dtype=np.uint64)
    keep, cp = _caps_ptr(caps)
    rc = lib().or_sign_batch_capped(variant, seed & EMPTY, m, _ptr(ids), _ptr(w), _ptr(off), S,
                                    _ptr(keys), int(nthreads), _ptr(stats), cp)
    if rc:
        raise OracleError(rc)
    return (keys, stats) if return_stats else keys


def pminhash(seed: int, m: int, ids, weights):
    """P-MinHash keys (uint64[m]) of one weighted set (Sec. 1.1)."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    assert ids.shape == w.shape
    keys = np.zeros(m, dtype=np.uint64)
    rc = lib().or_pminhash(seed & EMPTY, m, _ptr(ids), _ptr(w), ids.size, _ptr(keys))
    if rc:
        raise OracleError(rc)
    return keys


def pminhash_batch(seed: int, m: int, ids, weights, offsets, nthreads: int = 1):
    """P-MinHash keys (uint64[num_sets, m]) of a CSR batch."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    S = off.size - 1
    keys = np.zeros((S, m), dtype=np.uint64)
    rc = lib().or_pminhash_batch(seed & EMPTY, m, _ptr(ids), _ptr(w), _ptr(off), S, _ptr(keys), int(nthreads))
    if rc:
        raise OracleError(rc)
    return keys


def bbit_words(m: int, b: int) -> int:
    return (m * b + 63) // 64


def bbit_pack(ids, m: int, b: int):
    """b-bit reduction (Sec. 1.3) of signatures given by their element ids
    (uint64[num_sigs, m]; 0 = empty), packed into uint64[num_sigs, words]."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64).reshape(-1, m)
    out = np.zeros((ids.shape[0], bbit_words(m, b)), dtype=np.uint64)
    rc = lib().or_bbit_pack(_ptr(ids), ids.shape[0], m, b, _ptr(out))
    if rc:
        raise OracleError(rc)
    return out


def bbit_equal(a, c, m: int, b: int) -> int:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.uint64)
    return int(lib().or_bbit_equal(_ptr(a), _ptr(c), m, b))


def bbit_estimate(equal: int, m: int, b: int) -> float:
    """J estimate from b-bit signatures: components of different elements
    agree with probability 2^-b, so E[equal/m] = J + (1 - J) 2^-b and
    (equal/m - 2^-b) / (1 - 2^-b) is unbiased (the bias Sec. 1.3 says must be
    accounted for)."""
    r = 2.0 ** -b
    return (equal / m - r) / (1.0 - r)


def decode(keys, ids):
    """(idx uint32, val float64, id uint64) per component, for one set."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    m = keys.size
    idx = np.zeros(m, dtype=np.uint32)
    val = np.zeros(m, dtype=np.float64)
    idv = np.zeros(m, dtype=np.uint64)
    lib().or_decode(_ptr(keys), m, _ptr(ids), _ptr(idx), _ptr(val), _ptr(idv))
    return idx, val, idv


# --------------------------------------------------------------------------- #
# similarity and statistics (numpy, fp64)

def jp_definition(wa: dict, wb: dict) -> float:
    """J_P written out from its definition: sum over d of
    1 / sum over d' of max(wA(d')/wA(d), wB(d')/wB(d)); elements with a zero
    weight in either set contribute nothing (their inner sum is infinite)."""
    keys = set(wa) | set(wb)
    total = 0.0
    for d in keys:
        a, b = wa.get(d, 0.0), wb.get(d, 0.0)
        if a <= 0 or b <= 0:
            continue
        inner = 0.0
        for e in keys:
            inner += max(wa.get(e, 0.0) / a, wb.get(e, 0.0) / b)
        total += 1.0 / inner
    return total


def jp_exact(wa: dict, wb: dict) -> Fraction:
    """Same definition in exact rational arithmetic (for integer/rational weights)."""
    keys = set(wa) | set(wb)
    total = Fraction(0)
    for d in keys:
        a, b = Fraction(wa.get(d, 0)), Fraction(wb.get(d, 0))
        if a <= 0 or b <= 0:
            continue
        inner = Fraction(0)
        for e in keys:
            inner += max(Fraction(wa.get(e, 0)) / a, Fraction(wb.get(e, 0)) / b)
        total += 1 / inner
    return total


def jp_sorted(ids_a, w_a, ids_b, w_b) -> float:
    """J_P in O(N log N).  For d in both sets with ratio r(d) = wA(d)/wB(d):
    max(wA(d')/wA(d), wB(d')/wB(d)) equals wA(d')/wA(d) exactly when
    r(d') >= r(d), so the inner sum is (1/wA(d)) * sum_{r(d')>=r(d)} wA(d')
    + (1/wB(d)) * sum_{r(d')<r(d)} wB(d') with r = +inf for d' only in A and
    r = 0 for d' only in B."""
    ids_a = np.asarray(ids_a, dtype=np.uint64)
    ids_b = np.asarray(ids_b, dtype=np.uint64)
    w_a = np.asarray(w_a, dtype=np.float64)
    w_b = np.asarray(w_b, dtype=np.float64)
    ua, ia = np.unique(ids_a, return_index=True)
    ub, ib = np.unique(ids_b, return_index=True)
    allid = np.union1d(ua, ub)
    wa = np.zeros(allid.size)
    wb = np.zeros(allid.size)
    wa[np.searchsorted(allid, ua)] = w_a[ia]
    wb[np.searchsorted(allid, ub)] = w_b[ib]
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(wb > 0, wa / np.where(wb > 0, wb, 1.0), np.inf)
    r = np.where((wa == 0) & (wb > 0), 0.0, r)
    order = np.argsort(r, kind="stable")
    rs, was, wbs = r[order], wa[order], wb[order]
    # suffix sums of wA over r' >= r (ties included), prefix sums of wB over r' < r
    first = np.searchsorted(rs, rs, side="left")
    suf_a = np.concatenate([np.cumsum(was[::-1])[::-1], [0.0]])
    pre_b = np.concatenate([[0.0], np.cumsum(wbs)])
    both = (was > 0) & (wbs > 0)
    D = suf_a[first[both]] / was[both] + pre_b[first[both]] / wbs[both]
    return float(np.sum(1.0 / D))


def estimate(id_a, idx_a, id_b, idx_b) -> float:
    """Estimator of eq. (3): fraction of components with equal element ids,
    empty components never counting as equal."""
    id_a = np.asarray(id_a, dtype=np.uint64)
    id_b = np.asarray(id_b, dtype=np.uint64)
    idx_a = np.asarray(idx_a, dtype=np.uint32)
    idx_b = np.asarray(idx_b, dtype=np.uint32)
    eq = (id_a == id_b) & (idx_a != IDX_EMPTY) & (idx_b != IDX_EMPTY)
    return float(np.count_nonzero(eq)) / id_a.size


def alpha_superminhash(m: int, u: int) -> Fraction:
    """Variance factor alpha(m, u) of SuperMinHash, eq. (8), exact."""
    if u <= 1 or m == 1:  # one component, or one element: nothing to correlate
        return Fraction(1)
    num = sum(Fraction(l) ** u * ((l + 1) ** u + (l - 1) ** u - 2 * l ** u) for l in range(1, m))
    den = Fraction(m - 1) ** (u - 1) * Fraction(m) ** u * (u - 1)
    return 1 - num / den


def mse_moments(J: float, m: int, c: int):
    """Expectation and variance of the empirical MSE over c pairs for
    independent components (Sec. 3.1)."""
    mean = J * (1 - J) / m
    var = (J * J * (1 - J) ** 2) / (m * m * c) * (2 - 6.0 / m) + J * (1 - J) / (m ** 3 * c)
    return mean, var


def harmonic(n: int) -> float:
    return float(np.sum(1.0 / np.arange(1, n + 1)))
