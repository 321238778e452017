"""Pins of the oracle's random-stream primitives against mathematics.

Each test checks an oracle function against something other than itself: the
C library (as an accuracy reference only), closed forms from the paper, or a
distribution law with a stated significance level.
"""
import json
import math
import os
import struct

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def ulp(x: float) -> float:
    return math.ulp(x)


def test_log_accuracy_against_libm(oracle):
    rng = np.random.default_rng(1)
    # the uniforms the streams feed to the logarithm: k * 2^-53, k in [1, 2^53]
    ks = np.concatenate([rng.integers(1, 2**53, size=20000), np.arange(1, 200), 2**53 - np.arange(0, 200)])
    worst = 0.0
    for k in ks:
        x = float(k) * 2.0 ** -53
        ref = math.log(x)
        got = oracle.spec_log(x)
        if ref == 0.0:
            assert got == 0.0
            continue
        worst = max(worst, abs(got - ref) / ulp(ref))
    assert worst <= 2.0, worst
    # wide-range arguments (used for per-m constants)
    for x in np.exp(rng.uniform(-700, 700, size=5000)):
        ref = math.log(x)
        assert abs(oracle.spec_log(x) - ref) <= 2 * ulp(ref)


def test_stream_log_accuracy_against_libm(oracle):
    """The table-driven logarithm of the streams (every 32-bit uniform grid
    point class, plus general arguments) within 2 ulp of the C library."""
    rng = np.random.default_rng(11)
    ks = np.concatenate([rng.integers(1, 2**32 + 1, size=40000), np.arange(1, 300), 2**32 - np.arange(0, 300)])
    for k in ks:
        x = float(k) * 2.0 ** -32
        ref = math.log(x)
        got = oracle.stream_log(x)
        if ref == 0.0:
            assert got == 0.0
        else:
            assert abs(got - ref) <= 2 * ulp(ref), (x, got, ref)
    # every table cell, both sides of the sqrt(2) split
    for j in range(128):
        for frac in (0.0, 0.25, 0.5, 0.999):
            y = 1.0 + (j + frac) / 128.0
            for e in (-40, -1, 0, 3):
                x = math.ldexp(y, e)
                ref = math.log(x)
                assert abs(oracle.stream_log(x) - ref) <= 2 * ulp(ref), (j, frac, e)


def test_log_exact_points(oracle):
    assert oracle.spec_log(1.0) == 0.0
    for k in range(-60, 61):
        assert abs(oracle.spec_log(2.0 ** k) - k * math.log(2)) <= 2 * ulp(k * math.log(2) or 1.0)


def test_log1p_accuracy(oracle):
    rng = np.random.default_rng(2)
    for u in np.concatenate([np.exp(rng.uniform(np.log(1e-12), 0, 4000)), rng.uniform(1, 1e6, 2000),
                             1.0 / np.arange(1, 20000)]):
        ref = math.log1p(u)
        assert abs(oracle.spec_log1p(u) - ref) <= 2 * ulp(ref), u


def test_expm1_accuracy(oracle):
    for t in np.linspace(0, math.log(2), 5001)[1:]:
        ref = math.expm1(t)
        assert abs(oracle.spec_expm1(t) - ref) <= 2 * ulp(ref), t
    assert oracle.spec_expm1(0.0) == 0.0


def test_word_stream_against_published_splitmix64(oracle):
    """The word stream's first words from key 1234567 are the published
    SplitMix64 outputs from that seed: this pins the mix constants, the
    golden-ratio increment and the counter addressing (tests/golden/
    splitmix64_reference.json names the source)."""
    gold = json.load(open(os.path.join(os.path.dirname(GOLDEN), "splitmix64_reference.json")))
    K = gold["seed"]
    want = [int(v) for v in gold["outputs"]]
    assert [oracle.word(K, 0, t) for t in range(len(want))] == want
    # counter c = (i << 8) | t: point 1 slot 0 is output 257 of the generator
    z = K
    for _ in range(257):
        z = (z + 0x9E3779B97F4A7C15) & (2**64 - 1)
    assert oracle.word(K, 1, 0) == oracle.mix64(z)


def test_mix64_is_a_bijection_step(oracle):
    """The SplitMix64 output function is a composition of invertible steps
    (xor-shift by >= 27 bits, multiplication by odd constants): invert it with
    the modular inverses and recover the input."""
    def inv_xorshift(y, s):
        x = y
        for _ in range(64 // s + 1):
            x = y ^ (x >> s)
        return x & (2**64 - 1)

    c1, c2 = 0xBF58476D1CE4E5B9, 0x94D049BB133111EB
    i1, i2 = pow(c1, -1, 2**64), pow(c2, -1, 2**64)
    rng = np.random.default_rng(3)
    for z in [0, 1, 2**64 - 1] + [int(v) for v in rng.integers(0, 2**63, size=200)]:
        y = oracle.mix64(z)
        x = inv_xorshift(y, 31)
        x = (x * i2) & (2**64 - 1)
        x = inv_xorshift(x, 27)
        x = (x * i1) & (2**64 - 1)
        x = inv_xorshift(x, 30)
        assert x == z


def test_word_stream_avalanche(oracle):
    """Flipping one input bit of the element key flips about half the output
    bits of every word (binomial(64, 1/2) mean 32)."""
    rng = np.random.default_rng(4)
    flips = []
    for _ in range(300):
        K = int(rng.integers(0, 2**63))
        b = int(rng.integers(0, 64))
        for i in (1, 2, 1000):
            flips.append(bin(oracle.word(K, i, 0) ^ oracle.word(K ^ (1 << b), i, 0)).count("1"))
    flips = np.array(flips)
    assert abs(flips.mean() - 32.0) < 0.5
    assert abs(flips.var() - 16.0) < 2.5


def test_exp1_distribution(oracle):
    """Exp(1) from the high 32 bits of a word by inversion."""
    rng = np.random.default_rng(5)
    K = int(rng.integers(0, 2**63))
    xs = np.array([oracle.exp1_of_word(oracle.word(K, i, 0)) for i in range(1, 40001)])
    assert xs.min() >= 0.0 and not np.signbit(xs).any()
    assert stats.kstest(xs, "expon").pvalue > 1e-3
    assert abs(xs.mean() - 1.0) < 4 * 1.0 / math.sqrt(xs.size)


def test_lemire_uniform(oracle):
    rng = np.random.default_rng(6)
    for s in (1, 3, 7, 1000, 4096, 16383):
        K = int(rng.integers(0, 2**63))
        draws = np.array([oracle.lemire(K, i, s) for i in range(1, 30001)])
        assert draws.min() >= 0 and draws.max() < s
        if s == 1:
            assert (draws == 0).all()
        elif s <= 1000:
            counts = np.bincount(draws, minlength=s)
            assert stats.chisquare(counts).pvalue > 1e-3
        else:
            assert stats.kstest(draws / s, "uniform").pvalue > 1e-3


def test_lemire_redraw_path_and_cap(oracle):
    """Lemire's rejection (a biased low product half is redrawn from the next
    slot) and its cap of 8 redraws (Sec. 3 bounds every loop), forced with the
    validation floor: the label equals the one computed here from the words."""
    K, s = 31337, 1000
    for floor in (1 << 31, (1 << 32) - 1):
        for redraws in (0, 1, 3, 8):
            for i in range(1, 200):
                want = None
                thr = max((2**32 - s) % s, floor)
                prod = (oracle.word(K, i, 0) & 0xFFFFFFFF) * s
                r = 1
                while r <= redraws and (prod & 0xFFFFFFFF) < thr:
                    prod = (oracle.word(K, i, r) & 0xFFFFFFFF) * s
                    r += 1
                want = prod >> 32
                assert oracle.lemire(K, i, s, redraws, floor) == want
    # without the floor the default threshold leaves these draws alone
    assert all(oracle.lemire(K, i, s) == ((oracle.word(K, i, 0) & 0xFFFFFFFF) * s) >> 32 or
               ((oracle.word(K, i, 0) & 0xFFFFFFFF) * s) & 0xFFFFFFFF < (2**32 - s) % s for i in range(1, 2000))


def _te_cdf(lam):
    return lambda x: (1 - np.exp(-lam * x)) / (1 - math.exp(-lam))


@pytest.mark.parametrize("m", [2, 4, 16, 256, 4096])
def test_truncated_exponential_law(oracle, m):
    """Exp(lambda; 0, 1) of Sec. 2.8 has CDF (1 - e^{-lambda x})/(1 - e^{-lambda})."""
    lam, a, c1 = oracle.constants(3, m)[:3]
    rng = np.random.default_rng(7 + m)
    K = int(rng.integers(0, 2**63))
    xs = np.array([oracle.trunc_exp(K, i, lam, a, c1) for i in range(1, 30001)])
    assert xs.min() >= 0.0 and xs.max() < 1.0
    assert stats.kstest(xs, _te_cdf(lam)).pvalue > 1e-3


def _remainder_cdf(lam):
    """CDF of the density proportional to e^{-lambda x} - e^{-lambda} on [0, 1):
    what is left of Exp(lambda; 0, 1) once its uniform part (weight
    lambda/(e^lambda - 1)) is taken away."""
    tot = (1 - math.exp(-lam)) / lam - math.exp(-lam)
    return lambda x: ((1 - np.exp(-lam * x)) / lam - x * math.exp(-lam)) / tot


@pytest.mark.parametrize("variant,m,i", [(3, 2, 0), (3, 4, 0), (3, 16, 0), (4, 64, 63), (4, 64, 40)])
def test_truncated_exponential_second_branch_law(oracle, variant, m, i):
    """The draws that miss the uniform part follow the remainder of the density
    (the sampler's proposals, tangent and chord tests and expm1 test together),
    so the mixture is exactly Exp(lambda; 0, 1)."""
    lam, a, c1 = oracle.constants(variant, m, i)[:3]
    K = 4242 + m + i
    xs = []
    pt = 1
    while len(xs) < 6000:
        if c1 * (float(oracle.word(K, pt, 0) >> 32) * 2.0 ** -32) >= 1.0:
            xs.append(oracle.trunc_exp(K, pt, lam, a, c1))
        pt += 1
    assert stats.kstest(np.array(xs), _remainder_cdf(lam)).pvalue > 1e-3


def test_truncated_exponential_proposal_cap(oracle):
    """With one proposal allowed, a rejected proposal is returned as it is: the
    capped path gives the first proposal's x whatever the tests decide."""
    m = 2
    lam, a, c1 = oracle.constants(3, m)[:3]
    K = 99
    capped = diff = 0
    for pt in range(1, 4000):
        if c1 * (float(oracle.word(K, pt, 0) >> 32) * 2.0 ** -32) < 1.0:
            continue
        x1 = float(oracle.word(K, pt, 16) >> 11) * 2.0 ** -53
        assert oracle.trunc_exp(K, pt, lam, a, c1, rounds=1) == x1
        capped += 1
        diff += oracle.trunc_exp(K, pt, lam, a, c1) != x1
    assert capped > 500 and diff > 100  # the uncapped sampler rejects some first proposals


def test_truncated_exponential_law_rate_log2(oracle):
    """The largest rate ProbMinHash4 uses, lambda_{m-1} = log 2 (Sec. 2.8)."""
    m = 64
    lam, a, c1 = oracle.constants(4, m, m - 1)[:3]
    assert lam == pytest.approx(math.log(2), rel=1e-15)
    assert a == 1.0
    K = 12345
    xs = np.array([oracle.trunc_exp(K, i, lam, a, c1) for i in range(1, 30001)])
    assert stats.kstest(xs, _te_cdf(lam)).pvalue > 1e-3


def test_truncated_exponential_fast_path_rate(oracle):
    """Pr(first test succeeds) = (m-1) log(1 + 1/(m-1)), and log 2 ~ 69.3% at
    the worst rate (Sec. 2.8)."""
    gold = json.load(open(GOLDEN))
    for m, lam_idx in ((16, None), (256, None), (64, 63)):
        if lam_idx is None:
            c1 = oracle.constants(3, m)[2]
            expect = (m - 1) * math.log1p(1.0 / (m - 1))
        else:
            c1 = oracle.constants(4, m, lam_idx)[2]
            expect = gold["te_fast_path_worst"]["probability"]
        K = 777 + m
        N = 40000
        hits = sum(1 for i in range(1, N + 1)
                   if c1 * (float(oracle.word(K, i, 0) >> 32) * 2.0 ** -32) < 1.0)
        sd = math.sqrt(expect * (1 - expect) / N)
        tol = max(4 * sd, gold["te_fast_path_worst"]["tolerance"] if lam_idx else 0)
        assert abs(hits / N - expect) < tol + 4 * sd


def test_constants_closed_forms(oracle):
    """Per-m constants against their definitions in high precision."""
    import mpmath
    mpmath.mp.prec = 200
    for m in (2, 3, 64, 1024, 4096, 16384):
        lam, a, c1 = oracle.constants(3, m)[:3]
        L = mpmath.log(1 + mpmath.mpf(1) / (m - 1))
        assert abs(lam - float(L)) <= 2 * ulp(float(L))
        assert a == 1.0 / (m - 1)  # e^lambda - 1 = 1/(m-1)
        ref = (mpmath.e ** L - 1) / L
        assert abs(c1 - float(ref)) <= 4 * ulp(float(ref)), (m, c1, ref)
    for m in (2, 5, 64, 1024):
        row1 = oracle.constants(4, m, 1)
        assert row1[3] == 1.0  # gamma_1 = log(1+1/(m-1))/lambda_1 = 1 exactly
        assert row1[5] == pytest.approx(1.0 / row1[0], rel=0)  # delta = 1/lambda_1
        prev = 0.0
        for i in range(1, m):
            row = oracle.constants(4, m, i)
            Li = mpmath.log(1 + mpmath.mpf(1) / (m - i))
            assert abs(row[0] - float(Li)) <= 2 * ulp(float(Li))
            assert row[1] == 1.0 / (m - i)
            g = row[3]
            ref = float(mpmath.log(1 + mpmath.mpf(i) / (m - i)) / mpmath.log(1 + mpmath.mpf(1) / (m - 1)))
            assert abs(g - ref) <= 8 * ulp(ref)
            assert g > prev  # boundaries strictly increase
            prev = g
    for m in (1, 7, 100):
        for i in range(1, m + 1):
            assert oracle.constants(2, m, i)[0] == m / (m - i + 1)


def test_fisher_yates_uniform_permutations(oracle):
    """Labels of ProbMinHash2/4 at m = 4: the four labels of one element form a
    uniformly random permutation (Sec. 2.4, sampling without replacement)."""
    from itertools import permutations
    perms = {p: k for k, p in enumerate(permutations(range(4)))}
    counts = np.zeros(24)
    for K in range(1, 24001):
        _, ls = oracle.stream(2, 4, oracle.mix64(K), 1.0, 4)
        counts[perms[tuple(int(v) for v in ls)]] += 1
    assert stats.chisquare(counts).pvalue > 1e-3


def test_key_packing(oracle):
    """Key = value bits with the low 20 fraction bits replaced by the position:
    integer order is (truncated value, position) order."""
    assert oracle.key(1.0, 5) == (struct.unpack("<Q", struct.pack("<d", 1.0))[0] | 5)
    rng = np.random.default_rng(8)
    xs = np.sort(np.exp(rng.uniform(-50, 50, 2000)))
    keys = [oracle.key(float(x), 7) for x in xs]
    assert all(a <= b for a, b in zip(keys, keys[1:]))
    assert oracle.key(2.0, 1) < oracle.key(2.0, 2) < oracle.key(math.nextafter(2.0, 3) + 2.0 ** -30, 0)
    assert oracle.key(0.0, 3) == 3


def test_stream_monotone_lower_bounds(oracle):
    """Point i of ProbMinHash3 lies in [winv (i-1), ...) and of ProbMinHash4 in
    [winv gamma_{i-1}, ...) (Sec. 2.5, 2.6); ProbMinHash1/2 streams never
    decrease (Sec. 2.3, 2.4)."""
    for v in (1, 2, 3, 4):
        m = 64
        for K in (1, 99, 2**40 + 3):
            K = oracle.mix64(K)
            winv = 3.7
            xs, ls = oracle.stream(v, m, K, winv, 2000 if v in (1, 3) else m)
            assert (ls < m).all()
            if v in (1, 2):
                assert (np.diff(xs) >= 0).all()
            if v == 3:
                lb = winv * np.arange(xs.size)
                assert (xs >= lb).all()
            if v == 4:
                g = np.array([0.0] + [oracle.constants(4, m, i)[3] for i in range(1, m)])
                assert (xs >= winv * g).all()
            if v in (2, 4):
                assert sorted(ls.tolist()) == list(range(m))


def test_value_and_label_of_one_word_are_independent(oracle):
    """The value uniform (high half) and the label (low half) of a point come
    from one word; they must be independent: chi-square on the joint table of
    value decile x label for m = 10."""
    counts = np.zeros((10, 10))
    K = oracle.mix64(99)
    for i in range(1, 50001):
        u = (oracle.word(K, i, 0) >> 32) / 2.0 ** 32
        counts[int(u * 10), oracle.lemire(K, i, 10)] += 1
    chi2, pval, _, _ = stats.chi2_contingency(counts)
    assert pval > 1e-3
