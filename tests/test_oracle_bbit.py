"""Pins of the oracle's b-bit reduction (Sec. 1.3, algorithm "Reduction to a
b-bit signature") and of the bias-corrected estimator.

What the reduction must do, independently of how it hashes: a component's
field depends only on (element id, component index), so equal ids in a
component always agree; different ids agree with probability 2^-b, and
independently across components (the paper's reason for hashing the index
too); the packed layout holds every field where the stated layout puts it.
With Pr[agree] = J + (1 - J) 2^-b, (equal/m - 2^-b)/(1 - 2^-b) estimates J
without bias, checked on P-MinHash signatures of pairs with known J_P.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O

SEED = 0x5EED


def _fields(packed, m, b):
    words = np.asarray(packed, dtype=np.uint64)
    out = np.zeros(m, dtype=np.uint64)
    for k in range(m):
        bit = k * b
        out[k] = (int(words[bit // 64]) >> (bit % 64)) & ((1 << b) - 1)
    return out


@pytest.mark.parametrize("b", [1, 2, 4, 8, 16])
def test_layout_and_equal_ids_agree(b):
    m = 333
    rng = np.random.default_rng(b)
    ids = rng.integers(0, 2**64 - 1, size=(2, m), dtype=np.uint64)
    ids[1, ::3] = ids[0, ::3]  # every third component shares its element
    p = O.bbit_pack(ids, m, b)
    assert p.shape == (2, O.bbit_words(m, b))
    for s in range(2):
        want = np.array([O.lib().or_bbit_hash(int(ids[s, k]), k + 1) & ((1 << b) - 1) for k in range(m)],
                        dtype=np.uint64)
        assert np.array_equal(_fields(p[s], m, b), want)
    f0, f1 = _fields(p[0], m, b), _fields(p[1], m, b)
    assert np.all(f0[::3] == f1[::3])
    assert O.bbit_equal(p[0], p[1], m, b) == int(np.sum(f0 == f1))
    # padding bits of the last word stay zero
    used = m * b - 64 * (O.bbit_words(m, b) - 1)
    if used < 64:
        assert int(p[0, -1]) >> used == 0


@pytest.mark.parametrize("b", [1, 2, 4, 8])
def test_different_ids_agree_with_probability_2_pow_minus_b(b):
    """Two fixed different ids over m = 2^16 components: Binomial(m, 2^-b)."""
    m = 1 << 16
    ids = np.zeros((2, m), dtype=np.uint64)
    ids[0, :] = 123456789
    ids[1, :] = 987654321
    p = O.bbit_pack(ids, m, b)
    c = O.bbit_equal(p[0], p[1], m, b)
    r = 2.0 ** -b
    assert stats.binom.ppf(1e-6, m, r) <= c <= stats.binom.ppf(1 - 1e-6, m, r), (c, m * r)


def test_agreements_across_components_are_independent():
    """Many id pairs, b = 1: per-component agreement counts over pairs match
    Binomial(pairs, 1/2) per component and the per-pair counts Binomial(m, 1/2)
    (a shared hash across components would correlate them)."""
    m, pairs = 512, 400
    rng = np.random.default_rng(8)
    a = rng.integers(1, 2**64 - 1, size=(pairs, m), dtype=np.uint64)
    c = rng.integers(1, 2**64 - 1, size=(pairs, m), dtype=np.uint64)
    fa = O.bbit_pack(a, m, 1)
    fc = O.bbit_pack(c, m, 1)
    eq = np.array([[int(_fields(fa[i], m, 1)[k] == _fields(fc[i], m, 1)[k]) for k in range(m)]
                   for i in range(40)])
    per_pair = np.array([O.bbit_equal(fa[i], fc[i], m, 1) for i in range(pairs)])
    assert abs(per_pair.mean() - m / 2) < 5 * np.sqrt(m / 4 / pairs)
    assert abs(per_pair.var() / (m / 4) - 1) < 0.25  # a shared hash across components inflates this
    assert abs(eq.mean() - 0.5) < 0.02


@pytest.mark.parametrize("b", [1, 2, 4])
def test_corrected_estimator_is_unbiased(b):
    """P-MinHash signatures of overlapping sets, b-bit reduced: the corrected
    estimate lies within 5 sigma of J_P over 20 pairs pooled."""
    m = 4096
    rng = np.random.default_rng(30 + b)
    est, J = [], []
    for t in range(20):
        shared = rng.integers(1, 2**63, size=40, dtype=np.uint64)
        ida = np.concatenate([shared, rng.integers(1, 2**63, size=rng.integers(0, 40), dtype=np.uint64)])
        idb = np.concatenate([shared, rng.integers(1, 2**63, size=rng.integers(0, 40), dtype=np.uint64)])
        wa, wb = rng.exponential(size=ida.size), rng.exponential(size=idb.size)
        _, _, za = O.decode(O.pminhash(SEED, m, ida, wa), ida)
        _, _, zb = O.decode(O.pminhash(SEED, m, idb, wb), idb)
        p = O.bbit_pack(np.stack([za, zb]), m, b)
        est.append(O.bbit_estimate(O.bbit_equal(p[0], p[1], m, b), m, b))
        J.append(O.jp_sorted(ida, wa, idb, wb))
    est, J = np.array(est), np.array(J)
    r = 2.0 ** -b
    pr = J + (1 - J) * r
    sd = np.sqrt(np.sum(pr * (1 - pr) / m)) / (1 - r) / len(J)
    assert abs(est.mean() - J.mean()) < 5 * sd, (est.mean(), J.mean(), sd)


def test_bad_b_rejected():
    with pytest.raises(O.OracleError):
        O.bbit_pack(np.zeros((1, 8), dtype=np.uint64), 8, 3)
