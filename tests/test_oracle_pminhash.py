"""Pins of the oracle's P-MinHash (Sec. 1.1, the paper's O(nm) baseline).

P-MinHash gives each element of positive weight w one exponential value of
rate w per component and keeps, per component, the smallest.  What that fixes
independently of the implementation: the winner of a component is element d
with probability w_d / sum(w) (an exponential race), two sets agree in a
component with probability J_P (the defining collision law of Sec. 1.1), a
single element's values follow Exp(w), the signature is invariant under
scaling all weights by a power of two, values of a union are componentwise
minima of the parts' values, zero weights never win, and an empty set is all
empty.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O

SEED = 0x5EED


def _vals(keys):
    return (keys & ~np.uint64(O.POS_MASK)).view(np.float64)


def test_argmin_law():
    """Component winners: Binomial(m, w_d / W) for each element (5 sigma)."""
    m = 16384
    ids = np.array([11, 22, 33, 44, 55], dtype=np.uint64)
    w = np.array([1.0, 2.0, 3.0, 4.0, 0.5])
    idx, _, _ = O.decode(O.pminhash(SEED, m, ids, w), ids)
    counts = np.bincount(idx.astype(np.int64), minlength=ids.size)
    p = w / w.sum()
    z = (counts - m * p) / np.sqrt(m * p * (1 - p))
    assert np.all(np.abs(z) < 5), z


def test_collision_law_equals_jp():
    """Pr(z_k(A) = z_k(B)) = J_P: equal components ~ Binomial(m, J_P)."""
    m = 16384
    rng = np.random.default_rng(3)
    shared = rng.integers(0, 2**63, size=30, dtype=np.uint64)
    ida = np.concatenate([shared, rng.integers(0, 2**63, size=10, dtype=np.uint64)])
    idb = np.concatenate([shared, rng.integers(0, 2**63, size=25, dtype=np.uint64)])
    wa = rng.exponential(size=ida.size)
    wb = rng.exponential(size=idb.size)
    _, _, za = O.decode(O.pminhash(SEED, m, ida, wa), ida)
    _, _, zb = O.decode(O.pminhash(SEED, m, idb, wb), idb)
    J = O.jp_definition(dict(zip(ida.tolist(), wa)), dict(zip(idb.tolist(), wb)))
    c = int(np.sum(za == zb))
    assert stats.binom.ppf(1e-6, m, J) <= c <= stats.binom.ppf(1 - 1e-6, m, J), (c, m * J)


def test_single_element_values_are_exponential():
    """One element of weight w: the m values are Exp(w) (KS test)."""
    m = 8192
    w = 2.5
    keys = O.pminhash(SEED, m, np.array([7], dtype=np.uint64), np.array([w]))
    x = _vals(keys)
    assert stats.kstest(x, "expon", args=(0, 1 / w)).pvalue > 1e-4
    assert abs(x.mean() * w - 1) < 5 / np.sqrt(m)


def test_power_of_two_scaling_invariance():
    """Scaling every weight by 2^k scales every value exactly: same winners."""
    rng = np.random.default_rng(5)
    ids = rng.integers(0, 2**64 - 1, size=50, dtype=np.uint64)
    w = rng.exponential(size=50)
    a = O.pminhash(SEED, 512, ids, w)
    b = O.pminhash(SEED, 512, ids, w * 2.0**20)
    assert np.array_equal(a & np.uint64(O.POS_MASK), b & np.uint64(O.POS_MASK))
    assert np.array_equal(_vals(a) * 2.0**-20, _vals(b))


def test_union_values_are_componentwise_minima():
    """Values depend on (seed, id, w, k) only: the values of A u B are the
    componentwise minima of those of A and of B."""
    rng = np.random.default_rng(6)
    ids = rng.integers(0, 2**64 - 1, size=40, dtype=np.uint64)
    w = rng.exponential(size=40)
    m = 300
    a = _vals(O.pminhash(SEED, m, ids[:25], w[:25]))
    b = _vals(O.pminhash(SEED, m, ids[25:], w[25:]))
    ab = _vals(O.pminhash(SEED, m, ids, w))
    assert np.array_equal(ab, np.minimum(a, b))


def test_zero_weights_never_win_and_empty_sets():
    ids = np.array([1, 2, 3, 4], dtype=np.uint64)
    w = np.array([0.0, 1.5, 0.0, 0.25])
    _, _, z = O.decode(O.pminhash(SEED, 256, ids, w), ids)
    _, _, z2 = O.decode(O.pminhash(SEED, 256, ids[[1, 3]], w[[1, 3]]), ids[[1, 3]])
    assert np.array_equal(z, z2)
    assert np.all(O.pminhash(SEED, 64, ids, np.zeros(4)) == np.uint64(O.EMPTY))
    assert np.all(O.pminhash(SEED, 64, ids[:0], w[:0]) == np.uint64(O.EMPTY))


def test_errors():
    ids = np.array([1, 2], dtype=np.uint64)
    for bad in (-1.0, np.nan, np.inf, 1e-310):
        with pytest.raises(O.OracleError) as e:
            O.pminhash(SEED, 8, ids, np.array([1.0, bad]))
        assert e.value.code == O.ERR_WEIGHT
    with pytest.raises(O.OracleError) as e:
        O.pminhash(SEED, 0, ids, np.ones(2))
    assert e.value.code == O.ERR_M_RANGE


def test_batch_equals_single():
    rng = np.random.default_rng(7)
    sizes = rng.integers(0, 40, size=30)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    ids = rng.integers(0, 2**64 - 1, size=int(off[-1]), dtype=np.uint64)
    w = rng.exponential(size=ids.size)
    kb = O.pminhash_batch(SEED, 128, ids, w, off, nthreads=4)
    for s in range(30):
        a, b = int(off[s]), int(off[s + 1])
        assert np.array_equal(kb[s], O.pminhash(SEED, 128, ids[a:b], w[a:b]))
