"""Pins of the oracle's signature algorithms.

The sequential algorithms (stop limit, lower-bound tests, the lazily
initialised permutation) are checked against a brute force that shares none of the stop logic: it
generates every point of every stream and takes per-label minima (eq. (1) with
the hash values of eq. (9)).  The interleaved variants of Sec. 2.7 must give
identical signatures.  Special cases and invariances follow from the
definitions.
"""
import numpy as np
import pytest

from paper_1911_00675_amd import workloads as W

SEED = 0x5EED


def _rand_set(rng, n, law):
    ids = rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64)
    if law == "wide":
        w = np.exp(rng.uniform(np.log(1e-300), np.log(1e300), size=n))
    elif law == "ones":
        w = np.ones(n)
    else:
        w = rng.exponential(size=n) + 1e-12
    return ids, w


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_sequential_equals_brute_force(oracle, variant):
    rng = np.random.default_rng(100 + variant)
    ms = [1, 2, 3, 4, 5, 8, 16, 64] if variant <= 2 else [2, 3, 4, 5, 8, 16, 64]
    for m in ms:
        for trial in range(40):
            n = int(rng.integers(1, 9))
            ids, w = _rand_set(rng, n, ("exp", "wide", "ones")[trial % 3])
            seed = int(rng.integers(0, 2**63))
            seq = oracle.sign(variant, seed, m, ids, w)
            brute = oracle.sign(variant, seed, m, ids, w, mode=oracle.MODE_BRUTE)
            assert np.array_equal(seq, brute), (variant, m, n, trial)


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_sequential_equals_brute_force_under_forced_caps(oracle, variant):
    """The capped paths (Sec. 3: bounded loops) -- a short stream cap for
    ProbMinHash1/3, one proposal for the truncated-exponential sampler, few
    Lemire redraws with a floor that forces them -- give the same signature
    whether the stop rule prunes or every point is generated."""
    rng = np.random.default_rng(150 + variant)
    ms = [1, 2, 3, 16, 64] if variant <= 2 else [2, 3, 16, 64]
    hit = 0
    for caps in (oracle.Caps(imax=3, te_rounds=1, redraws=1, lemire_floor=1 << 31),
                 oracle.Caps(imax=1, te_rounds=2, redraws=0, lemire_floor=3 << 30),
                 oracle.Caps(imax=17, te_rounds=1, redraws=8, lemire_floor=(1 << 32) - 1)):
        for m in ms:
            for trial in range(25):
                n = int(rng.integers(1, 9))
                ids, w = _rand_set(rng, n, ("exp", "wide", "ones")[trial % 3])
                seed = int(rng.integers(0, 2**63))
                seq = oracle.sign(variant, seed, m, ids, w, caps=caps)
                brute = oracle.sign(variant, seed, m, ids, w, mode=oracle.MODE_BRUTE, caps=caps)
                assert np.array_equal(seq, brute), (variant, m, n, trial)
                hit += not np.array_equal(seq, oracle.sign(variant, seed, m, ids, w))
    assert hit > 20  # the caps change results: the capped paths ran


@pytest.mark.parametrize("variant", [1, 3])
def test_stream_cap_truncates(oracle, variant):
    """A stream cap of I points: the oracle's stream of a single element has
    exactly I points, and the signature of one element fills at most I
    components."""
    caps = oracle.Caps(imax=5)
    xs, ls = oracle.stream(variant, 64, 12345, 1.0, 100, caps=caps)
    assert np.count_nonzero(xs) <= 5 and xs[5:].max() == 0.0
    keys = oracle.sign(variant, SEED, 64, np.array([7], dtype=np.uint64), np.array([1.0]), caps=caps)
    assert 1 <= int(np.count_nonzero(keys != oracle.EMPTY)) <= 5


@pytest.mark.parametrize("variant", [1, 3])
def test_interleaved_equals_sequential(oracle, variant):
    """ProbMinHash1a == ProbMinHash1 and ProbMinHash3a == ProbMinHash3 (Sec. 2.7)."""
    rng = np.random.default_rng(200 + variant)
    for m in (2, 16, 256):
        for n in (1, 5, 50, 500, 3000):
            ids, w = _rand_set(rng, n, "exp")
            a = oracle.sign(variant, SEED, m, ids, w)
            b = oracle.sign(variant, SEED, m, ids, w, mode=oracle.MODE_INTERLEAVED)
            assert np.array_equal(a, b), (m, n)


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_brute_force_medium(oracle, variant):
    """Sequential == brute force at m = 256 with a few hundred elements."""
    rng = np.random.default_rng(300 + variant)
    for n in (1, 20, 300):
        ids, w = _rand_set(rng, n, "exp")
        assert np.array_equal(oracle.sign(variant, 9, 256, ids, w),
                              oracle.sign(variant, 9, 256, ids, w, mode=oracle.MODE_BRUTE))


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_single_element(oracle, variant):
    """n = 1: every component holds the only element (position 0)."""
    m = 128
    for K in range(5):
        keys = oracle.sign(variant, K, m, np.array([K * 7 + 1], dtype=np.uint64), np.array([0.3]))
        idx, val, ids = oracle.decode(keys, np.array([K * 7 + 1], dtype=np.uint64))
        assert (idx == 0).all() and (ids == K * 7 + 1).all() and np.isfinite(val).all()


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_empty_and_zero_weights(oracle, variant):
    m = 16
    keys = oracle.sign(variant, 1, m, np.zeros(0, dtype=np.uint64), np.zeros(0))
    assert (keys == oracle.EMPTY).all()
    idx, val, ids = oracle.decode(keys, np.zeros(0, dtype=np.uint64))
    assert (idx == oracle.IDX_EMPTY).all() and np.isinf(val).all() and (ids == 0).all()
    # a zero weight removes the element (Sec. 1.1: weight 0 means absent)
    ids = np.array([11, 22, 33], dtype=np.uint64)
    a = oracle.sign(variant, 1, m, ids, np.array([0.5, 0.0, 0.25]))
    b = oracle.sign(variant, 1, m, ids[[0, 2]], np.array([0.5, 0.25]))
    ia, _, da = oracle.decode(a, ids)
    ib, _, db = oracle.decode(b, ids[[0, 2]])
    assert np.array_equal(da, db)


def test_argument_errors(oracle):
    ids = np.array([1, 2], dtype=np.uint64)
    for bad in (-1.0, float("nan"), float("inf"), 1e-310):
        with pytest.raises(oracle.OracleError) as e:
            oracle.sign(1, 0, 8, ids, np.array([1.0, bad]))
        assert e.value.code == oracle.ERR_WEIGHT
    for v in (3, 4):
        with pytest.raises(oracle.OracleError) as e:
            oracle.sign(v, 0, 1, ids, np.array([1.0, 1.0]))
        assert e.value.code == oracle.ERR_VARIANT_M
    for m in (0, 16385):
        with pytest.raises(oracle.OracleError) as e:
            oracle.sign(1, 0, m, ids, np.array([1.0, 1.0]))
        assert e.value.code == oracle.ERR_M_RANGE
    for bad_variant in (0, 9):  # 5..8 are the binary specialisations
        with pytest.raises(oracle.OracleError):
            oracle.sign(bad_variant, 0, 8, ids, np.array([1.0, 1.0]))


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_order_independence(oracle, variant):
    """The signature is a function of the weighted set, not of the input order:
    permuting the elements permutes the positions and nothing else."""
    rng = np.random.default_rng(400 + variant)
    for n in (3, 40, 700):
        ids, w = _rand_set(rng, n, "exp")
        perm = rng.permutation(n)
        a = oracle.sign(variant, SEED, 256, ids, w)
        b = oracle.sign(variant, SEED, 256, ids[perm], w[perm])
        ia, va, da = oracle.decode(a, ids)
        ib, vb, db = oracle.decode(b, ids[perm])
        assert np.array_equal(da, db) and np.array_equal(va, vb)
        assert np.array_equal(ia, perm[ib])


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_power_of_two_scale_invariance(oracle, variant):
    """J_P and the signature are scale invariant (Sec. 1.1); scaling every
    weight by 2^k scales every point by 2^-k exactly, so positions agree
    bit for bit and values scale exactly."""
    rng = np.random.default_rng(500 + variant)
    ids, w = _rand_set(rng, 300, "exp")
    a = oracle.sign(variant, SEED, 256, ids, w)
    b = oracle.sign(variant, SEED, 256, ids, w * 2.0 ** 40)
    ia, va, _ = oracle.decode(a, ids)
    ib, vb, _ = oracle.decode(b, ids)
    assert np.array_equal(ia, ib)
    assert np.array_equal(va * 2.0 ** -40, vb)


def test_same_set_and_disjoint_sets(oracle):
    rng = np.random.default_rng(600)
    for v in (1, 2, 3, 4):
        ids, w = _rand_set(rng, 200, "exp")
        a = oracle.decode(oracle.sign(v, 3, 256, ids, w), ids)
        b = oracle.decode(oracle.sign(v, 3, 256, ids[::-1].copy(), w[::-1].copy()), ids[::-1].copy())
        assert oracle.estimate(a[2], a[0], b[2], b[0]) == 1.0
        ids2, w2 = _rand_set(rng, 200, "exp")
        c = oracle.decode(oracle.sign(v, 3, 256, ids2, w2), ids2)
        assert oracle.estimate(a[2], a[0], c[2], c[0]) == 0.0


def test_without_replacement_point_bound(oracle):
    """ProbMinHash2/4 generate at most m points per element (Sec. 2.4, 2.6)."""
    rng = np.random.default_rng(700)
    for v in (2, 4):
        for n in (1, 3, 30):
            ids, w = _rand_set(rng, n, "exp")
            _, st = oracle.sign(v, 1, 64, ids, w, return_stats=True)
            assert st[0] <= 64 * n
        _, st = oracle.sign(v, 1, 64, ids[:1], w[:1], return_stats=True)
        assert st[0] == 64  # a single element needs all m labels


def test_pmh1_expected_points(oracle):
    """Expected points of ProbMinHash1 with weights in random order:
    m H_m H_n (Sec. 2.3)."""
    m, n, S = 256, 100, 400
    b = W.random_sets(21, S, n, n, "exp")
    _, st = oracle.sign_batch(1, SEED, m, b.ids, b.weights, b.offsets, nthreads=4, return_stats=True)
    expect = S * m * oracle.harmonic(m) * oracle.harmonic(n)
    assert abs(st[0] / expect - 1.0) < 0.03, st[0] / expect


def test_batch_equals_single(oracle):
    b = W.random_sets(22, 50, 0, 300, "pareto")
    keys = oracle.sign_batch(3, SEED, 64, b.ids, b.weights, b.offsets, nthreads=3)
    for s in range(b.num_sets):
        ids, w = b.set(s)
        assert np.array_equal(keys[s], oracle.sign(3, SEED, 64, ids, w))


def test_frozen_oracle_keys(oracle):
    """The oracle reproduces the stored fixture written by
    tests/golden/make_oracle_golden.py (which calls only the oracle)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_keys.json")
    data = json.load(open(path))
    for case in data["cases"]:
        ids = np.array([int(x) for x in case["ids"]], dtype=np.uint64)
        w = np.array([float.fromhex(x) for x in case["weights"]])
        keys = oracle.sign(case["variant"], data["seed"], case["m"], ids, w)
        assert [format(int(x), "016x") for x in keys] == case["keys"]
