"""Pins of the oracle's interleaved ProbMinHash1a / ProbMinHash3a (Sec. 2.7)
against the paper's space analysis: the buffer holds its most elements right
after the first pass, and

* ProbMinHash1a: an element enters if its first point is below the stop
  limit, roughly the (m H_m)-th smallest first point so far, so the expected
  buffer size is sum_{j=1..n} min(1, m H_m / j);
* ProbMinHash3a with unit weights (Sec. 2.9): min(n, m H_m), independent of n
  once n exceeds m H_m;
* ProbMinHash3a with weights of finite mean: a plateau independent of n.

Also: with fewer elements than components no first pass can fill every
component, so every element enters the buffer.
"""
import numpy as np
import pytest

import oracle as O


def _H(m):
    return sum(1.0 / k for k in range(1, m + 1))


def _buffer(variant, m, ids, w):
    _, st = O.sign(variant, 7, m, ids, w, mode=O.MODE_INTERLEAVED, return_stats=True)
    return int(st[2])


def _mean_buffer(variant, m, n, reps, weights, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(reps):
        ids = rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64)
        if weights == "unit":
            w = np.ones(n)
        elif weights == "exp":
            w = rng.exponential(size=n)
        else:
            w = (1.0 - rng.random(n)) ** (-1.0 / 1.5)  # Pareto(1, 1.5): finite mean
        out.append(_buffer(variant, m, ids, w))
    return float(np.mean(out))


@pytest.mark.parametrize("m,n,reps", [(64, 1000, 200), (64, 10000, 40), (256, 10000, 40)])
def test_pmh1a_buffer_matches_sum(m, n, reps):
    want = float(np.minimum(1.0, m * _H(m) / np.arange(1, n + 1)).sum())
    got = _mean_buffer(1, m, n, reps, "exp", seed=m + n)
    assert abs(got / want - 1.0) < 0.05, (got, want)


@pytest.mark.parametrize("m,n,reps", [(64, 1000, 200), (64, 10000, 40), (256, 10000, 40)])
def test_pmh3a_unit_weights_buffer_is_min_n_mhm(m, n, reps):
    want = min(n, m * _H(m))
    got = _mean_buffer(7, m, n, reps, "unit", seed=2 * m + n)  # variant 7: binary ProbMinHash3
    assert abs(got / want - 1.0) < 0.05, (got, want)


@pytest.mark.parametrize("weights", ["exp", "pareto"])
def test_pmh3a_weighted_buffer_plateaus(weights):
    """n = 10^4 -> 10^5 at m = 64: ProbMinHash3a's buffer stays within 10%,
    ProbMinHash1a's grows by the log n factor of its sum."""
    b3 = [_mean_buffer(3, 64, n, 20, weights, seed=n) for n in (10_000, 100_000)]
    b1 = [_mean_buffer(1, 64, n, 20, weights, seed=n + 1) for n in (10_000, 100_000)]
    assert abs(b3[1] / b3[0] - 1.0) < 0.10, b3
    assert b1[1] / b1[0] > 1.35, b1


@pytest.mark.parametrize("variant", [1, 3, 7])
def test_every_element_buffered_below_m(variant):
    rng = np.random.default_rng(variant)
    for n in (1, 5, 63):
        ids = rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64)
        w = np.ones(n) if variant == 7 else rng.exponential(size=n)
        assert _buffer(variant, 64, ids, w) == n


def test_sequential_mode_reports_no_buffer():
    ids = np.arange(1, 100, dtype=np.uint64)
    _, st = O.sign(1, 7, 16, ids, np.ones(ids.size), return_stats=True)
    assert int(st[2]) == 0
