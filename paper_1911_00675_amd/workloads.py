"""Seeded synthetic weighted-set generators (data only, no signature arithmetic).

The paper evaluates on synthetic sets of random 64-bit ids with weights drawn
from stated laws (Sec. 3, Sec. 3.1, Sec. 3.2); these generators produce the
five workloads this library is measured and checked on.  Everything is a pure
function of the data seed, returned as numpy arrays in CSR form:

    ids      uint64[N]   element ids
    weights  float64[N]  positive weights (normalised per set to sum 1)
    offsets  uint64[S+1] set s owns elements offsets[s] .. offsets[s+1]-1

Both the GPU tests/benchmark and the oracle-side tests draw their inputs from
here; the module holds no part of the hashing method.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

U64 = np.uint64


@dataclass
class Batch:
    ids: np.ndarray
    weights: np.ndarray
    offsets: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def num_sets(self) -> int:
        return int(self.offsets.size - 1)

    @property
    def num_elements(self) -> int:
        return int(self.offsets[-1])

    def set(self, s: int):
        a, b = int(self.offsets[s]), int(self.offsets[s + 1])
        return self.ids[a:b], self.weights[a:b]

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def subset(self, sets) -> "Batch":
        """Batch made of the given sets, in the given order."""
        sets = np.asarray(sets, dtype=np.int64)
        sizes = self.sizes()[sets]
        off = np.zeros(sets.size + 1, dtype=np.uint64)
        np.cumsum(sizes, out=off[1:])
        idx = np.concatenate([np.arange(self.offsets[s], self.offsets[s + 1], dtype=np.int64)
                              for s in sets]) if sets.size else np.zeros(0, dtype=np.int64)
        return Batch(self.ids[idx], self.weights[idx], off, dict(self.meta, parent_sets=sets))


def _rand_u64(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)


def _normalise(w: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    sizes = np.diff(offsets).astype(np.int64)
    nz = sizes > 0
    sums = np.zeros(sizes.size)
    sums[nz] = np.add.reduceat(w, offsets[:-1][nz].astype(np.int64))
    return w / np.repeat(np.where(sums > 0, sums, 1.0), sizes)


def _offsets(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    np.cumsum(sizes.astype(np.uint64), out=off[1:])
    return off


def _log_uniform_int(rng, lo: int, hi: int, n: int) -> np.ndarray:
    """floor(exp(U * ln(hi + 1))) restricted to [lo, hi] (log-uniform law)."""
    a, b = np.log(lo), np.log(hi + 1.0)
    v = np.floor(np.exp(rng.uniform(a, b, size=n))).astype(np.int64)
    return np.clip(v, lo, hi)


def _dedupe_pool_draws(rng, pool_idx: np.ndarray, set_of: np.ndarray, pool_size: int) -> np.ndarray:
    """Redraw pool indices that repeat within a set, so every set holds
    distinct ids.  (Fresh uniform 64-bit ids are not checked: two equal ids
    among the n <= 10^6 fresh ids of one set occur with probability below
    n^2 / 2^65 < 3e-8.)"""
    for _ in range(64):
        key = set_of.astype(np.int64) * pool_size + pool_idx.astype(np.int64)
        _, first = np.unique(key, return_index=True)
        dup = np.ones(key.size, dtype=bool)
        dup[first] = False
        if not dup.any():
            return pool_idx
        pool_idx[dup] = rng.integers(0, pool_size, size=int(dup.sum()))
    raise RuntimeError("could not make pool draws distinct")


# --------------------------------------------------------------------------- #
# The five workloads.

def plain_pairs(seed: int = 1, num_sets: int = 1000, n: int = 100, num_pairs: int = 200) -> Batch:
    """1,000 sets of exactly 100 elements; uniform 64-bit ids; Exp(1) weights
    normalised per set.  For j < 200, set 2j+1 shares 50 random ids of set 2j
    (with fresh weights), so the 200 pairs (2j, 2j+1) have nonzero J_P."""
    rng = np.random.default_rng(seed)
    ids = _rand_u64(rng, num_sets * n)
    half = n // 2
    for j in range(num_pairs):
        a, b = 2 * j * n, (2 * j + 1) * n
        pick = rng.choice(n, size=half, replace=False)
        ids[b:b + half] = ids[a + pick]
    w = rng.exponential(1.0, size=num_sets * n)
    w = np.where(w > 0, w, 1.0)
    off = _offsets(np.full(num_sets, n))
    return Batch(ids, _normalise(w, off), off,
                 dict(name="plain_pairs", seed=seed, pairs=[(2 * j, 2 * j + 1) for j in range(num_pairs)]))


def mixed_sizes(seed: int = 2, num_sets: int = 100_000, n_lo: int = 1, n_hi: int = 10_000,
                pool_size: int = 1_000_000, pool_frac: float = 0.2, pareto_shape: float = 1.5) -> Batch:
    """Sets with log-uniform sizes in [1, 10^4]; each id comes from a shared
    pool of 10^6 ids with probability 0.2 (so sets overlap), else a fresh
    uniform 64-bit id; Pareto(x_m = 1, shape 1.5) weights normalised per set."""
    rng = np.random.default_rng(seed)
    sizes = _log_uniform_int(rng, n_lo, n_hi, num_sets)
    off = _offsets(sizes)
    N = int(off[-1])
    pool = _rand_u64(rng, pool_size)
    ids = _rand_u64(rng, N)
    from_pool = rng.random(N) < pool_frac
    set_of = np.repeat(np.arange(num_sets, dtype=np.int64), sizes)
    pidx = _dedupe_pool_draws(rng, rng.integers(0, pool_size, size=int(from_pool.sum())), set_of[from_pool],
                              pool_size)
    ids[from_pool] = pool[pidx]
    w = (1.0 - rng.random(N)) ** (-1.0 / pareto_shape)
    return Batch(ids, _normalise(w, off), off, dict(name="mixed_sizes", seed=seed))


def skewed(seed: int = 3, num_sets: int = 10_000, large_frac: float = 0.1,
           small=(10, 100), large=(100_000, 1_000_000)) -> Batch:
    """Heavy size skew: 90% of sets log-uniform in [10, 100] elements, 10% in
    [10^5, 10^6], at random positions; uniform ids; weights uniform on (0, 1]
    normalised per set."""
    rng = np.random.default_rng(seed)
    is_large = rng.random(num_sets) < large_frac
    sizes = np.where(is_large, _log_uniform_int(rng, large[0], large[1], num_sets),
                     _log_uniform_int(rng, small[0], small[1], num_sets))
    off = _offsets(sizes)
    N = int(off[-1])
    ids = _rand_u64(rng, N)
    w = 1.0 - rng.random(N)  # (0, 1]
    return Batch(ids, _normalise(w, off), off, dict(name="skewed", seed=seed))


def serving_requests(seed: int = 4, num_requests: int = 220_000, rate: float = 50_000.0,
                     n_lo: int = 10, n_hi: int = 100_000) -> Batch:
    """Single-set requests with Poisson arrivals (exponential inter-arrival
    times at the given rate, seconds in meta['arrival']), log-uniform sizes in
    [10, 10^5], uniform ids, Exp(1) weights normalised per set."""
    rng = np.random.default_rng(seed)
    sizes = _log_uniform_int(rng, n_lo, n_hi, num_requests)
    off = _offsets(sizes)
    N = int(off[-1])
    ids = _rand_u64(rng, N)
    w = rng.exponential(1.0, size=N)
    w = np.where(w > 0, w, 1.0)
    arrival = np.cumsum(rng.exponential(1.0 / rate, size=num_requests))
    return Batch(ids, _normalise(w, off), off,
                 dict(name="serving_requests", seed=seed, rate=rate, arrival=arrival))


def _zipf_ranks(rng, a: float, n_max: int, size: int) -> np.ndarray:
    """Zipf(a) ranks on [1, n_max] by rejection-inversion (W. Hormann and
    G. Derflinger, "Rejection-inversion to generate variates from monotone
    discrete distributions", ACM TOMACS 6(3), 1996), vectorised."""
    q = float(a)

    def H(x):  # integral of x^-q
        return np.expm1((1.0 - q) * np.log(x)) / (1.0 - q)

    def Hinv(y):
        return np.exp(np.log1p(y * (1.0 - q)) / (1.0 - q))

    h = lambda x: np.exp(-q * np.log(x))
    hx1 = float(H(1.5) - 1.0)
    hn = float(H(n_max + 0.5))
    sq = float(2.0 - Hinv(H(2.5) - h(2.0)))
    out = np.empty(size, dtype=np.uint64)
    todo = np.arange(size)
    while todo.size:
        u = hn + rng.random(todo.size) * (hx1 - hn)
        x = Hinv(u)
        k = np.clip(np.floor(x + 0.5), 1, n_max)
        ok = (k - x <= sq) | (u >= H(k + 0.5) - h(k))
        out[todo[ok]] = k[ok].astype(np.uint64)
        todo = todo[~ok]
    return out


LARGE_BLOCK = 1000  # sets per independently seeded block of large_uniform


def large_block(seed: int = 5, block: int = 0, n: int = 1000, universe: int = 100_000_000,
                zipf_a: float = 1.1, num_sets: int = LARGE_BLOCK) -> Batch:
    """Sets [block*LARGE_BLOCK, +num_sets) of large_uniform, from the block's
    own generator (so blocks can be produced independently, e.g. by a process
    pool).  Each set holds the first n distinct ranks of an i.i.d. Zipf stream
    (2.25 n draws, more for the rare set that needs them)."""
    rng = np.random.default_rng([seed, block])
    out = np.empty((num_sets, n), dtype=np.uint64)
    draw = 9 * n // 4
    cand = _zipf_ranks(rng, zipf_a, universe, num_sets * draw)
    set_of = np.repeat(np.arange(num_sets, dtype=np.int64), draw)
    _, first = np.unique(set_of * (universe + 1) + cand.astype(np.int64), return_index=True)
    first.sort()  # distinct (set, rank) pairs in draw order, sets contiguous
    cnt = np.bincount(set_of[first], minlength=num_sets)
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    full = np.flatnonzero(cnt >= n)
    out[full] = cand[first[start[full][:, None] + np.arange(n)[None, :]]]
    for s in np.flatnonzero(cnt < n):  # keep drawing for this set until it holds n distinct ids
        got = cand[first[start[s]:start[s] + cnt[s]]]
        while got.size < n:
            got = np.concatenate([got, _zipf_ranks(rng, zipf_a, universe, draw)])
            _, f = np.unique(got, return_index=True)
            got = got[np.sort(f)]
        out[s] = got[:n]
    off = _offsets(np.full(num_sets, n))
    w = np.exp(rng.standard_normal(num_sets * n))
    return Batch(out.reshape(-1), _normalise(w, off), off, dict(name="large_uniform", seed=seed, block=block))


def large_uniform(seed: int = 5, num_sets: int = 1_000_000, n: int = 1000, universe: int = 100_000_000,
                  zipf_a: float = 1.1, first_set: int = 0) -> Batch:
    """Sets of exactly 1,000 distinct ids whose popularity follows Zipf(1.1)
    over a universe of 10^8 ids (id = rank), drawn without replacement within
    a set; log-normal(0, 1) weights normalised per set.  Sets [first_set,
    first_set + num_sets) of the full workload (first_set a multiple of
    LARGE_BLOCK), concatenated from independently seeded blocks."""
    if first_set % LARGE_BLOCK:
        raise ValueError("first_set must be a multiple of LARGE_BLOCK")
    parts = [large_block(seed, (first_set + s0) // LARGE_BLOCK, n, universe, zipf_a,
                         min(LARGE_BLOCK, num_sets - s0)) for s0 in range(0, num_sets, LARGE_BLOCK)]
    off = _offsets(np.full(num_sets, n))
    return Batch(np.concatenate([p.ids for p in parts]), np.concatenate([p.weights for p in parts]), off,
                 dict(name="large_uniform", seed=seed, first_set=first_set))


def weight_pairs(W, num_pairs: int, seed: int = 11):
    """Pairs of weighted sets realising a multiset W of weight pairs (Sec. 3.1):
    every pair (wA, wB) in W becomes one fresh random element that gets weight
    wA in set A and wB in set B (absent where the weight is 0).  Returns a
    Batch with sets (2j, 2j+1) forming pair j."""
    rng = np.random.default_rng(seed)
    W = [(float(a), float(b)) for a, b in W]
    ids_list, w_list, sizes = [], [], []
    for _ in range(num_pairs):
        e = _rand_u64(rng, len(W))
        for side in (0, 1):
            sel = [k for k, pr in enumerate(W) if pr[side] > 0]
            ids_list.append(e[sel])
            w_list.append(np.array([W[k][side] for k in sel], dtype=np.float64))
            sizes.append(len(sel))
    off = _offsets(np.array(sizes))
    return Batch(np.concatenate(ids_list), np.concatenate(w_list), off,
                 dict(name="weight_pairs", W=W, seed=seed))


def random_sets(seed: int, num_sets: int, n_lo: int, n_hi: int, weight_law: str = "exp") -> Batch:
    """Small generic batches for tests: sizes uniform in [n_lo, n_hi]."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=num_sets)
    off = _offsets(sizes)
    N = int(off[-1])
    ids = _rand_u64(rng, N)
    if weight_law == "exp":
        w = rng.exponential(1.0, size=N)
        w = np.where(w > 0, w, 1.0)
    elif weight_law == "pareto":
        w = (1.0 - rng.random(N)) ** (-1.0 / 1.5)
    elif weight_law == "ones":
        w = np.ones(N)
    elif weight_law == "wide":  # log-uniform over many decades
        w = np.exp(rng.uniform(np.log(1e-300), np.log(1e300), size=N))
    else:
        raise ValueError(weight_law)
    return Batch(ids, w, off, dict(name="random_sets", seed=seed, law=weight_law))


WORKLOADS = {
    "plain_pairs": plain_pairs,
    "mixed_sizes": mixed_sizes,
    "skewed": skewed,
    "serving_requests": serving_requests,
    "large_uniform": large_uniform,
}
