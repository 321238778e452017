"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Integer/byte work (keys, positions, ids) must be bit-exact; the floating-point
stream primitives must be bit-exact too, because every signature index is an
argmin over them (the tolerance is zero by construction of the reading).
"""
import numpy as np
import pytest

import oracle as O
from paper_1911_00675_amd import workloads as W

pytestmark = pytest.mark.gpu
SEED = 0x5EED


@pytest.fixture(scope="module")
def pmh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1911_00675_amd import pmh as P
    P.lib()
    O.build()
    return P


def _keys(ctx, b, mode="batched"):
    sig = ctx.hash_sets(_dev(b.ids), _dev(b.weights), _dev(b.offsets), mode=mode)
    st = ctx.status()
    return sig, st


def _dev(a):
    from paper_1911_00675_amd import pmh as P
    return P.to_device(a)


def _host(sig):
    return (sig.keys.cpu().numpy().view(np.uint64), sig.idx.cpu().numpy().view(np.uint32),
            sig.val.cpu().numpy(), sig.id.cpu().numpy().view(np.uint64))


# ----------------------------------------------------------------- primitives
def test_primitives_bitwise(pmh):
    print("primitives: log/log1p/expm1/exp1/mix64/trunc-exp/lemire/spacing", flush=True)
    m = 256
    ctx = pmh.Context(SEED, m, 3)
    rng = np.random.default_rng(1)
    ks = rng.integers(1, 2**53, size=20000)
    u = ks.astype(np.float64) * 2.0 ** -53
    u[:3] = [1.0, 2.0 ** -53, 0.5]
    got = ctx.debug_eval(0, u)
    want = np.array([O.spec_log(x) for x in u])
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    x = np.concatenate([1.0 / np.arange(1, 5000), np.exp(rng.uniform(-30, 12, 5000))])
    assert np.array_equal(ctx.debug_eval(1, x).view(np.uint64),
                          np.array([O.spec_log1p(v) for v in x]).view(np.uint64))
    t = np.linspace(0, np.log(2), 3001)
    assert np.array_equal(ctx.debug_eval(2, t).view(np.uint64),
                          np.array([O.spec_expm1(v) for v in t]).view(np.uint64))
    words = rng.integers(0, 2**63, size=20000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    words[:2] = [np.uint64(0), np.uint64(2**64 - 1)]
    assert np.array_equal(ctx.debug_eval(3, words).view(np.uint64),
                          np.array([O.exp1_of_word(int(wd)) for wd in words]).view(np.uint64))
    assert np.array_equal(ctx.debug_eval(4, words), np.array([O.mix64(int(wd)) for wd in words], dtype=np.uint64))
    lam, a, c1 = O.constants(3, m)[:3]
    Ks = rng.integers(0, 2**63, size=20000, dtype=np.uint64)
    te = ctx.debug_eval(5, Ks)
    want = np.array([O.trunc_exp(int(K), k + 1, lam, a, c1) for k, K in enumerate(Ks)])
    assert np.array_equal(te.view(np.uint64), want.view(np.uint64))
    assert (want >= 1.0 / c1).sum() > 10  # the second branch of the sampler is exercised
    lab = ctx.debug_eval(6, Ks)
    assert np.array_equal(lab, np.array([O.lemire(int(K), k + 1, m) for k, K in enumerate(Ks)], dtype=np.uint64))
    xs = np.concatenate([u, np.exp(rng.uniform(-700, 700, 5000))])
    assert np.array_equal(ctx.debug_eval(8, xs).view(np.uint64),
                          np.array([O.stream_log(v) for v in xs]).view(np.uint64))
    assert np.array_equal(ctx.table(9, 512).view(np.uint64), O.stream_log_table().view(np.uint64))
    # wave prefix sums of fixed-point spacings (chains: 64 lanes, mini-chains: 8, 4, 2)
    sp_in = rng.integers(0, 2**51, size=64 * 300, dtype=np.uint64)
    sp_in[:64] = np.uint64(2**51 - 1)  # largest spacings
    sp_in[64:128] = 0
    for what, g in ((9, 64), (10, 8), (11, 4), (12, 2)):
        want = np.cumsum(sp_in.reshape(-1, g), axis=1, dtype=np.uint64).reshape(-1)
        assert np.array_equal(ctx.debug_eval(what, sp_in), want), what
        tail = sp_in[:100]  # a partial last group: missing entries count as 0
        assert np.array_equal(ctx.debug_eval(what, tail),
                              np.concatenate([np.cumsum(tail[i:i + g], dtype=np.uint64) for i in range(0, 100, g)]))
    sp = ctx.debug_eval(7, Ks)
    want = np.array([int(O.exp1_of_word(O.word(int(K), k + 1, 0)) * 2.0 ** 32) for k, K in enumerate(Ks)],
                    dtype=np.uint64)
    assert np.array_equal(sp, want)
    ctx.close()


@pytest.mark.parametrize("m", [2, 3, 64, 1000, 4096])
def test_constant_tables_bitwise(pmh, m):
    print(f"tables m={m}", flush=True)
    c2 = pmh.Context(SEED, m, 2)
    beta = c2.table(0, m + 1)
    assert all(beta[i] == O.constants(2, m, i)[0] for i in range(1, m + 1))
    c2.close()
    c3 = pmh.Context(SEED, m, 3)
    sc = c3.table(7, 8)
    assert np.array_equal(sc[:3].view(np.uint64), O.constants(3, m)[:3].view(np.uint64))
    c3.close()
    c4 = pmh.Context(SEED, m, 4)
    lam, a, c1, gam, dgam = (c4.table(w, m) for w in (1, 2, 3, 5, 6))
    delta = c4.table(7, 8)[4]
    for i in range(1, m):
        ref = O.constants(4, m, i)
        got = np.array([lam[i], a[i], c1[i], gam[i], dgam[i], delta])
        assert np.array_equal(got.view(np.uint64), ref[:6].view(np.uint64)), i
    c4.close()


# ----------------------------------------------------------------- signatures
VARIANT_M = [(v, m) for v in (1, 2, 3, 4) for m in (1, 2, 3, 64, 100, 1024) if not (v >= 3 and m == 1)]


@pytest.mark.parametrize("variant,m", VARIANT_M)
def test_random_batches_bit_exact(pmh, variant, m):
    """Ragged batches (sizes 0..600, several weight laws): keys, positions,
    values and ids equal the oracle's in the batched, plain and graph forms."""
    print(f"random batch PMH{variant} m={m}", flush=True)
    ctx = pmh.Context(SEED, m, variant)
    for law, seed in (("exp", 1), ("pareto", 2), ("wide", 3), ("ones", 4)):
        b = W.random_sets(100 * variant + seed + m, 40, 0, 600, law)
        want = O.sign_batch(variant, SEED, m, b.ids, b.weights, b.offsets, nthreads=8)
        for mode in ("batched", "plain", "graph"):
            sig, st = _keys(ctx, b, mode)
            assert st == pmh.PMH_OK
            keys, idx, val, ids = _host(sig)
            assert np.array_equal(keys, want), (law, mode)
        for s in range(b.num_sets):
            si, _ = b.set(s)
            ri, rv, rid = O.decode(want[s], si)
            assert np.array_equal(idx[s], ri) and np.array_equal(ids[s], rid)
            assert np.array_equal(val[s].view(np.uint64), rv.view(np.uint64))
    ctx.close()


def test_plain_pairs_workload(pmh):
    """1,000 sets x 100 elements, m = 256, ProbMinHash1, one launch per set:
    bit-exact, and the 200 sharing pairs obey the collision law."""
    print("plain_pairs workload", flush=True)
    from scipy import stats
    b = W.plain_pairs()
    ctx = pmh.Context(SEED, 256, 1)
    sig, st = _keys(ctx, b, "plain")
    assert st == pmh.PMH_OK
    keys, idx, val, ids = _host(sig)
    want = O.sign_batch(1, SEED, 256, b.ids, b.weights, b.offsets, nthreads=8)
    assert np.array_equal(keys, want)
    num, var, outside = 0.0, 0.0, 0
    for sa, sb in b.meta["pairs"]:
        ia, wa = b.set(sa)
        ib, wb = b.set(sb)
        J = O.jp_sorted(ia, wa, ib, wb)
        c = round(pmh.estimate(ids[sa], idx[sa], ids[sb], idx[sb]) * 256)
        num += c - 256 * J
        var += 256 * J * (1 - J)
        outside += not (stats.binom.ppf(0.005, 256, J) <= c <= stats.binom.ppf(0.995, 256, J))
    assert abs(num / np.sqrt(var)) <= 2.576 and outside <= 6
    ctx.close()


def test_edge_cases(pmh):
    """Empty sets, single elements, zero weights, invalid weights (skipped and
    reported), extreme weights."""
    print("edge cases", flush=True)
    m = 64
    sizes = [0, 1, 0, 2, 1, 5, 0]
    rng = np.random.default_rng(9)
    N = sum(sizes)
    ids = rng.integers(0, 2**64 - 1, size=N, dtype=np.uint64)
    w = rng.exponential(size=N) + 0.01
    w[3] = 0.0
    w[5] = 1e-300
    w[6] = 1e300
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    b = W.Batch(ids, w, off)
    for v in (1, 2, 3, 4):
        ctx = pmh.Context(SEED, m, v)
        sig, st = _keys(ctx, b)
        assert st == pmh.PMH_OK
        want = O.sign_batch(v, SEED, m, ids, w, off)
        assert np.array_equal(_host(sig)[0], want)
        assert (_host(sig)[1][0] == 0xFFFFFFFF).all() and np.isinf(_host(sig)[2][0]).all()
        # invalid weights: skipped like zeros, reported once
        wb = w.copy()
        wb[4] = -1.0
        wb[7] = np.nan
        wb[8] = 1e-310
        sig, st = _keys(ctx, W.Batch(ids, wb, off))
        assert st == pmh.PMH_ERR_WEIGHT
        wz = wb.copy()
        wz[[4, 7, 8]] = 0.0
        assert np.array_equal(_host(sig)[0], O.sign_batch(v, SEED, m, ids, wz, off))
        assert ctx.status() == pmh.PMH_OK  # cleared after reading
        ctx.close()


def test_oversize_set_reported(pmh):
    print("oversize set", flush=True)
    n = (1 << 20) + 1
    rng = np.random.default_rng(10)
    b = W.Batch(rng.integers(0, 2**64 - 1, size=n + 3, dtype=np.uint64), np.ones(n + 3),
                np.array([0, 3, n + 3], dtype=np.uint64))
    ctx = pmh.Context(SEED, 32, 1)
    sig, st = _keys(ctx, b)
    assert st == pmh.PMH_ERR_SET_TOO_LARGE
    keys = _host(sig)[0]
    assert np.array_equal(keys[0], O.sign(1, SEED, 32, b.ids[:3], b.weights[:3]))
    assert (keys[1] == O.EMPTY).all()
    ctx.close()


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_schedule_invariance(pmh, variant):
    """The signature does not depend on the schedule: thresholds, rounds, lane
    or chain mode, waves per workgroup, grid size (reading: exact minimum over
    all points, Sec. 2 stop rule as pure pruning)."""
    print(f"schedule invariance PMH{variant}", flush=True)
    m = 256
    b = W.random_sets(500 + variant, 60, 0, 2000, "pareto")
    want = O.sign_batch(variant, SEED, m, b.ids, b.weights, b.offsets, nthreads=8)
    ctx = pmh.Context(SEED, m, variant)
    default = ctx.get_tuning().as_dict()
    configs = [dict(), dict(c0=-6.0, grow=1.3, max_rounds=12), dict(max_rounds=1), dict(chain_expect=0.0),
               dict(chain_expect=1e9, mini_expect=1e9, lane_budget=1000000), dict(lane_budget=1),
               dict(mini_expect=0.0), dict(mini_expect=0.0, chain_expect=1e9), dict(waves=1), dict(waves=2),
               dict(lane_budget=1, waves=1),
               dict(blocks_per_cu=1), dict(kmax_refresh=1), dict(c0=20.0), dict(waves=4),
               dict(waves=4, chain_expect=0.0),
               dict(waves=8), dict(waves=8, chain_expect=0.0),
               dict(kmax_refresh=3, max_rounds=1),
               # many thin rounds (ProbMinHash3 resumes each element near the
               # previous threshold) in every mode
               dict(c0=-3.0, grow=1.05, max_rounds=60),
               dict(c0=-3.0, grow=1.05, max_rounds=60, chain_expect=0.0),
               dict(c0=-3.0, grow=1.05, max_rounds=60, mini_expect=0.0, chain_expect=1e9),
               dict(c0=-3.0, grow=1.05, max_rounds=60, chain_expect=1e9, mini_expect=1e9, lane_budget=1000000)]
    for cfg in configs:
        ctx.set_tuning(**cfg)
        sig, st = _keys(ctx, b)
        assert st == pmh.PMH_OK
        assert np.array_equal(_host(sig)[0], want), cfg
        ctx.set_tuning(**default)
    ctx.close()


def _split_batch(seed):
    """Sets around the split thresholds, with empty sets and runs of zero
    weights (chunks with nothing to hash)."""
    rng = np.random.default_rng(seed)
    sizes = [0, 1, 63, 64, 65, 200, 1000, 4097, 3, 20000, 129, 0, 5000]
    n = sum(sizes)
    ids = rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64)
    w = rng.pareto(1.5, size=n) + 0.05
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    w[off[7]:off[7] + 100] = 0.0  # a whole chunk and a part of the next without weight
    w[off[12]:off[13]] = 0.0      # a split set without any weight
    return W.Batch(ids, w, off)


@pytest.mark.parametrize("variant,m", [(1, 64), (2, 64), (3, 64), (4, 64), (1, 1024), (3, 1024), (2, 300),
                                       (4, 300), (1, 1), (2, 1)])
def test_split_sets(pmh, variant, m):
    """Sets split across workgroups (chunks merged by atomic min, completion
    check, repair round) give the oracle's signature bit for bit, whichever
    output row holds the merge and however often the repair runs."""
    print(f"split sets PMH{variant} m={m}", flush=True)
    b = _split_batch(40 + variant)
    want = O.sign_batch(variant, SEED, m, b.ids, b.weights, b.offsets, nthreads=8)
    decoded = [O.decode(want[s], b.set(s)[0]) for s in range(b.num_sets)]
    ctx = pmh.Context(SEED, m, variant)
    default = ctx.get_tuning().as_dict()
    for cfg in (dict(split_log2=6), dict(split_log2=6, c0_split=-30.0), dict(split_log2=7, c0_split=40.0),
                dict(split_log2=2), dict(split_log2=12), dict(split_log2=6, waves=1, blocks_per_cu=1)):
        ctx.set_tuning(**cfg)
        for outputs in (("idx", "val", "id", "keys"), ("val",), ("id", "idx"), ("idx",)):
            for mode in ("batched", "graph"):
                sig = ctx.hash_sets(_dev(b.ids), _dev(b.weights), _dev(b.offsets), mode=mode, outputs=outputs)
                assert ctx.status() == pmh.PMH_OK
                got = {k: getattr(sig, k).cpu().numpy() for k in outputs}
                for s in range(b.num_sets):
                    ri, rv, rid = decoded[s]
                    if "keys" in got:
                        assert np.array_equal(got["keys"][s].view(np.uint64), want[s]), (cfg, mode, s)
                    if "idx" in got:
                        assert np.array_equal(got["idx"][s].view(np.uint32), ri), (cfg, mode, outputs, s)
                    if "val" in got:
                        assert np.array_equal(got["val"][s].view(np.uint64), rv.view(np.uint64)), (cfg, mode, s)
                    if "id" in got:
                        assert np.array_equal(got["id"][s].view(np.uint64), rid), (cfg, mode, outputs, s)
        ctx.set_tuning(**default)
    ctx.close()


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_large_m_four_waves(pmh, variant):
    """m = 4096, where contexts default to 4 waves per workgroup (8 for
    ProbMinHash2/4): ragged sets
    up to 70,000 elements (split ones included: above m = 2048 sets of
    >= 2^16 elements split) in the batched and graph
    forms, and the same keys with 1 and 2 waves."""
    print(f"m=4096 PMH{variant}", flush=True)
    m = 4096
    rng = np.random.default_rng(70 + variant)
    sizes = [0, 1, 3, 50, 700, 4096, 9000, 70000, 12, 2]
    ids = rng.integers(0, 2**64 - 1, size=sum(sizes), dtype=np.uint64)
    w = rng.uniform(size=sum(sizes)) + 1e-3
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    b = W.Batch(ids, w, off)
    want = O.sign_batch(variant, SEED, m, ids, w, off, nthreads=8)
    ctx = pmh.Context(SEED, m, variant)
    assert ctx.get_tuning().waves == (4 if variant in (1, 3) else 8)
    for cfg in (dict(), dict(split_log2=12), dict(waves=2), dict(waves=1), dict(waves=8)):
        ctx.set_tuning(**cfg)
        for mode in ("batched", "graph"):
            sig, st = _keys(ctx, b, mode)
            assert st == pmh.PMH_OK
            assert np.array_equal(_host(sig)[0], want), (cfg, mode)
    ctx.close()


def test_split_largest_set(pmh):
    """One set of 2^20 elements (the largest accepted) with the default split,
    alone and beside small sets."""
    print("split: 2^20-element set", flush=True)
    rng = np.random.default_rng(11)
    n = 1 << 20
    sizes = [5, n, 17]
    ids = rng.integers(0, 2**64 - 1, size=sum(sizes), dtype=np.uint64)
    w = rng.exponential(size=sum(sizes))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    b = W.Batch(ids, w, off)
    for variant, m in ((1, 1024), (4, 256)):
        want = O.sign_batch(variant, SEED, m, ids, w, off, nthreads=8)
        ctx = pmh.Context(SEED, m, variant)
        sig, st = _keys(ctx, b)
        assert st == pmh.PMH_OK
        assert np.array_equal(_host(sig)[0], want)
        sig, st = _keys(ctx, b.subset([1]))
        assert st == pmh.PMH_OK and np.array_equal(_host(sig)[0][0], want[1])
        ctx.close()


def test_alone_and_in_a_mix(pmh):
    """A set's signature is the same alone, in any batch, at any position."""
    print("alone vs mix", flush=True)
    b = W.random_sets(77, 100, 1, 3000, "exp")
    ctx = pmh.Context(SEED, 512, 3)
    full = _host(_keys(ctx, b)[0])[0]
    rng = np.random.default_rng(5)
    for s in rng.choice(b.num_sets, 8, replace=False):
        alone = _host(_keys(ctx, b.subset([s]))[0])[0][0]
        assert np.array_equal(alone, full[s])
        order = rng.permutation(b.num_sets)
        mixed = _host(_keys(ctx, b.subset(order))[0])[0]
        assert np.array_equal(mixed[np.where(order == s)[0][0]], full[s])
    ctx.close()


def test_graph_survives_work_buffer_growth(pmh):
    """A cached graph keeps its own work buffer: a graph call, then a batched
    call on more sets (which grows the context's shared work buffer), then the
    same graph call again gives the batched result."""
    print("graph after work-buffer growth", flush=True)
    m = 64
    small = W.random_sets(301, 40, 0, 300, "exp")
    big = W.random_sets(302, 3000, 0, 40, "exp")
    ctx = pmh.Context(SEED, m, 1)
    args = [_dev(small.ids), _dev(small.weights), _dev(small.offsets)]
    out = ctx.alloc_outputs(small.num_sets)
    ctx.hash_sets(*args, out=out, mode="graph")
    first = _host(out)[0].copy()
    ctx.hash_sets(_dev(big.ids), _dev(big.weights), _dev(big.offsets))
    out.keys.fill_(0)
    ctx.hash_sets(*args, out=out, mode="graph")
    assert ctx.status() == pmh.PMH_OK
    want = ctx.hash_sets(*args)
    assert np.array_equal(_host(out)[0], _host(want)[0])
    assert np.array_equal(first, _host(want)[0])
    ctx.close()


def test_estimate_pairs_device(pmh):
    """pmh_estimate_pairs (eq. (3) numerators on the device) against the
    oracle's estimator, pair by pair, with empty sets (all-empty components)
    and identical pairs among them."""
    print("estimate_pairs", flush=True)
    import torch
    for m in (1, 64, 1000):
        b = W.random_sets(310 + m, 120, 0, 400, "pareto")
        pos = [5, 17, 40, 41]  # repeated offsets: empty sets
        b = W.Batch(b.ids, b.weights, np.insert(b.offsets, pos, b.offsets[pos]))
        assert (b.sizes() == 0).sum() >= 4
        ctx = pmh.Context(SEED, m, 1)
        sig = ctx.hash_sets(_dev(b.ids), _dev(b.weights), _dev(b.offsets))
        keys, idx, val, ids = _host(sig)
        rng = np.random.default_rng(m)
        A = rng.integers(0, b.num_sets, size=500)
        B = rng.integers(0, b.num_sets, size=500)
        A[20:30] = pos[0] + np.arange(10) % 2  # empty against non-empty and empty
        B[:20] = A[:20]  # identical pairs
        ia, ib = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        counts = pmh.estimate_pairs(sig.id[ia].contiguous(), sig.idx[ia].contiguous(),
                                    sig.id[ib].contiguous(), sig.idx[ib].contiguous()).cpu().numpy()
        want = np.array([round(O.estimate(ids[a], idx[a], ids[c], idx[c]) * m) for a, c in zip(A, B)])
        assert np.array_equal(counts, want), m
        sizes = b.sizes()
        for r in range(20):
            assert counts[r] == (m if sizes[A[r]] > 0 else 0)
        empty = sizes[A] == 0
        assert (counts[empty] == 0).all()
        ctx.close()
