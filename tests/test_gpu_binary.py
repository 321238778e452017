"""GPU parity of the binary-weight specialisations (Sec. 2.9): the HIP path's
pmh_hash_sets_binary through the C ABI against the oracle's variants 5..8
(ProbMinHash1..4 specialised to unit weights), bit-exact keys, positions,
values and ids, in every schedule the persistent kernel can take (lane,
4-lane mini-chain and 64-lane chain modes, thin and single rounds, split sets
merged across workgroups), with empty sets and sets up to 2^20 elements.
ProbMinHash1/2 binary must also equal the weighted path with unit weights.
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


def _dev(a):
    from paper_1911_00675_amd import pmh as P
    return P.to_device(a)


def _want(variant, m, b):
    return O.sign_batch(variant + 4, SEED, m, b.ids, np.ones(b.ids.size), b.offsets, nthreads=8)


def _binary(ctx, b, outputs=("idx", "val", "id", "keys")):
    sig = ctx.hash_sets(_dev(b.ids), None, _dev(b.offsets), mode="binary", outputs=outputs)
    return sig, ctx.status()


def _check(sig, b, want, what=""):
    if sig.keys is not None:
        assert np.array_equal(sig.keys.cpu().numpy().view(np.uint64), want), what
    idx = sig.idx.cpu().numpy().view(np.uint32) if sig.idx is not None else None
    val = sig.val.cpu().numpy().view(np.uint64) if sig.val is not None else None
    ids = sig.id.cpu().numpy().view(np.uint64) if sig.id is not None else None
    for s in range(b.num_sets):
        ri, rv, rid = O.decode(want[s], b.set(s)[0])
        if idx is not None:
            assert np.array_equal(idx[s], ri), (what, s)
        if val is not None:
            assert np.array_equal(val[s], rv.view(np.uint64)), (what, s)
        if ids is not None:
            assert np.array_equal(ids[s], rid), (what, s)


@pytest.mark.parametrize("variant,m", [(1, 1), (2, 1), (1, 64), (2, 64), (3, 2), (4, 2), (3, 64), (4, 64),
                                       (1, 1024), (2, 1024), (3, 1024), (4, 1024), (3, 4096), (4, 4096)])
def test_binary_random_batches(pmh, variant, m):
    """Sizes 0..3,000 (split sets from 2^11 elements), all outputs, then
    positions only (no merge row, so no split)."""
    print(f"binary PMH{variant} m={m}", flush=True)
    b = W.random_sets(900 + 10 * variant + m, 24 if m < 4096 else 10, 0, 3000, "exp")
    want = _want(variant, m, b)
    ctx = pmh.Context(SEED, m, variant)
    sig, st = _binary(ctx, b)
    assert st == pmh.PMH_OK
    _check(sig, b, want, "all")
    sig, st = _binary(ctx, b, outputs=("idx",))
    assert st == pmh.PMH_OK
    _check(sig, b, want, "idx")
    ctx.close()


@pytest.mark.parametrize("variant", [1, 2])
def test_binary_pmh12_equal_weighted_unit_weights(pmh, variant):
    """With unit weights the weighted kernel computes 1/w = 1 and the same
    points: both device paths agree bit for bit."""
    b = W.random_sets(950 + variant, 30, 0, 2500, "exp")
    ctx = pmh.Context(SEED, 256, variant)
    sig, st = _binary(ctx, b, outputs=("keys",))
    assert st == pmh.PMH_OK
    ref = ctx.hash_sets(_dev(b.ids), _dev(np.ones(b.ids.size)), _dev(b.offsets), outputs=("keys",))
    assert ctx.status() == pmh.PMH_OK
    assert np.array_equal(sig.keys.cpu().numpy(), ref.keys.cpu().numpy())
    ctx.close()


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_binary_schedule_invariance(pmh, variant):
    """Thresholds, rounds (thin ones make ProbMinHash3 resume each element
    after the previous threshold), lane/mini/chain modes, waves and splits
    change nothing."""
    print(f"binary schedule invariance PMH{variant}", flush=True)
    m = 256
    rng = np.random.default_rng(960 + variant)
    sizes = [0, 1, 2, 63, 64, 65, 300, 1000, 0, 4097, 3, 9000, 129, 2000]
    ids = rng.integers(0, 2**64 - 1, size=sum(sizes), dtype=np.uint64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    b = W.Batch(ids, np.ones(ids.size), off)
    want = _want(variant, m, b)
    ctx = pmh.Context(SEED, m, variant)
    default = ctx.get_tuning().as_dict()
    configs = [dict(), dict(c0=-6.0, grow=1.3, max_rounds=12), dict(max_rounds=1), dict(chain_expect=0.0),
               dict(chain_expect=1e9, mini_expect=1e9, lane_budget=1000000), dict(lane_budget=1),
               dict(mini_expect=0.0, chain_expect=1e9), dict(waves=1), dict(waves=2), dict(c0=20.0),
               dict(c0=-3.0, grow=1.05, max_rounds=60),
               dict(c0=-3.0, grow=1.05, max_rounds=60, chain_expect=0.0),
               dict(c0=-3.0, grow=1.05, max_rounds=60, mini_expect=0.0, chain_expect=1e9),
               dict(split_log2=6), dict(split_log2=6, c0_split=-30.0), dict(split_log2=2)]
    for cfg in configs:
        ctx.set_tuning(**cfg)
        sig, st = _binary(ctx, b, outputs=("keys",))
        assert st == pmh.PMH_OK
        assert np.array_equal(sig.keys.cpu().numpy().view(np.uint64), want), cfg
        ctx.set_tuning(**default)
    ctx.close()


def test_binary_largest_set(pmh):
    """A set of 2^20 elements beside small ones (split with the default
    tuning); one above 2^20 is reported and left empty."""
    print("binary: 2^20-element set", flush=True)
    rng = np.random.default_rng(970)
    n = 1 << 20
    sizes = [5, n, 17]
    ids = rng.integers(0, 2**64 - 1, size=sum(sizes), dtype=np.uint64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    b = W.Batch(ids, np.ones(ids.size), off)
    for variant, m in ((1, 1024), (3, 1024), (4, 256)):
        ctx = pmh.Context(SEED, m, variant)
        sig, st = _binary(ctx, b, outputs=("keys",))
        assert st == pmh.PMH_OK
        assert np.array_equal(sig.keys.cpu().numpy().view(np.uint64), _want(variant, m, b)), variant
        ctx.close()
    big = W.Batch(rng.integers(0, 2**64 - 1, size=n + 4, dtype=np.uint64), np.ones(n + 4),
                  np.array([0, 3, n + 4], dtype=np.uint64))
    ctx = pmh.Context(SEED, 32, 3)
    sig, st = _binary(ctx, big, outputs=("keys",))
    assert st == pmh.PMH_ERR_SET_TOO_LARGE
    keys = sig.keys.cpu().numpy().view(np.uint64)
    assert np.array_equal(keys[0], _want(3, 32, big.subset([0]))[0])
    assert (keys[1] == O.EMPTY).all()
    ctx.close()


def test_binary_collision_law(pmh):
    """Binary ProbMinHash3/4 on the device: |A| = 500, |B| = 400, 300 shared
    (J = 1/2); equal ids over m = 4096 within 1e-6 binomial bounds."""
    from scipy import stats
    m = 4096
    rng = np.random.default_rng(971)
    shared = rng.integers(0, 2**63, size=300, dtype=np.uint64)
    ida = np.concatenate([shared, rng.integers(0, 2**63, size=200, dtype=np.uint64)])
    idb = np.concatenate([shared, rng.integers(0, 2**63, size=100, dtype=np.uint64)])
    b = W.Batch(np.concatenate([ida, idb]), np.ones(ida.size + idb.size),
                np.array([0, ida.size, ida.size + idb.size], dtype=np.uint64))
    for variant in (3, 4):
        ctx = pmh.Context(SEED, m, variant)
        sig, st = _binary(ctx, b, outputs=("id",))
        assert st == pmh.PMH_OK
        z = sig.id.cpu().numpy().view(np.uint64)
        c = int((z[0] == z[1]).sum())
        assert stats.binom.ppf(1e-6, m, 0.5) <= c <= stats.binom.ppf(1 - 1e-6, m, 0.5), (variant, c)
        ctx.close()
