"""GPU parity of P-MinHash (Sec. 1.1, the paper's O(nm) baseline): the HIP
kernels through the C ABI against the CPU oracle, bit-exact keys, positions,
values and ids, with and without split sets (chunks of 1,024 elements for
sets of >= 2^11 elements when a merge row is available), component passes
that do not fill the last thread group, empty sets, zero and invalid weights.
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


def _run(ctx, b, outputs=("idx", "val", "id", "keys")):
    from paper_1911_00675_amd import pmh as P
    sig = ctx.hash_sets(P.to_device(b.ids), P.to_device(b.weights), P.to_device(b.offsets), mode="pminhash",
                        outputs=outputs)
    return sig, ctx.status()


def _check(sig, b, want, m):
    keys = sig.keys.cpu().numpy().view(np.uint64) if sig.keys is not None else None
    idx = sig.idx.cpu().numpy().view(np.uint32)
    val = sig.val.cpu().numpy().view(np.uint64) if sig.val is not None else None
    ids = sig.id.cpu().numpy().view(np.uint64) if sig.id is not None else None
    if keys is not None:
        assert np.array_equal(keys, want)
    for s in range(b.num_sets):
        si, _ = b.set(s)
        ri, rv, rid = O.decode(want[s], si)
        assert np.array_equal(idx[s], ri), s
        if val is not None:
            assert np.array_equal(val[s], rv.view(np.uint64)), s
        if ids is not None:
            assert np.array_equal(ids[s], rid), s


@pytest.mark.parametrize("m", [1, 7, 256, 1024, 1500, 4096])
def test_pminhash_random_batches(pmh, m):
    """Sizes up to 3,000 (sets of >= 2^11 elements split into 1,024-element
    chunks), Pareto weights; all outputs, then idx only (no merge row: no
    split)."""
    print(f"pminhash m={m}", flush=True)
    b = W.random_sets(800 + m, 24 if m < 4096 else 10, 0, 3000, "pareto")
    want = O.pminhash_batch(SEED, m, b.ids, b.weights, b.offsets, nthreads=8)
    ctx = pmh.Context(SEED, m, 1 if m == 1 else 3)  # the variant plays no part
    sig, st = _run(ctx, b)
    assert st == pmh.PMH_OK
    _check(sig, b, want, m)
    sig, st = _run(ctx, b, outputs=("idx",))
    assert st == pmh.PMH_OK
    _check(sig, b, want, m)
    sig, st = _run(ctx, b, outputs=("idx", "id"))  # merge rows in the id output
    assert st == pmh.PMH_OK
    _check(sig, b, want, m)
    ctx.close()


def test_pminhash_edge_cases(pmh):
    """Empty sets, single elements, zero weights, extreme weights; invalid
    weights skipped like zeros and reported."""
    m = 64
    sizes = [0, 1, 0, 2, 1, 5, 0, 2100]
    rng = np.random.default_rng(19)
    N = sum(sizes)
    ids = rng.integers(0, 2**64 - 1, size=N, dtype=np.uint64)
    w = rng.exponential(size=N) + 0.01
    w[3] = 0.0
    w[5] = 1e-300
    w[6] = 1e300
    w[20:40] = 0.0
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    b = W.Batch(ids, w, off)
    ctx = pmh.Context(SEED, m, 1)
    sig, st = _run(ctx, b)
    assert st == pmh.PMH_OK
    _check(sig, b, O.pminhash_batch(SEED, m, ids, w, off), m)
    assert (sig.idx[0].cpu().numpy().view(np.uint32) == 0xFFFFFFFF).all()
    wb = w.copy()
    wb[4] = -1.0
    wb[7] = np.nan
    wb[2000] = 1e-310
    sig, st = _run(ctx, W.Batch(ids, wb, off))
    assert st == pmh.PMH_ERR_WEIGHT
    wz = wb.copy()
    wz[[4, 7, 2000]] = 0.0
    _check(sig, b, O.pminhash_batch(SEED, m, ids, wz, off), m)
    ctx.close()


def test_pminhash_oversize_set_reported(pmh):
    n = (1 << 20) + 1
    rng = np.random.default_rng(20)
    b = W.Batch(rng.integers(0, 2**64 - 1, size=n + 3, dtype=np.uint64), np.ones(n + 3),
                np.array([0, 3, n + 3], dtype=np.uint64))
    ctx = pmh.Context(SEED, 32, 1)
    sig, st = _run(ctx, b)
    assert st == pmh.PMH_ERR_SET_TOO_LARGE
    keys = sig.keys.cpu().numpy().view(np.uint64)
    assert np.array_equal(keys[0], O.pminhash(SEED, 32, b.ids[:3], b.weights[:3]))
    assert (keys[1] == O.EMPTY).all()
    ctx.close()


def test_pminhash_collision_law(pmh):
    """Device signatures of two overlapping sets agree in a fraction J_P of
    4096 components (binomial 1e-6 bounds)."""
    from scipy import stats
    m = 4096
    rng = np.random.default_rng(21)
    shared = rng.integers(0, 2**63, size=300, dtype=np.uint64)
    ida = np.concatenate([shared, rng.integers(0, 2**63, size=200, dtype=np.uint64)])
    idb = np.concatenate([shared, rng.integers(0, 2**63, size=100, dtype=np.uint64)])
    wa, wb = rng.exponential(size=ida.size), rng.exponential(size=idb.size)
    b = W.Batch(np.concatenate([ida, idb]), np.concatenate([wa, wb]),
                np.array([0, ida.size, ida.size + idb.size], dtype=np.uint64))
    ctx = pmh.Context(SEED, m, 1)
    sig, st = _run(ctx, b)
    assert st == pmh.PMH_OK
    z = sig.id.cpu().numpy().view(np.uint64)
    J = O.jp_sorted(ida, wa, idb, wb)
    c = int((z[0] == z[1]).sum())
    assert stats.binom.ppf(1e-6, m, J) <= c <= stats.binom.ppf(1 - 1e-6, m, J)
    ctx.close()
