"""GPU parity of the b-bit reduction (Sec. 1.3) and of the packed all-pairs
counts: bit-exact packed words against the oracle for every b, equal-field
counts against the oracle's unpacking count on ragged tiles (k not a
multiple of 64, m b not a multiple of 64), and the corrected estimate on
device signatures of overlapping sets within binomial bounds of J_P."""
import numpy as np
import pytest

import oracle as O

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


@pytest.mark.parametrize("b", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("m", [1, 63, 333, 1024, 4096, 16384])
def test_pack_and_allpairs_bit_exact(pmh, b, m):
    import torch
    print(f"bbit b={b} m={m}", flush=True)
    rng = np.random.default_rng(b * 1000 + m)
    k = 97
    ids = rng.integers(0, 2**64 - 1, size=(k, m), dtype=np.uint64)
    ids[1] = ids[0]                       # an identical pair
    ids[2, : m // 2] = ids[3, : m // 2]   # a half-equal pair
    ids[5] = 0                            # an empty signature
    want = O.bbit_pack(ids, m, b)
    dev = torch.from_numpy(ids.view(np.int64)).cuda()
    got = pmh.bbit_pack(dev, b)
    assert np.array_equal(got.cpu().numpy().view(np.uint64), want)
    counts = pmh.bbit_allpairs(got, m, b).cpu().numpy().view(np.uint16)
    for r in range(k):
        for c in range(0, k, 7 if r > 8 else 1):
            assert counts[r, c] == O.bbit_equal(want[r], want[c], m, b), (r, c)
    assert np.array_equal(counts, counts.T)
    assert (np.diag(counts) == m).all() and counts[0, 1] == m


def test_corrected_estimate_on_device_signatures(pmh):
    """ProbMinHash1 signatures (m = 4096) of overlapping sets, 1-bit reduced on
    the device: the corrected estimate of each pair within 1e-6 binomial
    bounds of J_P."""
    from scipy import stats
    from paper_1911_00675_amd import workloads as W
    m, b = 4096, 1
    rng = np.random.default_rng(41)
    sets = []
    for _ in range(6):
        shared = rng.integers(1, 2**63, size=200, dtype=np.uint64)
        a = np.concatenate([shared, rng.integers(1, 2**63, size=rng.integers(0, 300), dtype=np.uint64)])
        c = np.concatenate([shared, rng.integers(1, 2**63, size=rng.integers(0, 300), dtype=np.uint64)])
        sets += [(a, rng.exponential(size=a.size)), (c, rng.exponential(size=c.size))]
    ids = np.concatenate([s[0] for s in sets])
    w = np.concatenate([s[1] for s in sets])
    off = np.concatenate([[0], np.cumsum([s[0].size for s in sets])]).astype(np.uint64)
    ctx = pmh.Context(SEED, m, 1)
    sig = ctx.hash_sets(pmh.to_device(ids), pmh.to_device(w), pmh.to_device(off), outputs=("idx", "id"))
    assert ctx.status() == pmh.PMH_OK
    packed = pmh.bbit_pack(sig.id, b)
    counts = pmh.bbit_allpairs(packed, m, b).cpu().numpy().view(np.uint16)
    r = 2.0 ** -b
    for p in range(6):
        (ia, wa), (ib, wb) = sets[2 * p], sets[2 * p + 1]
        J = O.jp_sorted(ia, wa, ib, wb)
        pr = J + (1 - J) * r
        c = int(counts[2 * p, 2 * p + 1])
        assert stats.binom.ppf(1e-6, m, pr) <= c <= stats.binom.ppf(1 - 1e-6, m, pr), (p, c, m * pr)
        est = O.bbit_estimate(c, m, b)
        assert abs(est - J) < 6 * np.sqrt(pr * (1 - pr) / m) / (1 - r)
    ctx.close()


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_fused_epilogue_bit_exact(pmh, variant):
    """The b-bit words written by the hash kernel's epilogue
    (pmh_hash_sets_bbit) equal the oracle's packing of the oracle's
    signature ids for every b, on ragged batches with empty and split sets,
    with the other outputs present (sets split) or absent (no merge row, no
    split), and the separate pack kernel's words."""
    from paper_1911_00675_amd import workloads as W
    rng = np.random.default_rng(900 + variant)
    sizes = [0, 1, 3, 80, 70000, 0, 700, 5]  # split at every m here (2^15 up to m = 2048, 2^16 above)
    n = sum(sizes)
    b_ = W.Batch(rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64), rng.exponential(size=n) + 1e-3,
                 np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64))
    d = [pmh.to_device(a) for a in (b_.ids, b_.weights, b_.offsets)]
    for m in (2, 63, 1000, 4096):
        print(f"fused bbit PMH{variant} m={m}", flush=True)
        want_keys = O.sign_batch(variant, SEED, m, b_.ids, b_.weights, b_.offsets, nthreads=8)
        ids = np.stack([O.decode(want_keys[s], b_.set(s)[0])[2] for s in range(b_.num_sets)])
        ctx = pmh.Context(SEED, m, variant)
        for bb in (1, 2, 4, 8, 16):
            want = O.bbit_pack(ids, m, bb)
            for outputs in (("idx", "val", "id", "keys"), ()):
                sig = ctx.hash_sets(*d, outputs=outputs, bbit=bb)
                assert ctx.status() == pmh.PMH_OK
                assert np.array_equal(sig.bbit.cpu().numpy().view(np.uint64), want), (m, bb, outputs)
                if outputs:
                    assert np.array_equal(sig.keys.cpu().numpy().view(np.uint64), want_keys)
                    sep = pmh.bbit_pack(sig.id, bb).cpu().numpy().view(np.uint64)
                    assert np.array_equal(sep, want)
        ctx.close()
