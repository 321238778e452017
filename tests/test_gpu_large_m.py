"""GPU parity above m = 4096: m = 8192 and the largest m the device accepts
for each variant (pmh_max_m; keys, and for ProbMinHash2/4 the Fisher-Yates
label arrays, live in LDS).  Ragged batches with empty, single-element and
split sets, the binary specialisations (Sec. 2.9) and an incremental update
in two calls, bit-exact against the oracle."""
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


def _batch(seed):
    rng = np.random.default_rng(seed)
    sizes = [0, 1, 2, 7, 300, 2500, 70000, 13, 0, 90]  # 70,000 >= 2^16: split at these m
    n = sum(sizes)
    ids = rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64)
    w = rng.pareto(1.5, size=n) + 0.05
    return W.Batch(ids, w, np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64))


def _halves(b):
    out = []
    for first in (True, False):
        idx, sizes = [], []
        for s in range(b.num_sets):
            a, e = int(b.offsets[s]), int(b.offsets[s + 1])
            h = a + (e - a) // 2
            r = np.arange(a, h) if first else np.arange(h, e)
            idx.append(r)
            sizes.append(r.size)
        idx = np.concatenate(idx).astype(np.int64)
        out.append(W.Batch(b.ids[idx], b.weights[idx], np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)))
    return out


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_large_m_bit_exact(pmh, variant):
    max_m = int(pmh.lib().pmh_max_m(variant))
    assert max_m >= 8192
    for m in sorted({8192, max_m}):
        print(f"PMH{variant} m={m}", flush=True)
        b = _batch(7000 + variant + m)
        want = O.sign_batch(variant, SEED, m, b.ids, b.weights, b.offsets, nthreads=8)
        ctx = pmh.Context(SEED, m, variant)
        default = ctx.get_tuning().as_dict()
        for cfg in (dict(), dict(split_log2=12), dict(waves=1)):
            ctx.set_tuning(**cfg)
            for mode in ("batched", "graph"):
                sig = ctx.hash_sets(_dev(b.ids), _dev(b.weights), _dev(b.offsets), mode=mode)
                assert ctx.status() == pmh.PMH_OK
                assert np.array_equal(sig.keys.cpu().numpy().view(np.uint64), want), (m, cfg, mode)
            ctx.set_tuning(**default)
        for s in range(b.num_sets):  # decoded outputs of the last call
            ri, rv, rid = O.decode(want[s], b.set(s)[0])
            assert np.array_equal(sig.idx[s].cpu().numpy().view(np.uint32), ri)
            assert np.array_equal(sig.val[s].cpu().numpy().view(np.uint64), rv.view(np.uint64))
            assert np.array_equal(sig.id[s].cpu().numpy().view(np.uint64), rid)
        ones = np.ones_like(b.weights)
        wantb = O.sign_batch(variant + 4, SEED, m, b.ids, ones, b.offsets, nthreads=8)
        sig = ctx.hash_sets(_dev(b.ids), None, _dev(b.offsets), mode="binary")
        assert ctx.status() == pmh.PMH_OK
        assert np.array_equal(sig.keys.cpu().numpy().view(np.uint64), wantb), (m, "binary")
        st = ctx.new_state(b.num_sets)
        for part in _halves(b):
            ctx.update_sets(_dev(part.ids), _dev(part.weights), _dev(part.offsets), st)
        assert ctx.status() == pmh.PMH_OK
        assert np.array_equal(st.keys.cpu().numpy().view(np.uint64), want), (m, "update")
        ctx.close()
    with pytest.raises(pmh.PmhError):
        pmh.Context(SEED, max_m + 64, variant)
