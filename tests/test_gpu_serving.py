"""Serving: continuous batching returns, for every request, exactly the
signature the batched launch computes for the same set, whatever batch the
request landed in (a signature is a pure function of the set)."""
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
    return P


def _batched(pmh, ctx, b):
    sig = ctx.hash_sets(pmh.to_device(b.ids), pmh.to_device(b.weights), pmh.to_device(b.offsets))
    assert ctx.status() == pmh.PMH_OK
    return sig.idx.cpu().numpy().view(np.uint32), sig.id.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("variant", [1, 3])
def test_submit_fetch_equals_batched(pmh, variant):
    print(f"serving submit/fetch PMH{variant}", flush=True)
    b = W.random_sets(900 + variant, 120, 0, 5000, "exp")
    ctx = pmh.Context(SEED, 256, variant)
    idx_b, id_b = _batched(pmh, ctx, b)
    srv = pmh.Server(ctx, slots=3, slot_elems=1 << 20, slot_sets=64)
    tickets = [srv.submit(*b.set(s)) for s in range(b.num_sets)]
    got = {}
    while len(got) < len(tickets):
        for s, t in enumerate(tickets):
            if s not in got:
                r = srv.fetch(t)
                if r is not None:
                    got[s] = r
    for s in range(b.num_sets):
        idx, val, idv = got[s]
        assert np.array_equal(idx, idx_b[s]) and np.array_equal(idv, id_b[s]), s
    st = srv.stats()
    assert st["done"] == b.num_sets and st["batches"] >= 1
    srv.close()
    ctx.close()


def test_replay_alone_vs_mixed(pmh):
    """Poisson arrivals at 50k/s (requests overlap on the device) give the
    same signatures as each request hashed alone."""
    print("serving replay", flush=True)
    rq = W.serving_requests(num_requests=400, n_hi=20000)
    ctx = pmh.Context(SEED, 1024, 3)
    srv = pmh.Server(ctx, slots=4, slot_elems=1 << 21, slot_sets=512)
    lat, idx, idv, wall = srv.replay(rq.ids, rq.weights, rq.offsets, rq.meta["arrival"])
    st = srv.stats()
    srv.close()
    assert np.isfinite(lat).all() and (lat > 0).all() and wall > 0
    assert st["done"] == rq.num_sets
    idx_b, id_b = _batched(pmh, ctx, rq)
    assert np.array_equal(idx, idx_b) and np.array_equal(idv, id_b)
    # a few requests alone in a one-slot server, one at a time
    alone = pmh.Server(ctx, slots=1, slot_elems=1 << 20, slot_sets=1)
    for s in (0, 7, 123, 399):
        t = alone.submit(*rq.set(s))
        r = None
        while r is None:
            r = alone.fetch(t)
        assert np.array_equal(r[0], idx_b[s]) and np.array_equal(r[2], id_b[s])
    alone.close()
    # and against the CPU reference for a sample
    for s in (3, 200):
        ids, w = rq.set(s)
        want = O.decode(O.sign(3, SEED, 1024, ids, w), ids)
        assert np.array_equal(idx[s], want[0]) and np.array_equal(idv[s], want[2])
    ctx.close()
