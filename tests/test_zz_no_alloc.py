"""The no-allocation entry point pmh_hash_sets_noalloc against pmh_hash_sets:
bit-exact keys, positions, values and ids on two calls in a row, the second
with a smaller batch (the static work buffer keeps the first call's contents),
split sets included; more sets than the buffer holds are refused before any
device work."""
import ctypes

import numpy as np
import pytest

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


def _batch(seed, num_sets, hi, big):
    b = W.random_sets(seed, num_sets, 0, hi, "pareto")
    if not big:
        return b
    rng = np.random.default_rng(seed)
    n = 40000  # split into chunks at the default split threshold 2^15
    ids = np.concatenate([b.ids, rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64)])
    w = np.concatenate([b.weights, rng.exponential(size=n)])
    off = np.concatenate([b.offsets, [b.offsets[-1] + n]]).astype(np.uint64)
    return W.Batch(ids, w, off)


def _all(sig):
    return [getattr(sig, k).cpu().numpy().view(np.uint64 if k in ("id", "keys") else
                                               np.uint32 if k == "idx" else np.float64)
            for k in ("keys", "idx", "val", "id")]


@pytest.mark.parametrize("variant,m", [(1, 1024), (2, 64), (3, 256), (4, 64)])
def test_noalloc_equals_batched(pmh, variant, m):
    print(f"noalloc PMH{variant} m={m}", flush=True)
    ctx = pmh.Context(SEED, m, variant)
    batches = [_batch(1000 + variant, 3000, 600, True), _batch(2000 + variant, 700, 200, False)]
    args = [[pmh.to_device(b.ids), pmh.to_device(b.weights), pmh.to_device(b.offsets)] for b in batches]
    got = [ctx.hash_sets(*a, mode="noalloc") for a in args]  # two calls in a row, the second smaller
    assert ctx.status() == pmh.PMH_OK
    want = [ctx.hash_sets(*a) for a in args]
    assert ctx.status() == pmh.PMH_OK
    for gs, ws in zip(got, want):
        for g, w in zip(_all(gs), _all(ws)):
            assert np.array_equal(g.view(np.uint64) if g.dtype == np.float64 else g,
                                  w.view(np.uint64) if w.dtype == np.float64 else w)
    ctx.close()


def test_noalloc_limit(pmh):
    """2^20 + 1 sets are refused with PMH_ERR_SCRATCH_LIMIT before anything
    is read or enqueued."""
    import torch
    ctx = pmh.Context(SEED, 16, 1)
    d = torch.zeros(4, dtype=torch.int64, device="cuda")
    p = ctypes.c_void_p(d.data_ptr())
    rc = pmh.lib().pmh_hash_sets_noalloc(ctx._c, p, p, p, (1 << 20) + 1, None, None, None, p, None)
    assert rc == pmh.PMH_ERR_SCRATCH_LIMIT
    torch.cuda.synchronize()
    ctx.close()
