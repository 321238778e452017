"""Stored tunings: pmh_tuning_save / pmh_tuning_load key a tuning by the
device architecture, compute-unit count, m and variant; autotune with a cache
file reuses a stored result.  Tunings never change a signature."""
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


def test_save_load_keyed(pmh, tmp_path):
    path = str(tmp_path / "tune.txt")
    ctx = pmh.Context(SEED, 256, 1)
    ctx.set_tuning(c0=2.5, waves=1, chain_expect=33.0, split_log2=12)
    ctx.save_tuning(path)
    want = ctx.get_tuning().as_dict()
    ctx.set_tuning(c0=4.0)
    ctx.save_tuning(path)  # replaces the line of the same key
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and "gfx" in lines[0]
    other = pmh.Context(SEED, 512, 1)
    other.save_tuning(path)
    assert len(open(path).read().splitlines()) == 2
    fresh = pmh.Context(SEED, 256, 1)
    assert fresh.load_tuning(path)
    got = fresh.get_tuning().as_dict()
    assert got == dict(want, c0=4.0)
    assert not pmh.Context(SEED, 256, 3).load_tuning(path)
    assert not pmh.Context(SEED, 128, 1).load_tuning(path)
    # a loaded tuning changes no signature
    b = W.random_sets(3, 30, 0, 400, "pareto")
    d = [pmh.to_device(a) for a in (b.ids, b.weights, b.offsets)]
    k1 = fresh.hash_sets(*d).keys.cpu().numpy().view(np.uint64)
    assert np.array_equal(k1, O.sign_batch(1, SEED, 256, b.ids, b.weights, b.offsets, nthreads=8))


def test_autotune_cache(pmh, tmp_path):
    path = str(tmp_path / "tune.txt")
    b = W.random_sets(4, 200, 1, 300, "exp")
    d = [pmh.to_device(a) for a in (b.ids, b.weights, b.offsets)]
    ctx = pmh.Context(SEED, 128, 3)
    best = ctx.autotune(*d, trials=1, cache=path)
    again = pmh.Context(SEED, 128, 3)
    assert again.autotune(*d, trials=1, cache=path) == best
    assert again.get_tuning().as_dict() == best


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_default_tuning(pmh, variant):
    """pmh_init's defaults per variant and m (documented in pmh.h): thresholds,
    waves per workgroup, chain threshold and split threshold."""
    for m, waves in ((256, 2), (1024, 2), (2048, (4, 2, 4, 2)[variant - 1]), (4096, (4, 8, 4, 8)[variant - 1]),
                     (8192, 4)):
        t = pmh.Context(SEED, m, variant).get_tuning().as_dict()
        assert t["waves"] == waves, (m, t)
        assert t["c0"] == (2.0 if variant == 3 else 3.0)
        assert t["grow"] == (1.35 if variant == 3 else 2.0)
        assert t["chain_expect"] == {1: 48.0, 2: 16.0, 3: 48.0, 4: 32.0}[variant]
        assert t["split_log2"] == (16 if m > 2048 else 15)
