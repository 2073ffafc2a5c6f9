"""sparrow_ring_gather_static (the read-back that allocates nothing) against
sparrow_ring_gather on the same ring and slots, through the C-ABI."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _fill(ring, torch, n, nr, seed):
    rng = np.random.default_rng(seed)
    D = nr + 4
    s = rng.uniform(-0.1, 1.1, size=(n, D)).astype(np.float32)
    sn = rng.uniform(0.0, 1.0, size=(n, D)).astype(np.float32)
    a = rng.integers(0, 7, n).astype(np.int32)
    r = rng.normal(size=n).astype(np.float32)
    d = (rng.random(n) < 0.3).astype(np.uint8)
    dev = [torch.as_tensor(x).cuda() for x in (s, a, r, sn, d)]
    ring.push(*dev)


def _same(got, want, where):
    for k, (g, w) in enumerate(zip(got, want)):
        g, w = g.cpu().numpy(), w.cpu().numpy()
        assert g.shape == w.shape, (where, k)
        assert np.array_equal(g.view(np.uint8), w.view(np.uint8)), (where, k)


def test_gather_static_matches_gather():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_04180_amd import sparrow
    print("\n[case] ring gather_static vs gather: capacity 5000, 32 rays, two calls "
          "(3000 then 17 slots), a second ring on the same GPU", flush=True)
    nr = 32
    ring = sparrow.Ring(5000, nr, seed=4)
    _fill(ring, torch, 3000, nr, 1)
    _fill(ring, torch, 2600, nr, 2)  # wraps: size 5000, head 600
    rng = np.random.default_rng(5)
    first = rng.integers(0, ring.size, 3000).astype(np.int32)
    second = rng.integers(0, ring.size, 17).astype(np.int32)
    for sl, tag in ((first, "first call"), (second, "second, smaller call")):
        want = ring.gather(sl)
        got = ring.gather_static(sl)
        torch.cuda.synchronize()
        _same(got, want, tag)
    # another ring shares the GPU's staging array; its reads are its own
    other = sparrow.Ring(64, 8, seed=9)
    _fill(other, torch, 40, 8, 3)
    sl = np.arange(39, -1, -1, dtype=np.int32)
    _same(other.gather_static(sl), other.gather(sl), "second ring")
    _same(ring.gather_static(second), ring.gather(second), "first ring again")
    # limits: at most GATHER_STATIC_MAX slots, each stored; empty is fine
    with pytest.raises(sparrow.SparrowError):
        ring.gather_static(np.zeros(sparrow.GATHER_STATIC_MAX + 1, np.int32))
    with pytest.raises(sparrow.SparrowError):
        other.gather_static(np.array([40], np.int32))
    empty = ring.gather_static(np.zeros(0, np.int32))
    assert all(t.numel() == 0 for t in empty)
    assert ring.status() == 0 and other.status() == 0
