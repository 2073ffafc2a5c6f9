"""The seeded input generators (shared by the GPU path's tests and the
oracle's): determinism, the workload recipe's ranges, and that the pooled
generator reproduces the serial one map for map."""
from __future__ import annotations

import numpy as np

from paper_2305_04180_amd import inputs


def test_pooled_maps_equal_serial_maps():
    cfg = inputs.workload("c5", n_envs=48)
    a = inputs.make_maps(cfg)
    b = inputs.make_maps(cfg, workers=4)
    assert len(a.grids) == len(b.grids) == 48
    assert all(np.array_equal(x, y) for x, y in zip(a.grids, b.grids))
    assert np.array_equal(a.env_to_map, b.env_to_map)


def test_mixed_maps_follow_the_recipe():
    cfg = inputs.workload("c5", n_envs=24)
    maps = inputs.make_maps(cfg)
    for g in maps.grids:
        side = g.shape[0]
        assert g.shape == (side, side) and side in cfg["sides"]
        assert g[0].all() and g[-1].all() and g[:, 0].all() and g[:, -1].all()
        fill = g.mean()
        # border plus shapes up to a per-map fill drawn from U[0.05, 0.20]
        # (the last shape may overshoot a little)
        assert 0.05 <= fill <= 0.26, fill
