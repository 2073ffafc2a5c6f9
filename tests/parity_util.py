"""Helpers for the GPU-vs-oracle parity tests (tolerances and comparisons).

Bit-exact: hit indices, done, flags, rewards, the whole FP32 state, range
observations when sigma = 0, velocity and distance observations.
Tolerances (derived in the design notes):
  noisy ranges (normalised): 2e-6 absolute -- the GPU draws the Gaussian with
      FP32 log/cospi (a few ulp) against the oracle's FP64 Box-Muller, times
      sigma <= 2 cells, divided by the range;
  bearing / pi: 2e-6 absolute (FP32 atan2 within a few ulp of FP64, on
      bit-identical arguments).
"""
from __future__ import annotations

import numpy as np

RANGE_TOL = 2e-6
BEARING_TOL = 2e-6


def to_np(t):
    return t.detach().cpu().numpy()


def compare_obs(g, o, n_rays, noisy=True, where=""):
    g = np.asarray(g, np.float32)
    o = np.asarray(o, np.float32)
    assert g.shape == o.shape, where
    rg, ro = g[:, :n_rays], o[:, :n_rays]
    if noisy:
        d = np.abs(rg.astype(np.float64) - ro)
        assert d.max() <= RANGE_TOL, f"{where}: range obs differ by {d.max()} at {np.unravel_index(d.argmax(), d.shape)}"
    else:
        bad = np.argwhere(rg.view(np.uint32) != ro.view(np.uint32))
        assert bad.size == 0, f"{where}: range obs not bit-exact at {bad[:5]}: {rg[tuple(bad[0])]} vs {ro[tuple(bad[0])]}"
    ex = g[:, n_rays:n_rays + 3].view(np.uint32) != o[:, n_rays:n_rays + 3].view(np.uint32)
    assert not ex.any(), f"{where}: velocity/distance obs not bit-exact at {np.argwhere(ex)[:5]}"
    b = np.abs(g[:, n_rays + 3].astype(np.float64) - o[:, n_rays + 3])
    b = np.minimum(b, np.abs(b - 2.0))  # bearing wraps at +-1
    assert b.max() <= BEARING_TOL, f"{where}: bearing differs by {b.max()}"


def compare_state(gf, gi, of, oi, where=""):
    bad = np.argwhere(gf.view(np.uint32) != of.view(np.uint32))
    assert bad.size == 0, f"{where}: float state differs at (env, field) {bad[:5]}: {gf[tuple(bad[0])]!r} vs {of[tuple(bad[0])]!r}"
    badi = np.argwhere(gi != oi)
    assert badi.size == 0, f"{where}: int state differs at {badi[:5]}"


def compare_exact(g, o, name, where=""):
    g = np.asarray(g)
    o = np.asarray(o)
    if g.dtype == np.float32:
        bad = np.argwhere(g.view(np.uint32) != o.astype(np.float32).view(np.uint32))
    else:
        bad = np.argwhere(g != o)
    assert bad.size == 0, f"{where}: {name} differs at {bad[:5]}: {g[tuple(bad[0])]} vs {o[tuple(bad[0])]}"
