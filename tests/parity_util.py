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
    if g.shape[0] == 0:
        return
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


# ---- the actor: which greedy choices the kernel's precision cannot flip -------
def bf16_round(x):
    """Values rounded to bf16 (nearest even), as float64."""
    from paper_2305_04180_amd import inputs
    bits = inputs._to_bf16_bits(np.asarray(x, np.float32)).astype(np.uint32) << 16
    return bits.view(np.float32).astype(np.float64)


def qnet_f64_weights(dims, w):
    wf = (np.asarray(w).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    d0, h1, h2, A = dims
    W1 = wf[:h1 * d0].reshape(h1, d0)
    W2 = wf[h1 * d0:h1 * d0 + h2 * h1].reshape(h2, h1)
    W3 = wf[h1 * d0 + h2 * h1:].reshape(A, h2)
    return W1, W2, W3


def qnet_bound(dims, w, b, obs, in_tol=0.0):
    """First-order bound (Higham) on |Q_kernel - Q_fp64| per (row, action),
    from oracle-side values only: hidden activations stored in bf16 (relative
    u = 2^-9 each) and FP32 accumulation over K terms (gamma ~ K 2^-24),
    propagated with |W|; plus, when the kernel's input may differ from `obs`
    by up to in_tol per entry (noisy ranges, bearing), the change of every
    entry whose bf16 rounding that can flip, pushed through |W1|, |W2|, |W3|."""
    W1, W2, W3 = qnet_f64_weights(dims, w)
    h1, h2 = dims[1], dims[2]
    b = np.asarray(b, np.float64)
    obs = np.asarray(obs, np.float32)
    xb = bf16_round(obs)
    a1 = np.maximum(xb @ W1.T + b[:h1], 0)
    a2 = np.maximum(a1 @ W2.T + b[h1:h1 + h2], 0)
    u, gam = 2.0 ** -9, max(h1, h2) * 2.0 ** -24
    aW2, aW3 = np.abs(W2), np.abs(W3)
    bound = (u + gam) * (a2 @ aW3.T + (a1 @ aW2.T) @ aW3.T) + 1e-6
    if in_tol > 0:
        lo = bf16_round(obs.astype(np.float64) - in_tol)
        hi = bf16_round(obs.astype(np.float64) + in_tol)
        dx = np.maximum(np.abs(hi - xb), np.abs(lo - xb))
        if dx.any():
            bound = bound + ((dx @ np.abs(W1).T) @ aW2.T) @ aW3.T
    return bound


def _bf16_relu(z):
    """bf16(binary32(relu(z))): the kernel's activation store, monotone in z."""
    return bf16_round(np.maximum(z, 0.0).astype(np.float32))


def qnet_rounded_bound(dims, w, b, obs, in_tol=0.0):
    """Bound per (row, action) on |Q_kernel - Q_bf16act|, where Q_bf16act is
    the oracle's Q-network with hidden activations rounded to bf16
    (qnet_f64(..., round_act=True)). The kernel accumulates each layer in
    FP32 (error <= gamma_K sum |w x|, gamma_K ~ K 2^-24) before rounding to
    bf16, so a stored activation can differ from the oracle's only where that
    error (plus what earlier differences carry forward) reaches a bf16
    rounding boundary; the monotone store maps the error interval of each
    pre-activation to the interval of activations it can produce. Inputs may
    differ from `obs` by in_tol per entry. Oracle-side values only."""
    W1, W2, W3 = qnet_f64_weights(dims, w)
    d0, h1, h2, _ = dims
    b = np.asarray(b, np.float64)
    b1, b2, b3 = b[:h1], b[h1:h1 + h2], b[h1 + h2:]
    obs = np.asarray(obs, np.float32)
    aW1, aW2, aW3 = np.abs(W1), np.abs(W2), np.abs(W3)
    g = lambda k: (k + 2) * 2.0 ** -24  # FP32 sum of k products and a bias
    xb = bf16_round(obs)
    dx = np.zeros_like(xb)
    if in_tol > 0:
        lo = bf16_round(obs.astype(np.float64) - in_tol)
        hi = bf16_round(obs.astype(np.float64) + in_tol)
        dx = np.maximum(np.abs(hi - xb), np.abs(lo - xb))
    z1 = xb @ W1.T + b1
    e1 = g(d0) * ((np.abs(xb) + dx) @ aW1.T + np.abs(b1)) + dx @ aW1.T
    a1 = _bf16_relu(z1)
    d1 = np.maximum(np.abs(_bf16_relu(z1 + e1) - a1), np.abs(_bf16_relu(z1 - e1) - a1))
    z2 = a1 @ W2.T + b2
    e2 = g(h1) * ((a1 + d1) @ aW2.T + np.abs(b2)) + d1 @ aW2.T
    a2 = _bf16_relu(z2)
    d2 = np.maximum(np.abs(_bf16_relu(z2 + e2) - a2), np.abs(_bf16_relu(z2 - e2) - a2))
    q = a2 @ W3.T + b3
    eq = g(h2 + 8) * ((a2 + d2) @ aW3.T + np.abs(b3)) + d2 @ aW3.T + 1e-7 * (1 + np.abs(q))
    return eq


def settled_greedy(q64, bound):
    """Oracle greedy action per row and whether no error within `bound` can
    change it (gap to the runner-up above both rows' bounds)."""
    order = np.argsort(-q64, 1, kind="stable")
    top, second = order[:, 0], order[:, 1]
    rows = np.arange(len(q64))
    gap = q64[rows, top] - q64[rows, second]
    return top, gap > bound[rows, top] + bound[rows, second]


def compare_reward(g, o, tol, where=""):
    """Rewards: bit-exact (tol = 0), or within tol where the reward has an
    atan2 term (Eq. (11)'s r_alpha; FP32 atan2 within a few ulp of FP64)."""
    if tol == 0:
        compare_exact(g, o, "reward", where)
        return
    d = np.abs(np.asarray(g, np.float64) - np.asarray(o, np.float64))
    assert d.size == 0 or d.max() <= tol, f"{where}: reward differs by {d.max()}"


def compare_obs_relative(g, o, n_rays, noisy=True, where=""):
    """Relative-pose observations [ranges | (x-tx)/D, (y-ty)/D, alpha/pi,
    v_l/v_max, v_a/omega_max]: ranges as compare_obs, the pose and velocity
    entries bit-exact, alpha/pi within BEARING_TOL (wrapping at +-1)."""
    g = np.asarray(g, np.float32)
    o = np.asarray(o, np.float32)
    assert g.shape == o.shape, where
    rg, ro = g[:, :n_rays], o[:, :n_rays]
    if noisy:
        d = np.abs(rg.astype(np.float64) - ro)
        assert d.size == 0 or d.max() <= RANGE_TOL, f"{where}: range obs differ by {d.max()}"
    else:
        assert np.array_equal(rg.view(np.uint32), ro.view(np.uint32)), f"{where}: range obs"
    for k in (0, 1, 3, 4):
        col = n_rays + k
        bad = np.argwhere(g[:, col].view(np.uint32) != o[:, col].view(np.uint32))
        assert bad.size == 0, f"{where}: state entry {k} differs at rows {bad[:5].ravel()}"
    b = np.abs(g[:, n_rays + 2].astype(np.float64) - o[:, n_rays + 2])
    b = np.minimum(b, np.abs(b - 2.0))
    assert b.size == 0 or b.max() <= BEARING_TOL, f"{where}: alpha differs by {b.max()}"


def actor_lockstep(orc, dims, w, b, eps, o_obs, acts, rew, done, where, reward_tol=0.0,
                   obs_steps=None, hits_steps=None, live=None, min_live=0.9):
    """Step the oracle with its own FP64 actor + VEM next to a GPU rollout
    (acts, rew, done: [K][N]) and compare; eps is the per-env VEM array, or
    a function of the step index giving it. Explored actions equal the
    oracle's draw; a greedy action equals the oracle's bf16-activation argmax
    wherever qnet_rounded_bound settles it; an env stays compared while its
    actions equal the FP64 actor's (its trajectory is then the oracle's).
    With obs_steps / hits_steps ([K][N][...] from a traced rollout), every
    step's observation and hit indices of the compared envs are checked too.
    live: the envs still on the oracle's trajectory when the rollout starts
    (default all); at least min_live of them must stay on it.
    Returns the mask of envs compared to the end and the oracle's last
    observation."""
    import oracle
    K, N = acts.shape
    live = np.ones(N, bool) if live is None else live.copy()
    n_settled = n_greedy = n_agree = 0
    for t in range(K):
        q64 = oracle.qnet_f64(dims, w, b, o_obs)
        a_o, ex = orc.vem(q64, eps(t) if callable(eps) else eps)
        exb = ex.astype(bool)
        q_ra = oracle.qnet_f64(dims, w, b, o_obs, round_act=True)
        top, settled = settled_greedy(q_ra, qnet_rounded_bound(dims, w, b, o_obs, RANGE_TOL))
        w_ = f"{where} t={t}"
        compare_exact(acts[t][live & exb], a_o[live & exb], "explored actions", w_)
        m = live & ~exb & settled
        compare_exact(acts[t][m], top[m], "settled greedy actions", w_)
        n_greedy += int((live & ~exb).sum())
        n_settled += int(m.sum())
        n_agree += int((live & ~exb & (acts[t] == a_o)).sum())
        live &= acts[t] == a_o
        r = orc.step(a_o, hit_k=hits_steps is not None)
        compare_reward(rew[t][live], r["reward"][live], reward_tol, w_)
        compare_exact(done[t][live], r["done"][live], "done", w_)
        if hits_steps is not None:
            compare_exact(hits_steps[t][live], r["hit_k"][live], "hit_k", w_)
        if obs_steps is not None:
            compare_obs(obs_steps[t][live], r["obs"][live], obs_steps.shape[2] - 4, True, w_ + " obs")
        o_obs = r["obs"]
    print(f"{where}: {live.sum()} of {N} envs compared over {K} steps; {n_settled} of "
          f"{n_greedy} greedy choices settled by the bound; agreement with the FP64 actor "
          f"{n_agree / max(n_greedy, 1):.5f}", flush=True)
    assert live.mean() >= min_live, (live.sum(), N)
    assert n_agree >= 0.995 * n_greedy
    return live, o_obs


def qnet_f64_threads(dims, w, b, obs, round_act=False, workers=16):
    """oracle.qnet_f64 over row chunks on a thread pool (the C call releases
    the GIL); same values as one call."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    obs = np.ascontiguousarray(obs, np.float32)
    if obs.shape[0] < 4096:
        return oracle.qnet_f64(dims, w, b, obs, round_act=round_act)
    chunks = np.array_split(obs, 4 * workers)
    with ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(lambda c: oracle.qnet_f64(dims, w, b, c, round_act=round_act), chunks))
    return np.concatenate(parts)


class ExploreDraws:
    """VEM exploration flags of n envs by global step, from the oracle's own
    VEM (the envs share one small map: only the draw counters matter)."""

    def __init__(self, seed, n, eps):
        import oracle
        from paper_2305_04180_amd import inputs
        cfg = inputs.workload("c2", n_envs=n, seed=seed)
        maps = inputs.single_maps([np.zeros((16, 16), np.uint8)], n_envs=n)
        self.orc = oracle.Oracle(cfg, maps)
        self.eps = np.ascontiguousarray(eps, np.float32)
        self.q0 = np.zeros((n, 7))

    def flags(self, g):
        self.orc.global_step = int(g)
        _, ex = self.orc.vem(self.q0, self.eps)
        return ex.astype(bool)


def traced_actor_rows(env, launches, K, sample):
    """Fused rollouts with every step traced (sparrow_rollout_trace): for the
    sampled envs, the observation each step's actor saw, the action it took
    and the global step, row by row (step-major)."""
    import torch
    prev = to_np(env.obs)[sample]
    obs_in, acts, steps = [], [], []
    for _ in range(launches):
        g0 = env.global_step
        a, _, _, _, obs_t, _ = env.rollout_trace(K, True)
        torch.cuda.synchronize()
        o = to_np(obs_t)[:, sample]
        obs_in.append(np.concatenate([prev[None], o[:-1]]))
        acts.append(to_np(a)[:, sample])
        steps.append(g0 + np.arange(K))
        prev = o[-1]
    return np.concatenate(obs_in), np.concatenate(acts), np.concatenate(steps)
