"""GPU parity of the collection loop pieces (Sec. 3.1.2, Alg. 1 steps 2-5 and
Alg. 2 step 1): the device experience buffer against the oracle's ring, the
68-512-512-7 actor against the FP64 oracle, and a small act -> step -> add ->
sample loop of the full-collection workload next to the oracle's own loop."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2305_04180_amd import inputs
from tests.parity_util import (BEARING_TOL, RANGE_TOL, compare_exact, compare_obs,
                               compare_state, qnet_bound, qnet_rounded_bound, settled_greedy,
                               to_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def banner(msg):
    print(f"\n[case] {msg}", flush=True)


def synthetic(rng, n, nr):
    """Seeded transitions with the observation layout, including values on
    and next to the storage format's rounding ties."""
    D = nr + 4
    s = rng.uniform(-0.1, 1.1, size=(n, D)).astype(np.float32)
    s[:, nr:] = rng.normal(0, 2, size=(n, 4)).astype(np.float32)
    sn = rng.uniform(0, 1, size=(n, D)).astype(np.float32)
    sn[:, nr:] = rng.normal(0, 0.5, size=(n, 4)).astype(np.float32)
    sf = rng.uniform(0, 1, size=(n, D)).astype(np.float32)
    special_r = np.array([0.5, 1.5 / 255, 2.5 / 255, 0.0, 1.0, -0.0, 254.5 / 255], np.float32)
    special_h = np.array([1 + 2 ** -11, 1 + 3 * 2 ** -11, 3 * 2 ** -25, 65520.0, 65504.0,
                          -2 ** -24, 1e-30], np.float32)
    for k in range(min(n, len(special_r))):
        s[k, k % nr] = special_r[k]
        s[k, nr + k % 4] = special_h[k]
    a = rng.integers(0, 7, n).astype(np.int32)
    r = rng.normal(size=n).astype(np.float32)
    d = (rng.random(n) < 0.3).astype(np.uint8)
    return s, a, r, sn, d, sf


def to_gpu(torch, *arrs):
    return [torch.as_tensor(np.ascontiguousarray(x)).cuda() for x in arrs]


def compare_read(g, o, where):
    names = ("s", "a", "r", "s_next", "done")
    for gi, oi, nm in zip(g, o, names):
        compare_exact(to_np(gi), oi, nm, where)


def test_ring_push_gather_sample_match_oracle(torch_gpu):
    """Pushes of assorted sizes (empty, full, wrapping), with and without
    terminal observations: every stored slot and every sample bit-exact."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    for cap, nr in ((1000, 64), (37, 32), (4096, 7)):
        banner(f"ring cap={cap} n_rays={nr}")
        ring = sparrow.Ring(cap, nr, seed=123)
        oring = oracle.Ring(cap, nr, seed=123)
        rng = np.random.default_rng(cap)
        for step, n in enumerate((min(300, cap), 0, cap, 17 % cap or 1, min(999, cap), 5)):
            s, a, r, sn, d, sf = synthetic(rng, n, nr)
            use_final = step % 2 == 0
            gs, ga, gr, gsn, gd, gsf = to_gpu(torch, s, a, r, sn, d, sf)
            ring.push(gs, ga, gr, gsn, gd, gsf if use_final else None)
            oring.push(s, a, r, sn, d, sf if use_final else None)
            assert (ring.size, ring.head) == (oring.size, oring.head)
            slots = np.arange(ring.size)
            got = ring.gather(slots)
            torch.cuda.synchronize()
            compare_read(got, oring.gather(slots), f"cap {cap} push {step}")
            for draw in (0, 1, 2**31 + 5):
                *vals, idx = ring.sample(256, draw)
                torch.cuda.synchronize()
                *ovals, oidx = oring.sample(256, draw)
                compare_exact(to_np(idx), oidx.astype(np.int32), "idx", f"draw {draw}")
                compare_read(vals, ovals, f"cap {cap} push {step} draw {draw}")
        assert ring.status() == 0


def test_ring_errors(torch_gpu):
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    banner("ring argument errors")
    ring = sparrow.Ring(8, 4)
    with pytest.raises(sparrow.SparrowError):
        ring.sample(4, 0)  # empty
    s, a, r, sn, d, _ = synthetic(np.random.default_rng(0), 9, 4)
    gs, ga, gr, gsn, gd = to_gpu(torch, s, a, r, sn, d)
    with pytest.raises(sparrow.SparrowError):
        ring.push(gs, ga, gr, gsn, gd)  # 9 > capacity
    with pytest.raises(ValueError):
        ring.push(gs[:3], ga[:4], gr[:4], gsn[:4], gd[:4])  # short buffer
    ring.push(gs[:3].contiguous(), ga[:3].contiguous(), gr[:3].contiguous(),
              gsn[:3].contiguous(), gd[:3].contiguous())
    with pytest.raises(sparrow.SparrowError):
        ring.gather([3])  # only slots 0..2 are stored
    assert ring.status() == 0 and ring.size == 3


def test_ring_full_capacity_2_22(torch_gpu):
    """2^22 slots of 64-ray transitions (the full-collection workload's
    buffer), filled past one wrap by 129 adds of 32768; samples bit-exact."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    cap, nr, n = 1 << 22, 64, 32768
    banner(f"ring cap=2^22 n_rays=64, 129 adds of {n}")
    ring = sparrow.Ring(cap, nr, seed=5)
    oring = oracle.Ring(cap, nr, seed=5)
    rng = np.random.default_rng(22)
    batches = [synthetic(rng, n, nr) for _ in range(3)]
    gpu_batches = [to_gpu(torch, *bt) for bt in batches]
    for k in range(129):
        s, a, r, sn, d, sf = batches[k % 3]
        gs, ga, gr, gsn, gd, gsf = gpu_batches[k % 3]
        ring.push(gs, ga, gr, gsn, gd, gsf)
        oring.push(s, a, r, sn, d, sf)
    assert ring.size == oring.size == cap and ring.head == oring.head == n
    for draw in range(8):
        *vals, idx = ring.sample(256, draw)
        torch.cuda.synchronize()
        *ovals, oidx = oring.sample(256, draw)
        compare_exact(to_np(idx), oidx.astype(np.int32), "idx", f"draw {draw}")
        compare_read(vals, ovals, f"2^22 draw {draw}")
    # the oldest slots hold the last adds (the wrap overwrote the first)
    slots = np.array([0, n - 1, n, cap - 1])
    compare_read(ring.gather(slots), oring.gather(slots), "2^22 wrap edges")


def _actor512(env, cfg):
    from paper_2305_04180_amd import sparrow
    dims = (env.obs_dim, 512, 512, 7)
    w, b, _ = inputs.qnet_weights(dims)
    import oracle
    eps = oracle.vem_epsilon(env.n, env.n, 0.01, 0.29)
    env.set_qnet(dims, w, b, env.vem_epsilon(env.n, 0.01, 0.29))
    return dims, w, b, eps


def test_actor_512_forward_parity(torch_gpu):
    """68-512-512-7 in BF16 on MFMA (weights streamed from L2) vs the FP64
    oracle on the oracle's observations plus random rows; a ragged row count
    spanning many 64-row passes."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    cfg = inputs.workload("c5", n_envs=50)
    banner("actor 68-512-512-7 forward on 3203 rows")
    maps = inputs.make_maps(cfg)
    env = sparrow.Env(cfg, maps)
    orc = oracle.Oracle(cfg, maps)
    dims, w, b, eps = _actor512(env, cfg)
    rows = [orc.reset()[0]]
    for _ in range(20):
        rows.append(orc.step(orc.uniform_actions())["obs"])
    rng = np.random.default_rng(11)
    rows.append(rng.uniform(-1.2, 1.2, size=(2153, 68)).astype(np.float32))
    obs = np.concatenate(rows)
    assert obs.shape == (3203, 68)
    q, greedy = env.qnet_forward(torch.as_tensor(obs).cuda())
    torch.cuda.synchronize()
    q = to_np(q).astype(np.float64)
    greedy = to_np(greedy)
    q64 = oracle.qnet_f64(dims, w, b, obs)
    bound = qnet_bound(dims, w, b, obs)
    dq = np.abs(q - q64)
    print(f"max|dQ| {dq.max():.2e}, max dQ/bound {(dq / bound).max():.3f}", flush=True)
    assert np.all(dq <= bound), (dq.max(), (dq / bound).max())
    top, settled = settled_greedy(q64, bound)
    assert np.array_equal(greedy[settled], top[settled])
    agree = (greedy == q64.argmax(1)).mean()
    q_ra = oracle.qnet_f64(dims, w, b, obs, round_act=True)
    eq = qnet_rounded_bound(dims, w, b, obs)
    assert np.all(np.abs(q - q_ra) <= eq), (np.abs(q - q_ra) / eq).max()
    top_ra, settled_ra = settled_greedy(q_ra, eq)
    assert np.array_equal(greedy[settled_ra], top_ra[settled_ra])
    print(f"greedy agreement with FP64 {agree:.5f}; bf16-activation oracle: max|dQ| "
          f"{np.abs(q - q_ra).max():.2e}, settled {settled_ra.mean():.4f}", flush=True)
    # the FP32 summation bound over 512 terms is worst case: about 90 % of
    # the rows are settled by it (an emulation of the kernel's arithmetic on
    # the CPU stays below a tenth of the bound)
    assert agree >= 0.995 and settled_ra.mean() >= 0.85
    q7, g7 = env.qnet_forward(torch.as_tensor(obs[:7]).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(to_np(g7), greedy[:7])
    with pytest.raises(sparrow.SparrowError):
        env.rollout(4, True)  # the fused rollout needs the width-256 actor


def _near_level_tie(x, tol):
    """Ranges within tol of a rounding tie of the uint8 levels."""
    p = np.clip(x.astype(np.float64), 0, 1) * 255.0
    return np.abs(p - np.floor(p) - 0.5) <= tol * 255.0 + 1e-9


def _f16_unsettled(x, tol):
    import oracle
    out = np.zeros(x.shape, bool)
    for k, v in np.ndenumerate(x):
        c = oracle.f16_rne(float(v))
        out[k] = oracle.f16_rne(float(v) - tol) != c or oracle.f16_rne(float(v) + tol) != c
    return out


def _compare_stored_obs(g, o, raw, nr, where):
    """A transition read back from the GPU ring vs the oracle ring's, where
    the GPU stored its own observation (noisy ranges and the bearing within
    tolerance of the oracle's): levels and binary16 codes are equal except
    where the oracle's raw value lies within that tolerance of a rounding
    tie, where the neighbouring code is allowed."""
    g, o = np.asarray(g, np.float32), np.asarray(o, np.float32)
    lv_g, lv_o = np.rint(g[:, :nr] * 255.0), np.rint(o[:, :nr] * 255.0)
    tie = _near_level_tie(raw[:, :nr], RANGE_TOL)
    dl = np.abs(lv_g - lv_o)
    assert np.all(dl[~tie] == 0) and np.all(dl <= 1), f"{where}: range levels differ"
    compare_exact(g[:, nr:nr + 3], o[:, nr:nr + 3], "stored scalars", where)
    bg, bo = g[:, nr + 3], o[:, nr + 3]
    uns = _f16_unsettled(raw[:, nr + 3], BEARING_TOL)
    assert np.array_equal(bg[~uns].view(np.uint32), bo[~uns].view(np.uint32)), f"{where}: bearing"
    assert np.all(np.abs(bg - bo) <= 2 * np.spacing(np.abs(bo).astype(np.float16)).astype(np.float32) + 1e-12)


def test_collection_loop_small(torch_gpu):
    """The full-collection workload at N = 40 for 24 steps: width-512 actor +
    VEM, the step with AutoReset, an add of (s, a, r, s', done) every step and
    a 256-draw sample every 8 steps, next to the same loop run by the oracle
    with its own FP64 actor."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    cfg = inputs.workload("c5", n_envs=40)
    N, T, nr = 40, 24, cfg["n_rays"]
    D = nr + 4
    banner(f"collection loop N={N}, {T} steps")
    maps = inputs.make_maps(cfg)
    env = sparrow.Env(cfg, maps)
    orc = oracle.Oracle(cfg, maps)
    dims, w, b, eps = _actor512(env, cfg)
    ring = sparrow.Ring(1 << 12, nr, seed=9)
    oring = oracle.Ring(1 << 12, nr, seed=9)
    cur = env.reset()
    nxt = torch.zeros_like(cur)
    fo = torch.zeros_like(cur)
    act = torch.zeros(N, dtype=torch.int32, device=env.device)
    rew = torch.zeros(N, dtype=torch.float32, device=env.device)
    done = torch.zeros(N, dtype=torch.uint8, device=env.device)
    o_obs, _ = orc.reset()
    live = np.ones(N, bool)
    live_at = []          # live mask of each step's transitions
    raw_s, raw_sn = [], []  # the oracle's raw observations per step
    for t in range(T):
        env.act(cur, act)
        fo.zero_()
        env.step(act, obs=nxt, reward=rew, done=done, final_obs=fo)
        ring.push(cur, act, rew, nxt, done, fo)
        q64 = oracle.qnet_f64(dims, w, b, o_obs)
        a_o, ex = orc.vem(q64, eps)
        q_ra = oracle.qnet_f64(dims, w, b, o_obs, round_act=True)
        top, settled = settled_greedy(q_ra, qnet_rounded_bound(dims, w, b, o_obs, RANGE_TOL))
        r = orc.step(a_o, final_obs=True)
        sn_o = np.where(r["done"][:, None].astype(bool), r["final_obs"], r["obs"])
        oring.push(o_obs, a_o, r["reward"], r["obs"], r["done"], r["final_obs"])
        torch.cuda.synchronize()
        g_a = to_np(act)
        exb = ex.astype(bool)
        compare_exact(g_a[live & exb], a_o[live & exb], "explored actions", f"t={t}")
        m = live & ~exb & settled
        compare_exact(g_a[m], top[m], "settled greedy actions", f"t={t}")
        live &= g_a == a_o
        compare_exact(to_np(rew)[live], r["reward"][live], "reward", f"t={t}")
        compare_exact(to_np(done)[live], r["done"][live], "done", f"t={t}")
        compare_obs(to_np(nxt)[live], r["obs"][live], nr, True, f"t={t}")
        live_at.append(live.copy())
        raw_s.append(o_obs.copy())
        raw_sn.append(sn_o.copy())
        o_obs = r["obs"]
        cur, nxt = nxt, cur
        if t % 8 == 7:
            gs, ga, gr, gsn, gd, gidx = ring.sample(256, t // 8)
            torch.cuda.synchronize()
            os_, oa, orw, osn, od, oidx = oring.sample(256, t // 8)
            gidx = to_np(gidx)
            compare_exact(gidx, oidx.astype(np.int32), "sampled slots", f"t={t}")
            ts, es = gidx // N, gidx % N
            ok = np.array([live_at[ti][ei] for ti, ei in zip(ts, es)])
            assert ok.mean() >= 0.8
            rs = np.stack([raw_s[ti][ei] for ti, ei in zip(ts, es)])
            rsn = np.stack([raw_sn[ti][ei] for ti, ei in zip(ts, es)])
            _compare_stored_obs(to_np(gs)[ok], os_[ok], rs[ok], nr, f"sample {t // 8} s")
            _compare_stored_obs(to_np(gsn)[ok], osn[ok], rsn[ok], nr, f"sample {t // 8} s'")
            compare_exact(to_np(ga)[ok], oa[ok], "sampled a", f"t={t}")
            compare_exact(to_np(gr)[ok], orw[ok], "sampled r", f"t={t}")
            compare_exact(to_np(gd)[ok], od[ok], "sampled done", f"t={t}")
    print(f"{live.sum()} of {N} envs compared through {T} steps", flush=True)
    assert live.mean() >= 0.9
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf[live], gi[live], of[live], oi[live], "collection loop final")
    assert env.status() == 0 and ring.status() == 0


def _oracle_collect(orc, oring, o_obs, K, actions_fn, raw, terminal=True):
    """The oracle's side of a collecting rollout from observation o_obs: K
    steps, each adding its N transitions (s' = the terminal observation
    where done, or the post-reset one with terminal=False) to the oracle's
    ring; raw collects (s, s') per step for the tie-aware comparison.
    Returns the per-step (a, r, done) and the last observation."""
    rows = []
    for t in range(K):
        a = actions_fn(t, o_obs)
        r = orc.step(a, final_obs=True)
        if terminal:
            sn = np.where(r["done"][:, None].astype(bool), r["final_obs"], r["obs"])
            oring.push(o_obs, a, r["reward"], r["obs"], r["done"], r["final_obs"])
        else:
            sn = r["obs"]
            oring.push(o_obs, a, r["reward"], r["obs"], r["done"])
        raw.append((o_obs.copy(), sn.copy()))
        rows.append((a, r["reward"], r["done"]))
        o_obs = r["obs"]
    return rows, o_obs


def _compare_ring_slots(ring, oring, slots, raw_s, raw_sn, nr, where, mask=None):
    g = ring.gather(slots)
    o = oring.gather(slots)
    g = [to_np(x) for x in g]
    keep = np.ones(len(slots), bool) if mask is None else mask
    _compare_stored_obs(g[0][keep], o[0][keep], raw_s[keep], nr, f"{where} s")
    _compare_stored_obs(g[3][keep], o[3][keep], raw_sn[keep], nr, f"{where} s'")
    compare_exact(g[1][keep], o[1][keep], "a", where)
    compare_exact(g[2][keep], o[2][keep], "r", where)
    compare_exact(g[4][keep], o[4][keep], "done", where)


@pytest.mark.parametrize("wl,variant,terminal", [("c1", (8, 64), True), ("c2", (8, 64), True),
                                                 ("c2", (4, 32), True), ("c2", (2, 16), True),
                                                 ("c2", (8, 64), False), ("c1", (4, 16), False)])
def test_rollout_collect_uniform_matches_oracle_ring(torch_gpu, wl, variant, terminal):
    """Alg. 1 steps 2-5 in one kernel: after an add of 7 transitions, two
    collecting rollouts (K = 24, then K = 12, so the second wraps a
    1500-slot ring and overwrites slots with done bits set) with uniform
    actions; every stored slot against the oracle's ring filled by its own
    step-and-add loop, the step-major outputs and the final state against
    the oracle. terminal: s' of done transitions is the terminal observation
    (else the post-reset one)."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    cfg = inputs.workload(wl, n_envs=45)
    N, nr = 45, cfg["n_rays"]
    banner(f"collecting rollout {wl} N={N} variant={variant} terminal={terminal}, "
           f"7 added, K=24 then 12, ring 1500")
    maps = inputs.make_maps(cfg)
    env = sparrow.Env(cfg, maps)
    orc = oracle.Oracle(cfg, maps)
    env.set_variant(1, *variant)
    env.reset()
    o_obs, _ = orc.reset()
    ring = sparrow.Ring(1500, nr, seed=4)
    oring = oracle.Ring(1500, nr, seed=4)
    rng = np.random.default_rng(5)
    pre = (rng.uniform(0, 1, (7, nr + 4)).astype(np.float32), rng.integers(0, 7, 7).astype(np.int32),
           rng.normal(size=7).astype(np.float32), rng.uniform(0, 1, (7, nr + 4)).astype(np.float32),
           np.ones(7, np.uint8))  # every added transition done: its bits must be kept
    ring.push(*to_gpu(torch, *pre))
    oring.push(*pre)
    raw = []
    slot_raw = {k: (pre[0][k], pre[3][k]) for k in range(7)}
    for K in (24, 12):
        head = ring.head
        acts = torch.zeros(K, N, dtype=torch.int32, device=env.device)
        rew = torch.zeros(K, N, dtype=torch.float32, device=env.device)
        done = torch.zeros(K, N, dtype=torch.uint8, device=env.device)
        env.rollout_collect(ring, K, False, acts, rew, done, terminal_obs=terminal)
        torch.cuda.synchronize()
        first = len(raw)
        rows, o_obs = _oracle_collect(orc, oring, o_obs, K, lambda t, o: orc.uniform_actions(),
                                      raw, terminal)
        for t, (a, r, d) in enumerate(rows):
            w = f"{wl} {variant} K={K} t={t}"
            compare_exact(to_np(acts[t]), a, "actions", w)
            compare_exact(to_np(rew[t]), r, "reward", w)
            compare_exact(to_np(done[t]), d, "done", w)
            for i in range(N):
                slot_raw[(head + t * N + i) % 1500] = (raw[first + t][0][i], raw[first + t][1][i])
        assert (ring.size, ring.head) == (oring.size, oring.head)
        # every stored slot, after each rollout (the first keeps the 7 added
        # transitions and their done bits in the word it shares with them)
        slots = np.arange(ring.size)
        rs = np.stack([slot_raw[s][0] for s in slots])
        rsn = np.stack([slot_raw[s][1] for s in slots])
        _compare_ring_slots(ring, oring, slots, rs, rsn, nr, f"{wl} {variant} K={K} ring")
    # the second rollout wrapped over the 7 added transitions and the first
    # rollout's oldest ones
    assert ring.size == 1500 and ring.head == (7 + 36 * N) % 1500
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf, gi, of, oi, f"{wl} {variant} final")
    compare_obs(to_np(env.obs), o_obs, nr, wl != "c1", "final obs")
    # samples of the collected buffer
    for draw in (0, 7):
        *vals, idx = ring.sample(256, draw)
        torch.cuda.synchronize()
        *ovals, oidx = oring.sample(256, draw)
        compare_exact(to_np(idx), oidx.astype(np.int32), "idx", f"draw {draw}")
    assert env.status() == 0 and ring.status() == 0


def test_rollout_collect_fused_actor_lockstep(torch_gpu):
    """The collecting rollout with the fused BF16 actor + VEM: the oracle runs
    its own FP64 actor; transitions of envs whose actions have equalled the
    FP64 actor's so far are compared slot by slot."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    cfg = inputs.workload("c2", n_envs=45)
    N, nr, K = 45, cfg["n_rays"], 20
    banner(f"collecting fused rollout c2 N={N} K={K}")
    maps = inputs.make_maps(cfg)
    env = sparrow.Env(cfg, maps)
    orc = oracle.Oracle(cfg, maps)
    dims = (env.obs_dim, 256, 256, 7)
    w, b, _ = inputs.qnet_weights(dims)
    eps = oracle.vem_epsilon(N, N, 0.01, 0.29)
    env.set_qnet(dims, w, b, env.vem_epsilon(N, 0.01, 0.29))
    env.reset()
    o_obs, _ = orc.reset()
    ring = sparrow.Ring(2048, nr, seed=2)
    oring = oracle.Ring(2048, nr, seed=2)
    acts = torch.zeros(K, N, dtype=torch.int32, device=env.device)
    env.rollout_collect(ring, K, True, acts)
    torch.cuda.synchronize()
    g_acts = to_np(acts)
    live = np.ones(N, bool)
    live_at = []

    def fp64_actor(t, o_obs):
        nonlocal live
        a_o, ex = orc.vem(oracle.qnet_f64(dims, w, b, o_obs), eps)
        exb = ex.astype(bool)
        q_ra = oracle.qnet_f64(dims, w, b, o_obs, round_act=True)
        top, settled = settled_greedy(q_ra, qnet_rounded_bound(dims, w, b, o_obs, RANGE_TOL))
        compare_exact(g_acts[t][live & exb], a_o[live & exb], "explored actions", f"t={t}")
        m = live & ~exb & settled
        compare_exact(g_acts[t][m], top[m], "settled greedy actions", f"t={t}")
        live = live & (g_acts[t] == a_o)
        live_at.append(live.copy())
        return a_o
    raw = []
    _oracle_collect(orc, oring, o_obs, K, fp64_actor, raw)
    print(f"{live.sum()} of {N} envs compared through {K} steps", flush=True)
    assert live.mean() >= 0.9
    assert (ring.size, ring.head) == (oring.size, oring.head) == (K * N, K * N)
    slots = np.arange(K * N)
    mask = np.concatenate(live_at)
    rs = np.concatenate([x[0] for x in raw])
    rsn = np.concatenate([x[1] for x in raw])
    _compare_ring_slots(ring, oring, slots, rs, rsn, nr, "fused ring", mask)
    assert env.status() == 0 and ring.status() == 0


def test_rollout_collect_rejects_mismatched_ring(torch_gpu):
    from paper_2305_04180_amd import sparrow
    cfg = inputs.workload("c1")
    banner("collecting rollout argument errors")
    env = sparrow.Env(cfg, inputs.make_maps(cfg))
    env.reset()
    N = cfg["n_envs"]
    with pytest.raises(sparrow.SparrowError):
        env.rollout_collect(sparrow.Ring(4 * N, cfg["n_rays"] + 1), 2, False)  # ray count
    small = sparrow.Ring(4 * N - 1, cfg["n_rays"])
    with pytest.raises(sparrow.SparrowError):
        env.rollout_collect(small, 4, False)  # 4 N > capacity
    env.rollout_collect(small, 3, False)
    assert small.size == 3 * N and small.head == 3 * N
    assert env.status() == 0 and small.status() == 0


@pytest.mark.parametrize("wl,variant,terminal", [("c2", (1, 64), True), ("c3", (8, 32), True),
                                                 ("c2", (4, 16), False)])
def test_step_collect_matches_oracle_ring(torch_gpu, wl, variant, terminal):
    """The plain step that adds its transitions to the ring itself, with the
    actions given from outside (here the uniform draws, which the oracle
    makes on its own): 30 steps of 45 envs into a 1000-slot ring (it wraps),
    every stored slot against the oracle's step-and-add loop."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    cfg = inputs.workload(wl, n_envs=45)
    N, nr = 45, cfg["n_rays"]
    banner(f"collecting step {wl} N={N} variant={variant} terminal={terminal}, 30 steps, ring 1000")
    maps = inputs.make_maps(cfg)
    env = sparrow.Env(cfg, maps)
    orc = oracle.Oracle(cfg, maps)
    env.set_variant(0, *variant)
    env.reset()
    o_obs, _ = orc.reset()
    ring = sparrow.Ring(1000, nr, seed=6)
    oring = oracle.Ring(1000, nr, seed=6)
    raw, slot_raw = [], {}
    flags = torch.zeros(N, dtype=torch.uint8, device=env.device)
    for t in range(30):
        head = ring.head
        a = env.random_actions()
        env.step_collect(ring, a, flags=flags, terminal_obs=terminal)
        torch.cuda.synchronize()
        rows, o_obs = _oracle_collect(orc, oring, o_obs, 1, lambda t_, o: orc.uniform_actions(),
                                      raw, terminal)
        a_o, r_o, d_o = rows[0]
        w = f"{wl} {variant} step {t}"
        compare_exact(to_np(a), a_o, "actions", w)
        compare_exact(to_np(env.reward), r_o, "reward", w)
        compare_exact(to_np(env.done), d_o, "done", w)
        compare_obs(to_np(env.obs), o_obs, nr, True, w)
        for i in range(N):
            slot_raw[(head + i) % 1000] = (raw[-1][0][i], raw[-1][1][i])
        assert (ring.size, ring.head) == (oring.size, oring.head)
    slots = np.arange(ring.size)
    rs = np.stack([slot_raw[s][0] for s in slots])
    rsn = np.stack([slot_raw[s][1] for s in slots])
    _compare_ring_slots(ring, oring, slots, rs, rsn, nr, f"{wl} {variant} ring")
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf, gi, of, oi, f"{wl} {variant} final")
    assert env.status() == 0 and ring.status() == 0
