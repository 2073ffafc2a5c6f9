"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times (autotuned default variants, K = 64 rollouts): every env where the oracle can afford it, sampled envs otherwise."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2305_04180_amd import inputs
from tests.parity_util import actor_lockstep, compare_exact, compare_obs, compare_state, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def m_maps():
    return inputs.make_maps(inputs.workload("m"))


def banner(msg):
    print(f"\n[case] {msg}", flush=True)


def test_m4096_fused_rollout_every_env(torch_gpu, m_maps):
    """4096 envs, 366^2 maps, BF16 actor: one K = 32 fused rollout next to the oracle running its own FP64 actor on every env."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    cfg = inputs.workload("m")
    N, K = cfg["n_envs"], 32
    banner(f"fused rollout N={N} K={K} default variant")
    dims = cfg["qnet"]
    w, b, _ = inputs.qnet_weights(dims)
    eps = oracle.vem_epsilon(N, N, 0.01, 0.29)
    env = sparrow.Env(cfg, m_maps)
    env.set_qnet(dims, w, b, env.vem_epsilon(N, 0.01, 0.29))
    assert env.get_variant(1) == (8, 64)
    orc = oracle.Oracle(cfg, m_maps)
    env.reset()
    o_obs, _ = orc.reset()
    compare_obs(to_np(env.obs), o_obs, cfg["n_rays"], True, "reset")
    acts, rew, done, obs = env.rollout(K, True)
    torch.cuda.synchronize()
    live, o_obs = actor_lockstep(orc, dims, w, b, eps, o_obs, to_np(acts), to_np(rew),
                                 to_np(done), "m4096")
    # each greedy choice agrees with the FP64 actor ~99.7 % of the time, so
    # over ~26 greedy steps about 93 % of the envs keep the oracle's trajectory
    assert live.mean() >= 0.9
    compare_obs(to_np(obs)[live], o_obs[live], cfg["n_rays"], True, "final obs")
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf[live], gi[live], of[live], oi[live], "final state")
    # the next 32 steps traced (same kernel and variant): every step's
    # observation and hit indices of the envs still on the oracle's trajectory
    acts, rew, done, obs, obs_t, hits_t = env.rollout_trace(K, True)
    torch.cuda.synchronize()
    live, o_obs = actor_lockstep(orc, dims, w, b, eps, o_obs, to_np(acts), to_np(rew),
                                 to_np(done), "m4096 traced", obs_steps=to_np(obs_t),
                                 hits_steps=to_np(hits_t), live=live, min_live=0.8)
    compare_obs(to_np(obs)[live], o_obs[live], cfg["n_rays"], True, "traced final obs")
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf[live], gi[live], of[live], oi[live], "traced final state")


def test_m4096_plain_step_every_env(torch_gpu, m_maps):
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    cfg = inputs.workload("m")
    banner("plain step N=4096, 8 steps, default variant")
    env = sparrow.Env(cfg, m_maps)
    assert env.get_variant(0) == (1, 64)
    orc = oracle.Oracle(cfg, m_maps)
    env.reset()
    orc.reset()
    flags = torch.zeros(env.n, dtype=torch.uint8, device=env.device)
    for s in range(8):
        a = env.random_actions()
        env.step(a, flags=flags)
        r = orc.step(orc.uniform_actions(), hit_k=True)
        w = f"step {s}"
        compare_exact(to_np(env.debug_hits()), r["hit_k"], "hit_k", w)
        compare_exact(to_np(env.done), r["done"], "done", w)
        compare_exact(to_np(flags), r["flags"], "flags", w)
        compare_exact(to_np(env.reward), r["reward"], "reward", w)
        compare_obs(to_np(env.obs), r["obs"], cfg["n_rays"], True, w)
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf, gi, of, oi, "plain final")


def test_c3_uneven_sides_rollout_sampled(torch_gpu):
    """C3: 16384 envs with sides {64,128,256,366,512}, 64 rays, range 128,
    one persistent 64-step rollout after autotuning; the oracle steps
    every 32nd env."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    cfg = inputs.workload("c3")
    N, K = cfg["n_envs"], 64
    banner(f"c3 rollout N={N} K={K}, sampled oracle")
    maps = inputs.make_maps(cfg)
    env = sparrow.Env(cfg, maps)
    env.reset()
    rep = env.autotune(steps=4)
    print("autotune chose", rep.get("chosen"), flush=True)
    orc = oracle.Oracle(cfg, maps)
    orc.reset()
    acts, rew, done, obs = env.rollout(K, False)
    torch.cuda.synchronize()
    acts, rew, done = to_np(acts), to_np(rew), to_np(done)
    ids = np.arange(0, N, 32)
    for t in range(K):
        a = orc.uniform_actions()
        compare_exact(acts[t], a, "uniform actions", f"t={t}")
        r = orc.step_envs(ids, a)
        compare_exact(rew[t][ids], r["reward"][ids], "reward", f"t={t}")
        compare_exact(done[t][ids], r["done"][ids], "done", f"t={t}")
    compare_obs(to_np(obs)[ids], r["obs"][ids], cfg["n_rays"], True, "c3 final obs")
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf[ids], gi[ids], of[ids], oi[ids], "c3 final state")


def test_c5_full_collection_loop_sampled(torch_gpu):
    """C5 at its full size: 32768 envs on sides {256, 366, 512} (512
    distinct maps, each shared by 64 envs), 64 rays, range 128, the
    68-512-512-7 actor + VEM as a separate kernel, the step with terminal
    observations and the add of all 32768 transitions to a 2^22-slot ring,
    as the benchmark runs them. The oracle runs every 64th env with its own
    FP64 actor; while an env's actions equal the FP64 actor's, its steps
    and its stored transitions are compared."""
    import oracle
    from paper_2305_04180_amd import sparrow
    from tests.parity_util import RANGE_TOL, qnet_rounded_bound, settled_greedy
    from tests.test_gpu_collect import _compare_stored_obs
    torch = torch_gpu
    cfg = inputs.workload("c5")
    N, nr, T = cfg["n_envs"], cfg["n_rays"], 6
    banner(f"c5 full collection N={N}, {T} steps, every 64th env against the oracle")
    maps = inputs.make_maps(cfg, n_maps=512)
    maps.env_to_map = (np.arange(N) % 512).astype(np.int32)
    dims = cfg["qnet"]
    w, b, _ = inputs.qnet_weights(dims)
    eps = oracle.vem_epsilon(N, N, cfg["eps"][0], cfg["eps"][1] - cfg["eps"][0])
    env = sparrow.Env(cfg, maps)
    env.set_qnet(dims, w, b, env.vem_epsilon(N, cfg["eps"][0], cfg["eps"][1] - cfg["eps"][0]))
    cur = env.reset()
    env.autotune(steps=2)
    ring = sparrow.Ring(1 << 22, nr, seed=5)
    orc = oracle.Oracle(cfg, maps)
    o_obs, _ = orc.reset()
    ids = np.arange(0, N, 64)
    oring = oracle.Ring(T * len(ids), nr, seed=5)
    nxt, fo = torch.zeros_like(cur), torch.zeros_like(cur)
    act = torch.zeros(N, dtype=torch.int32, device=env.device)
    rew = torch.zeros(N, dtype=torch.float32, device=env.device)
    done = torch.zeros(N, dtype=torch.uint8, device=env.device)
    live = np.ones(len(ids), bool)
    live_at, raw = [], []
    for t in range(T):
        env.act(cur, act)
        fo.zero_()
        env.step(act, obs=nxt, reward=rew, done=done, final_obs=fo)
        ring.push(cur, act, rew, nxt, done, fo)
        # the oracle's own actor on the sampled envs
        q_full = np.zeros((N, dims[3]), np.float64)
        q_full[ids] = oracle.qnet_f64(dims, w, b, o_obs[ids])
        a_o, ex = orc.vem(q_full, eps)
        q_ra = oracle.qnet_f64(dims, w, b, o_obs[ids], round_act=True)
        top, settled = settled_greedy(q_ra, qnet_rounded_bound(dims, w, b, o_obs[ids], RANGE_TOL))
        r = orc.step_envs(ids, a_o, final_obs=True)
        torch.cuda.synchronize()
        g_a = to_np(act)[ids]
        exb = ex[ids].astype(bool)
        w_ = f"c5 t={t}"
        compare_exact(g_a[live & exb], a_o[ids][live & exb], "explored actions", w_)
        m = live & ~exb & settled
        compare_exact(g_a[m], top[m], "settled greedy actions", w_)
        live &= g_a == a_o[ids]
        compare_exact(to_np(rew)[ids][live], r["reward"][ids][live], "reward", w_)
        compare_exact(to_np(done)[ids][live], r["done"][ids][live], "done", w_)
        compare_obs(to_np(nxt)[ids][live], r["obs"][ids][live], nr, True, w_)
        d = r["done"][ids].astype(bool)
        sn = np.where(d[:, None], r["final_obs"][ids], r["obs"][ids])
        oring.push(o_obs[ids], a_o[ids], r["reward"][ids], r["obs"][ids], r["done"][ids],
                   r["final_obs"][ids])
        raw.append((o_obs[ids].copy(), sn))
        live_at.append(live.copy())
        o_obs = o_obs.copy()
        o_obs[ids] = r["obs"][ids]
        cur, nxt = nxt, cur
    print(f"{live.sum()} of {len(ids)} sampled envs compared through {T} steps", flush=True)
    assert live.mean() >= 0.9
    assert ring.size == T * N
    slots = np.concatenate([t * N + ids for t in range(T)])
    g = [to_np(x) for x in ring.gather(slots)]
    o = oring.gather(np.arange(T * len(ids)))
    mask = np.concatenate(live_at)
    rs = np.concatenate([x[0] for x in raw])
    rsn = np.concatenate([x[1] for x in raw])
    _compare_stored_obs(g[0][mask], o[0][mask], rs[mask], nr, "c5 ring s")
    _compare_stored_obs(g[3][mask], o[3][mask], rsn[mask], nr, "c5 ring s'")
    compare_exact(g[1][mask], o[1][mask], "ring a", "c5")
    compare_exact(g[2][mask], o[2][mask], "ring r", "c5")
    compare_exact(g[4][mask], o[4][mask], "ring done", "c5")
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    lid = ids[live]
    compare_state(gf[lid], gi[lid], of[lid], oi[lid], "c5 final state")
    assert env.status() == 0 and ring.status() == 0


def test_rollout_partial_group_after_full_group(torch_gpu):
    """One more group than the grid has workgroups (eight envs per group, one
    workgroup per CU): a workgroup stages a full group and then the last,
    partial one, whose maps do not overwrite all of the first group's words
    in LDS. Uniform actions, every env against the oracle."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    N, K = 8 * n_cu + 5, 16
    cfg = inputs.workload("c2", n_envs=N)
    banner(f"rollout uniform c2 N={N} ({n_cu} CUs) K={K}")
    maps = inputs.make_maps(cfg)
    env = sparrow.Env(cfg, maps)
    assert env.get_variant(1) == (8, 64)
    orc = oracle.Oracle(cfg, maps)
    env.reset()
    orc.reset()
    for rep in range(2):
        acts, rew, done, obs = env.rollout(K, use_qnet=False)
        torch.cuda.synchronize()
        for t in range(K):
            a = orc.uniform_actions()
            r = orc.step(a, hit_k=True)
            w = f"rollout {rep} t={t}"
            compare_exact(to_np(acts[t]), a, "actions", w)
            compare_exact(to_np(rew[t]), r["reward"], "reward", w)
            compare_exact(to_np(done[t]), r["done"], "done", w)
        compare_obs(to_np(obs), r["obs"], cfg["n_rays"], True, f"rollout {rep} final obs")
        compare_exact(to_np(env.debug_hits()), r["hit_k"], "hit_k", f"rollout {rep} final")
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf, gi, of, oi, "partial group final")
