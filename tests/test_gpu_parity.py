"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle.

Every case prints its name, sizes and seed before touching the GPU.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2305_04180_amd import inputs
from tests.parity_util import actor_lockstep, qnet_bound, qnet_rounded_bound, settled_greedy, compare_exact, compare_obs, compare_state, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def banner(msg):
    print(f"\n[case] {msg}", flush=True)


def make(cfg, maps, torch_gpu):
    import oracle
    from paper_2305_04180_amd import sparrow
    env = sparrow.Env(cfg, maps)
    orc = oracle.Oracle(cfg, maps)
    return env, orc


def run_steps(env, orc, steps, torch_gpu, noisy, final_obs=True, check_state_every=1,
              actions_fn=None, where=""):
    torch = torch_gpu
    n, nr, D = env.n, env.n_rays, env.obs_dim
    fo = torch.zeros(n, D, dtype=torch.float32, device=env.device) if final_obs else None
    flags = torch.zeros(n, dtype=torch.uint8, device=env.device)
    total_done = 0
    for s in range(steps):
        a_o = orc.uniform_actions() if actions_fn is None else actions_fn(s)
        a_g = env.random_actions()
        if actions_fn is None:
            compare_exact(to_np(a_g), a_o, "uniform actions", f"{where} step {s}")
        else:
            a_g.copy_(torch.as_tensor(a_o))
        if fo is not None:
            fo.zero_()
        env.step(a_g, flags=flags, final_obs=fo)
        r = orc.step(a_o, final_obs=final_obs, hit_k=True)
        w = f"{where} step {s}"
        compare_exact(to_np(env.debug_hits()), r["hit_k"], "hit_k", w)
        compare_exact(to_np(env.done), r["done"], "done", w)
        compare_exact(to_np(flags), r["flags"], "flags", w)
        compare_exact(to_np(env.reward), r["reward"], "reward", w)
        compare_obs(to_np(env.obs), r["obs"], nr, noisy, w)
        if final_obs:
            dn = r["done"].astype(bool)
            if dn.any():
                compare_obs(to_np(fo)[dn], r["final_obs"][dn], nr, noisy, w + " final_obs")
        if check_state_every and (s % check_state_every == 0 or s == steps - 1):
            gf, gi = env.get_state()
            of, oi = orc.get_state()
            compare_state(gf, gi, of, oi, w)
        total_done += int(r["done"].sum())
    return total_done


def test_reset_parity_c1(torch_gpu):
    cfg = inputs.workload("c1")
    banner(f"reset c1 N={cfg['n_envs']} seed={cfg['seed']}")
    maps = inputs.make_maps(cfg)
    env, orc = make(cfg, maps, torch_gpu)
    env.reset()
    o_obs, rc, o_hk = orc.reset(hit_k=True)
    assert rc == 0 and env.status() == 0
    compare_exact(to_np(env.debug_hits()), o_hk, "hit_k", "reset")
    compare_obs(to_np(env.obs), o_obs, env.n_rays, noisy=False, where="reset")
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf, gi, of, oi, "reset")


def test_step_parity_c1_1000_steps(torch_gpu):
    """The minimum slice: C1 (N=16, 128^2, 32 rays), 1000 steps, bit-exact."""
    cfg = inputs.workload("c1")
    banner(f"step c1 N={cfg['n_envs']} 1000 steps")
    maps = inputs.make_maps(cfg)
    env, orc = make(cfg, maps, torch_gpu)
    env.reset()
    orc.reset()
    dones = run_steps(env, orc, 1000, torch_gpu, noisy=False, check_state_every=10, where="c1")
    assert dones > 50  # episodes end and AutoReset runs
    assert env.status() == 0


@pytest.mark.parametrize("variant", [(1, 16), (2, 32), (4, 32), (8, 64), (4, 16), (8, 32)])
def test_step_parity_c2_ragged(torch_gpu, variant):
    """C2 physics (366^2 mixed maps, full randomisation, noise, delay) with a
    ragged batch of 37 envs, every step kernel variant."""
    cfg = inputs.workload("c2", n_envs=37)
    banner(f"step c2 N=37 variant={variant} 150 steps")
    maps = inputs.make_maps(cfg)
    env, orc = make(cfg, maps, torch_gpu)
    env.set_variant(0, *variant)
    env.reset()
    orc.reset()
    run_steps(env, orc, 150, torch_gpu, noisy=True, check_state_every=5, where=f"c2 {variant}")


def test_step_parity_uneven_maps_64_rays(torch_gpu):
    """C3-style uneven map sides with 64 rays and range 128, 29 envs."""
    cfg = inputs.workload("c3", n_envs=29)
    banner("step c3-style N=29 uneven sides, 64 rays, 100 steps")
    maps = inputs.make_maps(cfg)
    env, orc = make(cfg, maps, torch_gpu)
    env.reset()
    orc.reset()
    run_steps(env, orc, 100, torch_gpu, noisy=True, check_state_every=10, where="c3")


def test_rollout_uniform_parity(torch_gpu):
    """Persistent rollout with uniform actions == the oracle stepped K times."""
    torch = torch_gpu
    cfg = inputs.workload("c2", n_envs=45)
    K = 24
    banner(f"rollout uniform c2 N=45 K={K}")
    maps = inputs.make_maps(cfg)
    for variant in [(8, 64), (8, 32), (4, 32), (2, 16)]:
        env, orc = make(cfg, maps, torch)
        env.set_variant(1, *variant)
        env.reset()
        orc.reset()
        # the first launch returns every step's observation and hit indices
        acts, rew, done, obs, obs_t, hits_t = env.rollout_trace(K, use_qnet=False)
        torch.cuda.synchronize()
        obs_t, hits_t = to_np(obs_t), to_np(hits_t)
        for t in range(K):
            a = orc.uniform_actions()
            r = orc.step(a, hit_k=True)
            w = f"rollout {variant} t={t}"
            compare_exact(to_np(acts[t]), a, "actions", w)
            compare_exact(to_np(rew[t]), r["reward"], "reward", w)
            compare_exact(to_np(done[t]), r["done"], "done", w)
            compare_exact(hits_t[t], r["hit_k"], "hit_k", w)
            compare_obs(obs_t[t], r["obs"], env.n_rays, True, w + " obs")
        compare_obs(to_np(obs), r["obs"], env.n_rays, True, "rollout final obs")
        compare_exact(to_np(env.debug_hits()), r["hit_k"], "hit_k", "rollout final")
        gf, gi = env.get_state()
        of, oi = orc.get_state()
        compare_state(gf, gi, of, oi, f"rollout {variant} final")
        assert env.global_step == orc.global_step
        # a second rollout continues from the new step counter
        acts2, rew2, done2, obs2 = env.rollout(K, use_qnet=False)
        torch.cuda.synchronize()
        for t in range(K):
            a = orc.uniform_actions()
            r = orc.step(a)
            compare_exact(to_np(rew2[t]), r["reward"], "reward", f"replay t={t}")
            compare_exact(to_np(done2[t]), r["done"], "done", f"replay t={t}")
        gf, gi = env.get_state()
        of, oi = orc.get_state()
        compare_state(gf, gi, of, oi, f"rollout replay {variant}")


def test_reset_failure_reports_ereset(torch_gpu):
    from paper_2305_04180_amd import sparrow
    cfg = inputs.workload("c1", n_envs=3)
    banner("reset failure on a full map")
    g = np.ones((32, 32), np.uint8)
    maps = inputs.single_maps([g], n_envs=3)
    env = sparrow.Env(cfg, maps)
    env.reset()
    assert env.status() == sparrow.ERESET


def _qnet_setup(cfg, env):
    dims = (env.obs_dim, 256, 256, 7)
    w, b, _ = inputs.qnet_weights(dims)
    import oracle
    # the library computes its own schedule; the oracle's copy is the oracle's
    env.set_qnet(dims, w, b, env.vem_epsilon(env.n, 0.01, 0.29))
    eps = oracle.vem_epsilon(env.n, env.n, 0.01, 0.29)
    return dims, w, b, eps


def test_qnet_forward_parity(torch_gpu):
    """BF16 MFMA Q-network vs the FP64 oracle on identical observations."""
    import oracle
    torch = torch_gpu
    cfg = inputs.workload("c2", n_envs=64)
    banner("qnet forward 36-256-256-7 on 2112 observations")
    maps = inputs.make_maps(cfg)
    env, orc = make(cfg, maps, torch)
    dims, w, b, eps = _qnet_setup(cfg, env)
    rows = [orc.reset()[0]]
    for _ in range(16):
        rows.append(orc.step(orc.uniform_actions())["obs"])
    rng = np.random.default_rng(9)
    rows.append(rng.uniform(-1.2, 1.2, size=(1024, 36)).astype(np.float32))
    obs = np.concatenate(rows)
    obs_t = torch.as_tensor(obs).cuda()
    q, greedy = env.qnet_forward(obs_t)
    torch.cuda.synchronize()
    q = to_np(q).astype(np.float64)
    greedy = to_np(greedy)
    q64 = oracle.qnet_f64(dims, w, b, obs, round_act=False)    # FP64 reference
    # first-order bound of the kernel's arithmetic on identical inputs
    bound = qnet_bound(dims, w, b, obs)
    dq = np.abs(q - q64)
    assert np.all(dq <= bound), (dq.max(), (dq / bound).max())
    assert np.array_equal(greedy, q.argmax(1))
    agree = (greedy == q64.argmax(1)).mean()
    top, clear = settled_greedy(q64, bound)
    print(f"max|dQ| vs fp64 {dq.max():.2e} (max dQ/bound {(dq / bound).max():.3f}), "
          f"agreement {agree:.5f}, clear-gap agreement "
          f"{(greedy[clear] == top[clear]).mean():.5f} ({clear.sum()} of {len(clear)} rows)")
    assert agree >= 0.995
    assert np.array_equal(greedy[clear], top[clear])
    # against the oracle with bf16 hidden activations: a tight bound
    q_ra = oracle.qnet_f64(dims, w, b, obs, round_act=True)
    eq = qnet_rounded_bound(dims, w, b, obs)
    assert np.all(np.abs(q - q_ra) <= eq), (np.abs(q - q_ra) / eq).max()
    top_ra, settled = settled_greedy(q_ra, eq)
    print(f"bf16-activation oracle: max|dQ| {np.abs(q - q_ra).max():.2e}, settled "
          f"{settled.mean():.4f}", flush=True)
    assert settled.mean() >= 0.95
    assert np.array_equal(greedy[settled], top_ra[settled])
    # partial rows and n = 0
    q5, g5 = env.qnet_forward(obs_t[:5].contiguous())
    torch.cuda.synchronize()
    assert np.array_equal(to_np(g5), greedy[:5])


def test_act_kernel_vem(torch_gpu):
    """The separate actor kernel on the oracle's observations: explored envs
    take the oracle's VEM draw, the rest the oracle's greedy action wherever
    the precision bound settles it."""
    import oracle
    torch = torch_gpu
    cfg = inputs.workload("c2", n_envs=300)
    banner("actor kernel (qnet + VEM) N=300")
    maps = inputs.make_maps(cfg)
    env, orc = make(cfg, maps, torch)
    dims, w, b, eps = _qnet_setup(cfg, env)
    env.reset()
    o_obs, _ = orc.reset()
    env.global_step = orc.global_step = 7
    a = env.act(torch.as_tensor(o_obs).cuda())
    torch.cuda.synchronize()
    q64 = oracle.qnet_f64(dims, w, b, o_obs)
    a_o, ex = orc.vem(q64, eps)
    exb = ex.astype(bool)
    q_ra = oracle.qnet_f64(dims, w, b, o_obs, round_act=True)
    top, settled = settled_greedy(q_ra, qnet_rounded_bound(dims, w, b, o_obs))
    compare_exact(to_np(a)[exb], a_o[exb], "explored actions", "act")
    m = ~exb & settled
    compare_exact(to_np(a)[m], top[m], "settled greedy actions", "act")
    print(f"settled {settled.mean():.4f}", flush=True)
    assert settled.mean() >= 0.95 and 0 < ex.sum() < 300


def test_fused_rollout_parity(torch_gpu):
    """Fused BF16 actor + step rollout against the oracle running its own
    FP64 actor: exploration draws and every settled greedy choice equal,
    rewards, dones, final observation and state equal for the envs whose
    trajectories provably coincide."""
    torch = torch_gpu
    cfg = inputs.workload("c2", n_envs=45)
    K = 16
    banner(f"fused rollout N=45 K={K}")
    maps = inputs.make_maps(cfg)
    for variant in [(8, 64), (8, 32), (4, 16)]:
        env, orc = make(cfg, maps, torch)
        dims, w, b, eps = _qnet_setup(cfg, env)
        env.set_variant(1, *variant)
        env.reset()
        o_obs, _ = orc.reset()
        acts, rew, done, obs, obs_t, hits_t = env.rollout_trace(K, use_qnet=True)
        torch.cuda.synchronize()
        live, o_obs = actor_lockstep(orc, dims, w, b, eps, o_obs, to_np(acts), to_np(rew),
                                     to_np(done), f"fused {variant}", obs_steps=to_np(obs_t),
                                     hits_steps=to_np(hits_t))
        compare_obs(to_np(obs)[live], o_obs[live], env.n_rays, True, f"fused {variant} final obs")
        gf, gi = env.get_state()
        of, oi = orc.get_state()
        compare_state(gf[live], gi[live], of[live], oi[live], f"fused {variant} final")


def test_autotune_preserves_state(torch_gpu):
    torch = torch_gpu
    cfg = inputs.workload("c2", n_envs=40)
    banner("autotune then step N=40")
    maps = inputs.make_maps(cfg)
    env, orc = make(cfg, maps, torch)
    _qnet_setup(cfg, env)
    env.reset()
    orc.reset()
    rep = env.autotune(steps=3)
    assert "chosen" in rep and len(rep["step"]) == 12
    assert env.global_step == orc.global_step
    run_steps(env, orc, 20, torch, noisy=True, check_state_every=5, where="after autotune")


def test_fused_rollout_64_rays_obs68(torch_gpu):
    """The 68-wide observation actor (64 rays): Q-network 68-256-256-7 on
    the oracle's observations, and a fused rollout on uneven map sides."""
    import oracle
    torch = torch_gpu
    cfg = inputs.workload("c3", n_envs=21)
    K = 12
    banner(f"fused rollout, 64 rays, obs 68, N=21, K={K}")
    maps = inputs.make_maps(cfg)
    env, orc = make(cfg, maps, torch)
    dims, w, b, eps = _qnet_setup(cfg, env)
    assert dims[0] == 68
    env.reset()
    o_obs, _ = orc.reset()
    q, greedy = env.qnet_forward(torch.as_tensor(o_obs).cuda())
    torch.cuda.synchronize()
    q64 = oracle.qnet_f64(dims, w, b, o_obs)
    assert np.all(np.abs(to_np(q).astype(np.float64) - q64) <= qnet_bound(dims, w, b, o_obs))
    q_ra = oracle.qnet_f64(dims, w, b, o_obs, round_act=True)
    eq = qnet_rounded_bound(dims, w, b, o_obs)
    assert np.all(np.abs(to_np(q).astype(np.float64) - q_ra) <= eq)
    top, settled = settled_greedy(q_ra, eq)
    assert np.array_equal(to_np(greedy)[settled], top[settled])
    acts, rew, done, obs = env.rollout(K, use_qnet=True)
    torch.cuda.synchronize()
    live, o_obs = actor_lockstep(orc, dims, w, b, eps, o_obs, to_np(acts), to_np(rew),
                                 to_np(done), "obs68")
    compare_obs(to_np(obs)[live], o_obs[live], env.n_rays, True, "obs68 final")
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf[live], gi[live], of[live], oi[live], "obs68 final")


def test_vem_schedule_rollout_and_act(torch_gpu):
    """VEM with the exploring interval shrinking from 45 envs to 3 over 10
    vectorized steps (T = 450 transitions), inside a 16-step fused rollout and
    in the separate actor kernel: every explored action equals the oracle's
    draw at that step's scheduled probabilities."""
    import oracle
    torch = torch_gpu
    cfg = inputs.workload("c2", n_envs=45)
    K, N = 16, 45
    banner("VEM schedule: OR 45 -> 3 over 450 transitions, rollout K=16 and act")
    maps = inputs.make_maps(cfg)
    env, orc = make(cfg, maps, torch)
    dims, w, b, _ = _qnet_setup(cfg, env)
    sched = (0.01, 0.8, N, 3, 10 * N)
    env.set_vem_schedule(*sched)
    env.reset()
    o_obs, _ = orc.reset()
    g0 = orc.global_step
    eps_fn = lambda t: oracle.vem_schedule_epsilon(N, g0 + t, *sched)
    # step 0 is global step 1 (after the reset): T = 45, m = 45 - floor(42 * 45 / 450) = 41
    assert (eps_fn(0) > 0.01).sum() == 40 and (eps_fn(12) > 0.01).sum() == 2
    acts, rew, done, obs = env.rollout(K, use_qnet=True)
    torch.cuda.synchronize()
    live, o_obs = actor_lockstep(orc, dims, w, b, eps_fn, o_obs, to_np(acts), to_np(rew),
                                 to_np(done), "vem schedule")
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf[live], gi[live], of[live], oi[live], "vem schedule final")
    # the actor kernel at a step in the middle of the decay
    env.global_step = orc.global_step = 5
    a = env.act(torch.as_tensor(o_obs).cuda())
    torch.cuda.synchronize()
    a_o, ex = orc.vem(oracle.qnet_f64(dims, w, b, o_obs), eps_fn(5 - g0))
    exb = ex.astype(bool)
    assert exb.any()
    compare_exact(to_np(a)[exb], a_o[exb], "explored actions", "act with schedule")
    from paper_2305_04180_amd import sparrow
    with pytest.raises(sparrow.SparrowError):
        env.set_vem_schedule(0.01, 0.8, 3, 4, 10)  # or_final > or_start


def test_vem_epsilon_matches_oracle(torch_gpu):
    """The library's per-env VEM schedule (Sec. 3.1.1) against the oracle's,
    bit for bit, for the workloads' interval and for short, single and empty
    exploring intervals."""
    import oracle
    cfg = inputs.workload("c1", n_envs=300)
    banner("vem epsilon schedule N=300")
    maps = inputs.make_maps(cfg)
    from paper_2305_04180_amd import sparrow
    env = sparrow.Env(cfg, maps)
    for m, e_min, e_max in ((300, 0.01, 0.29), (17, 0.01, 0.8), (1, 0.05, 0.5), (0, 0.2, 0.3),
                            (2, 0.0, 1.0)):
        got = to_np(env.vem_epsilon(m, e_min, e_max))
        want = oracle.vem_epsilon(300, m, e_min, e_max)
        compare_exact(got.view(np.uint32), want.view(np.uint32), "eps", f"m={m}")
    with pytest.raises(sparrow.SparrowError):
        env.vem_epsilon(301, 0.01, 0.29)


def test_failed_set_qnet_keeps_the_installed_network(torch_gpu):
    """A set_qnet that fails leaves the network installed before it in place:
    the actor keeps giving the same actions."""
    torch = torch_gpu
    from paper_2305_04180_amd import sparrow
    cfg = inputs.workload("c2", n_envs=64)
    banner("set_qnet failure path N=64")
    maps = inputs.make_maps(cfg)
    env = sparrow.Env(cfg, maps)
    env.reset()
    dims, w, b, _ = _qnet_setup(cfg, env)
    obs = env.obs.clone()
    a0 = env.act(obs).clone()
    with pytest.raises(sparrow.SparrowError) as ei:
        env.set_qnet((env.obs_dim, 384, 384, 7), np.zeros(384 * (36 + 384 + 7), np.uint16),
                     np.zeros(384 * 2 + 7, np.float32), np.zeros(env.n, np.float32))
    assert ei.value.code == sparrow.EUNSUPPORTED
    a1 = env.act(obs)
    torch.cuda.synchronize()
    compare_exact(to_np(a1), to_np(a0), "actions after a failed set_qnet", "set_qnet")


def test_autotune_cache(torch_gpu, tmp_path):
    """sparrow_autotune_cached: the first call times the variants and records
    the choice; an env of the same shape reads it back without timing; an
    env of another shape misses the record."""
    from paper_2305_04180_amd import sparrow
    cfg = inputs.workload("c2", n_envs=40)
    banner("autotune cache N=40")
    maps = inputs.make_maps(cfg)
    path = tmp_path / "autotune.jsonl"
    env = sparrow.Env(cfg, maps)
    _qnet_setup(cfg, env)
    env.reset()
    rep = env.autotune(steps=2, cache=path)
    assert "step" in rep and not rep.get("cached")
    chosen = (env.get_variant(0), env.get_variant(1))
    assert len(path.read_text().splitlines()) == 1
    env2 = sparrow.Env(cfg, maps)
    _qnet_setup(cfg, env2)
    env2.reset()
    env2.set_variant(0, 1, 16)
    env2.set_variant(1, 1, 16)
    rep2 = env2.autotune(steps=2, cache=path)
    assert rep2.get("cached") is True
    assert (env2.get_variant(0), env2.get_variant(1)) == chosen
    assert len(path.read_text().splitlines()) == 1
    cfg3 = inputs.workload("c2", n_envs=41)
    env3 = sparrow.Env(cfg3, inputs.make_maps(cfg3))
    _qnet_setup(cfg3, env3)
    env3.reset()
    assert not env3.autotune(steps=2, cache=path).get("cached")
    assert len(path.read_text().splitlines()) == 2
    assert env.status() == env2.status() == env3.status() == 0
