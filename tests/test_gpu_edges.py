"""GPU edge cases against the oracle: maximum sizes, degenerate physics and
geometry, small batches, and rollout corner cases."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2305_04180_amd import inputs
from tests.parity_util import compare_exact, compare_obs, compare_state, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def banner(msg):
    print(f"\n[case] {msg}", flush=True)


def lockstep(cfg, maps, torch, steps, noisy=True, variants=((0, 1, 64), (0, 8, 32))):
    """Step the library and the oracle side by side, comparing everything."""
    import oracle
    from paper_2305_04180_amd import sparrow
    for kern, epw, L in variants:
        env = sparrow.Env(cfg, maps)
        env.set_variant(kern, epw, L)
        orc = oracle.Oracle(cfg, maps)
        env.reset()
        o_obs, rc, o_hk = orc.reset(hit_k=True)
        w0 = f"{cfg.get('label', cfg['name'])} variant {(epw, L)} reset"
        compare_exact(to_np(env.debug_hits()), o_hk, "hit_k", w0)
        compare_obs(to_np(env.obs), o_obs, cfg["n_rays"], noisy, w0)
        fo = torch.zeros(env.n, env.obs_dim, dtype=torch.float32, device=env.device)
        flags = torch.zeros(env.n, dtype=torch.uint8, device=env.device)
        for s in range(steps):
            a = env.random_actions()
            fo.zero_()
            env.step(a, flags=flags, final_obs=fo)
            r = orc.step(orc.uniform_actions(), final_obs=True, hit_k=True)
            w = f"{cfg.get('label', cfg['name'])} variant {(epw, L)} step {s}"
            compare_exact(to_np(env.debug_hits()), r["hit_k"], "hit_k", w)
            compare_exact(to_np(env.done), r["done"], "done", w)
            compare_exact(to_np(flags), r["flags"], "flags", w)
            compare_exact(to_np(env.reward), r["reward"], "reward", w)
            compare_obs(to_np(env.obs), r["obs"], cfg["n_rays"], noisy, w)
            dn = r["done"].astype(bool)
            if dn.any():
                compare_obs(to_np(fo)[dn], r["final_obs"][dn], cfg["n_rays"], noisy, w + " final")
            if (~dn).any():  # rows of envs that are not done stay untouched
                assert np.all(to_np(fo)[~dn] == 0.0), w
        gf, gi = env.get_state()
        of, oi = orc.get_state()
        compare_state(gf, gi, of, oi, f"{cfg.get('label', cfg['name'])} {(epw, L)} final")
        assert env.status() == orc.status


def test_max_side_512_and_128_rays(torch_gpu):
    """512 x 512 maps (the largest side), 128 rays, range 255, robot radius 8."""
    cfg = inputs.workload("c2", n_envs=9, n_rays=128, range=255.0, robot_r=8.0, sides=(512,),
                          label="max")
    banner("512^2 maps, 128 rays, range 255, r = 8")
    maps = inputs.make_maps(cfg)
    lockstep(cfg, maps, torch_gpu, 30, variants=((0, 1, 64), (0, 4, 16), (0, 2, 32)))


def test_single_env_single_ray_full_circle(torch_gpu):
    cfg = inputs.workload("c2", n_envs=1, n_rays=1, fov=0.0, label="one")
    banner("N = 1, one ray")
    lockstep(cfg, inputs.make_maps(cfg), torch_gpu, 80)
    cfg2 = inputs.workload("c2", n_envs=3, n_rays=7, fov=2 * math.pi, label="circle")
    banner("N = 3, 7 rays over a full circle")
    lockstep(cfg2, inputs.make_maps(cfg2), torch_gpu, 60)


def test_degenerate_physics(torch_gpu):
    """K = 1 (velocity never follows the command), always two-step delay,
    no noise, truncation every step, huge arrival radius."""
    base = inputs.workload("c2", n_envs=11, label="deg")
    for change in (dict(K_lo=1.0, K_hi=1.0), dict(delay_lo=2, delay_hi=2),
                   dict(sigma_lo=0.0, sigma_hi=0.0), dict(t_max=1),
                   dict(arrive_r=60.0), dict(dt_lo=0.2, dt_hi=0.2, vmax_lo=15.0, vmax_hi=15.0)):
        cfg = dict(base, **change)
        banner(f"degenerate physics {change}")
        noisy = cfg["sigma_hi"] > 0
        lockstep(cfg, inputs.make_maps(cfg), torch_gpu, 25, noisy=noisy,
                 variants=((0, 1, 64),))


def test_unbordered_empty_and_tiny_maps(torch_gpu):
    """No border (rays leave the map: outside counts as a hit), a map with
    no obstacles, and mixed tiny sides shared by several envs. The 9 x 12 map
    leaves some starts with no target farther than the arrival radius, so the
    sticky reset error and its candidate-0 fallback are compared as well."""
    g_empty = np.zeros((40, 40), np.uint8)
    g_open = np.zeros((300, 200), np.uint8)  # non-square
    g_open[100:110, 50:150] = 1
    g_small = np.zeros((9, 12), np.uint8)
    maps = inputs.single_maps([g_empty, g_open, g_small], env_to_map=[0, 1, 2, 1, 0, 2, 1])
    cfg = inputs.workload("c2", n_envs=7, label="unbordered")
    banner("unbordered / empty / tiny maps shared by envs")
    lockstep(cfg, maps, torch_gpu, 60, variants=((0, 1, 64), (0, 8, 16)))


def test_rollout_lengths_and_interleaving(torch_gpu):
    """K = 1 and K = 7 rollouts interleaved with plain steps, each checked
    against the oracle; launches of different K reuse one slot table."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    cfg = inputs.workload("c2", n_envs=19, label="interleave")
    banner("rollout K = 1, 7 interleaved with steps")
    maps = inputs.make_maps(cfg)
    env = sparrow.Env(cfg, maps)
    orc = oracle.Oracle(cfg, maps)
    env.reset()
    orc.reset()
    for K in (1, 7, 1, 7):
        acts, rew, done, obs = env.rollout(K, False)
        torch.cuda.synchronize()
        for t in range(K):
            a = orc.uniform_actions()
            r = orc.step(a)
            compare_exact(to_np(rew[t]), r["reward"], "reward", f"K={K} t={t}")
            compare_exact(to_np(done[t]), r["done"], "done", f"K={K} t={t}")
        compare_obs(to_np(obs), r["obs"], cfg["n_rays"], True, f"K={K}")
        a = env.random_actions()
        env.step(a)
        r = orc.step(orc.uniform_actions())
        compare_exact(to_np(env.reward), r["reward"], "reward", f"step after K={K}")
    gf, gi = env.get_state()
    of, oi = orc.get_state()
    compare_state(gf, gi, of, oi, "interleaved")


def test_set_state_roundtrip_and_errors(torch_gpu):
    from paper_2305_04180_amd import sparrow
    cfg = inputs.workload("c1", n_envs=5, label="state")
    banner("set/get state, argument errors")
    env = sparrow.Env(cfg, inputs.make_maps(cfg))
    env.reset()
    f, i = env.get_state()
    f2 = f.copy()
    f2[:, 0] += 1.0
    env.set_state(f2, i)
    g, j = env.get_state()
    assert np.array_equal(g.view(np.uint32), f2.view(np.uint32)) and np.array_equal(i, j)
    bad = i.copy()
    bad[0, 1] = 3  # delay 3 is out of range
    with pytest.raises(sparrow.SparrowError):
        env.set_state(f, bad)
    with pytest.raises(sparrow.SparrowError):
        env.set_variant(0, 3, 32)
    with pytest.raises(sparrow.SparrowError):
        env.rollout(4, True)  # no Q-network installed
    with pytest.raises(sparrow.SparrowError):  # unequal hidden widths are unsupported
        env.set_qnet((36, 256, 512, 7), np.zeros(36 * 256 + 256 * 512 + 7 * 512, np.uint16),
                     np.zeros(256 + 512 + 7, np.float32), np.zeros(5, np.float32))
    with pytest.raises(ValueError):  # weights that do not match the dims
        env.set_qnet((36, 256, 256, 7), np.zeros(100, np.uint16), np.zeros(519, np.float32),
                     np.zeros(5, np.float32))
    assert env.status() == 0


def test_windowed_step_extreme_poses(torch_gpu):
    """The plain step stages only the map rows within range of the robot.
    Poses at the map's edges, far outside it (the staged rows are clamped to
    the map's) and with the range reaching past both ends, on 512-row maps
    with range 128 and on maps shorter than the window; terminal
    observations at those poses and the steps after the AutoReset against
    the oracle."""
    import oracle
    from paper_2305_04180_amd import sparrow
    torch = torch_gpu
    rng = np.random.default_rng(17)
    grids = []
    for H, W in ((512, 512), (300, 40), (200, 512)):
        g = (rng.random((H, W)) < 0.02).astype(np.uint8)
        grids.append(g)
    maps = inputs.single_maps(grids, env_to_map=[0, 0, 0, 0, 0, 0, 1, 1, 2, 2, 0, 2])
    cfg = inputs.workload("c3", n_envs=12, label="window")
    banner("windowed step: edge and outside poses, 512 rows, range 128")
    for variant in ((1, 64), (4, 32), (8, 16)):
        env = sparrow.Env(cfg, maps)
        env.set_variant(0, *variant)
        orc = oracle.Oracle(cfg, maps)
        env.reset()
        orc.reset()
        f, iv = orc.get_state()
        # x, y: inside near each edge, far outside, and mid-map
        poses = [(256.5, 0.2), (256.5, 511.9), (3.5, 140.0), (508.5, 300.0), (256.5, -40.0),
                 (256.5, 700.0), (-25.0, 256.0), (20.5, 300.3), (100.0, 100.0), (300.0, 199.5),
                 (256.0, 256.0), (-1e4, -1e4)]
        for k, (x, y) in enumerate(poses):
            f[k, 0], f[k, 1] = x, y
        env.set_state(f, iv)
        orc.set_state(f, iv)
        fo = torch.zeros(env.n, env.obs_dim, dtype=torch.float32, device=env.device)
        flags = torch.zeros(env.n, dtype=torch.uint8, device=env.device)
        for s in range(6):
            a = env.random_actions()
            fo.zero_()
            env.step(a, flags=flags, final_obs=fo)
            r = orc.step(orc.uniform_actions(), final_obs=True, hit_k=True)
            w = f"window {variant} step {s}"
            compare_exact(to_np(env.debug_hits()), r["hit_k"], "hit_k", w)
            compare_exact(to_np(env.done), r["done"], "done", w)
            compare_exact(to_np(flags), r["flags"], "flags", w)
            compare_exact(to_np(env.reward), r["reward"], "reward", w)
            compare_obs(to_np(env.obs), r["obs"], cfg["n_rays"], True, w)
            dn = r["done"].astype(bool)
            if dn.any():
                compare_obs(to_np(fo)[dn], r["final_obs"][dn], cfg["n_rays"], True, w + " final")
            if s == 0:  # the outside poses collide at once
                assert dn[[4, 5, 6, 11]].all(), w
        gf, gi = env.get_state()
        of, oi = orc.get_state()
        compare_state(gf, gi, of, oi, f"window {variant} final")
        assert env.status() == orc.status


def rollout_lockstep(cfg, maps, torch, K, variants=((8, 64), (8, 32))):
    """Fused rollouts (uniform actions) against the oracle stepped K times."""
    import oracle
    from paper_2305_04180_amd import sparrow
    noisy = cfg["sigma_hi"] > 0
    for epw, L in variants:
        env = sparrow.Env(cfg, maps)
        env.set_variant(1, epw, L)
        orc = oracle.Oracle(cfg, maps)
        env.reset()
        orc.reset()
        acts, rew, done, obs = env.rollout(K, use_qnet=False)
        torch.cuda.synchronize()
        w0 = f"{cfg.get('label', cfg['name'])} rollout {(epw, L)}"
        for t in range(K):
            a = orc.uniform_actions()
            r = orc.step(a, hit_k=True)
            compare_exact(to_np(acts[t]), a, "actions", f"{w0} t={t}")
            compare_exact(to_np(rew[t]), r["reward"], "reward", f"{w0} t={t}")
            compare_exact(to_np(done[t]), r["done"], "done", f"{w0} t={t}")
        compare_obs(to_np(obs), r["obs"], cfg["n_rays"], noisy, f"{w0} final")
        compare_exact(to_np(env.debug_hits()), r["hit_k"], "hit_k", f"{w0} final")
        gf, gi = env.get_state()
        of, oi = orc.get_state()
        compare_state(gf, gi, of, oi, f"{w0} final state")


def test_fused_rollout_edge_maps_and_ray_counts(torch_gpu):
    """The fused rollout's unit-step march at its extremes: 512^2 maps with
    128 rays to range 255; one ray (all 64 lanes of the env on it, the
    longest overshoot past a hit); 7 rays over a full circle; tiny unbordered
    maps of one word per row; and maps of different row lengths (the march
    then clamps per axis)."""
    torch = torch_gpu
    cfg = inputs.workload("c2", n_envs=9, n_rays=128, range=255.0, robot_r=8.0, sides=(512,),
                          label="max")
    banner("rollout: 512^2 maps, 128 rays, range 255, r = 8")
    rollout_lockstep(cfg, inputs.make_maps(cfg), torch, 24)
    cfg = inputs.workload("c2", n_envs=1, n_rays=1, fov=0.0, label="one")
    banner("rollout: N = 1, one ray")
    rollout_lockstep(cfg, inputs.make_maps(cfg), torch, 40, variants=((8, 64),))
    cfg = inputs.workload("c2", n_envs=3, n_rays=7, fov=2 * math.pi, label="circle")
    banner("rollout: N = 3, 7 rays over a full circle")
    rollout_lockstep(cfg, inputs.make_maps(cfg), torch, 30, variants=((8, 64),))
    g_a = np.zeros((20, 25), np.uint8)
    g_a[8:12, 5:9] = 1
    g_b = np.zeros((25, 20), np.uint8)
    g_b[3:5, 10:18] = 1
    cfg = inputs.workload("c2", n_envs=6, robot_r=2.0, arrive_r=2.0, range=40.0,
                          label="tiny")
    banner("rollout: tiny unbordered maps, one word per row")
    rollout_lockstep(cfg, inputs.single_maps([g_a, g_b], env_to_map=[0, 1, 0, 1, 1, 0]),
                     torch, 30)
    g_empty = np.zeros((40, 40), np.uint8)
    g_open = np.zeros((300, 200), np.uint8)
    g_open[100:110, 50:150] = 1
    cfg = inputs.workload("c2", n_envs=5, label="mixed")
    banner("rollout: maps of different row lengths")
    rollout_lockstep(cfg, inputs.single_maps([g_empty, g_open], env_to_map=[0, 1, 1, 0, 1]),
                     torch, 30)
