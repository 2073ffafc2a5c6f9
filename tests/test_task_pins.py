"""Pins of the oracle's paper-faithful task variant (Sec. 4.3.1): the five
actions against the target velocities the paper lists, Eq. (11) term by term
on hand-built maps (each term switched on and off by a pose or state chosen
for it), the terminal rewards, the relative-pose state, and the r_d disk
test against a brute-force FP64 cell walk.

The paper leaves the shapes of r_d1, r_d2 and r_alpha open, so these pins fix
the oracle to its reading of them (linear, clipped at zero), not to values
printed in the paper: parity with the paper is unpinned for this variant."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2305_04180_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
F32 = np.float32


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def constants():
    return json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))


def paper_task():
    return constants()["sec431_task"]


def env(grid, task=True, **kw):
    cfg = inputs.workload("c1", n_envs=1)
    cfg.update(dict(dt_lo=0.1, dt_hi=0.1, K_lo=0.0, K_hi=0.0, mu_lo=1.0, mu_hi=1.0,
                    vmax_lo=10.0, vmax_hi=10.0, sigma_lo=0.0, sigma_hi=0.0, delay_lo=0,
                    delay_hi=0, t_max=10_000, n_rays=27))
    cfg.update(kw)
    o = oracle.Oracle(cfg, inputs.single_maps([grid], n_envs=1))
    if task:
        t = paper_task()
        o.set_task(n_actions=5, reward=oracle.REWARD_EQ11, state=oracle.STATE_RELATIVE,
                   arrive_reward=t["arrive_reward"], collide_reward=t["collide_reward"],
                   plan_dist=100.0, near_dist=15.0, weights=tuple(t["weights"]))
    o.reset()
    return o, cfg


def put(o, **fields):
    f, i = o.get_state()
    for k, v in fields.items():
        if k in oracle.STATE_F:
            f[:, oracle.STATE_F.index(k)] = v
        else:
            i[:, oracle.STATE_I.index(k)] = v
    o.set_state(f, i)


def test_five_actions_are_the_listed_target_velocities():
    """Sec. 4.3.1 lists [v_l, v_a] per action: turn left [0.36 cm/s, 1],
    straight-left [18, 1], straight [18, 0], straight-right [18, -1], turn
    right [0.36, -1], with 18 cm/s the maximal linear velocity (Table 7) and
    1 rad/s the maximal angular one. With K = 0, mu = 1 and no delay the new
    velocity is the target velocity itself (Eq. (5))."""
    c = constants()
    vmax_cm = c["table7_simulation_parameters"]["max_linear_velocity_cm_s"]
    g = np.zeros((64, 64), np.uint8)
    for a, act in enumerate(c["sec431_actions"]):
        v_cm, w = act["v_cm_s"], act["w_rad_s"]
        o, cfg = env(g)
        put(o, x=32.5, y=32.5, phi=1.0, vl=0.0, va=0.0, K=0.0, mu=1.0, vmax=10.0, delay=0,
            tx=60.5, ty=60.5)
        o.step(np.array([a], np.int32))
        f, _ = o.get_state()
        frac = F32(v_cm / vmax_cm)  # 0.02 or 1
        assert f[0, 3] == F32(frac * F32(10.0)), (a, f[0, 3])
        assert f[0, 4] == F32(F32(w) * F32(cfg["omega_max"])), (a, f[0, 4])
    # an id past the five acts as stop: zero target velocity
    o, _ = env(g)
    put(o, x=32.5, y=32.5, vl=0.0, va=0.0, K=0.0, delay=0, tx=60.5, ty=60.5)
    o.step(np.array([5], np.int32))
    f, _ = o.get_state()
    assert f[0, 3] == 0.0 and f[0, 4] == 0.0


def test_five_action_env_equals_seven_action_env_on_the_mapped_rows():
    """Whole steps (ranges, reward, state) of the 5-action task equal those
    of the 7-action table driven with rows {0, 1, 3, 5, 6}."""
    cfg = inputs.workload("c2", n_envs=6, n_rays=27)
    maps = inputs.make_maps(cfg)
    a5 = oracle.Oracle(cfg, maps)
    a7 = oracle.Oracle(cfg, maps)
    a5.set_task(n_actions=5)
    a5.reset()
    a7.reset()
    rows = np.array([0, 1, 3, 5, 6])
    rng = np.random.default_rng(4)
    for s in range(40):
        act = rng.integers(0, 5, 6).astype(np.int32)
        r5 = a5.step(act, hit_k=True)
        r7 = a7.step(rows[act], hit_k=True)
        for k in ("obs", "reward", "done", "hit_k"):
            assert np.array_equal(r5[k], r7[k]), (s, k)


def eq11(d1, d2, rv, alpha_over_pi, rd, D=100.0, w=(0.3, 0.1, 0.3, 0.3, 0.1)):
    """Eq. (11) with the reading's terms, binary32 in the oracle's order."""
    invD = F32(1.0 / D)
    rd1 = max(F32(1.0) - F32(d1) * invD, F32(0.0))
    rd2 = max(F32(1.0) - F32(d2) * invD, F32(0.0))
    ra = F32(1.0) - abs(F32(alpha_over_pi))
    w = [F32(x) for x in w]
    r = w[0] * F32(rd1)
    r = F32(r + w[1] * F32(rd2))
    r = F32(r + w[2] * F32(rv))
    r = F32(r + w[3] * ra)
    r = F32(r + w[4] * F32(rd))
    return r


def step_still(o, **state):
    """One step with the pose held (dt = 0, K = 1: velocities kept)."""
    put(o, dt=0.0, K=1.0, delay=0, **state)
    return o.step(np.array([2], np.int32))


def test_eq11_terms_switch_one_at_a_time():
    g = np.zeros((128, 256), np.uint8)  # no border: cells outside count as obstacles
    o, cfg = env(g)
    vmax = 10.0
    # facing the target (forward = (-cos phi, -sin phi) = +x at phi = pi):
    # alpha = 0; v_l above half of v_max; nothing within the margin
    base = dict(x=40.5, y=60.5, phi=math.pi, tx=70.5, ty=60.5, vl=6.0, va=0.0, vmax=vmax)
    r = step_still(o, **base)
    assert r["done"][0] == 0
    assert r["reward"][0] == eq11(30.0, 0.0, 1.0, 0.0, 0.0)
    # d2 term: target 40 cells off in y as well (alpha now atan2 of the offset)
    r = step_still(o, **dict(base, ty=100.5))
    alpha = math.atan2(40.0, 30.0) / math.pi
    assert abs(r["reward"][0] - eq11(30.0, 40.0, 1.0, alpha, 0.0)) <= 1e-6
    # d1 past D: r_d1 clips at zero
    r = step_still(o, **dict(base, x=30.5, tx=140.5))
    assert r["reward"][0] == eq11(110.0, 0.0, 1.0, 0.0, 0.0)
    # v_l exactly half of v_max: r_v = 0 ("exceeds" is strict)
    r = step_still(o, **dict(base, vl=5.0))
    assert r["reward"][0] == eq11(30.0, 0.0, 0.0, 0.0, 0.0)
    # facing away: alpha = pi, r_alpha = 0
    r = step_still(o, **dict(base, phi=0.0))
    assert r["reward"][0] == eq11(30.0, 0.0, 1.0, 1.0, 0.0)
    # r_d: an occupied cell whose nearest point is 17.9 cells from the centre
    # (robot radius 3 + margin 15 = 18) gives -1; at 18.1 it does not
    for gap, rd in ((17.9, -1.0), (18.1, 0.0)):
        g2 = np.zeros((128, 256), np.uint8)
        cx = int(math.floor(40.5 + gap))  # cell [cx, cx + 1] x [60, 61]
        g2[60, cx] = 1
        o2, _ = env(g2)
        x = float(cx) - gap
        r = step_still(o2, **dict(base, x=x))
        assert r["reward"][0] == eq11(70.5 - F32(x), 0.0, 1.0, 0.0, rd), (gap, r["reward"][0])
    # terminal rewards: arrival (within r_a = 4 of the target) and collision
    r = step_still(o, **dict(base, x=68.5))
    assert r["done"][0] == 1 and r["reward"][0] == F32(75.0)
    g3 = np.zeros((128, 256), np.uint8)
    g3[60, 42] = 1
    o3, _ = env(g3)
    r = step_still(o3, **base)
    assert r["done"][0] == 1 and r["reward"][0] == F32(-10.0)


def test_relative_state():
    """[ranges | (x - tx)/D, (y - ty)/D, alpha/pi, v_l/v_max, v_a/omega_max]:
    32 entries with 27 rays."""
    g = np.zeros((128, 128), np.uint8)
    o, cfg = env(g)
    assert o.obs_dim == paper_task()["state_length"]
    st = dict(x=40.25, y=70.75, phi=0.4, tx=90.5, ty=20.5, vl=3.0, va=-0.5, vmax=10.0)
    r = step_still(o, **st)
    ob = r["obs"][0]
    D = F32(1.0 / 100.0)
    assert ob[27] == F32(F32(40.25) - F32(90.5)) * D
    assert ob[28] == F32(F32(70.75) - F32(20.5)) * D
    fx, fy = -math.cos(0.4), -math.sin(0.4)
    dx, dy = 90.5 - 40.25, 20.5 - 70.75
    alpha = math.atan2(dy * fx - dx * fy, dx * fx + dy * fy) / math.pi
    assert abs(ob[29] - alpha) <= 1e-6
    assert ob[30] == F32(3.0) / F32(10.0) and ob[31] == F32(-0.5) / F32(cfg["omega_max"])


def test_near_disk_matches_brute_force():
    """The r_d test (any occupied cell within robot_r + near_dist of the
    centre, touching included) against an FP64 walk over every cell."""
    rng = np.random.default_rng(9)
    g = (rng.random((200, 200)) < 0.0015).astype(np.uint8)
    o, cfg = env(g)
    R = 3.0 + 15.0
    seen = {True: 0, False: 0}
    for _ in range(300):
        px, py = rng.uniform(-5, 205, 2).astype(np.float32)
        dmin = math.inf  # FP64 distance from the centre to the nearest occupied cell
        for j in range(int(py) - 22, int(py) + 23):
            for i in range(int(px) - 22, int(px) + 23):
                occ = i < 0 or j < 0 or i >= 200 or j >= 200 or g[j, i]
                if not occ:
                    continue
                dx = max(i - float(px), 0.0, float(px) - (i + 1))
                dy = max(j - float(py), 0.0, float(py) - (j + 1))
                dmin = min(dmin, math.hypot(dx, dy))
        got = o.near(0, float(px), float(py))
        if abs(dmin - R) > 1e-4:  # away from the binary32 rounding of the boundary
            assert got == (dmin < R), (px, py, dmin)
            seen[got] += 1
    assert seen[True] > 20 and seen[False] > 20


def test_task_rejects_bad_values():
    g = np.zeros((32, 32), np.uint8)
    o, _ = env(g, task=False)
    for bad in (dict(n_actions=6), dict(reward=2), dict(state=3), dict(plan_dist=0.0),
                dict(near_dist=-1.0)):
        with pytest.raises(ValueError):
            o.set_task(**bad)
