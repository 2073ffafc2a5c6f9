"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks one part of the oracle against something other than itself:
a library routine (rocRAND's Philox, libm sin/cos, torch float64 linear
layers and bf16 rounding), a closed form of Eq. (5)/(6), hand-built maps whose
ranges follow from geometry, a brute-force FP64 voxel walk, or statistics.
"""
from __future__ import annotations

import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2305_04180_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def base_cfg(**kw):
    cfg = inputs.workload("c1", n_envs=1)
    cfg.update(dict(dt_lo=0.1, dt_hi=0.1, K_lo=0.6, K_hi=0.6, mu_lo=1.0, mu_hi=1.0,
                    vmax_lo=10.0, vmax_hi=10.0, sigma_lo=0.0, sigma_hi=0.0, delay_lo=0,
                    delay_hi=0, t_max=10_000))
    cfg.update(kw)
    return cfg


def one_env(grid, **kw):
    cfg = base_cfg(**kw)
    maps = inputs.single_maps([grid], n_envs=cfg["n_envs"])
    return oracle.Oracle(cfg, maps), cfg


def put(o, **fields):
    """Overwrite state fields of every env."""
    f, i = o.get_state()
    for k, v in fields.items():
        if k in oracle.STATE_F:
            f[:, oracle.STATE_F.index(k)] = v
        else:
            i[:, oracle.STATE_I.index(k)] = v
    o.set_state(f, i)


def get(o, name):
    f, i = o.get_state()
    if name in oracle.STATE_F:
        return f[:, oracle.STATE_F.index(name)]
    return i[:, oracle.STATE_I.index(name)]


# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------
_MASK = 0xFFFFFFFF


def philox_py(ctr, key):
    """Philox4x32-10 written here from its definition (Salmon et al., SC'11:
    ten rounds of two 32x32->64 multiplies by 0xD2511F53 and 0xCD9E8D57, the
    high halves xored with the other counter words and the round key, the key
    bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85): a second
    implementation, independent of the oracle's C code."""
    c = [int(v) & _MASK for v in ctr]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for _ in range(10):
        p0, p1 = 0xD2511F53 * c[0], 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & _MASK, p1 & _MASK, ((p0 >> 32) ^ c[3] ^ k1) & _MASK,
             p0 & _MASK]
        k0, k1 = (k0 + 0x9E3779B9) & _MASK, (k1 + 0xBB67AE85) & _MASK
    return c


def test_philox_matches_rocrand_engine(tmp_path):
    """The oracle's Philox equals rocRAND's Philox4x32-10 engine (a library
    implementation of the same SC'11 generator) on random counters and keys."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    exe = tmp_path / "philox_probe"
    subprocess.check_call([hipcc, "-O1", "--offload-arch=gfx950", "-o", str(exe),
                           os.path.join(HERE, "philox_rocrand_probe.cpp")],
                          stderr=subprocess.DEVNULL, cwd=str(tmp_path))
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2**32, size=(512, 4), dtype=np.uint64)
    ctr[:, 1] %= 2**30  # the probe encodes (c0, c1) as a 4x offset
    ctr[:8] = 0
    ctr[1, 0], ctr[2, 2], ctr[3, 3] = 1, 1, 1
    key = rng.integers(0, 2**32, size=(512, 2), dtype=np.uint64)
    key[0] = 0
    lines = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctr, key))
    out = subprocess.run([str(exe)], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(v) for v in l.split()] for l in out.stdout.strip().split("\n")], np.uint64)
    got = np.stack([oracle.philox4x32_10(c.astype(np.uint32), k.astype(np.uint32))
                    for c, k in zip(ctr, key)]).astype(np.uint64)
    assert np.array_equal(got, ref)
    # the tests' own Python Philox (used to pin the reset order) agrees too
    py = np.array([philox_py(c, k) for c, k in zip(ctr, key)], np.uint64)
    assert np.array_equal(py, ref)


def test_philox_uniformity_chi2():
    """Output words are uniform: chi^2 over 256 bins of the top byte, for
    counters that differ only in the env index (as the simulator draws them)."""
    n = 1 << 16
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 1] = 17
    ctr[:, 2] = 4
    out = oracle.philox_batch(ctr, [1, 0])
    for w in range(4):
        counts = np.bincount(out[:, w] >> 24, minlength=256)
        exp = n / 256
        chi2 = ((counts - exp) ** 2 / exp).sum()
        # 255 dof: mean 255, sd ~22.6; 5 sd bound
        assert chi2 < 255 + 5 * 22.6, (w, chi2)
    # successive counters decorrelate: lag-1 correlation of word 0
    x = out[:, 0].astype(np.float64)
    r = np.corrcoef(x[:-1], x[1:])[0, 1]
    assert abs(r) < 5 / math.sqrt(n)


# --------------------------------------------------------------------------
# sincos_f32 (Cody-Waite + Taylor) against libm in FP64
# --------------------------------------------------------------------------
def _ulp32(x):
    x = np.abs(np.asarray(x, np.float64)).astype(np.float32)
    return np.spacing(np.maximum(x, np.float32(np.finfo(np.float32).tiny))).astype(np.float64)


def test_sincos_f32_within_2ulp_of_libm():
    rng = np.random.default_rng(1)
    phi = np.concatenate([
        np.linspace(-np.pi, np.pi, 1 << 20, dtype=np.float64).astype(np.float32),
        rng.uniform(-3.2, 3.2, 1 << 18).astype(np.float32),
        np.float32([0.0, -0.0, np.pi / 2, -np.pi / 2, np.pi, -np.pi, np.pi / 4, 3 * np.pi / 4,
                    1e-30, -1e-20, 1e-8]),
    ])
    s, c = oracle.sincos_batch(phi)
    ref_s = np.sin(phi.astype(np.float64))
    ref_c = np.cos(phi.astype(np.float64))
    es = np.abs(s - ref_s) / _ulp32(ref_s)
    ec = np.abs(c - ref_c) / _ulp32(ref_c)
    assert es.max() <= 2.0, (es.max(), phi[es.argmax()])
    assert ec.max() <= 2.0, (ec.max(), phi[ec.argmax()])
    # exact at zero, symmetric
    s0, c0 = oracle.sincos_f32(0.0)
    assert s0 == 0.0 and c0 == 1.0
    s1, c1 = oracle.sincos_batch(-phi[:1000])
    s2, c2 = oracle.sincos_batch(phi[:1000])
    assert np.array_equal(s1, -s2) and np.array_equal(c1, c2)


# --------------------------------------------------------------------------
# Kinematics: Eq. (5) and Eq. (6) closed forms
# --------------------------------------------------------------------------
def _open_map(side=256):
    return np.zeros((side, side), np.uint8)


def test_eq5_geometric_series_and_eq6_straight_line():
    """Constant command, omega = 0 (action 3): v_t = mu v_hat (1 - K^t) +
    K^t v_0 (Eq. (5) iterated), heading constant, and
    x_t = x_0 - dt cos(phi_0) sum_s v_s (Eq. (6))."""
    o, cfg = one_env(_open_map(512), K_lo=0.6, K_hi=0.6, mu_lo=0.8, mu_hi=0.8)
    o.reset()
    phi0 = np.float32(0.3)
    put(o, x=100.0, y=120.0, phi=phi0, vl=0.0, va=0.0, tx=500.0, ty=500.0, dprev=1000.0)
    vhat = 0.8 * 1.0 * 10.0
    xs, vs = [], []
    for t in range(1, 40):
        o.step([3])
        vs.append(float(get(o, "vl")[0]))
        xs.append((float(get(o, "x")[0]), float(get(o, "y")[0])))
        assert get(o, "phi")[0] == phi0
        v_closed = vhat * (1 - 0.6 ** t)
        assert abs(vs[-1] - v_closed) <= 1e-5 * vhat
    sum_v = np.cumsum(np.array(vs, np.float64))
    for t, (x, y) in enumerate(xs):
        xc = 100.0 - 0.1 * math.cos(float(phi0)) * sum_v[t]
        yc = 120.0 - 0.1 * math.sin(float(phi0)) * sum_v[t]
        assert abs(x - xc) < 1e-4 and abs(y - yc) < 1e-4


def test_eq5_K0_reaches_command_in_one_step_and_clamps():
    o, cfg = one_env(_open_map(), K_lo=0.0, K_hi=0.0, mu_lo=1.0, mu_hi=1.0)
    o.reset()
    put(o, x=128.0, y=128.0, phi=0.0, vl=0.0, va=0.0)
    o.step([1])  # full speed, turn left
    assert get(o, "vl")[0] == np.float32(10.0)
    assert get(o, "va")[0] == np.float32(1.0)
    # velocities above the limits are clamped (Eq. (5) then the limits)
    put(o, vl=50.0, va=-7.0, K=0.5)
    o.step([3])
    assert get(o, "vl")[0] == np.float32(10.0)
    assert get(o, "va")[0] == np.float32(-1.0)


def test_eq6_uses_old_heading_and_new_velocity():
    """Semi-implicit pose update: x' = x - dt v' cos(phi) with phi before the step."""
    o, cfg = one_env(_open_map(), K_lo=0.0, K_hi=0.0)
    o.reset()
    put(o, x=128.0, y=128.0, phi=0.0, vl=0.0, va=0.0)
    o.step([1])  # v' = 10, w' = 1, old phi = 0
    assert get(o, "x")[0] == np.float32(128.0 - 0.1 * 10.0)
    assert get(o, "y")[0] == np.float32(128.0)  # sin(0) = 0 exactly
    assert get(o, "phi")[0] == np.float32(0.1)


def test_stop_keeps_pose_exactly_and_heading_wraps():
    o, cfg = one_env(_open_map(), K_lo=0.0, K_hi=0.0)
    o.reset()
    put(o, x=100.25, y=90.5, phi=1.0, vl=0.0, va=0.0, delay=0)
    for _ in range(5):
        o.step([7])  # out-of-table id: stop
    assert get(o, "x")[0] == np.float32(100.25) and get(o, "y")[0] == np.float32(90.5)
    # heading wraps into (-pi, pi]
    put(o, phi=np.float32(3.1), va=0.0)
    o.step([0])  # turn left at 1 rad/s for 0.1 s -> 3.2 -> wraps
    p = float(get(o, "phi")[0])
    assert -math.pi < p <= math.pi and abs(p - (3.2 - 2 * math.pi)) < 1e-6


def test_control_delay_fifo():
    """Delay d applies the action issued d steps earlier; the queue starts at stop."""
    for d in (0, 1, 2):
        o, cfg = one_env(_open_map(), K_lo=0.0, K_hi=0.0, delay_lo=d, delay_hi=d)
        o.reset()
        put(o, x=128.0, y=128.0, phi=0.0, vl=0.0, va=0.0)
        seq = [1, 5, 3, 0, 6]
        got = []
        for a in seq:
            o.step([a])
            got.append(float(get(o, "va")[0]))
        wmap = {1: 1.0, 5: -1.0, 3: 0.0, 0: 1.0, 6: -1.0}
        expect = [0.0] * d + [wmap[a] for a in seq[:len(seq) - d]]
        assert got == expect, (d, got, expect)


def test_vectorization_equals_single_env_rows():
    """Eq. (7)/(8) are Eq. (5)/(6) row by row: env i of a batch evolves exactly
    as env i of another batch whose other rows differ."""
    cfg = inputs.workload("c2", n_envs=12)
    maps = inputs.make_maps(cfg)
    cfg_b = dict(cfg, n_envs=20)
    maps_b = inputs.make_maps(cfg_b)
    maps_b.grids[:12] = maps.grids  # same maps for the shared envs
    a = oracle.Oracle(cfg, maps)
    b = oracle.Oracle(cfg_b, maps_b)
    oa, _ = a.reset()
    ob, _ = b.reset()
    assert np.array_equal(oa, ob[:12])
    rng = np.random.default_rng(3)
    for _ in range(60):
        act = rng.integers(0, 7, 20).astype(np.int32)
        ra = a.step(act[:12])
        rb = b.step(act)
        for k in ("obs", "reward", "done", "flags"):
            assert np.array_equal(ra[k], rb[k][:12]), k


def test_fp64_shadow_kinematics_gate():
    """One-step FP32 kinematics stay within 1e-5 (relative, floors 1 cell,
    1 rad, v_max) of the FP64 shadow over a randomised C2 run."""
    cfg = inputs.workload("c2", n_envs=32)
    o = oracle.Oracle(cfg, inputs.make_maps(cfg))
    o.reset()
    st = oracle.Stats()
    for _ in range(100):
        o.step(o.uniform_actions(), stats=st)
    d = st.as_dict()
    assert d["kin_steps"] == 3200
    for k in ("max_rel_x", "max_rel_y", "max_rel_phi", "max_rel_vl", "max_rel_va"):
        assert d[k] <= 1e-5, (k, d[k])
    assert d["ties_coll"] == 0


# --------------------------------------------------------------------------
# LiDAR ray march
# --------------------------------------------------------------------------
def test_empty_unbordered_map_gives_max_range():
    R = 100
    side = 2 * R + 7
    o, cfg = one_env(np.zeros((side, side), np.uint8), range=float(R), n_rays=32)
    o.reset()
    put(o, x=side / 2, y=side / 2, phi=0.37, vl=0.0, va=0.0)
    r = o.step([7], hit_k=True)
    assert np.all(r["hit_k"] == -1)
    assert np.all(r["obs"][0, :32] == 1.0)


def test_robot_inside_block_hits_at_zero_and_collides():
    g = np.zeros((64, 64), np.uint8)
    g[20:40, 20:40] = 1
    o, cfg = one_env(g, n_rays=32)
    o.reset()
    put(o, x=30.5, y=30.5, phi=0.0, vl=0.0, va=0.0, tx=5.5, ty=5.5, dprev=30.0)
    for th in np.linspace(-math.pi, math.pi, 37):
        assert o.march(0, 30.5, 30.5, float(np.cos(th)), float(np.sin(th))) == 0
    r = o.step([7], final_obs=True)
    assert np.all(r["final_obs"][0, :32] == 0.0)  # every terminal range is 0
    assert r["flags"][0] & oracle.F_COLL and r["done"][0] == 1 and r["reward"][0] == -10.0
    # the post-reset observation is taken at a free pose
    assert r["obs"][0, :32].min() > 0.0


@pytest.mark.parametrize("phi,axis,sign", [(0.0, 0, -1), (math.pi, 0, +1),
                                            (math.pi / 2, 1, -1), (-math.pi / 2, 1, +1)])
def test_axis_aligned_wall_distance(phi, axis, sign):
    """A 3-ray 180-degree fan at a cell centre: the centre ray hits a wall
    column X (or row Y) at d = |X - floor(x0)| (- 1 when approaching from
    above), the side rays run along the other axis."""
    side = 101
    g = np.zeros((side, side), np.uint8)
    x0 = 50.5
    dist = 17
    # forward = (-cos phi, -sin phi)
    wall = int(math.floor(x0)) + sign * dist
    if axis == 0:
        g[:, wall] = 1
    else:
        g[wall, :] = 1
    o, cfg = one_env(g, n_rays=3, fov=math.pi, range=60.0)
    o.reset()
    put(o, x=x0, y=x0, phi=np.float32(phi), vl=0.0, va=0.0)
    r = o.step([7], hit_k=True)
    kc = r["hit_k"][0, 1]
    assert kc == dist, (kc, dist)
    # side rays run parallel to the wall: they end at the map edge
    edge = int(side - math.floor(x0))  # samples until x >= side along +axis
    for j in (0, 2):
        assert r["hit_k"][0, j] in (edge, int(math.floor(x0)) + 1), r["hit_k"][0]


def _dda_path(grid, x, y, ux, uy, tmax):
    """Amanatides & Woo (1987) voxel traversal in FP64: every cell the segment
    from (x, y) along u crosses, as (cell, t_entry, t_exit, occupied), until
    tmax or the first cell outside the map (which counts as occupied)."""
    H, W = grid.shape
    ix, iy = math.floor(x), math.floor(y)
    step_x = 1 if ux > 0 else -1
    step_y = 1 if uy > 0 else -1
    inf = float("inf")
    tdx = abs(1.0 / ux) if ux != 0 else inf
    tdy = abs(1.0 / uy) if uy != 0 else inf
    tx = ((ix + 1 - x) / ux if ux > 0 else (x - ix) / -ux) if ux != 0 else inf
    ty = ((iy + 1 - y) / uy if uy > 0 else (y - iy) / -uy) if uy != 0 else inf
    t = 0.0
    path = []
    while t <= tmax:
        outside = not (0 <= ix < W and 0 <= iy < H)
        occ = outside or grid[iy, ix] != 0
        t_exit = min(tx, ty)
        path.append(((ix, iy), t, t_exit, occ))
        if outside:
            break
        if tx < ty:
            t = tx
            tx += tdx
            ix += step_x
        else:
            t = ty
            ty += tdy
            iy += step_y
    return path


def test_march_against_fp64_voxel_walk():
    """Unit-step march vs an exact FP64 traversal on random maps. With t* the
    entry distance of the first occupied cell crossed: the march hits no
    earlier than t*; when it hits that cell, t* <= d < t* + ds; it may step
    past it only when the ray's chord through it is shorter than ds (a
    corner); and its hit cell lies on the traversal (up to FP32 sample
    rounding at a cell boundary, counted as a tie)."""
    cfg = inputs.workload("c2", n_envs=4)
    maps = inputs.make_maps(cfg)
    o = oracle.Oracle(cfg, maps)
    rng = np.random.default_rng(11)
    n_first = n_skip = n_tie = n_none = 0
    for trial in range(1500):
        m = int(rng.integers(0, 4))
        grid = maps.grids[m]
        while True:
            x, y = rng.uniform(2, 364, 2)
            if grid[int(y), int(x)] == 0:
                break
        th = rng.uniform(-math.pi, math.pi)
        ux, uy = np.float32(math.cos(th)), np.float32(math.sin(th))
        x, y = np.float32(x), np.float32(y)
        k = o.march(m, x, y, ux, uy)
        path = _dda_path(grid, float(x), float(y), float(ux), float(uy), 100.0)
        occ = [p for p in path if p[3]]
        first = occ[0] if occ else None
        if k < 0:
            n_none += 1
            # nothing up to R: every occupied cell crossed before R is a corner
            for c, t0, t1, _ in occ:
                if t0 <= 99.0:
                    assert t1 - t0 < 1.0 + 1e-4, (c, t0, t1)
            continue
        assert first is not None and k >= first[1] - 1e-4
        px = float(np.float32(x + np.float32(np.float32(k) * ux)))
        py = float(np.float32(y + np.float32(np.float32(k) * uy)))
        cell = (math.floor(px), math.floor(py))
        on_path = {p[0] for p in path}
        if cell not in on_path:
            n_tie += 1
            continue
        if cell == first[0]:
            n_first += 1
            assert first[1] - 1e-4 <= k < first[1] + 1.0 + 1e-4, (k, first)
        else:
            n_skip += 1
            assert first[2] - first[1] < 1.0 + 1e-4, (k, first)
    assert n_first + n_skip + n_tie + n_none == 1500
    assert n_first > 900 and n_tie <= 5
    assert n_skip < n_first  # every skip above was checked to be a corner


def test_supersampled_march_agrees_with_voxel_walk():
    """Pins the brute force itself: a x64 super-sampled FP64 march finds the
    traversal's first occupied cell."""
    cfg = inputs.workload("c2", n_envs=1)
    grid = inputs.make_maps(cfg).grids[0]
    rng = np.random.default_rng(12)
    for _ in range(200):
        while True:
            x, y = rng.uniform(2, 364, 2)
            if grid[int(y), int(x)] == 0:
                break
        th = rng.uniform(-math.pi, math.pi)
        ux, uy = math.cos(th), math.sin(th)
        occ = [p for p in _dda_path(grid, x, y, ux, uy, 100.0) if p[3]]
        first = occ[0] if occ else None
        hit = None
        for s in range(0, 100 * 64 + 1):
            t = s / 64.0
            cx, cy = math.floor(x + t * ux), math.floor(y + t * uy)
            if not (0 <= cx < 366 and 0 <= cy < 366) or grid[cy, cx]:
                hit = (cx, cy)
                break
        if first is None:
            assert hit is None
        else:
            assert hit is not None
            # same cell, or a corner thinner than 1/64 that the samples missed
            assert hit == first[0] or abs(first[1] - s / 64.0) < 1.0 / 32


# --------------------------------------------------------------------------
# Collision geometry
# --------------------------------------------------------------------------
def test_collision_touching_distance_is_inclusive():
    g = np.zeros((40, 40), np.uint8)
    g[10, 10] = 1  # square [10, 11] x [10, 11]
    o, cfg = one_env(g, robot_r=5.0)
    # axis: distance exactly 5 from the square's right edge
    assert o.collides(0, 16.0, 10.5)
    assert not o.collides(0, float(np.nextafter(np.float32(16.0), np.float32(20.0))), 10.5)
    # diagonal 3-4-5 from the corner (11, 11)
    assert o.collides(0, 14.0, 15.0)
    assert not o.collides(0, float(np.nextafter(np.float32(14.0), np.float32(20.0))), 15.0)
    # outside the map counts as occupied
    o2, _ = one_env(np.zeros((40, 40), np.uint8), robot_r=3.0)
    assert o2.collides(0, 3.0, 20.0) and not o2.collides(0, 3.0001, 20.0)


# --------------------------------------------------------------------------
# Reward, termination, truncation (Sec. 4.3.1)
# --------------------------------------------------------------------------
def test_reward_progress_arrival_timeout():
    o, cfg = one_env(_open_map(), K_lo=0.0, K_hi=0.0, t_max=6, arrive_r=4.0)
    o.reset()
    # target straight ahead (forward = -x at phi = 0), 10 cells away
    put(o, x=100.5, y=100.5, phi=0.0, vl=0.0, va=0.0, tx=90.5, ty=100.5, dprev=10.0, t=0)
    r = o.step([3])  # moves 1 cell toward the target
    assert r["done"][0] == 0 and abs(r["reward"][0] - (1.0 - 0.01)) < 1e-5
    r = o.step([3])
    assert abs(r["reward"][0] - 0.99) < 1e-5
    # now 8 away; after 4 more steps 4 away -> arrival (+10, terminated)
    for _ in range(3):
        r = o.step([3])
        assert r["done"][0] == 0
    r = o.step([3])
    assert r["done"][0] == 1 and r["reward"][0] == 10.0
    assert r["flags"][0] == oracle.F_TERM | oracle.F_ARRIVE
    # timeout: turning in place for t_max steps truncates, shaping reward kept
    o.reset()
    put(o, x=100.5, y=100.5, phi=0.0, vl=0.0, va=0.0, tx=50.5, ty=50.5,
        dprev=float(np.float32(math.hypot(50, 50))), t=0)
    for s in range(6):
        r = o.step([7])
    assert r["done"][0] == 1 and r["flags"][0] == oracle.F_TRUNC
    assert abs(r["reward"][0] + 0.01) < 1e-6


def test_collision_beats_arrival_and_autoreset_clears_episode():
    g = np.zeros((64, 64), np.uint8)
    g[30, 35] = 1
    o, cfg = one_env(g, arrive_r=4.0)
    o.reset()
    put(o, x=32.5, y=30.5, phi=0.0, vl=0.0, va=0.0, tx=33.5, ty=30.5, dprev=1.0, t=3)
    r = o.step([7], final_obs=True)
    assert r["done"][0] == 1 and r["reward"][0] == -10.0
    assert r["flags"][0] == oracle.F_TERM | oracle.F_COLL
    # AutoReset: new episode, zero velocity, empty FIFO, free start
    assert get(o, "t")[0] == 0 and get(o, "vl")[0] == 0 and get(o, "q0")[0] == oracle.STOP
    x, y = get(o, "x")[0], get(o, "y")[0]
    assert not o.collides(0, x, y)
    # the terminal observation shows the terminal pose: distance 1 cell
    assert abs(r["final_obs"][0, cfg["n_rays"] + 2] * math.sqrt(2) * 64 - 1.0) < 1e-5


def test_reset_draws_within_ranges_and_free():
    cfg = inputs.workload("c2", n_envs=64)
    maps = inputs.make_maps(cfg)
    o = oracle.Oracle(cfg, maps)
    _, rc = o.reset()
    assert rc == 0
    f, i = o.get_state()
    S = {k: f[:, n] for n, k in enumerate(oracle.STATE_F)}
    for name, lo, hi in (("dt", 0.05, 0.2), ("K", 0.0, 0.6), ("mu", 0.5, 1.0),
                         ("vmax", 5.0, 15.0), ("sigma", 0.0, 2.0)):
        assert S[name].min() >= np.float32(lo) and S[name].max() < np.float32(hi) + 1e-6, name
    assert set(np.unique(i[:, 1])) <= {0, 1, 2}
    for e in range(64):
        assert not o.collides(e, S["x"][e], S["y"][e])
        assert not o.collides(e, S["tx"][e], S["ty"][e])
        assert (S["tx"][e] - S["x"][e]) ** 2 + (S["ty"][e] - S["y"][e]) ** 2 > 16.0
        assert S["x"][e] % 1.0 == 0.5 and S["y"][e] % 1.0 == 0.5


def _disk_free(grid, px, py, r):
    """Brute force over every cell of the map and a margin around it: no
    occupied cell (outside the map counts as occupied) whose square lies
    within distance r of (px, py), touching included."""
    H, W = grid.shape
    for j in range(int(math.floor(py - r)) - 2, int(math.floor(py + r)) + 3):
        for i in range(int(math.floor(px - r)) - 2, int(math.floor(px + r)) + 3):
            occ = not (0 <= i < W and 0 <= j < H) or grid[j, i] != 0
            if not occ:
                continue
            dx = max(i - px, 0.0, px - (i + 1))
            dy = max(j - py, 0.0, py - (j + 1))
            if dx * dx + dy * dy <= r * r:
                return False
    return True


def test_reset_takes_first_free_candidate_and_documented_words():
    """Reading R10 (Sec. 3.2.4 per-episode randomisation, Sec. 3.2.5 reset),
    pinned with draws the test makes itself (its own Philox, above): the
    cells of the first start and target candidates are made occupied, and
    the oracle must take the first candidate in counter order whose disk is
    free (the target also farther than the arrival radius from the start).
    Each randomised parameter must come from its documented Philox word:
    (RESET_DR, 0) words 0-3 -> dt, K, mu, v_max; (RESET_DR, 1) words 0-2 ->
    sigma, delay, heading."""
    seed = (5 << 32) | 123
    key = (seed & _MASK, seed >> 32)
    side, n_envs, g = 48, 3, 0
    cfg = base_cfg(n_envs=n_envs, seed=seed, dt_lo=0.05, dt_hi=0.2, K_lo=0.0, K_hi=0.6,
                   mu_lo=0.5, mu_hi=1.0, vmax_lo=5.0, vmax_hi=15.0, sigma_lo=0.0,
                   sigma_hi=2.0, delay_lo=0, delay_hi=2, arrive_r=4.0)
    r, ra = cfg["robot_r"], cfg["arrive_r"]

    def cand(i, purpose, n):
        w = philox_py((i, g, purpose, n), key)
        return (w[0] * side) >> 32, (w[1] * side) >> 32  # floor(w * side / 2^32)

    grids, want = [], []
    for i in range(n_envs):
        grid = np.zeros((side, side), np.uint8)
        blocked_s, blocked_t = 2 + i, 1 + i  # leading candidates made occupied
        for n in range(blocked_s):
            cx, cy = cand(i, 2, n)
            grid[cy, cx] = 1
        for n in range(blocked_t):
            cx, cy = cand(i, 3, n)
            grid[cy, cx] = 1
        ns = next(n for n in range(1024) if _disk_free(grid, cand(i, 2, n)[0] + 0.5,
                                                         cand(i, 2, n)[1] + 0.5, r))
        sx, sy = cand(i, 2, ns)[0] + 0.5, cand(i, 2, ns)[1] + 0.5

        def target_ok(n):
            px, py = cand(i, 3, n)[0] + 0.5, cand(i, 3, n)[1] + 0.5
            return _disk_free(grid, px, py, r) and (px - sx) ** 2 + (py - sy) ** 2 > ra * ra
        nt = next(n for n in range(1024) if target_ok(n))
        assert ns >= blocked_s and nt >= blocked_t
        grids.append(grid)
        want.append((ns, nt, sx, sy, cand(i, 3, nt)[0] + 0.5, cand(i, 3, nt)[1] + 0.5))
    maps = inputs.Maps(grids=grids, env_to_map=np.arange(n_envs, dtype=np.int32))
    o = oracle.Oracle(cfg, maps)
    assert o.global_step == g
    _, rc = o.reset()
    assert rc == 0
    f32 = np.float32
    u24 = lambda w: f32(w >> 8) * f32(2.0 ** -24)
    for i in range(n_envs):
        ns, nt, sx, sy, tx, ty = want[i]
        for name, v in (("x", sx), ("y", sy), ("tx", tx), ("ty", ty)):
            assert get(o, name)[i] == f32(v), (i, name, ns, nt)
        a = philox_py((i, g, 1, 0), key)
        b = philox_py((i, g, 1, 1), key)
        span = lambda lo, hi: f32(cfg[hi]) - f32(cfg[lo])
        exp = {"dt": f32(cfg["dt_lo"]) + span("dt_lo", "dt_hi") * u24(a[0]),
               "K": f32(cfg["K_lo"]) + span("K_lo", "K_hi") * u24(a[1]),
               "mu": f32(cfg["mu_lo"]) + span("mu_lo", "mu_hi") * u24(a[2]),
               "vmax": f32(cfg["vmax_lo"]) + span("vmax_lo", "vmax_hi") * u24(a[3]),
               "sigma": f32(cfg["sigma_lo"]) + span("sigma_lo", "sigma_hi") * u24(b[0]),
               "phi": u24(b[2]) * f32(2.0 * math.pi) - f32(math.pi)}
        for name, v in exp.items():
            assert get(o, name)[i].view(np.uint32) == f32(v).view(np.uint32), (i, name)
        assert get(o, "delay")[i] == cfg["delay_lo"] + ((b[1] * 3) >> 32)


def test_full_map_fails_reset():
    o, cfg = one_env(np.ones((20, 20), np.uint8))
    _, rc = o.reset()
    assert rc == -4 and o.status == -4


def test_reset_is_deterministic_and_seeded():
    cfg = inputs.workload("c2", n_envs=8)
    maps = inputs.make_maps(cfg)
    a, _ = oracle.Oracle(cfg, maps).reset()
    b, _ = oracle.Oracle(cfg, maps).reset()
    c, _ = oracle.Oracle(dict(cfg, seed=2), maps).reset()
    assert np.array_equal(a, b) and not np.array_equal(a, c)


# --------------------------------------------------------------------------
# Noise and observation normalisation
# --------------------------------------------------------------------------
def test_noise_zero_sigma_exact_and_gaussian_moments():
    g = np.zeros((200, 200), np.uint8)
    g[:, 150] = 1
    n = 256
    o, cfg = one_env(g, n_envs=n, n_rays=1, fov=0.0, range=100.0, sigma_lo=1.5, sigma_hi=1.5)
    o.reset()
    # forward = +x at phi = pi: the wall at column 150 is 149.5 - 100 + ... away
    put(o, x=100.5, y=100.5, phi=np.float32(math.pi), vl=0.0, va=0.0, tx=10.5, ty=10.5,
        dprev=200.0, t=0)
    samples = []
    for _ in range(20):
        r = o.step(np.full(n, 7, np.int32), hit_k=True)
        assert np.all(r["hit_k"][:, 0] == 50)
        samples.append(r["obs"][:, 0] * 100.0 - 50.0)
    z = np.concatenate(samples).astype(np.float64)
    m, v = z.mean(), z.var()
    se = 1.5 / math.sqrt(z.size)
    assert abs(m) < 4 * se, m
    assert abs(v - 2.25) < 4 * 2.25 * math.sqrt(2.0 / z.size), v
    o0, _ = one_env(g, n_envs=n, n_rays=1, fov=0.0, range=100.0)
    o0.reset()
    put(o0, x=100.5, y=100.5, phi=np.float32(math.pi), vl=0.0, va=0.0, tx=10.5, ty=10.5,
        dprev=200.0, t=0)
    r = o0.step(np.full(n, 7, np.int32))
    assert np.all(r["obs"][:, 0] == np.float32(50.0) * np.float32(1.0 / 100.0))


def test_observation_bearing_and_distance():
    o, cfg = one_env(_open_map(100), n_rays=4)
    o.reset()
    nr = 4
    # heading phi = 0 moves along -x (Eq. (6)); counter-clockwise (left) of it
    # is -y, so a target at -y has bearing +pi/2
    for (tx, ty), want in (((40.5, 50.5), 0.0), ((50.5, 40.5), 0.5), ((50.5, 60.5), -0.5),
                           ((60.5, 50.5), 1.0)):
        put(o, x=50.5, y=50.5, phi=0.0, vl=0.0, va=0.0, tx=tx, ty=ty, dprev=10.0, t=0)
        r = o.step([7])
        b = float(r["obs"][0, nr + 3])
        assert min(abs(b - want), abs(abs(b) - 1.0) if want == 1.0 else 9) < 1e-6, (tx, ty, b)
        assert abs(r["obs"][0, nr + 2] - 10.0 / (math.sqrt(2) * 100)) < 1e-6


# --------------------------------------------------------------------------
# VEM and the Q-network
# --------------------------------------------------------------------------
def test_vem_epsilon_schedule():
    """Exploiting interval at E_min, exploring interval linear to
    E_min + E_max across env index (Sec. 3.1.1)."""
    e = oracle.vem_epsilon(8192, 8192, 0.01, 0.29)
    assert np.allclose(e, np.linspace(0.01, 0.3, 8192, dtype=np.float64), atol=1e-7)
    e2 = oracle.vem_epsilon(16, 3, 0.01, 0.8)
    assert np.all(e2[:13] == np.float32(0.01))
    assert np.allclose(e2[13:], [0.01, 0.41, 0.81])


def test_vem_extremes_and_rates():
    cfg = inputs.workload("c2", n_envs=4096)
    maps = inputs.single_maps([np.zeros((64, 64), np.uint8)], n_envs=4096)
    o = oracle.Oracle(cfg, maps)
    rng = np.random.default_rng(2)
    q = rng.normal(size=(4096, 7))
    greedy = q.argmax(1)
    a0, ex0 = o.vem(q, np.zeros(4096, np.float32))
    assert np.array_equal(a0, greedy) and ex0.sum() == 0
    a1, ex1 = o.vem(q, np.ones(4096, np.float32))
    assert ex1.all()
    counts = np.bincount(a1, minlength=7)
    exp = 4096 / 7
    assert ((counts - exp) ** 2 / exp).sum() < 6 + 5 * math.sqrt(12)
    eps = np.full(4096, 0.3, np.float32)
    tot = 0
    for g in range(10):
        o.global_step = g
        _, ex = o.vem(q, eps)
        tot += int(ex.sum())
    p = tot / 40960
    assert abs(p - 0.3) < 4 * math.sqrt(0.3 * 0.7 / 40960)
    # ties go to the lowest index
    qt = np.zeros((4096, 7))
    qt[:, 2] = qt[:, 5] = 1.0
    at, _ = o.vem(qt, np.zeros(4096, np.float32))
    assert np.all(at == 2)


def test_qnet_f64_matches_torch_float64():
    """FP64 Q-network = torch float64 Linear/ReLU stack (a library routine) on
    the same bf16 weights; the input rounding = torch's bf16 conversion."""
    import torch
    dims = (36, 256, 256, 7)
    w, b, _ = inputs.qnet_weights(dims)
    rng = np.random.default_rng(4)
    obs = rng.uniform(-1.2, 1.2, size=(50, 36)).astype(np.float32)
    q = oracle.qnet_f64(dims, w, b, obs)
    wt = torch.from_numpy(w.astype(np.int32) << 16).to(torch.int32).view(torch.float32).double()
    W1 = wt[:256 * 36].reshape(256, 36)
    W2 = wt[256 * 36:256 * 36 + 256 * 256].reshape(256, 256)
    W3 = wt[256 * 36 + 256 * 256:].reshape(7, 256)
    bt = torch.from_numpy(b).double()
    x = torch.from_numpy(obs).to(torch.bfloat16).double()
    h = torch.relu(torch.nn.functional.linear(x, W1, bt[:256]))
    h = torch.relu(torch.nn.functional.linear(h, W2, bt[256:512]))
    qt = torch.nn.functional.linear(h, W3, bt[512:]).numpy()
    assert np.allclose(q, qt, rtol=1e-12, atol=1e-12)
    # bf16 rounding of single values agrees with torch (round to nearest even)
    vals = np.float32([1.0, 1.00390625, 1.01171875, -3.3, 1e-3, 0.099999994, 65504.0])
    for v in vals:
        tb = torch.tensor([v]).to(torch.bfloat16).view(torch.int16).item() & 0xFFFF
        assert oracle.bf16_rne(float(v)) == tb
    qa = oracle.qnet_f64(dims, w, b, obs, round_act=True)
    assert np.abs(qa - q).max() < 0.05 and not np.array_equal(qa, q)


def test_paper_constants_fixture():
    """Table 7 defaults and the Sec. 4.3.1 action list (tests/golden) against
    the fixed-physics workload and the action table ratios."""
    import json
    with open(os.path.join(HERE, "golden", "paper_constants.json")) as f:
        pc = json.load(f)
    t7 = pc["table7_simulation_parameters"]
    c1 = inputs.workload("c1")
    assert c1["K_lo"] == c1["K_hi"] == t7["K"]
    assert c1["dt_lo"] == c1["dt_hi"] == t7["control_interval_s"]
    assert c1["omega_max"] == t7["max_angular_velocity_rad_s"]
    acts = pc["sec431_actions"]
    vmax = t7["max_linear_velocity_cm_s"]
    o, cfg = one_env(_open_map(), K_lo=0.0, K_hi=0.0)
    o.reset()
    for a, ident in zip(acts, (0, 1, 3, 5, 6)):
        put(o, x=128.0, y=128.0, phi=0.0, vl=0.0, va=0.0)
        o.step([ident])
        assert abs(get(o, "vl")[0] / 10.0 - a["v_cm_s"] / vmax) < 1e-7
        assert get(o, "va")[0] == np.float32(a["w_rad_s"])


def test_free_disk_means_no_hit_inside_radius():
    """For a collision-free pose, no ray can hit at a sample closer than the
    robot radius (such a cell would have been a collision): the first
    k_free = 3 samples (t = 0, 1, 2 < r = 3) never hit. The HIP march starts
    at k_free for such poses, so this property is what keeps it exact."""
    cfg = inputs.workload("c2", n_envs=8)
    maps = inputs.make_maps(cfg)
    o = oracle.Oracle(cfg, maps)
    rng = np.random.default_rng(21)
    checked = 0
    for _ in range(3000):
        m = int(rng.integers(0, 8))
        x, y = (float(np.float32(v)) for v in rng.uniform(-2, 368, 2))
        if o.collides(m, x, y):
            continue
        for th in rng.uniform(-math.pi, math.pi, 8):
            k = o.march(m, x, y, float(np.float32(math.cos(th))), float(np.float32(math.sin(th))))
            assert k == -1 or k >= 3, (m, x, y, th, k)
            checked += 1
    assert checked > 5000


def test_vem_or_decays_linearly_table6():
    """Table 6 (Sparrow): the exploring interval shrinks from 16 to 3 envs
    over 500K transitions. A linear decay loses its k-th env when the line
    16 - 13 T / decay first reaches 16 - k, i.e. at T = ceil(k decay / 13)."""
    import json
    from fractions import Fraction
    hp = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))["table6_sparrow_framework"]
    s, f, dec = hp["or_start"], hp["or_final"], hp["or_decay_steps_T"]
    assert oracle.vem_or(0, s, f, dec) == s
    assert oracle.vem_or(dec, s, f, dec) == f and oracle.vem_or(10 ** 12, s, f, dec) == f
    for k in range(1, s - f + 1):
        t_k = math.ceil(Fraction(k * dec, s - f))
        assert oracle.vem_or(t_k, s, f, dec) == s - k, k
        assert oracle.vem_or(t_k - 1, s, f, dec) == s - k + 1, k
    assert oracle.vem_or(12345, s, f, 0) == f  # no decay: the final interval
    # with the Table 6 probabilities the last env explores at E_min + E_max
    e = oracle.vem_schedule_epsilon(16, 0, hp["E_min"], hp["E_max"], s, f, dec)
    assert e[0] == np.float32(0.01) and e[-1] == np.float32(0.81)
    e_end = oracle.vem_schedule_epsilon(16, dec, hp["E_min"], hp["E_max"], s, f, dec)
    assert np.all(e_end[:13] == np.float32(0.01)) and np.allclose(e_end[13:], [0.01, 0.41, 0.81])
