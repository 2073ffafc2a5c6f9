"""Seeded synthetic inputs for the Sparrow step: workload presets and maps.

This module holds no arithmetic of the method itself. It produces the data a
caller hands to the library (and that the tests hand to the oracle): binary
occupancy grids shaped like the paper's training maps (Sec. 4.3.2 trains on
maps with randomly generated obstacles; Sec. 4.3.3 names blocky, fence-shaped
and mixed obstacle types), the per-env map assignment, configuration presets,
and Q-network weights. The paper's own map images are not available, so these
generators stand in for them.

Maps use numpy's PCG64 generator seeded from (230504180, workload id, map
index); the simulation's own random draws come from Philox inside the method
and are not made here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MAP_SEED = 230504180

# Per-env domain randomisation ranges and the rest of the physics. Velocities
# are in cells per second: a v_max of 0.5-1.5 cells per nominal 0.1 s control
# interval (Table 7) is 5-15 cells/s.
_DR_FULL = dict(dt_lo=0.05, dt_hi=0.2, K_lo=0.0, K_hi=0.6, mu_lo=0.5, mu_hi=1.0,
                vmax_lo=5.0, vmax_hi=15.0, omega_max=1.0, sigma_lo=0.0, sigma_hi=2.0,
                delay_lo=0, delay_hi=2)
# Fixed physics at the Table 7 defaults (K = 0.6, interval 0.1 s, no delay,
# v_max 1 cell per interval, no noise).
_DR_FIXED = dict(dt_lo=0.1, dt_hi=0.1, K_lo=0.6, K_hi=0.6, mu_lo=1.0, mu_hi=1.0,
                 vmax_lo=10.0, vmax_hi=10.0, omega_max=1.0, sigma_lo=0.0, sigma_hi=0.0,
                 delay_lo=0, delay_hi=0)

_COMMON = dict(n_actions=7, fov=math.radians(270.0), ds=1.0, robot_r=3.0, arrive_r=4.0,
               t_max=500, seed=1)

# Workload presets. "sides" lists the square map sides drawn uniformly per map.
WORKLOADS = {
    # plain step, fixed physics, 128^2 rectangle maps
    "c1": dict(_COMMON, **_DR_FIXED, n_envs=16, sides=(128,), style="rects", n_rays=32,
               range=64.0, steps=1000, qnet=None),
    # plain step, full randomisation, one 366^2 mixed map per env
    "c2": dict(_COMMON, **_DR_FULL, n_envs=4096, sides=(366,), style="mixed", n_rays=32,
               range=100.0, steps=10000, qnet=None),
    # batching: uneven sides, 64 rays, 64-step rollouts
    "c3": dict(_COMMON, **_DR_FULL, n_envs=16384, sides=(64, 128, 256, 366, 512),
               style="mixed", n_rays=64, range=128.0, steps=64, qnet=None),
    # fused actor, precision report
    "c4": dict(_COMMON, **_DR_FULL, n_envs=8192, sides=(366,), style="mixed", n_rays=32,
               range=100.0, steps=2048, qnet=(36, 256, 256, 7), eps=(0.01, 0.3)),
    # full collection loop
    "c5": dict(_COMMON, **_DR_FULL, n_envs=32768, sides=(256, 366, 512), style="mixed",
               n_rays=64, range=128.0, steps=10000, qnet=(68, 512, 512, 7), eps=(0.01, 0.3)),
    # the headline workload: c2 physics driven by c4's actor
    "m": dict(_COMMON, **_DR_FULL, n_envs=4096, sides=(366,), style="mixed", n_rays=32,
              range=100.0, steps=10000, qnet=(36, 256, 256, 7), eps=(0.01, 0.3)),
    # the paper's own task (Sec. 4.3.1/4.3.2) on c2's maps and physics: 27 rays,
    # 5 actions, Eq. (11) reward with +75 / -10, the 32-entry relative-pose
    # state and the 32-256-128-5 network. Cell size read as 2 cm: the 30 cm
    # margin of r_d is 15 cells; the planning distance D is 100 cells.
    "p": dict(_COMMON, **_DR_FULL, n_envs=4096, sides=(366,), style="mixed", n_rays=27,
              range=100.0, steps=2048, qnet=(32, 256, 128, 5), eps=(0.01, 0.3),
              task=dict(n_actions=5, reward=1, state=1, arrive_reward=75.0,
                        collide_reward=-10.0, plan_dist=100.0, near_dist=15.0,
                        weights=(0.3, 0.1, 0.3, 0.3, 0.1))),
}
WORKLOAD_IDS = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5, "m": 2, "p": 2}


def workload(name: str, **overrides) -> dict:
    cfg = dict(WORKLOADS[name])
    cfg.update(overrides)
    cfg["name"] = name
    return cfg


@dataclass
class Maps:
    """Ragged set of uint8 [H][W] grids (0 = free) plus the env->map table."""
    grids: list = field(default_factory=list)
    env_to_map: np.ndarray = None

    def flat(self):
        width = np.array([g.shape[1] for g in self.grids], np.int32)
        height = np.array([g.shape[0] for g in self.grids], np.int32)
        sizes = width.astype(np.int64) * height
        offsets = np.zeros(len(self.grids), np.int64)
        offsets[1:] = np.cumsum(sizes)[:-1]
        cells = np.concatenate([g.reshape(-1) for g in self.grids]).astype(np.uint8)
        return cells, offsets, width, height, np.ascontiguousarray(self.env_to_map, np.int32)


def _rng(wid: int, i: int) -> np.random.Generator:
    return np.random.default_rng([MAP_SEED, wid, i])


def _border(g: np.ndarray) -> None:
    g[0, :] = 1
    g[-1, :] = 1
    g[:, 0] = 1
    g[:, -1] = 1


def rect_map(side: int, rng: np.random.Generator, fill: float = 0.10) -> np.ndarray:
    """1-cell border, axis-aligned rectangles of 2..16 cells until the
    interior fill reaches `fill`."""
    g = np.zeros((side, side), np.uint8)
    _border(g)
    inner = (side - 2) * (side - 2)
    filled = 0
    while filled < fill * inner:
        w, h = int(rng.integers(2, 17)), int(rng.integers(2, 17))
        x0, y0 = int(rng.integers(1, side - 1)), int(rng.integers(1, side - 1))
        x1, y1 = min(x0 + w, side - 1), min(y0 + h, side - 1)
        reg = g[y0:y1, x0:x1]
        filled += int((reg == 0).sum())
        reg[...] = 1
    return g


def mixed_map(side: int, rng: np.random.Generator) -> np.ndarray:
    """1-cell border, then walls (p=0.3), rectangles (p=0.4) and discs (p=0.3)
    until a per-map fill drawn from U[0.05, 0.20] is reached. Shape sizes
    scale with side / 366."""
    g = np.zeros((side, side), np.uint8)
    _border(g)
    target = float(rng.uniform(0.05, 0.20)) * side * side
    filled = int(g.sum())
    sc = side / 366.0
    while filled < target:
        kind = rng.random()
        if kind < 0.3:  # wall
            thick = int(rng.integers(1, 3))
            length = int(rng.integers(8, max(9, side // 3 + 1)))
            x0, y0 = int(rng.integers(0, side)), int(rng.integers(0, side))
            if rng.random() < 0.5:
                reg = g[y0:y0 + thick, x0:x0 + length]
            else:
                reg = g[y0:y0 + length, x0:x0 + thick]
        elif kind < 0.7:  # rectangle
            w = max(1, int(round(int(rng.integers(3, 25)) * sc)))
            h = max(1, int(round(int(rng.integers(3, 25)) * sc)))
            x0, y0 = int(rng.integers(0, side)), int(rng.integers(0, side))
            reg = g[y0:y0 + h, x0:x0 + w]
        else:  # disc, cell-centre test in integers: (2dx)^2 + (2dy)^2 <= (2r)^2
            r = max(1, int(round(int(rng.integers(2, 11)) * sc)))
            cx, cy = int(rng.integers(0, side)), int(rng.integers(0, side))
            ys = np.arange(max(0, cy - r), min(side, cy + r + 1))
            xs = np.arange(max(0, cx - r), min(side, cx + r + 1))
            if len(ys) == 0 or len(xs) == 0:
                continue
            m = ((2 * (xs[None, :] - cx)) ** 2 + (2 * (ys[:, None] - cy)) ** 2) <= (2 * r) ** 2
            sub = g[ys[0]:ys[-1] + 1, xs[0]:xs[-1] + 1]
            filled += int(((sub == 0) & m).sum())
            sub[m] = 1
            continue
        filled += int((reg == 0).sum())
        reg[...] = 1
    return g


def _maps_chunk(job):
    cfg, first, n = job
    return make_maps(cfg, n_maps=n, first=first).grids


def make_maps(cfg: dict, n_maps: int | None = None, first: int = 0, workers: int = 1) -> Maps:
    """One map per env (env i uses map i), sides drawn per map from cfg['sides'].
    Map i depends only on (workload, i), so `workers` > 1 (a fork pool; call
    it before the process touches the GPU) gives the same maps faster."""
    n = cfg["n_envs"] if n_maps is None else n_maps
    if workers > 1 and n >= 4 * workers:
        import multiprocessing as mp
        step = -(-n // (4 * workers))
        jobs = [(cfg, first + lo, min(step, n - lo)) for lo in range(0, n, step)]
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_maps_chunk, jobs)
        return Maps(grids=[g for part in parts for g in part],
                    env_to_map=np.arange(n, dtype=np.int32))
    wid = WORKLOAD_IDS.get(cfg.get("name", "c2"), 0)
    grids = []
    for i in range(first, first + n):
        rng = _rng(wid, i)
        sides = cfg["sides"]
        side = int(sides[int(rng.integers(0, len(sides)))]) if len(sides) > 1 else int(sides[0])
        if cfg.get("style") == "rects":
            grids.append(rect_map(side, rng))
        else:
            grids.append(mixed_map(side, rng))
    return Maps(grids=grids, env_to_map=np.arange(n, dtype=np.int32))


def ascii_map(text: str) -> np.ndarray:
    """Hand-built map from ASCII art: '#' occupied, anything else free. The
    first line of `text` is row 0 (y = 0)."""
    rows = [r for r in text.strip("\n").split("\n")]
    w = max(len(r) for r in rows)
    g = np.zeros((len(rows), w), np.uint8)
    for y, r in enumerate(rows):
        for x, ch in enumerate(r):
            g[y, x] = 1 if ch == "#" else 0
    return g


def single_maps(grids, n_envs: int | None = None, env_to_map=None) -> Maps:
    grids = list(grids)
    if env_to_map is None:
        n = len(grids) if n_envs is None else n_envs
        env_to_map = np.arange(n, dtype=np.int32) % len(grids)
    return Maps(grids=grids, env_to_map=np.asarray(env_to_map, np.int32))


def qnet_weights(dims, seed: int = 7):
    """Kaiming-uniform weights U(+-sqrt(6/fan_in)) rounded to bf16 (RNE) and
    biases U(+-1/sqrt(fan_in)) in f32. Layout: W_l row-major [out][in]
    concatenated over layers; biases concatenated. Returns (w_bf16 uint16,
    b f32, w f32 masters)."""
    rng = np.random.default_rng([MAP_SEED, 99, seed])
    ws, bs = [], []
    for fan_in, fan_out in zip(dims[:-1], dims[1:]):
        bound = math.sqrt(6.0 / fan_in)
        ws.append(rng.uniform(-bound, bound, size=(fan_out, fan_in)).astype(np.float32))
        bb = 1.0 / math.sqrt(fan_in)
        bs.append(rng.uniform(-bb, bb, size=fan_out).astype(np.float32))
    w32 = np.concatenate([w.reshape(-1) for w in ws]).astype(np.float32)
    b32 = np.concatenate(bs).astype(np.float32)
    return _to_bf16_bits(w32), b32, w32


def _to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even float32 -> bf16 bit patterns (data preparation)."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    return r
