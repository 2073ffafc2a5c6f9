"""Benchmark of the vectorized Sparrow step on one MI355X.

Workload (default): 4096 envs, each with its own 366 x 366 synthetic map,
32 LiDAR rays over 270 degrees with range 100, full per-env randomisation,
auto-reset; actions from the BF16 Q-network 36-256-256-7 with per-env
epsilon linearly spaced in [0.01, 0.3] (VEM).

A "step" is one vectorized step of all N envs: actor + simulator step.
  fused : K-step rollouts of the persistent kernel (actor fused, maps in LDS),
          one launch per K steps; the headline value
  plain : per step, uniform random actions + the plain step kernel
  plain+actor : per step, the separate actor kernel + the plain step kernel
  fused+collect : the fused rollouts adding every step's transitions to a
          device ring inside the kernel (reported beside the headline)
The fused path is timed over --repeats runs of exactly --steps steps each
(HIP events on the launch stream); value is the median run. Prints one JSON
line (rank 0, N=1 only).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_HBM_GBS = 8000.0
MI355X_CUS, MI355X_CLOCK_GHZ = 256, 2.4
# LDS: 128 B/clk/CU (the CDNA3 figure; CDNA4's is measured by the LDS probe,
# and the roofline takes the larger of the two)
MI355X_LDS_GBS = MI355X_CUS * 128 * MI355X_CLOCK_GHZ
# 32-bit vector lane-ops per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (the 157.3 TFLOP/s FP32 figure counts an FMA as 2 and packed FP32 as 2)
MI355X_VALU_TOPS = MI355X_CUS * 4 * 16 * MI355X_CLOCK_GHZ / 1e3
MI355X_BF16_TFLOPS = 2500.0

# Algorithmic work of one env-step, from the method's definition (not from
# the kernel's instruction count):
#   per marched ray sample: t_k (1), position x + t*u, y + t*u (4),
#     floor (2), outside-map clamp (2), row multiply-add (1), word shift (1),
#     address add (1), bit test (1)                              = 13 lane-ops
#   per ray: Philox4x32-10 (10 rounds x (2 mul-lo, 2 mul-hi, 4 xor,
#     2 key adds)) = 100, Box-Muller + noise add + clip + scale = 10 -> 110
#   per env: delay FIFO, command, Eq. (5), Eq. (6), wrap (~30), sincos (~30),
#     disk collision over <= 49 cells x 10 (~490), arrival/reward (~12),
#     observation scalars incl. atan2 (~40), VEM draw (~105)      = 707
ALG_OPS_PER_SAMPLE = 13
ALG_OPS_PER_RAY = 110
ALG_OPS_PER_ENV = 707
# The paper task's Eq. (11) adds per env-step: r_d1, r_d2, r_v (~12), r_alpha
# (the bearing's atan2 and |alpha|, ~45), the weighted sum (~10), and r_d,
# the margin-disk test (radius r + 15 = 18 cells, a 38-row box): per row, the
# run of cells within the disk around the robot's column (a square root and
# the two ends' exact per-cell tests, ~20) and one to three word reads (~10)
# -> 38 x 30 = 1,140
ALG_OPS_PER_ENV_EQ11 = 12 + 45 + 10 + 38 * 30
# LDS bytes of one env-step beyond the march's one word per sample: the
# collision test's 7 rows x 2 words x 4 B
LDS_COLLISION_BYTES = 56
# HBM bytes of one plain step of one env: the rows of its packed map within
# range of the robot (staged into LDS every step) + SoA state read and
# written (15 x 4 B x 2) + action (4) +
# obs and the library's copy (2 x 4 x obs_dim) + reward (4) + done (1) +
# per-ray hit indices (2 x n_rays)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def under_profiler():
    """True when a profiler's library is preloaded: it initialises the GPU
    before main() runs, so no fork pool may be started."""
    pre = os.environ.get("LD_PRELOAD", "")
    return "rocprof" in pre or any(k.startswith(("ROCP_", "ROCPROF")) for k in os.environ)


def map_workers():
    return 1 if under_profiler() else max(1, min(16, os.cpu_count() or 1))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000, help="timed vectorized steps per run")
    ap.add_argument("--warmup", type=int, default=256)
    ap.add_argument("--repeats", type=int, default=15, help="timed runs; the median is reported")
    ap.add_argument("--workload", default="m")
    ap.add_argument("--rollout", type=int, default=64, help="steps per fused rollout launch")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=10000,
                    help="plain-step leg length (the domain-randomized plain workload's 10^4 steps)")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the full-collection leg (32768 envs, ring buffer)")
    ap.add_argument("--c5-steps", type=int, default=2048)
    ap.add_argument("--c5-warmup", type=int, default=64)
    ap.add_argument("--no-k256", action="store_true",
                    help="skip the headline steps in 256-step launches")
    ap.add_argument("--no-task", action="store_true",
                    help="skip the paper's own task (27 rays, 5 actions, Eq. (11), 32-256-128-5)")
    ap.add_argument("--no-asl", action="store_true",
                    help="skip the actor/learner leg paced by the time feedback mechanism")
    ap.add_argument("--roofline-launches", type=int, default=16,
                    help="K-step launches timed for the roofline (K = --rollout), whatever --steps is")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the batching leg (16384 envs, uneven sides, 64 rays)")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the precision leg (8192 envs, 2048 traced fused steps)")
    ap.add_argument("--no-peaks", action="store_true", help="skip the LDS / HBM / MFMA probes")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--learner-only", action="store_true",
                    help="only run the learner leg and print its result (for kernel traces)")
    return ap.parse_args()


def copy_calibration(mb):
    """A plain copy kernel of known size: the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    n = mb * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4, "launches": 3}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(cfg, maps, w, b, seconds, cores=None):
    """The oracle (FP32 step + FP64 Q-network + VEM) on the host cores, on a
    bounded sample of envs, one Python thread per core over env shards (the
    C calls release the GIL)."""
    import oracle
    n_sample = 256
    cores = cores or min(os.cpu_count() or 1, 16)
    sub = dict(cfg, n_envs=n_sample)
    from paper_2305_04180_amd import inputs
    smaps = inputs.Maps(grids=maps.grids[:n_sample], env_to_map=np.arange(n_sample, dtype=np.int32))
    o = oracle.Oracle(sub, smaps)
    obs, _ = o.reset()
    dims = cfg["qnet"]
    D = o.obs_dim
    # the oracle's own VEM schedule over the full batch, first n_sample envs
    eps = oracle.vem_epsilon(cfg["n_envs"], cfg["n_envs"], cfg["eps"][0],
                             cfg["eps"][1] - cfg["eps"][0])
    eps_s = np.ascontiguousarray(eps[:n_sample])
    shards = np.array_split(np.arange(n_sample), cores)
    acts = np.zeros(n_sample, np.int32)
    rew = np.zeros(n_sample, np.float32)
    done = np.zeros(n_sample, np.uint8)
    nobs = np.zeros_like(obs)

    def actor_and_step(sh):
        e0, e1 = int(sh[0]), int(sh[-1]) + 1
        q = oracle.qnet_f64(dims, w, b, obs[e0:e1])
        # VEM for the shard's envs (same counters as the full batch)
        full_q = np.zeros((n_sample, 7))
        full_q[e0:e1] = q
        a, _ = o.vem(full_q, eps_s)
        acts[e0:e1] = a[e0:e1]
        o.step_range(e0, e1, acts, nobs, rew, done)

    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        th = [threading.Thread(target=actor_and_step, args=(sh,)) for sh in shards if len(sh)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        o.advance()
        obs[:] = nobs
        steps += 1
    dt = time.perf_counter() - t0
    return {"value": n_sample * steps / dt, "unit": "env-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{n_sample} of the {cfg['n_envs']} envs (same maps/physics), {steps} steps, "
                      f"FP64 Q-network + VEM + FP32 step, {dt:.1f} s"}


def cpu_plain(cfg, maps, seconds, n_sample=256, cores=None, max_steps=None):
    """The oracle's plain step (FP32, uniform random actions drawn by the
    oracle itself) on the host cores, on a bounded sample of envs of the
    workload, one Python thread per core over env shards."""
    import oracle
    from paper_2305_04180_amd import inputs
    n_sample = min(n_sample, cfg["n_envs"])
    cores = cores or min(os.cpu_count() or 1, 16)
    sub = dict(cfg, n_envs=n_sample)
    emap = np.asarray(maps.env_to_map[:n_sample])
    used = np.unique(emap)
    remap = np.searchsorted(used, emap).astype(np.int32)
    smaps = inputs.Maps(grids=[maps.grids[k] for k in used], env_to_map=remap)
    o = oracle.Oracle(sub, smaps)
    obs, _ = o.reset()
    shards = [sh for sh in np.array_split(np.arange(n_sample), cores) if len(sh)]
    rew = np.zeros(n_sample, np.float32)
    done = np.zeros(n_sample, np.uint8)
    nobs = np.zeros_like(obs)

    def step(sh, acts):
        o.step_range(int(sh[0]), int(sh[-1]) + 1, acts, nobs, rew, done)

    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and (max_steps is None or steps < max_steps):
        acts = o.uniform_actions()
        if len(shards) == 1:
            step(shards[0], acts)
        else:
            th = [threading.Thread(target=step, args=(sh, acts)) for sh in shards]
            for t in th:
                t.start()
            for t in th:
                t.join()
        o.advance()
        steps += 1
    dt = time.perf_counter() - t0
    return {"value": round(n_sample * steps / dt, 1), "unit": "env-steps/s", "cores": len(shards),
            "kind": "oracle",
            "sample": f"{n_sample} of the {cfg['n_envs']} envs (same maps/physics), {steps} steps, "
                      f"FP32 step with uniform actions, {dt:.1f} s"}


def c1_leg(with_cpu):
    """The small plain workload: 16 envs on 128^2 rectangle maps, 32 rays to
    range 64, fixed physics, uniform random actions, its 1000 steps, one
    sparrow_step per step (launch-bound at 16 envs); the oracle runs the same
    1000 steps on one host thread beside it."""
    import torch
    from paper_2305_04180_amd import inputs, sparrow
    cfg = inputs.workload("c1")
    maps = inputs.make_maps(cfg)
    env = sparrow.Env(cfg, maps)
    env.reset()
    a_buf = torch.zeros(cfg["n_envs"], dtype=torch.int32, device="cuda")
    for _ in range(16):
        env.random_actions(a_buf)
        env.step(a_buf)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = cfg["steps"]
    e0.record(stream)
    for _ in range(steps):
        env.random_actions(a_buf)
        env.step(a_buf)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert env.status() == 0
    out = {"value": round(cfg["n_envs"] * steps / (ms / 1e3), 1), "unit": "env-steps/s",
           "n_envs": cfg["n_envs"], "steps": steps, "ms_per_step": round(ms / steps, 5),
           "config": {"workload": "16 envs, own 128x128 rectangle map each (10% fill, border), "
                                  "32 rays/270 deg/range 64, dt 0.1 s, no delay, uniform actions"}}
    if with_cpu:
        out["cpu_baseline"] = cpu_plain(cfg, maps, 60.0, n_sample=cfg["n_envs"], cores=1,
                                        max_steps=steps)
    return out


def collection_c5(cfg, maps, steps, warmup, fused_add=False):
    """The full collection loop (Alg. 1 steps 2-5 with Alg. 2 step 1's
    sampling): per step the 68-512-512-7 actor + VEM (separate kernel), the
    step with AutoReset, and an add of the N transitions to the 2^22-slot
    device ring (fused_add: by the step kernel itself; else a separate add
    kernel); every 8 steps a uniform mini-batch of 256."""
    import torch
    from paper_2305_04180_amd import inputs, sparrow
    N, nr = cfg["n_envs"], cfg["n_rays"]
    D = nr + 4
    dims = cfg["qnet"]
    w, b, _ = inputs.qnet_weights(dims)
    env = sparrow.Env(cfg, maps)
    env.set_qnet(dims, w, b, env.vem_epsilon(N, cfg["eps"][0], cfg["eps"][1] - cfg["eps"][0]))
    ring = sparrow.Ring(1 << 22, nr, seed=cfg["seed"])
    cur = env.reset()
    env.autotune(steps=4)
    dev = env.device
    nxt = torch.zeros_like(cur)
    fo = torch.zeros_like(cur)
    act = torch.zeros(N, dtype=torch.int32, device=dev)
    rew = torch.zeros(N, dtype=torch.float32, device=dev)
    done = torch.zeros(N, dtype=torch.uint8, device=dev)
    B = 256
    sb = (torch.zeros(B, D, device=dev), torch.zeros(B, dtype=torch.int32, device=dev),
          torch.zeros(B, device=dev), torch.zeros(B, D, device=dev),
          torch.zeros(B, dtype=torch.uint8, device=dev))
    sidx = torch.zeros(B, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    state = {"cur": cur, "nxt": nxt, "t": 0}

    def one(ev=None):
        c, n_, t = state["cur"], state["nxt"], state["t"]
        marks = [] if ev is not None else None

        def mark():
            if marks is not None:
                e = torch.cuda.Event(enable_timing=True)
                e.record(stream)
                marks.append(e)
        mark()
        env.act(c, act)
        mark()
        if fused_add:
            # the step adds the transitions itself (s = c, the step's own copy)
            env.step_collect(ring, act, obs=n_, reward=rew, done=done)
            mark()
        else:
            env.step(act, obs=n_, reward=rew, done=done, final_obs=fo)
            mark()
            ring.push(c, act, rew, n_, done, fo)
        mark()
        if t % 8 == 7:
            ring.sample(B, t // 8, outs=sb, idx=sidx)
        mark()
        state["cur"], state["nxt"], state["t"] = n_, c, t + 1
        if ev is not None:
            ev.append(marks)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        one()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert env.status() == 0 and ring.status() == 0
    # per-phase times from a separate pass with events between the calls
    evs = []
    for _ in range(64):
        one(evs)
    torch.cuda.synchronize()
    names = ("act", "step", "add", "sample")
    phase = {k: float(np.mean([m[i].elapsed_time(m[i + 1]) for m in evs])) for i, k in
             enumerate(names)}
    mlp_flops = 2.0 * (dims[0] * dims[1] + dims[1] * dims[2] + dims[2] * dims[3])
    # the plain step stages the rows within range of each robot (taken at
    # the loop's final state)
    map_bytes = env_window_bytes(maps, cfg, env.get_state()[0][:, 1])
    step_bytes = map_bytes + N * (15 * 4 * 2 + 4 + 4 * D * 2 + 4 + 1 + 2 * nr)
    add_bytes = N * (3 * 4 * D + 4 + 4 + 1) + N * (2 * nr + 2 * 8 + 1 + 4)
    return {
        "metric": "env-steps/s of the full collection loop: actor 68-512-512-7 bf16 + VEM, step, "
                  "add to a 2^22-slot device ring, 256-draw sample every 8 steps",
        "value": round(N * steps / (ms / 1e3), 1), "unit": "env-steps/s",
        "n_envs": N, "steps": steps, "warmup": warmup, "ms_per_step": round(ms / steps, 5),
        "add": "inside the step kernel" if fused_add else "separate add kernel",
        "config": {"workload": "32768 envs, own map each, sides {256,366,512}, 64 rays/270 deg/"
                               "range 128, full DR, Q-MLP 68-512-512-7 bf16, eps linspace(0.01,0.3)",
                   "ring_slots": 1 << 22, "bytes_per_transition": 2 * nr + 2 * 8 + 1 + 4 + 0.125,
                   "minibatch": B, "sample_every": 8},
        "variants": {"step": env.get_variant(0)},
        "phase_ms_per_step": {k: round(v, 4) for k, v in phase.items()},
        "actor_mfma": {"achieved_tflops": round(mlp_flops * N / (phase["act"] / 1e3) / 1e12, 2),
                       "peak": MI355X_BF16_TFLOPS,
                       "frac": round(mlp_flops * N / (phase["act"] / 1e3) / 1e12 / MI355X_BF16_TFLOPS, 4)},
        "step_hbm": {"alg_bytes": int(step_bytes),
                     "achieved_gbs": round(step_bytes / (phase["step"] / 1e3) / 1e9, 1),
                     "frac": round(step_bytes / (phase["step"] / 1e3) / 1e9 / MI355X_HBM_GBS, 4)},
        "add_hbm": {"alg_bytes": int(add_bytes),
                    "achieved_gbs": round(add_bytes / (phase["add"] / 1e3) / 1e9, 1)},
    }


def paper_task(lds_peak, steps=2048, K=64):
    """The paper's own task (Sec. 4.3.1/4.3.2) at 4096 envs on 366^2 maps:
    27 rays, five actions, Eq. (11) reward, 32-entry relative-pose state,
    the 32-256-128-5 actor with VEM; fused rollouts and the plain step."""
    import torch
    from paper_2305_04180_amd import inputs, sparrow
    cfg = inputs.workload("p")
    N = cfg["n_envs"]
    maps = inputs.make_maps(cfg)
    dims = cfg["qnet"]
    w, b, _ = inputs.qnet_weights(dims)
    env = sparrow.Env(cfg, maps)
    env.set_qnet(dims, w, b, env.vem_epsilon(N, cfg["eps"][0], cfg["eps"][1] - cfg["eps"][0]))
    env.reset()
    env.autotune(steps=8)
    acts = torch.zeros(K, N, dtype=torch.int32, device="cuda")
    rew = torch.zeros(K, N, dtype=torch.float32, device="cuda")
    done = torch.zeros(K, N, dtype=torch.uint8, device="cuda")
    for _ in range(2):
        env.rollout(K, True, acts, rew, done)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps // K):
        env.rollout(K, True, acts, rew, done)
    e1.record(stream)
    torch.cuda.synchronize()
    fused_ms = e0.elapsed_time(e1)
    fused = N * (steps // K) * K / (fused_ms / 1e3)
    roof = fused_roofline(env, cfg, maps, K, 8, stream, lds_peak,
                          extra_env_ops=ALG_OPS_PER_ENV_EQ11,
                          kernel="k_rollout<64, QNetCfg<64,256,128>, false, true> "
                                 "(paper task: 27 rays, 5 actions, Eq. (11))")
    a = torch.zeros(N, dtype=torch.int32, device="cuda")
    for _ in range(16):
        env.random_actions(a)
        env.step(a)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(256):
        env.random_actions(a)
        env.step(a)
    e1.record(stream)
    torch.cuda.synchronize()
    plain = N * 256 / (e0.elapsed_time(e1) / 1e3)
    assert env.status() == 0
    return {"workload": "4096 envs, own 366x366 map each, 27 rays/270 deg/range 100, full DR, "
                        "5 actions, Eq. (11) reward (+75/-10, margin 15 cells, D 100 cells), "
                        "32-entry relative-pose state, Q-MLP 32-256-128-5 bf16",
            "fused_env_steps_per_s": round(fused, 1), "plain_env_steps_per_s": round(plain, 1),
            "fused_steps": (steps // K) * K, "plain_steps": 256,
            "roofline": roof,
            "variants": {"step": env.get_variant(0), "rollout": env.get_variant(1)}}


def learner_leg(updates=200, batch=256):
    """The DDQN update (Alg. 2 step 2) on its own: back-to-back updates on
    resident 256-row mini-batches of the 36-256-256-7 network, HIP events
    around them. Algorithmic FLOP per update: three forward passes (online
    s, online s', target s') and the backward pass of one (about two
    forwards), FP32 on the matrix cores in three launches."""
    import torch
    from paper_2305_04180_amd import inputs, sparrow
    dims = (36, 256, 256, 7)
    _, b, w32 = inputs.qnet_weights(dims)
    L = sparrow.Learner(dims, w32, b, max_batch=batch)
    g = torch.Generator(device="cuda").manual_seed(1)
    s = torch.rand(batch, dims[0], device="cuda", generator=g)
    sn = torch.rand(batch, dims[0], device="cuda", generator=g)
    a = torch.randint(0, dims[3], (batch,), device="cuda", dtype=torch.int32, generator=g)
    r = torch.randn(batch, device="cuda", generator=g)
    d = (torch.rand(batch, device="cuda", generator=g) < 0.1).to(torch.uint8)
    for _ in range(10):
        L.update(s, a, r, sn, d)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(updates):
        L.update(s, a, r, sn, d)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / updates
    fwd = 2.0 * batch * (dims[0] * dims[1] + dims[1] * dims[2] + dims[2] * dims[3])
    flop = 5.0 * fwd
    tf = flop / (ms / 1e3) / 1e12
    return {"updates": updates, "minibatch": batch, "network": list(dims),
            "ms_per_update": round(ms, 4), "updates_per_s": round(1e3 / ms, 1),
            "roofline": {"bound": "latency", "achieved": round(tf, 3), "peak": 157.3,
                         "unit": "TFLOP/s", "frac": round(tf / 157.3, 5),
                         "flop_per_update": int(flop),
                         "note": "FP32 peak (vector and matrix alike); a 256-row update is three "
                                 "dependent launches (row-block forward, row-block backward, "
                                 "weight gradients with their Adam step), each bound by memory "
                                 "round trips rather than arithmetic"}}


def asl_tfm(seconds=3.0, n_envs=256, tps=32, batch=256, learn_start=8192):
    """Actor and learner side by side (Sec. 3.1.2, Alg. 1 and Alg. 2) on one
    GPU, paced by the time feedback mechanism: the actor thread steps the
    envs (actor kernel + step + add to the ring) on its stream, the learner
    thread samples a mini-batch and runs the DDQN update on its own; each
    reports its period and sleeps as told. Reports the TPS achieved against
    its target."""
    import threading
    import torch
    from paper_2305_04180_amd import inputs, sparrow
    cfg = inputs.workload("c2", n_envs=n_envs)
    maps = inputs.make_maps(cfg)
    N, D = n_envs, cfg["n_rays"] + 4
    dims = (D, 256, 256, 7)
    wb, b, w32 = inputs.qnet_weights(dims)
    s_act = torch.cuda.Stream()
    s_learn = torch.cuda.Stream()
    with torch.cuda.stream(s_act):
        env = sparrow.Env(cfg, maps, stream=s_act)
        env.set_qnet(dims, wb, b, env.vem_epsilon(N, 0.01, 0.8))
        ring = sparrow.Ring(1 << 20, cfg["n_rays"], seed=3, stream=s_act)
        cur = env.reset()
        nxt, fo = torch.zeros_like(cur), torch.zeros_like(cur)
        act = torch.zeros(N, dtype=torch.int32, device="cuda")
        rew = torch.zeros(N, dtype=torch.float32, device="cuda")
        done = torch.zeros(N, dtype=torch.uint8, device="cuda")
        sb = [torch.zeros(batch, D, device="cuda"), torch.zeros(batch, dtype=torch.int32, device="cuda"),
              torch.zeros(batch, device="cuda"), torch.zeros(batch, D, device="cuda"),
              torch.zeros(batch, dtype=torch.uint8, device="cuda")]
        sidx = torch.zeros(batch, dtype=torch.int32, device="cuda")
    learner = sparrow.Learner(dims, w32, b, max_batch=batch, stream=s_learn)
    rho = N * tps / batch
    tfm = sparrow.Tfm(rho)
    lock = threading.Lock()  # the sharer's occupancy flag (Sec. 3.1.2)
    stop = threading.Event()
    counts = {"v": 0, "b": 0, "v_time": 0.0, "b_time": 0.0}
    state = {"cur": cur, "nxt": nxt}

    def actor():
        while not stop.is_set():
            t0 = time.perf_counter()
            with torch.cuda.stream(s_act):
                env.act(state["cur"], act)
                env.step(act, obs=state["nxt"], reward=rew, done=done, final_obs=fo)
                with lock:
                    ring.push(state["cur"], act, rew, state["nxt"], done, fo)
            s_act.synchronize()
            state["cur"], state["nxt"] = state["nxt"], state["cur"]
            dt = time.perf_counter() - t0
            tfm.actor(dt)
            counts["v"] += 1
            counts["v_time"] += dt
            z = tfm.actor_sleep
            if z > 0:
                time.sleep(z)

    def learn():
        while not stop.is_set():
            if ring.size < learn_start:
                time.sleep(0.001)
                continue
            t0 = time.perf_counter()
            with lock:
                with torch.cuda.stream(s_act):  # ordered after the adds
                    ring.sample(batch, counts["b"], outs=sb, idx=sidx)
                    ev = torch.cuda.Event()
                    ev.record(s_act)
            s_learn.wait_event(ev)
            with torch.cuda.stream(s_learn):
                learner.update(*sb)
            s_learn.synchronize()
            dt = time.perf_counter() - t0
            tfm.learner(dt)
            counts["b"] += 1
            counts["b_time"] += dt
            z = tfm.learner_sleep
            if z > 0:
                time.sleep(z)

    ta, tl = threading.Thread(target=actor), threading.Thread(target=learn)
    ta.start()
    tl.start()
    # measure once the learner has started
    while ring.size < learn_start:
        time.sleep(0.01)
    time.sleep(0.5)
    v0, b0, t0 = counts["v"], counts["b"], time.perf_counter()
    time.sleep(seconds)
    v1, b1, t1 = counts["v"], counts["b"], time.perf_counter()
    stop.set()
    ta.join()
    tl.join()
    assert env.status() == 0 and ring.status() == 0
    dv, db = v1 - v0, b1 - b0
    return {"n_envs": N, "target_tps": tps, "minibatch": batch, "rho": rho,
            "achieved_tps": round(batch * db / max(N * dv, 1), 3),
            "vectorized_steps_per_s": round(dv / (t1 - t0), 1),
            "updates_per_s": round(db / (t1 - t0), 1),
            "mean_actor_period_ms": round(1e3 * counts["v_time"] / max(counts["v"], 1), 4),
            "mean_learner_period_ms": round(1e3 * counts["b_time"] / max(counts["b"], 1), 4),
            "window_s": round(t1 - t0, 2)}


def kernel_source_hash():
    """sha1 of the HIP sources (kernels and the host side that launches
    them): identifies the kernel build that a counter summary in profiles/
    was taken from."""
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2305_04180_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()


def counter_traffic(kernel_key):
    """A per-launch figure from the committed rocprofv3 counter summary:
    HBM bytes (FETCH_SIZE x calibration + WRITE_SIZE) for the
    traffic_bytes_per_launch_* keys, the VALU busy fraction for valu_busy_*;
    None when the summary was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "counters_m4096.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.strip().strip("|").strip()
        if ":" in line and line.split(":")[0].strip() in ("source_sha1", kernel_key):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha1") != kernel_source_hash() or kernel_key not in vals:
        return None
    v = float(vals[kernel_key])
    return int(v) if v.is_integer() else v


def env_map_bytes(maps):
    """Packed LDS-ready bytes of all maps: one set word, then H + 2 rows of
    ceil((W + 2) / 32) words, padded to 16 bytes."""
    tot = 0
    for g in maps.grids:
        H, W = g.shape
        words = 1 + ((W + 2 + 31) // 32) * (H + 2)
        tot += ((words + 3) // 4) * 16
    return tot


def env_window_bytes(maps, cfg, y):
    """Bytes the windowed step stages for envs whose robots are at rows y
    (float array [N]): the rows within ceil(max(range, r)) + 2 of the
    robot's row, clipped to the map's rows -1..H, plus the word in front."""
    win = math.ceil(max(cfg["range"], cfg["robot_r"])) + 2
    tot = 0
    for e, m in enumerate(maps.env_to_map):
        H, W = maps.grids[m].shape
        wpr = (W + 2 + 31) // 32
        cy = min(max(math.floor(float(y[e])), -1), H)
        rows = min(H, cy + win) - max(-1, cy - win) + 1
        tot += 4 * (rows * wpr + 1)
    return tot


def peaks(skip):
    """The device's own peak rates from the library's probes (LDS reads of 16
    and 4 bytes per lane, an HBM copy, dense BF16 MFMA)."""
    if skip:
        return None
    from paper_2305_04180_amd import sparrow
    out = {}
    for name, kind, size, iters, unit in (
            ("lds_b128", sparrow.PEAK_LDS128, 0, 2048, "GB/s"),
            ("lds_b32", sparrow.PEAK_LDS32, 0, 2048, "GB/s"),
            ("hbm_copy", sparrow.PEAK_HBM_COPY, 1 << 30, 8, "GB/s"),
            ("mfma_bf16", sparrow.PEAK_MFMA_BF16, 0, 256, "TFLOP/s")):
        rate, _ = sparrow.peak(kind, size, iters)
        out[name] = round(rate / (1e12 if unit == "TFLOP/s" else 1e9), 1)
    out["units"] = {"lds_b128": "GB/s", "lds_b32": "GB/s", "hbm_copy": "GB/s (read + write)",
                    "mfma_bf16": "TFLOP/s"}
    out["per_cu_clk"] = {"lds_b128_bytes": round(out["lds_b128"] / MI355X_CUS / MI355X_CLOCK_GHZ, 1),
                         "lds_b32_bytes": round(out["lds_b32"] / MI355X_CUS / MI355X_CLOCK_GHZ, 1)}
    return out


def fused_roofline(env, cfg, maps, K, launches, stream, lds_peak, extra_env_ops=0,
                   kernel="", counter_key=None, lds_b32_peak=None):
    """Roofline of the fused rollout kernel on its own K-step launches (HIP
    events around each on the launch stream), whatever the
    metric's step count. Algorithmic work per launch (N K env-steps):
      LDS  4 B per marched sample of the definition (k = 0 .. first hit, or
           0 .. M without one; counted over one traced launch) + the
           collision test's 56 B per env-step + the maps staged once
      HBM  maps once + state in and out + final observation and hit indices
           + per step reward, done and action
      MFMA the Q-network's 2 (d0 h1 + h1 h2 + h2 A) FLOP per env-step
    bound / frac: the largest of the three fractions (published peaks for HBM
    and MFMA; for LDS the larger of 128 B/clk/CU and the probe's
    measurement). The vector-ALU lane-op count is reported beside it, and
    so are the LDS fraction against the probe's 4-byte read rate (the
    march's own access width) and the VALU busy fraction that the committed
    counter summary measured on the same kernel sources."""
    import torch
    N, nr, D = cfg["n_envs"], cfg["n_rays"], env.obs_dim
    dims = cfg["qnet"]
    acts = torch.zeros(K, N, dtype=torch.int32, device="cuda")
    rew = torch.zeros(K, N, dtype=torch.float32, device="cuda")
    done = torch.zeros(K, N, dtype=torch.uint8, device="cuda")
    obs = torch.zeros(N, D, dtype=torch.float32, device="cuda")
    env.rollout(K, True, acts, rew, done, obs)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(launches)]
    for a, b2 in ev:
        a.record(stream)
        env.rollout(K, True, acts, rew, done, obs)
        b2.record(stream)
    torch.cuda.synchronize()
    launch_ms = np.array([a.elapsed_time(b2) for a, b2 in ev])
    _, _, _, _, _, hits_t = env.rollout_trace(K, True)
    torch.cuda.synchronize()
    M = int(cfg["range"] / cfg["ds"])
    h = hits_t.to(torch.int64)
    samples = float(torch.where(h < 0, torch.full_like(h, M), h).add(1).sum().item()) / (K * N)
    del hits_t, h
    assert env.status() == 0
    avg_s = float(launch_ms.mean()) / 1e3
    es = N * K
    maps_b = env_map_bytes(maps)
    lds_b = (4.0 * samples + LDS_COLLISION_BYTES) * es + maps_b
    hbm_b = maps_b + N * (15 * 4 * 2 + 4 * D * 2 + 2 * nr + 4) + es * (4 + 1 + 4)
    flops = 2.0 * (dims[0] * dims[1] + dims[1] * dims[2] + dims[2] * dims[3]) * es
    ops = (ALG_OPS_PER_SAMPLE * samples + ALG_OPS_PER_RAY * nr + ALG_OPS_PER_ENV
           + extra_env_ops) * es
    lds_gbs, hbm_gbs = lds_b / avg_s / 1e9, hbm_b / avg_s / 1e9
    mfma_tf, alu_t = flops / avg_s / 1e12, ops / avg_s / 1e12
    fr = {"lds": lds_gbs / lds_peak, "hbm": hbm_gbs / MI355X_HBM_GBS,
          "mfma": mfma_tf / MI355X_BF16_TFLOPS}
    bound = max(fr, key=fr.get)
    ach = {"lds": (lds_gbs, lds_peak, "GB/s"), "hbm": (hbm_gbs, MI355X_HBM_GBS, "GB/s"),
           "mfma": (mfma_tf, MI355X_BF16_TFLOPS, "TFLOP/s")}[bound]
    return {"bound": bound, "achieved": round(ach[0], 2), "peak": round(ach[1], 1), "unit": ach[2],
            "frac": round(fr[bound], 5),
            "traffic": counter_traffic(counter_key) if counter_key else None,
            "traffic_alg_bytes": int(hbm_b),
            "kernel": kernel, "rollout_k": K, "launches": launches,
            "avg_launch_ms": round(avg_s * 1e3, 4),
            "launch_ms_min_max": [round(float(launch_ms.min()), 4), round(float(launch_ms.max()), 4)],
            "samples_per_env_step": round(samples, 2),
            "lds_frac": round(fr["lds"], 5), "hbm_frac": round(fr["hbm"], 5),
            "mfma_frac": round(fr["mfma"], 5),
            "alg_per_launch": {"lds_bytes": int(lds_b), "hbm_bytes": int(hbm_b),
                               "mfma_flop": int(flops), "env_steps": es},
            "lds_b32_frac": round(lds_gbs / lds_b32_peak, 5) if lds_b32_peak else None,
            "valu_busy_counters": counter_traffic(counter_key.replace("traffic_bytes_per_launch",
                                                                      "valu_busy"))
            if counter_key else None,
            "alu": {"achieved": round(alu_t, 3), "peak": round(MI355X_VALU_TOPS, 2),
                    "unit": "T lane-ops/s", "frac": round(alu_t / MI355X_VALU_TOPS, 4),
                    "units": f"32-bit lane-ops from the definition: {ALG_OPS_PER_SAMPLE}/sample, "
                             f"{ALG_OPS_PER_RAY}/ray, {ALG_OPS_PER_ENV + extra_env_ops}/env; "
                             "peak 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz"}}


def c3_leg(cfg, maps, launches=16, K=64):
    """Batching workload: 16384 envs on uneven square maps (sides 64..512),
    64 rays to range 128, full randomisation; uniform random actions;
    autotuned variant; K = 64 rollouts."""
    import torch
    from paper_2305_04180_amd import sparrow
    N = cfg["n_envs"]
    env = sparrow.Env(cfg, maps)
    env.reset()
    tune = env.autotune(steps=4)
    stream = torch.cuda.current_stream()
    acts = torch.zeros(K, N, dtype=torch.int32, device="cuda")
    rew = torch.zeros(K, N, dtype=torch.float32, device="cuda")
    done = torch.zeros(K, N, dtype=torch.uint8, device="cuda")
    obs = torch.zeros(N, env.obs_dim, dtype=torch.float32, device="cuda")
    for _ in range(2):
        env.rollout(K, False, acts, rew, done, obs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(launches):
        env.rollout(K, False, acts, rew, done, obs)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert env.status() == 0
    return {"value": round(N * K * launches / (ms / 1e3), 1), "unit": "env-steps/s",
            "n_envs": N, "steps": K * launches, "rollout_k": K, "launches": launches,
            "ms_per_step": round(ms / (K * launches), 5),
            "config": {"workload": "16384 envs, own map each, sides uniform in {64,128,256,366,512}, "
                                   "64 rays/270 deg/range 128, full DR, uniform random actions, "
                                   "64-step rollouts, autotuned"},
            "variants": {"rollout": env.get_variant(1), "step": env.get_variant(0)},
            "autotune_chosen": tune.get("chosen")}


def c4_leg(cfg, maps, launches=16, K=64):
    """Precision workload's fused rollout at 8192 envs (366^2 maps, 32 rays,
    BF16 36-256-256-7 actor, eps linspace(0.01, 0.3)): env-steps/s of K = 64
    rollouts. Returns the env for the precision report."""
    import torch
    from paper_2305_04180_amd import sparrow
    N = cfg["n_envs"]
    dims = cfg["qnet"]
    w, b, _ = inputs_mod().qnet_weights(dims)
    env = sparrow.Env(cfg, maps)
    env.set_qnet(dims, w, b, env.vem_epsilon(N, cfg["eps"][0], cfg["eps"][1] - cfg["eps"][0]))
    env.reset()
    stream = torch.cuda.current_stream()
    acts = torch.zeros(K, N, dtype=torch.int32, device="cuda")
    rew = torch.zeros(K, N, dtype=torch.float32, device="cuda")
    done = torch.zeros(K, N, dtype=torch.uint8, device="cuda")
    obs = torch.zeros(N, env.obs_dim, dtype=torch.float32, device="cuda")
    env.rollout(K, True, acts, rew, done, obs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(launches):
        env.rollout(K, True, acts, rew, done, obs)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert env.status() == 0
    return env, {"value": round(N * K * launches / (ms / 1e3), 1), "unit": "env-steps/s",
                 "n_envs": N, "steps": K * launches, "rollout_k": K,
                 "variants": {"rollout": env.get_variant(1)}}


def inputs_mod():
    from paper_2305_04180_amd import inputs
    return inputs


def oracle_checks(cfg4, env4, cfg, maps, sample_every=32, launches=32, K=64):
    """Reports that need the oracle (run in the CPU leg):
    c4: 2048 fused steps at 8192 envs with every step traced; on every
        sample_every-th env, each greedy choice of the fused actor against the
        FP64 oracle network's argmax on the observation that step's actor saw
        (exploration draws from the oracle's own VEM), and max |dQ| of the
        actor kernel's Q values on those rows;
    m_shadow: the oracle's FP64 kinematics shadow on 256 envs of the headline
        workload over 500 uniform-action steps: largest one-step relative
        error against the 1e-5 tolerance, and the cell-boundary ties."""
    import torch
    import oracle
    from paper_2305_04180_amd import inputs
    from tests.parity_util import ExploreDraws, qnet_f64_threads, traced_actor_rows
    out = {}
    if env4 is not None:
        N = cfg4["n_envs"]
        dims = cfg4["qnet"]
        w, b, _ = inputs.qnet_weights(dims)
        e_min, e_span = cfg4["eps"][0], cfg4["eps"][1] - cfg4["eps"][0]
        sample = np.arange(0, N, sample_every)
        env4.reset()
        t0 = time.time()
        obs_in, acts, steps = traced_actor_rows(env4, launches, K, sample)
        draws = ExploreDraws(cfg4["seed"], N, oracle.vem_epsilon(N, N, e_min, e_span))
        ex = np.stack([draws.flags(g)[sample] for g in steps]).reshape(-1)
        x = obs_in.reshape(-1, env4.obs_dim)
        a = acts.reshape(-1)
        q, greedy = env4.qnet_forward(torch.as_tensor(x).cuda())
        torch.cuda.synchronize()
        q = q.cpu().numpy().astype(np.float64)
        greedy = greedy.cpu().numpy()
        q64 = qnet_f64_threads(dims, w, b, x, workers=min(16, os.cpu_count() or 1))
        top = q64.argmax(1)
        srt = np.sort(q64, axis=1)
        gap = srt[:, -1] - srt[:, -2]
        g = ~ex
        clear = g & (gap > 0.05)
        out["c4_precision"] = {
            "envs": N, "sampled_envs": int(len(sample)), "steps": int(launches * K),
            "rows": int(x.shape[0]), "greedy_rows": int(g.sum()),
            "greedy_agreement_vs_fp64": round(float((a[g] == top[g]).mean()), 6),
            "agreement_fp64_gap_over_0.05": round(float((a[clear] == top[clear]).mean()), 6),
            "rows_gap_over_0.05": int(clear.sum()),
            "fused_equals_actor_kernel": bool(np.array_equal(greedy[g], a[g])),
            "max_abs_dq": float(np.abs(q - q64).max()),
            "observations": "the rollout's own: the observation each step's actor saw "
                            f"(every step of {launches} traced K = {K} launches)",
            "seconds": round(time.time() - t0, 1)}
    # FP64 kinematics shadow and ties on a sample of the headline workload
    n_s = 256
    sub = dict(cfg, n_envs=n_s)
    smaps = inputs.Maps(grids=maps.grids[:n_s], env_to_map=np.arange(n_s, dtype=np.int32))
    o = oracle.Oracle(sub, smaps)
    o.reset()
    st = oracle.Stats()
    n_steps = 500
    for _ in range(n_steps):
        o.step(o.uniform_actions(), stats=st)
    d = st.as_dict()
    rel = max(d["max_rel_x"], d["max_rel_y"], d["max_rel_phi"], d["max_rel_vl"], d["max_rel_va"])
    out["m_shadow"] = {
        "envs": n_s, "steps": n_steps, "tolerance": 1e-5,
        "max_rel_one_step": rel, "within_tolerance": bool(rel <= 1e-5),
        "max_rel": {k: d[k] for k in ("max_rel_x", "max_rel_y", "max_rel_phi", "max_rel_vl",
                                      "max_rel_va")},
        "boundary_ties_ray_samples": int(d["ties_ray"]), "samples": int(d["samples"]),
        "boundary_ties_collision": int(d["ties_coll"]), "kin_steps": int(d["kin_steps"]),
        "what": "FP32 step against the FP64 shadow re-synced every step; ties = samples or "
                "collision tests whose cell differs between FP32 and FP64 positions "
                "(counted, not failed)"}
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU; envs are independent, so N GPUs would each run "
              "their own shard with no per-step exchange (see the design notes). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2305_04180_amd import inputs, sparrow

    if args.copy_mb:
        assert torch.cuda.is_available(), "bench.py needs the GPU"
        copy_calibration(args.copy_mb)
        return
    if args.learner_only:
        assert torch.cuda.is_available(), "bench.py needs the GPU"
        print(json.dumps({"learner": learner_leg()}), flush=True)
        return
    # maps of the other workloads, generated with a process pool before this
    # process touches the GPU (one process under a profiler, whose preloaded
    # library has already initialised it)
    maps5 = maps3 = maps4 = None
    cfg3, cfg4, cfg5 = inputs.workload("c3"), inputs.workload("c4"), inputs.workload("c5")
    for flag, cfg_x, name in ((args.no_c5, cfg5, "c5"), (args.no_c3, cfg3, "c3"),
                              (args.no_c4, cfg4, "c4")):
        if flag:
            continue
        t0 = time.time()
        mx = inputs.make_maps(cfg_x, workers=map_workers())
        log(f"[bench] {name}: {len(mx.grids)} maps in {time.time() - t0:.1f}s")
        if name == "c5":
            maps5 = mx
        elif name == "c3":
            maps3 = mx
        else:
            maps4 = mx
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    cfg = inputs.workload(args.workload)
    N = cfg["n_envs"]
    log(f"[bench] generating {N} maps ({cfg['sides']})")
    t0 = time.time()
    maps = inputs.make_maps(cfg)
    log(f"[bench] maps ready in {time.time() - t0:.1f}s")
    dims = cfg["qnet"]
    w, b, _ = inputs.qnet_weights(dims)

    env = sparrow.Env(cfg, maps)
    env.set_qnet(dims, w, b, env.vem_epsilon(N, cfg["eps"][0], cfg["eps"][1] - cfg["eps"][0]))
    env.reset()
    tune = {}
    if not args.no_tune:
        tune = env.autotune(steps=8)
        log(f"[bench] autotune: {json.dumps(tune)}")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    # ---------------- fused rollout ----------------
    # Each run times exactly args.steps vectorized steps: launches of K steps
    # (K = --rollout, or --steps when that is smaller) plus one shorter launch
    # for the remainder.
    K = min(args.rollout, args.steps)
    n_full, rem = divmod(args.steps, K)
    n_warm = max(1, math.ceil(args.warmup / K))
    acts = torch.zeros(K, N, dtype=torch.int32, device="cuda")
    rew = torch.zeros(K, N, dtype=torch.float32, device="cuda")
    done = torch.zeros(K, N, dtype=torch.uint8, device="cuda")
    obs = torch.zeros(N, env.obs_dim, dtype=torch.float32, device="cuda")
    log(f"[bench] fused warmup {n_warm} x {K} steps")
    for _ in range(n_warm):
        env.rollout(K, True, acts, rew, done, obs)
    if rem:
        env.rollout(rem, True, acts, rew, done, obs)
    torch.cuda.synchronize()

    def fused_run():
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(n_full)]
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        t_start.record(stream)
        for i in range(n_full):
            ev[i][0].record(stream)
            env.rollout(K, True, acts, rew, done, obs)
            ev[i][1].record(stream)
        if rem:
            env.rollout(rem, True, acts, rew, done, obs)
        t_end.record(stream)
        torch.cuda.synchronize()
        return (t_start.elapsed_time(t_end), time.perf_counter() - wall0,
                [a.elapsed_time(b2) for a, b2 in ev])

    runs = []
    for r in range(args.repeats):
        runs.append(fused_run())
        log(f"[bench] fused run {r}: {N * args.steps / (runs[-1][0] / 1e3) / 1e6:.1f} M env-steps/s")
    run_ms = [x[0] for x in runs]
    med = int(np.argsort(run_ms)[len(run_ms) // 2])
    fused_ms, wall, _ = runs[med]
    steps_fused = args.steps
    fused_rate = N * steps_fused / (fused_ms / 1e3)
    assert env.status() == 0
    log(f"[bench] fused: {fused_rate / 1e6:.1f} M env-steps/s ({fused_ms / steps_fused * 1e3:.2f} us/step)")

    # the LDS, HBM and MFMA probes run after the headline timing, so that
    # the MFMA probe's power draw does not precede it
    pk = peaks(args.no_peaks)
    if pk:
        log(f"[bench] peaks: {pk}")
    lds_peak = max(MI355X_LDS_GBS, pk["lds_b128"] if pk else 0.0)

    # ---------------- roofline of the fused kernel ----------------
    # on its own launches of the workload's rollout length, whatever --steps is
    KR = args.rollout
    roofline = fused_roofline(env, cfg, maps, KR, args.roofline_launches, stream, lds_peak,
                              kernel="k_rollout<64, QNetCfg<64,256,256>> (fused actor + step)",
                              counter_key="traffic_bytes_per_launch_k_rollout",
                              lds_b32_peak=pk["lds_b32"] if pk else None)
    log(f"[bench] roofline: {json.dumps(roofline)}")

    # ---------------- the same steps in 256-step launches ----------------
    # (the workload's rollouts are 64 steps; longer launches amortise the
    # per-launch map staging and launch over more steps)
    fused_k256 = None
    K2 = 256
    n2, rem2 = divmod(args.steps, K2)
    if args.no_k256:
        n2, rem2 = 0, 0
    a2 = torch.zeros(K2, N, dtype=torch.int32, device="cuda")
    r2 = torch.zeros(K2, N, dtype=torch.float32, device="cuda")
    d2 = torch.zeros(K2, N, dtype=torch.uint8, device="cuda")
    for _ in range(2 if n2 else 0):
        env.rollout(K2, True, a2, r2, d2, obs)
    if rem2:
        env.rollout(rem2, True, a2, r2, d2, obs)
    torch.cuda.synchronize()
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    k0.record(stream)
    for _ in range(n2):
        env.rollout(K2, True, a2, r2, d2, obs)
    if rem2:
        env.rollout(rem2, True, a2, r2, d2, obs)
    k1.record(stream)
    torch.cuda.synchronize()
    if n2:
        fused_k256 = N * args.steps / (k0.elapsed_time(k1) / 1e3)
        log(f"[bench] fused, 256-step launches: {fused_k256 / 1e6:.1f} M env-steps/s")

    # ---------------- fused rollout that also fills the ring ----------------
    # Alg. 1 steps 2-5 in one kernel: the same rollouts, each step's N
    # transitions added to a 2^22-slot device ring inside the kernel.
    ring = sparrow.Ring(1 << 22, cfg["n_rays"], seed=cfg["seed"])

    def collect_run(terminal):
        for _ in range(n_warm):
            env.rollout_collect(ring, K, True, obs=obs, terminal_obs=terminal)
        torch.cuda.synchronize()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(n_full):
            env.rollout_collect(ring, K, True, obs=obs, terminal_obs=terminal)
        if rem:
            env.rollout_collect(ring, rem, True, obs=obs, terminal_obs=terminal)
        c1.record(stream)
        torch.cuda.synchronize()
        assert env.status() == 0 and ring.status() == 0
        return c0.elapsed_time(c1)
    collect_ms = collect_run(True)
    collect_pr_ms = collect_run(False)
    fused_collect = {
        "value": round(N * args.steps / (collect_ms / 1e3), 1), "unit": "env-steps/s",
        "steps": args.steps, "ring_slots": 1 << 22, "ring_size": ring.size,
        "over_fused": round(fused_ms / collect_ms, 4),
        "post_reset_s_next_value": round(N * args.steps / (collect_pr_ms / 1e3), 1),
        "what": "fused rollout that adds (s, a, r, s', done) of every step to the device ring "
                "inside the kernel (uint8 ranges, binary16 scalars, int8 action, FP32 reward, "
                "done bit); s' of a done transition is its terminal observation (value) or the "
                "post-reset observation (post_reset_s_next_value)"}
    del ring
    log(f"[bench] fused+collect: {fused_collect['value'] / 1e6:.1f} M env-steps/s "
        f"(post-reset s': {fused_collect['post_reset_s_next_value'] / 1e6:.1f} M)")

    # ---------------- plain step ----------------
    P = args.plain_steps
    a_buf = torch.zeros(N, dtype=torch.int32, device="cuda")
    for _ in range(32):
        env.random_actions(a_buf)
        env.step(a_buf)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(P):
        env.random_actions(a_buf)
        env.step(a_buf)
    s1.record(stream)
    torch.cuda.synchronize()
    plain_ms = s0.elapsed_time(s1)
    plain_rate = N * P / (plain_ms / 1e3)
    log(f"[bench] plain: {plain_rate / 1e6:.1f} M env-steps/s")
    # plain step with the separate actor kernel
    q0 = torch.cuda.Event(enable_timing=True)
    q1 = torch.cuda.Event(enable_timing=True)
    q0.record(stream)
    for _ in range(P):
        env.act(env.obs, a_buf)
        env.step(a_buf)
    q1.record(stream)
    torch.cuda.synchronize()
    pa_rate = N * P / (q0.elapsed_time(q1) / 1e3)
    log(f"[bench] plain+actor: {pa_rate / 1e6:.1f} M env-steps/s")

    D, nr = env.obs_dim, cfg["n_rays"]
    win_bytes = env_window_bytes(maps, cfg, env.get_state()[0][:, 1])
    step_bytes = win_bytes + N * (15 * 4 * 2 + 4 + 4 * D * 2 + 4 + 1 + 2 * nr)
    plain_hbm = step_bytes * P / (plain_ms / 1e3) / 1e9
    plain_roofline = {"bound": "hbm", "achieved": round(plain_hbm, 1), "peak": MI355X_HBM_GBS,
                      "unit": "GB/s", "frac": round(plain_hbm / MI355X_HBM_GBS, 4),
                      "traffic": counter_traffic("traffic_bytes_per_launch_k_step"),
                      "traffic_alg_bytes": int(step_bytes),
                      "kernel": "k_step (one launch per step, map rows within range "
                                "staged) + k_actions",
                      "staged_map_bytes_per_step": int(win_bytes),
                      "whole_map_bytes": int(env_map_bytes(maps))}

    log("[bench] c1 (16 envs, 1000 plain steps)")
    c1 = c1_leg(not args.no_cpu)
    log(f"[bench] c1: {json.dumps(c1)}")

    c3 = None
    if maps3 is not None:
        log("[bench] c3 batching (16384 envs, uneven sides, 64 rays)")
        c3 = c3_leg(cfg3, maps3)
        log(f"[bench] c3: {c3['value'] / 1e6:.1f} M env-steps/s, variant {c3['variants']}")
    env4 = c4 = None
    if maps4 is not None:
        log("[bench] c4 fused rollout (8192 envs)")
        env4, c4 = c4_leg(cfg4, maps4)
        log(f"[bench] c4: {c4['value'] / 1e6:.1f} M env-steps/s")

    cpu = None
    c2_cpu = None
    checks = {}
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(cfg, maps, w, b, args.cpu_seconds)
        one = cpu_baseline(cfg, maps, w, b, args.cpu_seconds / 3, cores=1)
        cpu["single_thread_value"] = one["value"]
        cpu["cpu_model"] = cpu_model()
        cpu["nproc"] = os.cpu_count()
        log("[bench] cpu baselines of the plain workloads (oracle)")
        c2_cpu = cpu_plain(inputs.workload("c2"), maps, args.cpu_seconds / 3)
        c2_cpu["single_thread_value"] = cpu_plain(inputs.workload("c2"), maps,
                                                  args.cpu_seconds / 6, cores=1)["value"]
        if c3 is not None:
            c3["cpu_baseline"] = cpu_plain(cfg3, maps3, args.cpu_seconds / 3)
        log("[bench] oracle checks: c4 precision, kinematics shadow")
        checks = oracle_checks(cfg4, env4, cfg, maps)
        log(f"[bench] oracle checks: {json.dumps(checks)}")
    if c4 is not None and "c4_precision" in checks:
        c4["precision"] = checks["c4_precision"]
    env4 = None

    c5 = None
    if maps5 is not None:
        log("[bench] c5 full collection loop")
        c5 = collection_c5(cfg5, maps5, args.c5_steps, args.c5_warmup)
        # the same loop with the add done by the step kernel (sparrow_step_collect)
        log("[bench] c5 loop with the add inside the step")
        ins = collection_c5(cfg5, maps5, max(16, args.c5_steps // 4), args.c5_warmup,
                            fused_add=True)
        c5["add_in_step"] = {"value": ins["value"], "steps": ins["steps"],
                             "phase_ms_per_step": ins["phase_ms_per_step"]}
        log(f"[bench] c5: {c5['value'] / 1e6:.1f} M env-steps/s, phases {c5['phase_ms_per_step']}")

    ptask = None
    if not args.no_task:
        log("[bench] the paper's own task (Sec. 4.3.1/4.3.2)")
        ptask = paper_task(lds_peak)
        log(f"[bench] paper task: {ptask}")

    learner = None
    if not args.no_asl:
        log("[bench] learner updates back to back")
        learner = learner_leg()
        log(f"[bench] learner: {learner['ms_per_update']} ms per update")

    asl = None
    if not args.no_asl:
        log("[bench] actor + learner paced by the time feedback mechanism")
        asl = asl_tfm()
        log(f"[bench] asl: {asl}")

    out = {
        "metric": "env-steps/s at N=4096, 366^2 maps, 32 rays; fused BF16 vs plain; % HBM/LDS peak",
        "value": round(fused_rate, 1),
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": steps_fused,
        "warmup": n_warm * K + rem,
        "repeats": args.repeats,
        "run_values": [round(N * steps_fused / (m / 1e3), 1) for m in run_ms],
        "ms_per_step": round(fused_ms / steps_fused, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 sim + bf16 mfma actor",
        "data": "synthetic",
        "config": {"workload": "4096 envs, own 366x366 map each, 32 rays/270 deg/range 100, "
                               "full DR, Q-MLP 36-256-256-7 bf16, eps linspace(0.01,0.3)",
                   "n_envs": N, "rollout_k": K, "remainder_k": rem, "launches": n_full + (rem > 0),
                   "parallelism": "single GPU"},
        "plain_env_steps_per_s": round(plain_rate, 1),
        "plain_actor_env_steps_per_s": round(pa_rate, 1),
        "c2_plain": {"value": round(plain_rate, 1), "unit": "env-steps/s", "steps": P,
                     "what": "the plain leg is the domain-randomized plain workload: the same "
                             "4096 envs, maps and physics with uniform random actions, "
                             f"{P} steps",
                     "cpu_baseline": c2_cpu},
        "c1_plain": c1,
        "fused_over_plain": round(fused_rate / plain_rate, 3),
        "fused_collect": fused_collect,
        "fused_k256_env_steps_per_s": round(fused_k256, 1) if fused_k256 else None,
        "wall_s_timed": round(wall, 4),
        "variants": {"step": env.get_variant(0), "rollout": env.get_variant(1)},
        "kernel_source_sha1": kernel_source_hash(),
        "roofline": roofline,
        "plain_roofline": plain_roofline,
        "cpu_baseline": cpu,
        "precision": checks.get("c4_precision"),
        "kinematics_shadow": checks.get("m_shadow"),
        "peaks": pk,
        "c3_batching": c3,
        "c4_fused": c4,
        "collection_c5": c5,
        "paper_task": ptask,
        "paper_context": {"value": 8155.0, "unit": "env-steps/s", "kind": "context",
                          "hardware": "NVIDIA RTX 3090 + AMD 3990X (the paper's platform)",
                          "derived_from": "Table 4: maximal real-time factor 815.5 at N = 64, "
                                          "divided by the 0.1 s control interval of Table 7",
                          "note": "a different workload (map size and ray count not stated); "
                                  "not the target, so vs_baseline stays null"},
        "asl_tfm": asl,
        "learner": learner,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
