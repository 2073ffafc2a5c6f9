"""The precision workload at full size: 8192 envs on 366^2 maps, 32 rays, the
BF16 36-256-256-7 actor with per-env epsilon linearly spaced in [0.01, 0.3],
2048 fused steps (32 rollouts of 64 steps, every step traced). On a sample of
envs, every greedy choice the fused actor made is compared with the argmax of
the FP64 oracle network on the observation that step's actor saw (the
rollout's own observations), and the standalone actor kernel's Q values on
the same rows are held to the first-order error bound."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2305_04180_amd import inputs
from tests.parity_util import (ExploreDraws, qnet_bound, qnet_f64_threads, to_np,
                               traced_actor_rows)

pytestmark = pytest.mark.gpu


def test_c4_greedy_agreement_2048_steps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2305_04180_amd import sparrow
    cfg = inputs.workload("c4")
    N, K, launches = cfg["n_envs"], 64, 32
    sample = np.arange(0, N, 32)
    print(f"\n[case] c4 N={N} {launches}x{K} traced fused steps, {len(sample)} sampled envs",
          flush=True)
    maps = inputs.make_maps(cfg)
    dims = cfg["qnet"]
    w, b, _ = inputs.qnet_weights(dims)
    e_min, e_span = cfg["eps"][0], cfg["eps"][1] - cfg["eps"][0]
    env = sparrow.Env(cfg, maps)
    env.set_qnet(dims, w, b, env.vem_epsilon(N, e_min, e_span))
    env.reset()
    obs_in, acts, steps = traced_actor_rows(env, launches, K, sample)
    assert env.status() == 0
    draws = ExploreDraws(cfg["seed"], N, oracle.vem_epsilon(N, N, e_min, e_span))
    explored = np.stack([draws.flags(g)[sample] for g in steps])  # [2048, sampled envs]
    x = obs_in.reshape(-1, env.obs_dim)
    a = acts.reshape(-1)
    ex = explored.reshape(-1)
    # the standalone actor kernel gives the fused actor's greedy choice on the
    # same observation (same arithmetic), and its Q values
    q, greedy = env.qnet_forward(torch.as_tensor(x).cuda())
    torch.cuda.synchronize()
    q, greedy = to_np(q).astype(np.float64), to_np(greedy)
    assert np.array_equal(greedy[~ex], a[~ex]), int((greedy[~ex] != a[~ex]).sum())
    q64 = qnet_f64_threads(dims, w, b, x)
    dq = np.abs(q - q64)
    bound = qnet_bound(dims, w, b, x)
    assert np.all(dq <= bound), (dq.max(), (dq / bound).max())
    agree = float((a[~ex] == q64.argmax(1)[~ex]).mean())
    print(f"c4: {x.shape[0]} rows, {int((~ex).sum())} greedy; agreement with the FP64 actor "
          f"{agree:.5f}; max|dQ| {dq.max():.3e} (max dQ/bound {(dq / bound).max():.3f}); "
          f"explored {ex.mean():.4f}", flush=True)
    assert agree >= 0.995
