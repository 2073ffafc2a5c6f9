"""Pins of the learner oracle (Alg. 2 step 2: a DDQN update on a mini-batch;
Table 6 hyperparameters): finite differences of the loss, torch float64
autograd and torch's Adam (library routines), the double-Q target on a case
where the online and target networks disagree, and the target-network copy
period."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def tiny(seed=0, dims=(5, 6, 4, 3)):
    rng = np.random.default_rng(seed)
    d0, h1, h2, A = dims
    w = rng.normal(0, 0.7, h1 * d0 + h2 * h1 + A * h2).astype(np.float32)
    b = rng.normal(0, 0.3, h1 + h2 + A).astype(np.float32)
    return dims, w, b


def batch(rng, B, d0, A):
    s = rng.normal(size=(B, d0)).astype(np.float32)
    sn = rng.normal(size=(B, d0)).astype(np.float32)
    a = rng.integers(0, A, B).astype(np.int32)
    r = rng.normal(size=B).astype(np.float32)
    d = (rng.random(B) < 0.3).astype(np.uint8)
    return s, a, r, sn, d


def test_gradient_matches_central_differences():
    """gamma = 0 makes the target r, so the loss is a function of the online
    weights alone; lr = 0 keeps the weights for repeated evaluations."""
    dims, w, b = tiny(1)
    s, a, r, sn, d = batch(np.random.default_rng(2), 7, dims[0], dims[3])
    r *= 4  # some |delta| beyond the Huber knee
    L = oracle.Learner(dims, w, b, gamma=0.0, lr=0.0)
    loss, gw, gb = L.update(s, a, r, sn, d)
    h = 2e-5  # small enough that no ReLU or Huber kink lies within +-h here
    # float32 inputs: perturb by exactly representable steps in float64 space
    for idx in range(0, w.size, 3):
        wp, wm = w.astype(np.float64).copy(), w.astype(np.float64).copy()
        wp[idx] += h
        wm[idx] -= h
        lp = oracle.Learner(dims, wp.astype(np.float32), b, gamma=0.0, lr=0.0).update(s, a, r, sn, d)[0]
        lm = oracle.Learner(dims, wm.astype(np.float32), b, gamma=0.0, lr=0.0).update(s, a, r, sn, d)[0]
        hp = float(np.float32(wp[idx])) - float(w[idx])
        hm = float(w[idx]) - float(np.float32(wm[idx]))
        fd = (lp - lm) / (hp + hm)
        assert abs(fd - gw[idx]) <= 1e-7 + 1e-4 * abs(gw[idx]), (idx, fd, gw[idx])


def _torch_step(dims, w, b, s, a, r, sn, d, gamma, lr, k, wt=None, bt=None):
    torch = pytest.importorskip("torch")
    d0, h1, h2, A = dims
    t = lambda x: torch.tensor(np.asarray(x, np.float64))
    W = [t(w[:h1 * d0]).reshape(h1, d0), t(w[h1 * d0:h1 * d0 + h2 * h1]).reshape(h2, h1),
         t(w[h1 * d0 + h2 * h1:]).reshape(A, h2)]
    Bs = [t(b[:h1]), t(b[h1:h1 + h2]), t(b[h1 + h2:])]
    params = [p.requires_grad_() for p in W + Bs]
    Wt = [x.detach().clone() for x in W] if wt is None else [t(wt[:h1 * d0]).reshape(h1, d0),
          t(wt[h1 * d0:h1 * d0 + h2 * h1]).reshape(h2, h1), t(wt[h1 * d0 + h2 * h1:]).reshape(A, h2)]
    Bt = [x.detach().clone() for x in Bs] if bt is None else [t(bt[:h1]), t(bt[h1:h1 + h2]), t(bt[h1 + h2:])]

    def net(x, W_, B_):
        x = torch.relu(x @ W_[0].T + B_[0])
        x = torch.relu(x @ W_[1].T + B_[1])
        return x @ W_[2].T + B_[2]
    with torch.no_grad():
        a_star = net(t(sn), W, Bs).argmax(1)
        y = t(r) + gamma * (1 - t(d)) * net(t(sn), Wt, Bt).gather(1, a_star[:, None])[:, 0]
    q = net(t(s), W, Bs).gather(1, torch.tensor(a, dtype=torch.int64)[:, None])[:, 0]
    loss = torch.nn.functional.huber_loss(q, y, delta=k)
    loss.backward()
    grads = [p.grad.detach().clone() for p in params]
    opt = torch.optim.Adam(params, lr=lr, betas=(0.9, 0.999), eps=1e-8)
    opt.step()
    return float(loss), grads, [p.detach() for p in params]


def test_loss_gradients_and_adam_match_torch_float64():
    dims, w, b = tiny(3, dims=(6, 16, 8, 4))
    s, a, r, sn, d = batch(np.random.default_rng(4), 9, dims[0], dims[3])
    r *= 3
    L = oracle.Learner(dims, w, b, gamma=0.9, lr=1e-2, huber_k=1.0, target_every=0)
    loss, gw, gb = L.update(s, a, r, sn, d)
    tl, tg, tp = _torch_step(dims, w, b, s, a, r, sn, d, 0.9, 1e-2, 1.0)
    assert abs(loss - tl) <= 1e-12 * max(1.0, abs(tl))
    g_t = np.concatenate([g.reshape(-1).numpy() for g in tg[:3]])
    gb_t = np.concatenate([g.reshape(-1).numpy() for g in tg[3:]])
    np.testing.assert_allclose(gw, g_t, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(gb, gb_t, rtol=1e-10, atol=1e-13)
    w1, b1, _, _ = L.params()
    p_t = np.concatenate([p.reshape(-1).numpy() for p in tp[:3]])
    pb_t = np.concatenate([p.reshape(-1).numpy() for p in tp[3:]])
    np.testing.assert_allclose(w1, p_t, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(b1, pb_t, rtol=1e-12, atol=1e-14)


def test_double_q_target_uses_online_argmax_and_target_value():
    """After one update (target_every = 0 keeps the target at the initial
    weights) the online and target networks differ; build a batch where
    their argmax actions on s' differ and check the loss against torch's
    double-Q target, which differs from the plain max of the target."""
    torch = pytest.importorskip("torch")
    dims, w, b = tiny(5, dims=(4, 8, 8, 3))
    rng = np.random.default_rng(6)
    L = oracle.Learner(dims, w, b, gamma=0.9, lr=0.5, target_every=0)
    L.update(*batch(rng, 16, dims[0], dims[3]))
    w1, b1, wt, bt = L.params()
    cand = rng.normal(size=(400, dims[0])).astype(np.float32)
    qo, qt = L.q(cand), L.q(cand, target=True)
    pick = np.nonzero(qo.argmax(1) != qt.argmax(1))[0]
    assert pick.size >= 4
    sn = cand[pick[:4]]
    s, a, r, _, _ = batch(rng, 4, dims[0], dims[3])
    d = np.zeros(4, np.uint8)
    # a second learner in the same state (same seeds): online w1, target the
    # initial weights; its loss on this batch is torch's double-Q loss
    L3 = oracle.Learner(dims, w, b, gamma=0.9, lr=0.5, target_every=0)
    L3.update(*batch(np.random.default_rng(6), 16, dims[0], dims[3]))
    tl3, _, _ = _torch_step(dims, w1, b1, s, a, r, sn, d, 0.9, 0.0, 1.0, wt=wt, bt=bt)
    loss3 = L3.update(s, a, r, sn, d)[0]
    assert abs(loss3 - tl3) <= 1e-12
    q_on = L.q(sn)
    plain = r + 0.9 * qt[pick[:4]].max(1)
    double = r + 0.9 * qt[pick[:4]][np.arange(4), q_on.argmax(1)]
    assert not np.allclose(plain, double)


def test_target_network_copied_every_period():
    hp = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))["table6_sparrow_framework"]
    dims, w, b = tiny(7)
    rng = np.random.default_rng(8)
    L = oracle.Learner(dims, w, b, gamma=hp["gamma"], lr=1e-2, target_every=3)
    for step in range(1, 8):
        L.update(*batch(rng, 5, dims[0], dims[3]))
        w1, b1, wt, bt = L.params()
        if step % 3 == 0:
            assert np.array_equal(w1, wt) and np.array_equal(b1, bt), step
        else:
            assert not np.array_equal(w1, wt), step
    assert L.steps == 7
    with pytest.raises(ValueError):
        L.update(*batch(rng, 0, dims[0], dims[3]))


def simulate_asl(tfm, v_period, b_period, horizon):
    """Actor and learner running side by side in virtual time, each sleeping
    as the mechanism says after every step / update."""
    t_a = t_l = 0.0
    n_v = n_b = 0
    while min(t_a, t_l) < horizon:
        if t_a <= t_l:
            t_a += v_period
            tfm.actor(v_period)
            n_v += 1
            t_a += tfm.actor_sleep
        else:
            t_l += b_period
            tfm.learner(b_period)
            n_b += 1
            t_l += tfm.learner_sleep
    return n_v, n_b


@pytest.mark.parametrize("v,b", [(1.0, 0.05), (0.2, 0.3), (0.01, 0.001), (0.5, 0.0625)])
def test_tfm_holds_the_update_ratio_at_rho(v, b):
    """Eq. (TB2TV): with V = rho B the learner makes rho updates per
    vectorized step, so TPS = B_batch B_step / T_step stays at its target,
    whichever side is faster."""
    hp = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))["table6_sparrow_framework"]
    rho = hp["N"] * hp["TPS"] / hp["minibatch"]  # 16 * 256 / 256 = 16
    tfm = oracle.Tfm(rho)
    assert tfm.xi == 0.0  # nothing recorded yet
    n_v, n_b = simulate_asl(tfm, v, b, horizon=2000 * max(v, rho * b))
    assert abs(n_b / n_v - rho) / rho < 0.02, (n_v, n_b)
    # the slower side never sleeps
    if v > rho * b:
        assert tfm.actor_sleep == 0.0 and tfm.learner_sleep > 0.0
    else:
        assert tfm.actor_sleep > 0.0 and tfm.learner_sleep == 0.0
