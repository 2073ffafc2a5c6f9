"""CPU oracle of the vectorized Sparrow step (arXiv 2305.04180, Sec. 3.2).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product path (the HIP library
and its binding) never does. This module is the ctypes wrapper around the
plain C oracle in ``sparrow_oracle.c``; it shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "sparrow_oracle.c")
SRC_RING = os.path.join(HERE, "ring_oracle.c")
SRC_LEARNER = os.path.join(HERE, "learner_oracle.c")

STOP = 7
N_ACTIONS = 7
F_TERM, F_TRUNC, F_COLL, F_ARRIVE = 1, 2, 4, 8
P_RESET_DR, P_RESET_START, P_RESET_TARGET = 1, 2, 3
P_NOISE, P_NOISE_RESET, P_ACTION_UNIFORM, P_EXPLORE = 4, 5, 6, 7
STATE_F = ("x", "y", "phi", "vl", "va", "tx", "ty", "dprev", "dt", "K", "mu", "vmax", "sigma")
STATE_I = ("t", "delay", "q0", "q1")


def build(force: bool = True) -> str:
    """Compile the oracle with strict IEEE binary32 semantics."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", LIB_PATH, SRC, SRC_RING, SRC_LEARNER, "-lm"]
        subprocess.check_call(cmd)
    return LIB_PATH


class _Config(C.Structure):
    _fields_ = [
        ("n_envs", C.c_int32), ("n_rays", C.c_int32), ("n_actions", C.c_int32),
        ("fov", C.c_float), ("range", C.c_float), ("ds", C.c_float),
        ("robot_r", C.c_float), ("arrive_r", C.c_float), ("t_max", C.c_int32),
        ("dt_lo", C.c_float), ("dt_hi", C.c_float), ("K_lo", C.c_float), ("K_hi", C.c_float),
        ("mu_lo", C.c_float), ("mu_hi", C.c_float), ("vmax_lo", C.c_float),
        ("vmax_hi", C.c_float), ("omega_max", C.c_float), ("sigma_lo", C.c_float),
        ("sigma_hi", C.c_float), ("delay_lo", C.c_int32), ("delay_hi", C.c_int32),
        ("seed", C.c_uint64),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("max_rel_x", C.c_double), ("max_rel_y", C.c_double), ("max_rel_phi", C.c_double),
        ("max_rel_vl", C.c_double), ("max_rel_va", C.c_double),
        ("ties_ray", C.c_uint64), ("ties_coll", C.c_uint64), ("samples", C.c_uint64),
        ("rays", C.c_uint64), ("kin_steps", C.c_uint64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class _Task(C.Structure):
    _fields_ = [("n_actions", C.c_int32), ("reward", C.c_int32), ("state", C.c_int32),
                ("arrive_reward", C.c_float), ("collide_reward", C.c_float),
                ("plan_dist", C.c_float), ("near_dist", C.c_float), ("w_d1", C.c_float),
                ("w_d2", C.c_float), ("w_v", C.c_float), ("w_alpha", C.c_float),
                ("w_d", C.c_float)]


REWARD_PROGRESS, REWARD_EQ11 = 0, 1
STATE_TARGET, STATE_RELATIVE = 0, 1


class LearnerConfig(C.Structure):
    _fields_ = [("gamma", C.c_double), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("adam_eps", C.c_double), ("huber_k", C.c_double),
                ("target_every", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Config), C.c_int32, P, P, P, P, P]
        L.orc_destroy.argtypes = [P]
        L.orc_status.argtypes = [P]
        L.orc_status.restype = C.c_int32
        L.orc_global_step.argtypes = [P]
        L.orc_global_step.restype = C.c_uint32
        L.orc_set_global_step.argtypes = [P, C.c_uint32]
        L.orc_obs_dim.argtypes = [P]
        L.orc_obs_dim.restype = C.c_int32
        L.orc_reset.argtypes = [P, P, P]
        L.orc_reset.restype = C.c_int32
        L.orc_step_range.argtypes = [P, C.c_int32, C.c_int32, P, P, P, P, P, P, P, P]
        L.orc_step_range.restype = C.c_int32
        L.orc_advance.argtypes = [P]
        L.orc_step.argtypes = [P, P, P, P, P, P, P, P, P]
        L.orc_step.restype = C.c_int32
        L.orc_get_state.argtypes = [P, P, P]
        L.orc_set_state.argtypes = [P, P, P]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_sincos_f32.argtypes = [C.c_float, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.orc_sincos_batch.argtypes = [C.c_int32, P, P, P]
        L.orc_philox_batch.argtypes = [C.c_int32, P, P, P]
        L.orc_collides.argtypes = [P, C.c_int32, C.c_float, C.c_float]
        L.orc_collides.restype = C.c_int32
        L.orc_near.argtypes = [P, C.c_int32, C.c_float, C.c_float]
        L.orc_near.restype = C.c_int32
        L.orc_set_task.argtypes = [P, C.POINTER(_Task)]
        L.orc_set_task.restype = C.c_int32
        L.orc_march.argtypes = [P, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float]
        L.orc_march.restype = C.c_int32
        L.orc_ray_table.argtypes = [P, P, P]
        L.orc_bf16_rne.argtypes = [C.c_float]
        L.orc_bf16_rne.restype = C.c_uint16
        L.orc_qnet_f64.argtypes = [P, P, P, C.c_int32, P, C.c_int32, P]
        L.orc_vem.argtypes = [P, P, C.c_int32, P, P, P]
        L.orc_uniform_actions.argtypes = [P, P]
        L.orc_vem_epsilon.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double, P]
        L.orc_vem_or.restype = C.c_int32
        L.orc_vem_or.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int64]
        L.orc_ring_create.restype = P
        L.orc_ring_create.argtypes = [C.c_int64, C.c_int32, C.c_uint64]
        L.orc_ring_destroy.argtypes = [P]
        L.orc_ring_size.restype = C.c_int64
        L.orc_ring_size.argtypes = [P]
        L.orc_ring_head.restype = C.c_int64
        L.orc_ring_head.argtypes = [P]
        L.orc_ring_push.restype = C.c_int32
        L.orc_ring_push.argtypes = [P, C.c_int32, P, P, P, P, P, P]
        L.orc_ring_gather.restype = C.c_int32
        L.orc_ring_gather.argtypes = [P, C.c_int32, P, P, P, P, P, P]
        L.orc_ring_sample.restype = C.c_int32
        L.orc_ring_sample.argtypes = [P, C.c_int32, C.c_uint32, P, P, P, P, P, P]
        L.orc_learner_create.restype = P
        L.orc_learner_create.argtypes = [P, P, P, C.POINTER(LearnerConfig)]
        L.orc_learner_destroy.argtypes = [P]
        L.orc_learner_update.restype = C.c_int32
        L.orc_learner_update.argtypes = [P, C.c_int32, P, P, P, P, P, P, P, P]
        L.orc_learner_get.argtypes = [P, P, P, P, P]
        L.orc_learner_steps.restype = C.c_int64
        L.orc_learner_steps.argtypes = [P]
        L.orc_learner_q.argtypes = [P, C.c_int32, C.c_int32, P, P]
        L.orc_tfm_init.argtypes = [P, C.c_double]
        L.orc_tfm_actor.argtypes = [P, C.c_double]
        L.orc_tfm_learner.argtypes = [P, C.c_double]
        L.orc_tfm_xi.restype = C.c_double
        L.orc_tfm_xi.argtypes = [P]
        L.orc_f16_rne.restype = C.c_uint16
        L.orc_f16_rne.argtypes = [C.c_float]
        L.orc_f16_to_f32.restype = C.c_float
        L.orc_f16_to_f32.argtypes = [C.c_uint16]
        L.orc_quant_u8.restype = C.c_uint8
        L.orc_quant_u8.argtypes = [C.c_float]
        L.orc_dequant_u8.restype = C.c_float
        L.orc_dequant_u8.argtypes = [C.c_uint8]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def sincos_f32(phi: float):
    s, c = C.c_float(), C.c_float()
    lib().orc_sincos_f32(C.c_float(phi), C.byref(s), C.byref(c))
    return np.float32(s.value), np.float32(c.value)


def sincos_batch(phi):
    phi = np.ascontiguousarray(phi, dtype=np.float32)
    s = np.zeros_like(phi)
    c = np.zeros_like(phi)
    lib().orc_sincos_batch(phi.size, _p(phi), _p(s), _p(c))
    return s, c


def philox_batch(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(ctr)
    lib().orc_philox_batch(ctr.shape[0], _p(ctr), _p(k), _p(out))
    return out


def bf16_rne(f: float) -> int:
    return int(lib().orc_bf16_rne(C.c_float(f)))


def qnet_f64(dims, w_bf16, b_f32, obs, round_act=False):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    w = np.ascontiguousarray(w_bf16, dtype=np.uint16)
    b = np.ascontiguousarray(b_f32, dtype=np.float32)
    o = np.ascontiguousarray(obs, dtype=np.float32)
    n = o.shape[0]
    q = np.zeros((n, int(d[3])), np.float64)
    lib().orc_qnet_f64(_p(d), _p(w), _p(b), n, _p(o), int(bool(round_act)), _p(q))
    return q


def vem_or(T, or_start, or_final, decay):
    """Exploring-interval size after T transitions (linear decay, Sec. 3.1.1)."""
    return int(lib().orc_vem_or(int(T), int(or_start), int(or_final), int(decay)))


def vem_schedule_epsilon(n, g, e_min, e_max, or_start, or_final, decay):
    """Per-env VEM probabilities at global step g (T = n * g transitions)."""
    return vem_epsilon(n, vem_or(n * g, or_start, or_final, decay), e_min, e_max)


def vem_epsilon(n, m, e_min, e_max):
    out = np.zeros(n, np.float32)
    lib().orc_vem_epsilon(n, m, e_min, e_max, _p(out))
    return out


class Oracle:
    """One batch of N environments stepped on the CPU."""

    def __init__(self, cfg: dict, maps):
        self.cfg = dict(cfg)
        c = _Config()
        c.n_envs = cfg["n_envs"]
        c.n_rays = cfg["n_rays"]
        c.n_actions = N_ACTIONS
        for f in ("fov", "range", "ds", "robot_r", "arrive_r", "dt_lo", "dt_hi", "K_lo",
                  "K_hi", "mu_lo", "mu_hi", "vmax_lo", "vmax_hi", "omega_max",
                  "sigma_lo", "sigma_hi"):
            setattr(c, f, float(cfg[f]))
        c.t_max = cfg["t_max"]
        c.delay_lo = cfg["delay_lo"]
        c.delay_hi = cfg["delay_hi"]
        c.seed = cfg["seed"]
        self._c = c
        cells, offsets, width, height, env_to_map = maps.flat()
        self.maps = maps
        self._h = lib().orc_create(C.byref(c), len(width), _p(cells), _p(offsets), _p(width),
                                   _p(height), _p(env_to_map))
        if not self._h:
            raise ValueError("oracle rejected the configuration")
        self.n = c.n_envs
        self.obs_dim = c.n_rays + 4
        self.n_actions = N_ACTIONS

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    @property
    def status(self):
        return lib().orc_status(self._h)

    @property
    def global_step(self):
        return lib().orc_global_step(self._h)

    @global_step.setter
    def global_step(self, g):
        lib().orc_set_global_step(self._h, g)

    def reset(self, hit_k=False):
        obs = np.zeros((self.n, self.obs_dim), np.float32)
        hk = np.zeros((self.n, self.cfg["n_rays"]), np.int16) if hit_k else None
        rc = lib().orc_reset(self._h, _p(obs), _p(hk))
        return (obs, rc, hk) if hit_k else (obs, rc)

    def step(self, actions, final_obs=False, hit_k=False, stats: Stats | None = None):
        a = np.ascontiguousarray(actions, dtype=np.int32)
        obs = np.zeros((self.n, self.obs_dim), np.float32)
        rew = np.zeros(self.n, np.float32)
        done = np.zeros(self.n, np.uint8)
        flags = np.zeros(self.n, np.uint8)
        fo = np.zeros((self.n, self.obs_dim), np.float32) if final_obs else None
        hk = np.zeros((self.n, self.cfg["n_rays"]), np.int16) if hit_k else None
        rc = lib().orc_step(self._h, _p(a), _p(obs), _p(rew), _p(done), _p(flags), _p(fo),
                            _p(hk), C.byref(stats) if stats is not None else None)
        return dict(obs=obs, reward=rew, done=done, flags=flags, final_obs=fo, hit_k=hk, rc=rc)

    def step_range(self, e0, e1, actions, obs, rew, done, flags=None):
        return lib().orc_step_range(self._h, e0, e1, _p(actions), _p(obs), _p(rew), _p(done),
                                    _p(flags), None, None, None)

    def advance(self):
        lib().orc_advance(self._h)

    def step_envs(self, ids, actions, final_obs=False):
        """Step only the envs in `ids` (the others keep their state), then
        advance the global step. Returns full-size reward/done/obs (and
        final_obs) arrays whose rows outside `ids` are zero."""
        a = np.ascontiguousarray(actions, dtype=np.int32)
        obs = np.zeros((self.n, self.obs_dim), np.float32)
        rew = np.zeros(self.n, np.float32)
        done = np.zeros(self.n, np.uint8)
        fo = np.zeros((self.n, self.obs_dim), np.float32) if final_obs else None
        L = lib()
        for i in ids:
            i = int(i)
            L.orc_step_range(self._h, i, i + 1, _p(a), _p(obs), _p(rew), _p(done), None, _p(fo),
                             None, None)
        lib().orc_advance(self._h)
        return dict(obs=obs, reward=rew, done=done, final_obs=fo)

    def get_state(self):
        f = np.zeros((self.n, len(STATE_F)), np.float32)
        i = np.zeros((self.n, len(STATE_I)), np.int32)
        lib().orc_get_state(self._h, _p(f), _p(i))
        return f, i

    def set_state(self, f, i):
        f = np.ascontiguousarray(f, dtype=np.float32)
        i = np.ascontiguousarray(i, dtype=np.int32)
        assert f.shape == (self.n, len(STATE_F)) and i.shape == (self.n, len(STATE_I))
        lib().orc_set_state(self._h, _p(f), _p(i))

    def collides(self, m, px, py):
        return bool(lib().orc_collides(self._h, m, C.c_float(px), C.c_float(py)))

    def near(self, m, px, py):
        return bool(lib().orc_near(self._h, m, C.c_float(px), C.c_float(py)))

    def set_task(self, n_actions=7, reward=REWARD_PROGRESS, state=STATE_TARGET,
                 arrive_reward=10.0, collide_reward=-10.0, plan_dist=1.0, near_dist=0.0,
                 weights=(0.3, 0.1, 0.3, 0.3, 0.1)):
        """Task variant (Sec. 4.3.1): 5 or 7 actions, progress or Eq. (11)
        reward, target or relative-pose state (see the C header)."""
        t = _Task(n_actions, reward, state, arrive_reward, collide_reward, plan_dist, near_dist,
                  *weights)
        if lib().orc_set_task(self._h, C.byref(t)) != 0:
            raise ValueError("oracle rejected the task")
        self.n_actions = n_actions
        self.obs_dim = lib().orc_obs_dim(self._h)

    def march(self, m, x, y, ux, uy):
        return int(lib().orc_march(self._h, m, C.c_float(x), C.c_float(y), C.c_float(ux),
                                   C.c_float(uy)))

    def ray_table(self):
        c = np.zeros(self.cfg["n_rays"], np.float32)
        s = np.zeros(self.cfg["n_rays"], np.float32)
        lib().orc_ray_table(self._h, _p(c), _p(s))
        return c, s

    def uniform_actions(self):
        a = np.zeros(self.n, np.int32)
        lib().orc_uniform_actions(self._h, _p(a))
        return a

    def vem(self, q, eps):
        q = np.ascontiguousarray(q, dtype=np.float64)
        eps = np.ascontiguousarray(eps, dtype=np.float32)
        a = np.zeros(self.n, np.int32)
        ex = np.zeros(self.n, np.uint8)
        lib().orc_vem(self._h, _p(q), q.shape[1], _p(eps), _p(a), _p(ex))
        return a, ex


# ---------------------------------------------------------------------------
# Experience buffer (Sec. 3.1.2: Alg. 1 step 5 adds, Alg. 2 step 1 samples).
# Storage format and sampling rule: ring_oracle.h.
# ---------------------------------------------------------------------------
def f16_rne(f: float) -> int:
    return int(lib().orc_f16_rne(C.c_float(f)))


def f16_to_f32(h: int) -> float:
    return float(lib().orc_f16_to_f32(C.c_uint16(h)))


def quant_u8(o: float) -> int:
    return int(lib().orc_quant_u8(C.c_float(o)))


def dequant_u8(q: int) -> float:
    return float(lib().orc_dequant_u8(C.c_uint8(q)))


class Ring:
    """Ring of `capacity` transitions of observations with n_rays ranges."""

    def __init__(self, capacity: int, n_rays: int, seed: int):
        self.capacity, self.n_rays, self.D = int(capacity), int(n_rays), int(n_rays) + 4
        self._h = lib().orc_ring_create(self.capacity, self.n_rays, int(seed))
        if not self._h:
            raise MemoryError("orc_ring_create failed")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_ring_destroy(self._h)
            self._h = None

    @property
    def size(self) -> int:
        return int(lib().orc_ring_size(self._h))

    @property
    def head(self) -> int:
        return int(lib().orc_ring_head(self._h))

    def push(self, s, a, r, s_next, done, s_final=None):
        n = len(a)
        s = np.ascontiguousarray(s, np.float32).reshape(n, self.D)
        s_next = np.ascontiguousarray(s_next, np.float32).reshape(n, self.D)
        sf = None if s_final is None else np.ascontiguousarray(s_final, np.float32).reshape(n, self.D)
        a = np.ascontiguousarray(a, np.int32)
        r = np.ascontiguousarray(r, np.float32)
        d = np.ascontiguousarray(done, np.uint8)
        rc = lib().orc_ring_push(self._h, n, _p(s), _p(a), _p(r), _p(s_next), _p(sf), _p(d))
        if rc:
            raise ValueError("push rejected")

    def _outs(self, n):
        return (np.zeros((n, self.D), np.float32), np.zeros(n, np.int32), np.zeros(n, np.float32),
                np.zeros((n, self.D), np.float32), np.zeros(n, np.uint8))

    def gather(self, slots):
        slots = np.ascontiguousarray(slots, np.int64)
        s, a, r, sn, d = self._outs(len(slots))
        rc = lib().orc_ring_gather(self._h, len(slots), _p(slots), _p(s), _p(a), _p(r), _p(sn), _p(d))
        if rc:
            raise IndexError("slot outside the stored range")
        return s, a, r, sn, d

    def sample(self, B: int, draw: int):
        s, a, r, sn, d = self._outs(B)
        idx = np.zeros(B, np.int64)
        rc = lib().orc_ring_sample(self._h, B, draw, _p(s), _p(a), _p(r), _p(sn), _p(d), _p(idx))
        if rc:
            raise ValueError("empty ring")
        return s, a, r, sn, d, idx


# ---------------------------------------------------------------------------
# Learner (Alg. 2 step 2: DDQN update). Definitions: learner_oracle.h.
# ---------------------------------------------------------------------------
class Learner:
    def __init__(self, dims, w, b, gamma=0.98, lr=1e-4, beta1=0.9, beta2=0.999, adam_eps=1e-8,
                 huber_k=1.0, target_every=200):
        self.dims = tuple(int(d) for d in dims)
        d0, h1, h2, A = self.dims
        self.nw = h1 * d0 + h2 * h1 + A * h2
        self.nb = h1 + h2 + A
        w = np.ascontiguousarray(w, np.float32)
        b = np.ascontiguousarray(b, np.float32)
        assert w.size == self.nw and b.size == self.nb
        self.cfg = LearnerConfig(gamma, lr, beta1, beta2, adam_eps, huber_k, target_every)
        d = np.asarray(self.dims, np.int32)
        self._h = lib().orc_learner_create(_p(d), _p(w), _p(b), C.byref(self.cfg))
        if not self._h:
            raise MemoryError("orc_learner_create failed")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_learner_destroy(self._h)
            self._h = None

    def update(self, s, a, r, s_next, done):
        B = len(a)
        s = np.ascontiguousarray(s, np.float32)
        s_next = np.ascontiguousarray(s_next, np.float32)
        a = np.ascontiguousarray(a, np.int32)
        r = np.ascontiguousarray(r, np.float32)
        d = np.ascontiguousarray(done, np.uint8)
        loss = np.zeros(1, np.float64)
        gw = np.zeros(self.nw, np.float64)
        gb = np.zeros(self.nb, np.float64)
        rc = lib().orc_learner_update(self._h, B, _p(s), _p(a), _p(r), _p(s_next), _p(d),
                                      _p(loss), _p(gw), _p(gb))
        if rc:
            raise ValueError("empty mini-batch")
        return float(loss[0]), gw, gb

    def params(self):
        w, b = np.zeros(self.nw), np.zeros(self.nb)
        wt, bt = np.zeros(self.nw), np.zeros(self.nb)
        lib().orc_learner_get(self._h, _p(w), _p(b), _p(wt), _p(bt))
        return w, b, wt, bt

    @property
    def steps(self):
        return int(lib().orc_learner_steps(self._h))

    def q(self, x, target=False):
        x = np.ascontiguousarray(x, np.float32)
        q = np.zeros((x.shape[0], self.dims[3]), np.float64)
        lib().orc_learner_q(self._h, int(bool(target)), x.shape[0], _p(x), _p(q))
        return q


class Tfm:
    """Time feedback mechanism (Sec. 3.1.2, Eq. (TB2TV)); see learner_oracle.h."""

    class _S(C.Structure):
        _fields_ = [("rho", C.c_double), ("v_sum", C.c_double), ("b_sum", C.c_double),
                    ("v_n", C.c_int64), ("b_n", C.c_int64)]

    def __init__(self, rho):
        self._s = Tfm._S()
        lib().orc_tfm_init(C.byref(self._s), float(rho))

    def actor(self, seconds):
        lib().orc_tfm_actor(C.byref(self._s), float(seconds))

    def learner(self, seconds):
        lib().orc_tfm_learner(C.byref(self._s), float(seconds))

    @property
    def xi(self):
        return float(lib().orc_tfm_xi(C.byref(self._s)))

    @property
    def actor_sleep(self):
        return max(self.xi, 0.0)

    @property
    def learner_sleep(self):
        x = self.xi
        return -x / self._s.rho if x <= 0 else 0.0
