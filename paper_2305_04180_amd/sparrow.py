"""ctypes binding of libsparrow.so (the C-ABI in include/sparrow.h).

Argument marshalling only: every step of the simulation runs in the library's
HIP kernels. torch provides device memory and the stream; buffers are passed
as raw device pointers. There is no CPU fallback: without the built library
on a gfx950 device the constructor raises.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsparrow.so")

OK, EINVAL, ENOMEM, EHIP, ERESET, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FLAG_TERMINATED, FLAG_TRUNCATED, FLAG_COLLISION, FLAG_ARRIVAL = 1, 2, 4, 8
N_ACTIONS = 7
STATE_F = ("x", "y", "phi", "vl", "va", "tx", "ty", "dprev", "dt", "K", "mu", "vmax", "sigma")
STATE_I = ("t", "delay", "q0", "q1")

EXPORTS = (
    "sparrow_create", "sparrow_reset", "sparrow_step", "sparrow_random_actions",
    "sparrow_set_qnet", "sparrow_qnet_forward", "sparrow_act", "sparrow_rollout", "sparrow_rollout_trace",
    "sparrow_debug_hits", "sparrow_get_state", "sparrow_set_state", "sparrow_global_step",
    "sparrow_set_global_step", "sparrow_set_variant", "sparrow_get_variant",
    "sparrow_autotune", "sparrow_autotune_cached", "sparrow_status", "sparrow_destroy", "sparrow_last_error",
    "sparrow_set_vem_schedule", "sparrow_vem_epsilon", "sparrow_rollout_collect",
    "sparrow_step_collect",
    "sparrow_set_task",
    "sparrow_obs_dim",
    "sparrow_ring_create", "sparrow_ring_push", "sparrow_ring_sample", "sparrow_ring_gather",
    "sparrow_ring_gather_static", "sparrow_ring_size", "sparrow_ring_head", "sparrow_ring_status", "sparrow_ring_destroy",
    "sparrow_peak",
    "sparrow_learner_create", "sparrow_learner_update", "sparrow_learner_q",
    "sparrow_learner_export_bf16", "sparrow_learner_read", "sparrow_learner_steps",
    "sparrow_learner_destroy",
    "sparrow_tfm_create", "sparrow_tfm_actor_period", "sparrow_tfm_learner_period",
    "sparrow_tfm_xi", "sparrow_tfm_actor_sleep", "sparrow_tfm_learner_sleep",
    "sparrow_tfm_destroy",
)


class SparrowError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sparrow error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("n_envs", C.c_int32), ("n_rays", C.c_int32), ("n_actions", C.c_int32),
        ("fov_rad", C.c_float), ("range_cells", C.c_float), ("march_step", C.c_float),
        ("robot_radius", C.c_float), ("arrive_radius", C.c_float), ("timeout_steps", C.c_int32),
        ("dt_lo", C.c_float), ("dt_hi", C.c_float), ("K_lo", C.c_float), ("K_hi", C.c_float),
        ("mu_lo", C.c_float), ("mu_hi", C.c_float), ("vmax_lo", C.c_float),
        ("vmax_hi", C.c_float), ("omega_max", C.c_float), ("sigma_lo", C.c_float),
        ("sigma_hi", C.c_float), ("delay_lo", C.c_int32), ("delay_hi", C.c_int32),
        ("seed", C.c_uint64),
    ]


class LearnerConfig(C.Structure):
    _fields_ = [("gamma", C.c_float), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("adam_eps", C.c_float), ("huber_k", C.c_float),
                ("target_every", C.c_int32), ("max_batch", C.c_int32)]


class TaskStruct(C.Structure):
    _fields_ = [("n_actions", C.c_int32), ("reward", C.c_int32), ("state", C.c_int32),
                ("arrive_reward", C.c_float), ("collide_reward", C.c_float),
                ("plan_dist", C.c_float), ("near_dist", C.c_float), ("w_d1", C.c_float),
                ("w_d2", C.c_float), ("w_v", C.c_float), ("w_alpha", C.c_float),
                ("w_d", C.c_float)]


REWARD_PROGRESS, REWARD_EQ11 = 0, 1
STATE_TARGET, STATE_RELATIVE = 0, 1


class MapsStruct(C.Structure):
    _fields_ = [("n_maps", C.c_int32), ("cells", C.c_void_p), ("offsets", C.c_void_p),
                ("width", C.c_void_p), ("height", C.c_void_p), ("env_to_map", C.c_void_p)]


_lib = None


def lib(path: str = LIB_PATH):
    """Load the built library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        L = C.CDLL(path)
        P, I32, U32 = C.c_void_p, C.c_int32, C.c_uint32
        sig = {
            "sparrow_create": (I32, [C.POINTER(Config), C.POINTER(MapsStruct), P, C.POINTER(P)]),
            "sparrow_reset": (I32, [P, P]),
            "sparrow_step": (I32, [P, P, P, P, P, P, P]),
            "sparrow_random_actions": (I32, [P, P]),
            "sparrow_set_qnet": (I32, [P, P, P, P, P]),
            "sparrow_qnet_forward": (I32, [P, P, I32, P, P]),
            "sparrow_act": (I32, [P, P, P]),
            "sparrow_rollout": (I32, [P, I32, I32, P, P, P, P]),
            "sparrow_rollout_trace": (I32, [P, I32, I32, P, P, P, P, P, P]),
            "sparrow_rollout_collect": (I32, [P, P, I32, I32, I32, P, P, P, P]),
            "sparrow_set_task": (I32, [P, C.POINTER(TaskStruct)]),
            "sparrow_step_collect": (I32, [P, P, P, P, P, P, P, I32]),
            "sparrow_obs_dim": (I32, [P]),
            "sparrow_debug_hits": (I32, [P, P]),
            "sparrow_get_state": (I32, [P, P, P]),
            "sparrow_set_state": (I32, [P, P, P]),
            "sparrow_global_step": (U32, [P]),
            "sparrow_set_global_step": (None, [P, U32]),
            "sparrow_set_variant": (I32, [P, I32, I32, I32]),
            "sparrow_get_variant": (I32, [P, I32, C.POINTER(I32), C.POINTER(I32)]),
            "sparrow_autotune": (I32, [P, I32, C.c_char_p, I32]),
            "sparrow_autotune_cached": (I32, [P, I32, C.c_char_p, C.c_char_p, I32]),
            "sparrow_status": (I32, [P]),
            "sparrow_destroy": (None, [P]),
            "sparrow_last_error": (C.c_char_p, []),
            "sparrow_set_vem_schedule": (I32, [P, C.c_double, C.c_double, I32, I32, C.c_int64]),
            "sparrow_vem_epsilon": (I32, [P, I32, C.c_double, C.c_double, P]),
            "sparrow_learner_create": (I32, [P, P, P, C.POINTER(LearnerConfig), P, C.POINTER(P)]),
            "sparrow_learner_update": (I32, [P, I32, P, P, P, P, P, P]),
            "sparrow_learner_q": (I32, [P, I32, I32, P, P]),
            "sparrow_learner_export_bf16": (I32, [P, P, P]),
            "sparrow_learner_read": (I32, [P, P, P, P, P, P, P]),
            "sparrow_learner_steps": (C.c_int64, [P]),
            "sparrow_learner_destroy": (None, [P]),
            "sparrow_tfm_create": (I32, [C.c_double, C.POINTER(P)]),
            "sparrow_tfm_actor_period": (None, [P, C.c_double]),
            "sparrow_tfm_learner_period": (None, [P, C.c_double]),
            "sparrow_tfm_xi": (C.c_double, [P]),
            "sparrow_tfm_actor_sleep": (C.c_double, [P]),
            "sparrow_tfm_learner_sleep": (C.c_double, [P]),
            "sparrow_tfm_destroy": (None, [P]),
            "sparrow_ring_create": (I32, [I32, I32, C.c_uint64, P, C.POINTER(P)]),
            "sparrow_ring_push": (I32, [P, I32, P, P, P, P, P, P]),
            "sparrow_ring_sample": (I32, [P, I32, U32, P, P, P, P, P, P]),
            "sparrow_ring_gather": (I32, [P, I32, P, P, P, P, P, P]),
            "sparrow_ring_gather_static": (I32, [P, I32, P, P, P, P, P, P]),
            "sparrow_ring_size": (C.c_int64, [P]),
            "sparrow_ring_head": (C.c_int64, [P]),
            "sparrow_ring_status": (I32, [P]),
            "sparrow_ring_destroy": (None, [P]),
            "sparrow_peak": (I32, [I32, C.c_int64, I32, P, C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise SparrowError(rc, lib().sparrow_last_error().decode())
    return rc


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _buf(t, dtype, numel, device, name, nullable=False):
    """Check a caller's buffer before its pointer reaches a kernel: the
    C-ABI takes raw pointers and cannot see sizes, so a short, strided or
    mistyped tensor is rejected here rather than written out of bounds."""
    if t is None:
        if nullable:
            return None
        raise ValueError(f"{name}: buffer required")
    if not hasattr(t, "data_ptr") or t.dtype != dtype:
        raise ValueError(f"{name}: expected a {dtype} tensor, got {getattr(t, 'dtype', type(t))}")
    if t.device != device:
        raise ValueError(f"{name}: expected device {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name}: needs {numel} elements, has {t.numel()}")
    return t


def make_config(cfg: dict) -> Config:
    c = Config()
    c.n_envs, c.n_rays, c.n_actions = cfg["n_envs"], cfg["n_rays"], N_ACTIONS
    c.fov_rad, c.range_cells, c.march_step = cfg["fov"], cfg["range"], cfg["ds"]
    c.robot_radius, c.arrive_radius, c.timeout_steps = cfg["robot_r"], cfg["arrive_r"], cfg["t_max"]
    for f in ("dt_lo", "dt_hi", "K_lo", "K_hi", "mu_lo", "mu_hi", "vmax_lo", "vmax_hi",
              "omega_max", "sigma_lo", "sigma_hi"):
        setattr(c, f, float(cfg[f]))
    c.delay_lo, c.delay_hi, c.seed = cfg["delay_lo"], cfg["delay_hi"], cfg["seed"]
    return c


class Env:
    """N Sparrow environments on the current HIP device and torch stream."""

    def __init__(self, cfg: dict, maps, stream=None):
        import torch
        self.torch = torch
        self.cfg = dict(cfg)
        self.n = cfg["n_envs"]
        self.n_rays = cfg["n_rays"]
        self.obs_dim = self.n_rays + 4
        self.n_actions = N_ACTIONS
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        cells, offsets, width, height, env_to_map = maps.flat()
        self._keep = (cells, offsets, width, height, env_to_map)
        ms = MapsStruct(len(width), cells.ctypes.data, offsets.ctypes.data, width.ctypes.data,
                        height.ctypes.data, env_to_map.ctypes.data)
        self._c = make_config(cfg)
        h = C.c_void_p()
        _check(lib().sparrow_create(C.byref(self._c), C.byref(ms),
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        f32, u8, i32 = torch.float32, torch.uint8, torch.int32
        dev = self.device
        self.obs = torch.zeros(self.n, self.obs_dim, dtype=f32, device=dev)
        self.reward = torch.zeros(self.n, dtype=f32, device=dev)
        self.done = torch.zeros(self.n, dtype=u8, device=dev)
        self.flags = torch.zeros(self.n, dtype=u8, device=dev)
        self.actions = torch.zeros(self.n, dtype=i32, device=dev)
        if cfg.get("task"):
            self.set_task(**cfg["task"])

    def set_task(self, n_actions=7, reward=REWARD_PROGRESS, state=STATE_TARGET,
                 arrive_reward=10.0, collide_reward=-10.0, plan_dist=1.0, near_dist=0.0,
                 weights=(0.3, 0.1, 0.3, 0.3, 0.1)):
        """Task variant (Sec. 4.3.1): 5 or 7 actions, progress or Eq. (11)
        reward, target or relative-pose state. Drops the Q-network; reset
        before stepping."""
        t = TaskStruct(int(n_actions), int(reward), int(state), float(arrive_reward),
                       float(collide_reward), float(plan_dist), float(near_dist),
                       *[float(x) for x in weights])
        _check(lib().sparrow_set_task(self._h, C.byref(t)))
        self.n_actions = int(n_actions)
        self.obs_dim = int(lib().sparrow_obs_dim(self._h))
        self.obs = self.torch.zeros(self.n, self.obs_dim, dtype=self.torch.float32,
                                    device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            lib().sparrow_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- RL-API ---------------------------------------------------------------
    def _b(self, t, dtype, numel, name, nullable=False):
        return _buf(t, dtype, numel, self.device, name, nullable)

    def reset(self, obs=None):
        t = self.torch
        obs = self._b(self.obs if obs is None else obs, t.float32, self.n * self.obs_dim, "obs")
        _check(lib().sparrow_reset(self._h, _ptr(obs)))
        return obs

    def step(self, actions, obs=None, reward=None, done=None, flags=None, final_obs=None):
        t, n, D = self.torch, self.n, self.obs_dim
        actions = self._b(actions, t.int32, n, "actions")
        obs = self._b(self.obs if obs is None else obs, t.float32, n * D, "obs")
        reward = self._b(self.reward if reward is None else reward, t.float32, n, "reward")
        done = self._b(self.done if done is None else done, t.uint8, n, "done")
        flags = self._b(flags, t.uint8, n, "flags", nullable=True)
        final_obs = self._b(final_obs, t.float32, n * D, "final_obs", nullable=True)
        _check(lib().sparrow_step(self._h, _ptr(actions), _ptr(obs), _ptr(reward), _ptr(done),
                                  _ptr(flags), _ptr(final_obs)))
        return obs, reward, done

    def step_collect(self, ring, actions, obs=None, reward=None, done=None, flags=None,
                     terminal_obs=True):
        """One step that also adds its N transitions (s = the current
        observation, the given actions, r, s', done) to `ring`."""
        t, n, D = self.torch, self.n, self.obs_dim
        actions = self._b(actions, t.int32, n, "actions")
        obs = self._b(self.obs if obs is None else obs, t.float32, n * D, "obs")
        reward = self._b(self.reward if reward is None else reward, t.float32, n, "reward")
        done = self._b(self.done if done is None else done, t.uint8, n, "done")
        flags = self._b(flags, t.uint8, n, "flags", nullable=True)
        _check(lib().sparrow_step_collect(self._h, ring._h, _ptr(actions), _ptr(obs),
                                          _ptr(reward), _ptr(done), _ptr(flags),
                                          int(bool(terminal_obs))))
        return obs, reward, done

    def random_actions(self, out=None):
        out = self._b(self.actions if out is None else out, self.torch.int32, self.n, "actions")
        _check(lib().sparrow_random_actions(self._h, _ptr(out)))
        return out

    # -- actor ----------------------------------------------------------------
    def set_qnet(self, dims, w_bf16, b_f32, eps):
        torch = self.torch
        d = (C.c_int32 * 4)(*[int(x) for x in dims])
        nw = sum(int(dims[k]) * int(dims[k + 1]) for k in range(3))
        nb = int(dims[1]) + int(dims[2]) + int(dims[3])
        w = torch.as_tensor(np.asarray(w_bf16).view(np.int16)).to(self.device)
        b = torch.as_tensor(np.asarray(b_f32, np.float32)).to(self.device)
        if isinstance(eps, torch.Tensor):
            e = self._b(eps, torch.float32, self.n, "eps")
        else:
            e = torch.as_tensor(np.asarray(eps, np.float32)).to(self.device)
        for t, k, name in ((w, nw, "weights"), (b, nb, "biases"), (e, self.n, "eps")):
            if t.numel() != k:
                raise ValueError(f"{name}: expected {k} values for dims {tuple(dims)}, got {t.numel()}")
        _check(lib().sparrow_set_qnet(self._h, d, _ptr(w), _ptr(b), _ptr(e)))
        self._qkeep = (w, b, e)

    def vem_epsilon(self, m, e_min, e_max, out=None):
        """VEM's per-env exploration probabilities for a fixed exploring
        interval of the last m envs (sparrow_vem_epsilon), on the device."""
        t = self.torch
        out = t.zeros(self.n, dtype=t.float32, device=self.device) if out is None else out
        self._b(out, t.float32, self.n, "eps")
        _check(lib().sparrow_vem_epsilon(self._h, int(m), float(e_min), float(e_max), _ptr(out)))
        return out

    def set_vem_schedule(self, e_min, e_max, or_start, or_final, decay_transitions):
        """VEM with an exploring interval shrinking linearly over training."""
        _check(lib().sparrow_set_vem_schedule(self._h, float(e_min), float(e_max), int(or_start),
                                              int(or_final), int(decay_transitions)))

    def qnet_forward(self, obs, q=None, greedy=None):
        torch = self.torch
        n = obs.shape[0]
        self._b(obs, torch.float32, n * self.obs_dim, "obs")
        if obs.dim() != 2 or obs.shape[1] != self.obs_dim:
            raise ValueError(f"obs: expected shape [n, {self.obs_dim}], got {tuple(obs.shape)}")
        q = torch.zeros(n, self.n_actions, dtype=torch.float32, device=self.device) if q is None else q
        greedy = torch.zeros(n, dtype=torch.int32, device=self.device) if greedy is None else greedy
        self._b(q, torch.float32, n * self.n_actions, "q")
        self._b(greedy, torch.int32, n, "greedy")
        _check(lib().sparrow_qnet_forward(self._h, _ptr(obs), n, _ptr(q), _ptr(greedy)))
        return q, greedy

    def act(self, obs, actions=None):
        t = self.torch
        obs = self._b(obs, t.float32, self.n * self.obs_dim, "obs")
        actions = self._b(self.actions if actions is None else actions, t.int32, self.n, "actions")
        _check(lib().sparrow_act(self._h, _ptr(obs), _ptr(actions)))
        return actions

    def rollout(self, K, use_qnet, actions=None, reward=None, done=None, obs=None):
        torch = self.torch
        dev = self.device
        actions = torch.zeros(K, self.n, dtype=torch.int32, device=dev) if actions is None else actions
        reward = torch.zeros(K, self.n, dtype=torch.float32, device=dev) if reward is None else reward
        done = torch.zeros(K, self.n, dtype=torch.uint8, device=dev) if done is None else done
        obs = self.obs if obs is None else obs
        n = self.n
        self._b(actions, torch.int32, K * n, "actions", nullable=True)
        self._b(reward, torch.float32, K * n, "reward")
        self._b(done, torch.uint8, K * n, "done")
        self._b(obs, torch.float32, n * self.obs_dim, "obs")
        _check(lib().sparrow_rollout(self._h, K, int(bool(use_qnet)), _ptr(actions),
                                     _ptr(reward), _ptr(done), _ptr(obs)))
        return actions, reward, done, obs

    def rollout_trace(self, K, use_qnet, actions=None, reward=None, done=None, obs=None,
                      obs_steps=None, hits_steps=None):
        """rollout() that also returns every step's observation [K][N][obs_dim]
        and per-ray hit indices [K][N][n_rays] (sparrow_rollout_trace)."""
        torch = self.torch
        dev = self.device
        n = self.n
        actions = torch.zeros(K, n, dtype=torch.int32, device=dev) if actions is None else actions
        reward = torch.zeros(K, n, dtype=torch.float32, device=dev) if reward is None else reward
        done = torch.zeros(K, n, dtype=torch.uint8, device=dev) if done is None else done
        obs = self.obs if obs is None else obs
        if obs_steps is None:
            obs_steps = torch.zeros(K, n, self.obs_dim, dtype=torch.float32, device=dev)
        if hits_steps is None:
            hits_steps = torch.zeros(K, n, self.n_rays, dtype=torch.int16, device=dev)
        self._b(actions, torch.int32, K * n, "actions", nullable=True)
        self._b(reward, torch.float32, K * n, "reward")
        self._b(done, torch.uint8, K * n, "done")
        self._b(obs, torch.float32, n * self.obs_dim, "obs")
        self._b(obs_steps, torch.float32, K * n * self.obs_dim, "obs_steps")
        self._b(hits_steps, torch.int16, K * n * self.n_rays, "hits_steps")
        _check(lib().sparrow_rollout_trace(self._h, K, int(bool(use_qnet)), _ptr(actions),
                                           _ptr(reward), _ptr(done), _ptr(obs), _ptr(obs_steps),
                                           _ptr(hits_steps)))
        return actions, reward, done, obs, obs_steps, hits_steps

    def rollout_collect(self, ring, K, use_qnet, actions=None, reward=None, done=None, obs=None,
                        terminal_obs=True):
        """K fused steps that also add their K * N transitions to `ring`
        (Alg. 1 steps 2-5 in one kernel); the step-major actions, rewards and
        done flags are optional outputs here. terminal_obs: s' of a done
        transition is the terminal observation (else the post-reset one)."""
        torch = self.torch
        n = self.n
        obs = self.obs if obs is None else obs
        self._b(actions, torch.int32, K * n, "actions", nullable=True)
        self._b(reward, torch.float32, K * n, "reward", nullable=True)
        self._b(done, torch.uint8, K * n, "done", nullable=True)
        self._b(obs, torch.float32, n * self.obs_dim, "obs")
        _check(lib().sparrow_rollout_collect(self._h, ring._h, K, int(bool(use_qnet)),
                                             int(bool(terminal_obs)), _ptr(actions), _ptr(reward),
                                             _ptr(done), _ptr(obs)))
        return actions, reward, done, obs

    # -- inspection -----------------------------------------------------------
    def debug_hits(self):
        t = self.torch.zeros(self.n, self.n_rays, dtype=self.torch.int16, device=self.device)
        _check(lib().sparrow_debug_hits(self._h, _ptr(t)))
        return t

    def get_state(self):
        f = np.zeros((self.n, len(STATE_F)), np.float32)
        i = np.zeros((self.n, len(STATE_I)), np.int32)
        _check(lib().sparrow_get_state(self._h, f.ctypes.data, i.ctypes.data))
        return f, i

    def set_state(self, f, i):
        f = np.ascontiguousarray(f, np.float32)
        i = np.ascontiguousarray(i, np.int32)
        _check(lib().sparrow_set_state(self._h, f.ctypes.data, i.ctypes.data))

    @property
    def global_step(self):
        return int(lib().sparrow_global_step(self._h))

    @global_step.setter
    def global_step(self, g):
        lib().sparrow_set_global_step(self._h, int(g))

    def set_variant(self, kernel, envs_per_group, lanes_per_env):
        _check(lib().sparrow_set_variant(self._h, kernel, envs_per_group, lanes_per_env))

    def get_variant(self, kernel):
        a, b = C.c_int32(), C.c_int32()
        _check(lib().sparrow_get_variant(self._h, kernel, C.byref(a), C.byref(b)))
        return a.value, b.value

    def autotune(self, steps=8, cache=None):
        """Time the kernel variants and keep the fastest (sparrow_autotune);
        with cache (a file path), reuse the choice recorded there for the
        same device and workload shape (sparrow_autotune_cached)."""
        buf = C.create_string_buffer(1 << 16)
        if cache:
            _check(lib().sparrow_autotune_cached(self._h, steps, str(cache).encode(), buf, len(buf)))
        else:
            _check(lib().sparrow_autotune(self._h, steps, buf, len(buf)))
        return json.loads(buf.value.decode() or "{}")

    def status(self):
        return lib().sparrow_status(self._h)


class Ring:
    """Device experience buffer (sparrow_ring_*): batched adds of transitions
    (s, a, r, s', done) and uniform mini-batch sampling, on the current
    device and torch stream."""

    def __init__(self, capacity: int, n_rays: int, seed: int = 1, stream=None):
        import torch
        self.torch = torch
        self.capacity, self.n_rays, self.D = int(capacity), int(n_rays), int(n_rays) + 4
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib().sparrow_ring_create(self.capacity, self.n_rays, int(seed),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().sparrow_ring_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _b(self, t, dtype, numel, name, nullable=False):
        return _buf(t, dtype, numel, self.device, name, nullable)

    @property
    def size(self) -> int:
        return int(lib().sparrow_ring_size(self._h))

    @property
    def head(self) -> int:
        return int(lib().sparrow_ring_head(self._h))

    def push(self, s, a, r, s_next, done, s_final=None):
        t = self.torch
        n = int(a.numel())
        self._b(s, t.float32, n * self.D, "s")
        self._b(a, t.int32, n, "a")
        self._b(r, t.float32, n, "r")
        self._b(s_next, t.float32, n * self.D, "s_next")
        self._b(s_final, t.float32, n * self.D, "s_final", nullable=True)
        self._b(done, t.uint8, n, "done")
        _check(lib().sparrow_ring_push(self._h, n, _ptr(s), _ptr(a), _ptr(r), _ptr(s_next),
                                       _ptr(s_final), _ptr(done)))

    def _outs(self, n, outs):
        t, dev = self.torch, self.device
        if outs is not None:
            s, a, r, sn, d = outs
            self._b(s, t.float32, n * self.D, "s")
            self._b(a, t.int32, n, "a")
            self._b(r, t.float32, n, "r")
            self._b(sn, t.float32, n * self.D, "s_next")
            self._b(d, t.uint8, n, "done")
            return outs
        return (t.zeros(n, self.D, dtype=t.float32, device=dev), t.zeros(n, dtype=t.int32, device=dev),
                t.zeros(n, dtype=t.float32, device=dev), t.zeros(n, self.D, dtype=t.float32, device=dev),
                t.zeros(n, dtype=t.uint8, device=dev))

    def sample(self, B: int, draw: int, outs=None, idx=None):
        """B uniform draws over the stored slots (Philox counter (b, draw, 8, 0))."""
        s, a, r, sn, d = self._outs(B, outs)
        if idx is None:
            idx = self.torch.zeros(B, dtype=self.torch.int32, device=self.device)
        self._b(idx, self.torch.int32, B, "idx")
        _check(lib().sparrow_ring_sample(self._h, B, int(draw) & 0xFFFFFFFF, _ptr(s), _ptr(a),
                                         _ptr(r), _ptr(sn), _ptr(d), _ptr(idx)))
        return s, a, r, sn, d, idx

    def gather(self, slots):
        """Read back the given slots (host integers, each in [0, size))."""
        sl = np.ascontiguousarray(slots, np.int32)
        s, a, r, sn, d = self._outs(len(sl), None)
        _check(lib().sparrow_ring_gather(self._h, len(sl), sl.ctypes.data, _ptr(s), _ptr(a),
                                         _ptr(r), _ptr(sn), _ptr(d)))
        return s, a, r, sn, d

    def gather_static(self, slots):
        """gather() through sparrow_ring_gather_static: the slots are staged
        in the library's fixed per-GPU array (at most GATHER_STATIC_MAX), and
        the call allocates no device memory."""
        sl = np.ascontiguousarray(slots, np.int32)
        s, a, r, sn, d = self._outs(len(sl), None)
        _check(lib().sparrow_ring_gather_static(self._h, len(sl), sl.ctypes.data, _ptr(s), _ptr(a),
                                                _ptr(r), _ptr(sn), _ptr(d)))
        return s, a, r, sn, d

    def status(self) -> int:
        return lib().sparrow_ring_status(self._h)


class Learner:
    """The DDQN learner on the device (sparrow_learner_*): FP32 online and
    target networks with Adam; one update per mini-batch."""

    def __init__(self, dims, w_f32, b_f32, gamma=0.98, lr=1e-4, beta1=0.9, beta2=0.999,
                 adam_eps=1e-8, huber_k=1.0, target_every=200, max_batch=256, stream=None):
        import torch
        self.torch = torch
        self.dims = tuple(int(x) for x in dims)
        d0, h1, h2, A = self.dims
        self.nw = h1 * d0 + h2 * h1 + A * h2
        self.nb = h1 + h2 + A
        self.max_batch = int(max_batch)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        w = np.ascontiguousarray(w_f32, np.float32)
        b = np.ascontiguousarray(b_f32, np.float32)
        if w.size != self.nw or b.size != self.nb:
            raise ValueError(f"expected {self.nw} weights and {self.nb} biases for dims {self.dims}")
        self._cfg = LearnerConfig(gamma, lr, beta1, beta2, adam_eps, huber_k, target_every, max_batch)
        d = (C.c_int32 * 4)(*self.dims)
        h = C.c_void_p()
        _check(lib().sparrow_learner_create(d, w.ctypes.data, b.ctypes.data, C.byref(self._cfg),
                                            C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            lib().sparrow_learner_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, s, a, r, s_next, done):
        t = self.torch
        B = int(a.numel())
        d0 = self.dims[0]
        for x, dt, n, name in ((s, t.float32, B * d0, "s"), (a, t.int32, B, "a"),
                               (r, t.float32, B, "r"), (s_next, t.float32, B * d0, "s_next"),
                               (done, t.uint8, B, "done")):
            _buf(x, dt, n, self.device, name)
        _check(lib().sparrow_learner_update(self._h, B, _ptr(s), _ptr(a), _ptr(r), _ptr(s_next),
                                            _ptr(done), _ptr(self.loss)))
        return self.loss

    def q(self, x, target=False):
        t = self.torch
        n = x.shape[0]
        _buf(x, t.float32, n * self.dims[0], self.device, "x")
        q = t.zeros(n, self.dims[3], dtype=t.float32, device=self.device)
        _check(lib().sparrow_learner_q(self._h, int(bool(target)), n, _ptr(x), _ptr(q)))
        return q

    def export_bf16(self):
        t = self.torch
        w = t.zeros(self.nw, dtype=t.int16, device=self.device)
        b = t.zeros(self.nb, dtype=t.float32, device=self.device)
        _check(lib().sparrow_learner_export_bf16(self._h, _ptr(w), _ptr(b)))
        return w, b

    def read(self):
        """Synchronising host copies: w, b, wt, bt, and the last gradients gw, gb."""
        out = [np.zeros(n, np.float32) for n in (self.nw, self.nb, self.nw, self.nb, self.nw, self.nb)]
        _check(lib().sparrow_learner_read(self._h, *[o.ctypes.data for o in out]))
        return out

    @property
    def steps(self):
        return int(lib().sparrow_learner_steps(self._h))


class Tfm:
    """Time feedback mechanism (sparrow_tfm_*): the actor reports each
    vectorized step's duration, the learner each update's; the faster side
    sleeps as told (Sec. 3.1.2, Eq. (TB2TV))."""

    def __init__(self, rho):
        h = C.c_void_p()
        _check(lib().sparrow_tfm_create(float(rho), C.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            lib().sparrow_tfm_destroy(self._h)
            self._h = None

    def actor(self, seconds):
        lib().sparrow_tfm_actor_period(self._h, float(seconds))

    def learner(self, seconds):
        lib().sparrow_tfm_learner_period(self._h, float(seconds))

    @property
    def xi(self):
        return float(lib().sparrow_tfm_xi(self._h))

    @property
    def actor_sleep(self):
        return float(lib().sparrow_tfm_actor_sleep(self._h))

    @property
    def learner_sleep(self):
        return float(lib().sparrow_tfm_learner_sleep(self._h))


GATHER_STATIC_MAX = 65536  # SPARROW_GATHER_STATIC_MAX

PEAK_LDS128, PEAK_LDS32, PEAK_HBM_COPY, PEAK_MFMA_BF16 = 0, 1, 2, 3


def peak(kind: int, size: int = 0, iters: int = 4096, stream=None):
    """Peak-rate probe of the current device (sparrow_peak): returns
    (rate, seconds), rate in bytes/s for the LDS and HBM probes and FLOP/s
    for the MFMA probe. Synchronises."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    rate, secs = C.c_double(), C.c_double()
    _check(lib().sparrow_peak(int(kind), int(size), int(iters), C.c_void_p(st.cuda_stream),
                              C.byref(rate), C.byref(secs)))
    return rate.value, secs.value
