"""The C-ABI library loads and exports every symbol its header declares, and
rejects invalid arguments before touching a device (no GPU needed)."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2305_04180_amd import inputs, sparrow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sparrow.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sparrow_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sparrow.LIB_PATH):
        pytest.skip("libsparrow.so not built")
    return sparrow.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 18
    raw = C.CDLL(sparrow.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n
    assert set(names) == set(sparrow.EXPORTS)


def _create(cfg, maps):
    c = sparrow.make_config(cfg)
    cells, offsets, width, height, env_to_map = maps.flat()
    ms = sparrow.MapsStruct(len(width), cells.ctypes.data, offsets.ctypes.data,
                            width.ctypes.data, height.ctypes.data, env_to_map.ctypes.data)
    h = C.c_void_p()
    rc = sparrow.lib().sparrow_create(C.byref(c), C.byref(ms), None, C.byref(h))
    keep = (cells, offsets, width, height, env_to_map)
    return rc, h, keep


@pytest.mark.parametrize("change", [
    dict(n_envs=0), dict(n_rays=0), dict(n_rays=129), dict(range=0.0), dict(ds=0.0),
    dict(robot_r=0.0), dict(robot_r=9.0), dict(t_max=0), dict(delay_hi=3),
    dict(delay_lo=2, delay_hi=1), dict(vmax_lo=0.0), dict(sigma_lo=-1.0),
    dict(dt_lo=0.3, dt_hi=0.2),
])
def test_invalid_config_is_einval(lib, change):
    cfg = inputs.workload("c1", n_envs=2)
    cfg.update(change)
    maps = inputs.single_maps([np.zeros((16, 16), np.uint8)], n_envs=max(cfg["n_envs"], 1))
    rc, h, _ = _create(cfg, maps)
    assert rc == sparrow.EINVAL, (change, rc)
    assert not h.value
    assert lib.sparrow_last_error()


def test_bad_maps_are_einval(lib):
    cfg = inputs.workload("c1", n_envs=2)
    big = inputs.single_maps([np.zeros((513, 16), np.uint8)], n_envs=2)
    assert _create(cfg, big)[0] == sparrow.EINVAL
    badmap = inputs.single_maps([np.zeros((16, 16), np.uint8)], env_to_map=[0, 1])
    assert _create(cfg, badmap)[0] == sparrow.EINVAL
    h = C.c_void_p()
    assert lib.sparrow_create(None, None, None, C.byref(h)) == sparrow.EINVAL


def test_null_handle_calls_are_einval(lib):
    assert lib.sparrow_reset(None, None) == sparrow.EINVAL
    assert lib.sparrow_step(None, None, None, None, None, None, None) == sparrow.EINVAL
    assert lib.sparrow_rollout(None, 4, 0, None, None, None, None) == sparrow.EINVAL
    assert lib.sparrow_status(None) == sparrow.EINVAL
    assert lib.sparrow_set_variant(None, 0, 8, 32) == sparrow.EINVAL
    lib.sparrow_destroy(None)


def test_valid_config_without_gpu_fails_cleanly(lib):
    """On a host without a gfx950 device, create reports EHIP or EUNSUPPORTED."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cfg = inputs.workload("c1", n_envs=2)
    maps = inputs.single_maps([np.zeros((16, 16), np.uint8)], n_envs=2)
    rc, h, _ = _create(cfg, maps)
    assert rc in (sparrow.EHIP, sparrow.EUNSUPPORTED)
    assert not h.value


def test_binding_fails_loudly_without_library(tmp_path):
    import importlib
    mod = importlib.reload(sparrow)
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(RuntimeError):
            mod.lib(str(tmp_path / "missing.so"))
    finally:
        mod._lib = saved


def test_binding_does_no_vem_arithmetic():
    """VEM's per-env schedule comes from the library (sparrow_vem_epsilon);
    the binding only marshals arguments."""
    assert not hasattr(sparrow, "vem_epsilon")
    src = open(os.path.join(ROOT, "paper_2305_04180_amd", "sparrow.py")).read()
    assert "linspace" not in src and "e_max * frac" not in src


def test_product_path_never_touches_the_oracle():
    """The library sources and the binding name no oracle file or symbol."""
    pkg = os.path.join(ROOT, "paper_2305_04180_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower() or f == "inputs.py" and "import oracle" not in text, f
                assert "orc_" not in text, f


def test_binding_rejects_bad_buffers():
    """Short, strided, mistyped or misplaced buffers never reach the C-ABI."""
    import torch
    cpu = torch.device("cpu")
    ok = torch.zeros(8, dtype=torch.float32)
    assert sparrow._buf(ok, torch.float32, 8, cpu, "x") is ok
    assert sparrow._buf(None, torch.float32, 8, cpu, "x", nullable=True) is None
    for bad, kw in ((None, {}), (torch.zeros(7), {}), (torch.zeros(8, dtype=torch.float64), {}),
                    (torch.zeros(4, 4)[:, ::2], {}), (np.zeros(8, np.float32), {})):
        with pytest.raises(ValueError):
            sparrow._buf(bad, torch.float32, 8, cpu, "x", **kw)
    with pytest.raises(ValueError):
        sparrow._buf(ok, torch.float32, 8, torch.device("cuda", 0), "x")


def test_ring_argument_errors_without_device(lib):
    h = C.c_void_p()
    for cap, nr in ((0, 32), (1 << 27, 32), (16, 0), (16, 129)):
        assert lib.sparrow_ring_create(cap, nr, 1, None, C.byref(h)) == sparrow.EINVAL, (cap, nr)
        assert not h.value
    assert lib.sparrow_ring_create(16, 32, 1, None, None) == sparrow.EINVAL
    assert lib.sparrow_ring_push(None, 1, None, None, None, None, None, None) == sparrow.EINVAL
    assert lib.sparrow_ring_sample(None, 1, 0, None, None, None, None, None, None) == sparrow.EINVAL
    assert lib.sparrow_ring_gather(None, 0, None, None, None, None, None, None) == sparrow.EINVAL
    assert lib.sparrow_ring_status(None) == sparrow.EINVAL
    assert lib.sparrow_ring_size(None) == -1 and lib.sparrow_ring_head(None) == -1
    lib.sparrow_ring_destroy(None)


def test_vem_schedule_null_handle(lib):
    assert lib.sparrow_set_vem_schedule(None, 0.01, 0.8, 16, 3, 500000) == sparrow.EINVAL


def test_learner_argument_errors_without_device(lib):
    Cfg = lib.sparrow_learner_create.argtypes[3]._type_  # the class the loaded library uses
    cfg = Cfg(0.98, 1e-4, 0.9, 0.999, 1e-8, 1.0, 200, 256)
    w = np.zeros(10, np.float32)
    h = C.c_void_p()
    for dims in ((0, 4, 4, 2), (129, 4, 4, 2), (4, 513, 4, 2), (4, 4, 4, 17)):
        d = (C.c_int32 * 4)(*dims)
        assert lib.sparrow_learner_create(d, w.ctypes.data, w.ctypes.data, C.byref(cfg), None,
                                          C.byref(h)) == sparrow.EINVAL, dims
    bad = Cfg(0.98, 1e-4, 0.9, 0.999, 1e-8, 1.0, 200, 0)
    d = (C.c_int32 * 4)(4, 4, 4, 2)
    assert lib.sparrow_learner_create(d, w.ctypes.data, w.ctypes.data, C.byref(bad), None,
                                      C.byref(h)) == sparrow.EINVAL
    assert lib.sparrow_learner_update(None, 1, None, None, None, None, None, None) == sparrow.EINVAL
    assert lib.sparrow_learner_steps(None) == -1
    lib.sparrow_learner_destroy(None)


def test_tfm_matches_the_oracle(lib):
    """The pacing rule is host code: the library's and the oracle's sleep
    decisions agree exactly on a random record of periods."""
    import oracle
    with pytest.raises(sparrow.SparrowError):
        sparrow.Tfm(0.0)
    rng = np.random.default_rng(5)
    lt, ot = sparrow.Tfm(16.0), oracle.Tfm(16.0)
    assert lt.xi == ot.xi == 0.0
    for _ in range(500):
        if rng.random() < 0.3:
            v = float(rng.exponential(0.01))
            lt.actor(v), ot.actor(v)
        else:
            bb = float(rng.exponential(0.001))
            lt.learner(bb), ot.learner(bb)
        assert lt.xi == ot.xi
        assert lt.actor_sleep == ot.actor_sleep and lt.learner_sleep == ot.learner_sleep
