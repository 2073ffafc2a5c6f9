"""Pins of the experience-buffer oracle (Sec. 3.1.2: Alg. 1 step 5 adds the
batched transitions, Alg. 2 step 1 samples a mini-batch; Table 6 sizes).

Each test checks the oracle against something other than itself: IEEE 754
binary16 values worked out by hand, numpy's own float16 conversion (a library
routine), closed forms of the uint8 quantisation, an independent numpy model
of the ring, and statistics of the sampler.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


# ---- binary16 round to nearest even -----------------------------------------
HAND = [  # (value, binary16 bits) from the IEEE 754 encoding
    (0.0, 0x0000), (-0.0, 0x8000), (1.0, 0x3C00), (-2.0, 0xC000), (0.5, 0x3800),
    (65504.0, 0x7BFF),                      # largest finite
    (65519.99, 0x7BFF),                     # below the half-way point to 2^16
    (65520.0, 0x7C00),                      # tie between 65504 and 2^16 -> even -> inf
    (1e9, 0x7C00), (-math.inf, 0xFC00),
    (2.0 ** -14, 0x0400),                   # smallest normal
    (2.0 ** -24, 0x0001),                   # smallest subnormal
    (2.0 ** -25, 0x0000),                   # tie between 0 and 2^-24 -> even -> 0
    (1.5 * 2.0 ** -25, 0x0001),
    (3 * 2.0 ** -25, 0x0002),               # 1.5 units: tie -> even 2
    (2.0 ** -14 - 2.0 ** -25, 0x0400),      # 1023.5 units: tie -> 1024 = smallest normal
    (1.0 + 2.0 ** -11, 0x3C00),             # tie -> even mantissa 0
    (1.0 + 3 * 2.0 ** -11, 0x3C02),         # tie between ...01 and ...02 -> even
    (1.0 + 2.0 ** -11 + 2.0 ** -20, 0x3C01),  # just above the tie
    (1.0 / 3.0, 0x3555),
    (-0.1, 0xAE66),
]


@pytest.mark.parametrize("value,bits", HAND)
def test_f16_hand_values(value, bits):
    assert oracle.f16_rne(value) == bits, (value, hex(oracle.f16_rne(value)), hex(bits))


def test_f16_nan_stays_nan():
    h = oracle.f16_rne(float("nan"))
    assert (h & 0x7C00) == 0x7C00 and (h & 0x3FF) != 0


def test_f16_matches_numpy_on_random_and_boundary_floats():
    rng = np.random.default_rng(7)
    # uniform over binary32 bit patterns of moderate magnitude plus ties
    bits = rng.integers(0x2E000000, 0x48000000, size=200_000, dtype=np.uint32)
    bits = np.concatenate([bits, bits | 0x80000000])
    # exact ties of binary16 normals: low 13 fraction bits = 0x1000
    ties = (rng.integers(0x38800000, 0x477FE000, size=20_000, dtype=np.uint32) & ~np.uint32(0x1FFF)) | 0x1000
    f = np.concatenate([bits, ties]).view(np.float32)
    with np.errstate(over="ignore"):
        ref = f.astype(np.float16).view(np.uint16)
    got = np.array([oracle.f16_rne(float(x)) for x in f], np.uint16)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, [(float(f[i]), hex(got[i]), hex(ref[i])) for i in bad[:5]]


def test_f16_to_f32_is_exact_for_every_pattern():
    h = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    ref = h.view(np.float16).astype(np.float32)
    got = np.array([oracle.f16_to_f32(int(x)) for x in h], np.float32)
    finite = np.isfinite(ref)
    assert np.array_equal(got[finite].view(np.uint32), ref[finite].view(np.uint32))
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.array_equal(np.isinf(got), np.isinf(ref))


# ---- uint8 ranges -------------------------------------------------------------
def test_quant_u8_closed_forms():
    assert oracle.quant_u8(0.0) == 0 and oracle.quant_u8(1.0) == 255
    assert oracle.quant_u8(-0.3) == 0 and oracle.quant_u8(1.7) == 255
    assert oracle.quant_u8(float("nan")) == 0
    assert oracle.quant_u8(0.5) == 128          # 127.5: tie -> even
    assert oracle.quant_u8(1.5 / 255.0) == 2    # 1.5 (up to rounding of the quotient)
    for k in range(256):
        # every stored level reads back as k / 255 and quantises to itself
        v = oracle.dequant_u8(k)
        assert v == float(np.float32(k) / np.float32(255.0))
        assert oracle.quant_u8(v) == k
    # the error of a round trip is at most half a level
    xs = np.random.default_rng(3).random(20_000).astype(np.float32)
    back = np.array([oracle.dequant_u8(oracle.quant_u8(float(x))) for x in xs])
    assert np.abs(back - xs).max() <= 0.5 / 255.0 + 1e-7


# ---- the ring -----------------------------------------------------------------
class NumpyRing:
    """Independent model: a dict slot -> stored transition, quantised by numpy."""

    def __init__(self, cap, nr):
        self.cap, self.nr, self.head, self.size, self.slots = cap, nr, 0, 0, {}

    def enc(self, o):
        o = np.asarray(o, np.float32)
        r = np.clip(o[:self.nr], np.float32(0), np.float32(1))
        q = np.rint(r * np.float32(255.0)).astype(np.uint8)
        return q, o[self.nr:].astype(np.float16)

    def dec(self, enc):
        q, h = enc
        return np.concatenate([q.astype(np.float32) / np.float32(255.0), h.astype(np.float32)])

    def push(self, s, a, r, sn, d, sf=None):
        for i in range(len(a)):
            nxt = sf[i] if (sf is not None and d[i]) else sn[i]
            self.slots[(self.head + i) % self.cap] = (self.enc(s[i]), int(a[i]), np.float32(r[i]),
                                                     self.enc(nxt), int(bool(d[i])))
        self.head = (self.head + len(a)) % self.cap
        self.size = min(self.size + len(a), self.cap)

    def gather(self, k):
        es, a, r, en, d = self.slots[k]
        return self.dec(es), a, r, self.dec(en), d


def batch(rng, n, nr):
    D = nr + 4
    s = rng.random((n, D), dtype=np.float32)
    s[:, nr:] = rng.normal(size=(n, 4)).astype(np.float32)
    sn = rng.random((n, D), dtype=np.float32)
    sn[:, nr:] = rng.normal(size=(n, 4)).astype(np.float32)
    sf = rng.random((n, D), dtype=np.float32)
    a = rng.integers(0, 7, n).astype(np.int32)
    r = rng.normal(size=n).astype(np.float32)
    d = (rng.random(n) < 0.2).astype(np.uint8)
    return s, a, r, sn, d, sf


@pytest.mark.parametrize("cap,nr,pushes", [(37, 5, [10, 20, 30, 7]), (64, 32, [64, 64, 1]),
                                           (100, 64, [3, 0, 99, 50])])
def test_ring_wraps_and_keeps_the_latest(cap, nr, pushes):
    rng = np.random.default_rng(cap)
    orc = oracle.Ring(cap, nr, seed=5)
    ref = NumpyRing(cap, nr)
    for n in pushes:
        s, a, r, sn, d, sf = batch(rng, n, nr)
        use_final = n % 2 == 0
        orc.push(s, a, r, sn, d, sf if use_final else None)
        ref.push(s, a, r, sn, d, sf if use_final else None)
        assert orc.size == ref.size and orc.head == ref.head
        slots = np.arange(orc.size)
        gs, ga, gr, gsn, gd = orc.gather(slots)
        for k in slots:
            es, ea, er, esn, ed = ref.gather(int(k))
            assert np.array_equal(gs[k], es) and np.array_equal(gsn[k], esn), k
            assert ga[k] == ea and gr[k] == er and gd[k] == ed


def test_ring_rejects_oversize_push_and_bad_slots():
    orc = oracle.Ring(8, 4, seed=1)
    s, a, r, sn, d, _ = batch(np.random.default_rng(0), 9, 4)
    with pytest.raises(ValueError):
        orc.push(s, a, r, sn, d)
    with pytest.raises(ValueError):
        orc.sample(4, 0)                       # empty
    orc.push(s[:3], a[:3], r[:3], sn[:3], d[:3])
    with pytest.raises(IndexError):
        orc.gather([3])                        # only slots 0..2 are stored


def test_sample_is_uniform_in_range_and_deterministic():
    cap, nr = 97, 3
    orc = oracle.Ring(cap, nr, seed=11)
    rng = np.random.default_rng(1)
    s, a, r, sn, d, _ = batch(rng, cap, nr)
    orc.push(s, a, r, sn, d)
    counts = np.zeros(cap)
    for draw in range(400):
        *_, idx = orc.sample(256, draw)
        assert idx.min() >= 0 and idx.max() < cap
        counts += np.bincount(idx, minlength=cap)
    n = counts.sum()
    chi2 = float(((counts - n / cap) ** 2 / (n / cap)).sum())
    # 96 degrees of freedom: mean 96, sd ~13.9; 5 sd is far outside chance
    assert chi2 < 96 + 5 * math.sqrt(2 * 96), chi2
    a1 = orc.sample(64, 9)
    a2 = orc.sample(64, 9)
    assert all(np.array_equal(x, y) for x, y in zip(a1, a2))
    assert not np.array_equal(a1[-1], orc.sample(64, 10)[-1])
    # the sample returns what the gather returns at its indices
    s_, a_, r_, sn_, d_, idx = orc.sample(32, 3)
    gs, ga, gr, gsn, gd = orc.gather(idx)
    assert np.array_equal(s_, gs) and np.array_equal(a_, ga) and np.array_equal(sn_, gsn)


def test_sample_covers_only_stored_slots_before_wrap():
    orc = oracle.Ring(1000, 2, seed=4)
    s, a, r, sn, d, _ = batch(np.random.default_rng(2), 10, 2)
    orc.push(s, a, r, sn, d)
    *_, idx = orc.sample(5000, 1)
    assert set(np.unique(idx)) == set(range(10))
