"""Pins of the oracle's counter-based RNG and deterministic FP32 elementary
functions (CPU only).

  philox          published known-answer vectors (tests/golden)
  det_log         libm log, |err| <= 4 ulp-ish over (0, 1] and beyond
  det_sincos2pi   libm sin/cos of 2 pi u, |err| <= 2e-7
  det_rotvec_scale  2 atan2(n, w) / n against libm, incl. the n -> 0 limit
  gauss6          Box-Muller from the pinned Philox words recomputed with libm,
                  and a Kolmogorov-Smirnov normality check
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers(O):
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = O.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_det_log_accuracy(O):
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(0, 1, 2000), np.logspace(-7.2, 0, 500), [1.0, 0.5, 2 ** -24]])
    xs = xs[xs > 0].astype(np.float32)
    for x in xs:
        ref = math.log(float(x))
        got = O.det_log(float(x))
        assert abs(got - ref) <= 3e-7 * max(1.0, abs(ref)), (x, got, ref)
    assert O.det_log(1.0) == 0.0


def test_det_sincos_accuracy(O):
    us = np.concatenate([np.arange(4096) / 4096.0, np.random.default_rng(1).uniform(0, 1, 2000)]).astype(np.float32)
    for u in us:
        s, c = O.det_sincos2pi(float(u))
        a = 2 * math.pi * float(u)
        assert abs(s - math.sin(a)) < 3e-7 and abs(c - math.cos(a)) < 3e-7, (u, s, c)


def test_det_rotvec_scale(O):
    rng = np.random.default_rng(2)
    for _ in range(3000):
        th = rng.uniform(0, math.pi) if rng.random() < 0.8 else 10 ** rng.uniform(-9, -1)
        n, w = math.sin(th / 2), math.cos(th / 2)
        got = O.det_rotvec_scale(np.float32(n), np.float32(w))
        nf, wf = float(np.float32(n)), float(np.float32(w))
        ref = 2 * math.atan2(nf, wf) / nf if nf > 0 else 2.0 / wf
        assert abs(got - ref) <= 4e-7 * ref, (th, got, ref)
    assert O.det_rotvec_scale(0.0, 1.0) == 2.0


def test_gauss6_is_box_muller_of_philox_words(O):
    seed = 0x1234_5678_9ABC
    for (a, b, c, p) in [(0, 0, 0, 2), (7, 3, 1, 1), (123456, 99, 9, 2)]:
        z = O.gauss6(seed, a, b, c, p)
        key = [seed & 0xFFFFFFFF, seed >> 32]
        w = list(O.philox([a, b, c, (p << 16) | 0], key)) + list(O.philox([a, b, c, (p << 16) | 1], key))
        for k in range(3):
            u1 = ((int(w[2 * k]) >> 8) + 1) * 2.0 ** -24
            u2 = (int(w[2 * k + 1]) >> 8) * 2.0 ** -24
            r = math.sqrt(-2 * math.log(u1))
            assert abs(z[2 * k] - r * math.cos(2 * math.pi * u2)) < 2e-6
            assert abs(z[2 * k + 1] - r * math.sin(2 * math.pi * u2)) < 2e-6


def test_gauss6_normal_distribution(O):
    zs = np.array([O.gauss6(99, i, 1, 2, 2) for i in range(4000)]).ravel()
    assert abs(zs.mean()) < 0.03 and abs(zs.std() - 1) < 0.03
    assert stats.kstest(zs, "norm").pvalue > 1e-3


def test_uniform_init_and_lsh_frame(O):
    lo, hi = np.array([-1, 2, 0], np.float32), np.array([3, 5, 1], np.float32)
    P = O.init_uniform(5, 5000, lo, hi)
    q = P[:, :4].astype(np.float64)
    assert np.all(np.abs(np.linalg.norm(q, axis=1) - 1) < 1e-6)
    assert np.all(P[:, 4:7] >= lo) and np.all(P[:, 4:7] < hi)
    # Shoemake rotations are uniform: E[q q^T] = I/4 for a uniform unit quaternion
    C = (q.T @ q) / len(q)
    assert np.allclose(C, np.eye(4) / 4, atol=0.02)
    T = O.lsh_frame(5, 3, 4, lo, hi)
    assert abs(np.linalg.norm(T[:4]) - 1) < 1e-6
    assert not np.array_equal(T, O.lsh_frame(5, 3, 5, lo, hi))


def test_index_ranges_match_full_sets(O):
    # samples of a large particle set: particle i draws with its own index
    lo = np.array([0, 0, 0], np.float32); hi = np.array([10, 10, 3], np.float32)
    full = O.init_uniform(5, 300, lo, hi)
    assert np.array_equal(O.init_uniform_range(5, 120, 180, lo, hi), full[120:])
    TL = O.lsh_frame(5, 2, 1, lo, hi)
    codes = O.lsh_codes(full, TL, 1.0, 5.0, 2.5, 0.3, 20, 5, 2, 1)
    assert np.array_equal(O.lsh_codes(full[120:], TL, 1.0, 5.0, 2.5, 0.3, 20, 5, 2, 1, first_index=120), codes[120:])
