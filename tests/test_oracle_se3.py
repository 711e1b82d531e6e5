"""Pins of the oracle's SE(3) algebra (CPU only), against scipy's matrix
exponential and logarithm of 4x4 homogeneous matrices (Eq. 1, 5, 8).

  se3_exp / se3_log / se3_between   expm / logm, round trips
  det_qdist  q_ij = d^T W d with d = log(T_i^-1 T_j) (Eq. 7-8), FP32 program
             against the FP64 logm value; q_ii = 0; q_ij = q_ji (d_ji = -d_ij);
             continuity across the small-angle branch
"""
import numpy as np
import pytest

from _pinutil import between_ref, pose_to_M, random_pose8, se3_exp_ref, se3_log_ref, M_to_pose8


def test_exp_log_against_scipy(O):
    rng = np.random.default_rng(0)
    for _ in range(300):
        xi = np.concatenate([rng.normal(size=3) * rng.choice([1e-7, 1e-3, 0.5, 2.5]), rng.normal(size=3) * 3])
        if np.linalg.norm(xi[:3]) > 3.0:
            continue
        T = O.se3_exp(xi)
        M = se3_exp_ref(xi)
        P = pose_to_M(T)
        assert np.allclose(P, M, atol=1e-12)
        assert np.allclose(O.se3_log(T), xi, atol=1e-10)
        assert np.allclose(O.se3_log(T), se3_log_ref(M), atol=1e-9)


def test_between_against_scipy(O):
    rng = np.random.default_rng(1)
    for _ in range(200):
        Ti, Tj = random_pose8(rng), random_pose8(rng)
        assert np.allclose(O.se3_between(Ti, Tj), between_ref(Ti, Tj), atol=2e-6)


@pytest.mark.parametrize("scale", [1e-5, 1e-3, 0.05, 0.3, 1.0, 2.5])
def test_det_qdist_against_fp64(O, scale):
    rng = np.random.default_rng(int(scale * 1e6) + 3)
    sr, st = 5.0, 2.5
    W = np.array([sr] * 3 + [st] * 3)
    for _ in range(300):
        Ti = random_pose8(rng, tscale=10)
        M = pose_to_M(Ti) @ se3_exp_ref(np.concatenate([rng.normal(size=3) * scale, rng.normal(size=3) * scale]))
        Tj = M_to_pose8(M)
        d = between_ref(Ti, Tj)
        ref = float(np.sum(W * d * d))
        got = O.det_qdist(Ti, Tj, sr, st)
        # FP32 inputs + FP32 program: relative 1e-5 or the FP32 rounding of the poses
        assert abs(got - ref) <= 2e-5 * ref + 1e-9 * (1 + np.linalg.norm(Ti[4:7])) ** 2 * 50, (got, ref)


def test_det_qdist_invariants(O):
    rng = np.random.default_rng(4)
    for _ in range(200):
        Ti, Tj = random_pose8(rng), random_pose8(rng)
        assert O.det_qdist(Ti, Ti, 5.0, 2.5) == 0.0
        a, b = O.det_qdist(Ti, Tj, 5.0, 2.5), O.det_qdist(Tj, Ti, 5.0, 2.5)
        assert abs(a - b) <= 1e-5 * a
