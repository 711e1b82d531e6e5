"""Pins of the information matrix Omega = (Sigma^M + R Sigma^S R^T)^-1 of the
GICP term (Sec. III-C, Eq. (3)) and of the damped Gauss-Newton step (Eq. (4)),
CPU only.

The likelihood pins elsewhere use R = I, isotropic scan covariances or a zero
residual, so none of them can tell R Sigma^S R^T from R^T Sigma^S R.  Here one
map voxel holds a planar patch z = const (normal exactly z, so Sigma^M =
diag(1, 1, eps')), the one scan point has a rank-1 covariance along the sensor
x axis, and the particle's rotation R = R_z(90 deg) R_y(90 deg) sends the
sensor x axis to -z while R^T sends it to -y.  Every matrix in the term is then
diagonal in the map frame, and the cost, H_vv = R^T Omega R and b_v =
-R^T Omega e have closed forms written with divisions only.

The same construction pins the scan-to-scan GICP terms (target point with
covariance diag(1, 1, eps'), rotated source covariance).

Damping: psi = -(H + diag(lam_rel H_ii + lam_abs))^-1 b (Marquardt's diagonal
scaling) is pinned with a diagonal H of spread-out entries, where it reduces
to an elementwise division that a trace-scaled damping would not match, and
with a dense SPD H against numpy's solver.
"""
import numpy as np
import pytest

# q = (w, x, y, z) of R_z(90 deg) R_y(90 deg); exact in FP32, R has entries 0, +-1
Q_ZY = np.array([0.5, -0.5, 0.5, 0.5])
R_ZY = np.array([[0.0, -1.0, 0.0],
                 [0.0, 0.0, 1.0],
                 [-1.0, 0.0, 0.0]])
SIG2 = 0.04       # rank-1 scan variance along the sensor x axis
DELTA = 1e-4      # isotropic part of the scan covariance (keeps it positive definite)
EPS = 1e-3


def test_rotation_sends_x_to_minus_z():
    # the construction relies on R x = -z and R^T x = -y
    w, x, y, z = Q_ZY
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    Ry = np.array([[0.0, 0.0, 1.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0]])
    assert np.array_equal(R, Rz @ Ry)
    assert np.array_equal(R, R_ZY)
    assert np.array_equal(R @ [1, 0, 0], [0, 0, -1])
    assert np.array_equal(R.T @ [1, 0, 0], [0, -1, 0])


def _closed_form(e, eps_n):
    """cost, H_vv, b_v for Sigma^M = diag(1, 1, eps_n) and R Sigma^S R^T =
    sigma^2 z z^T + delta I (the scan's rank-1 covariance along sensor x,
    carried to the map frame), with the covariance entries as stored in FP32:
    C is diagonal, so Omega = diag(1 / C_mm)"""
    sxx = float(np.float32(SIG2 + DELTA))
    sd = float(np.float32(DELTA))
    w = np.array([1.0 / (1.0 + sd), 1.0 / (1.0 + sd), 1.0 / (eps_n + sxx)])
    cost = float(np.sum(w * e * e))
    Hvv = R_ZY.T @ np.diag(w) @ R_ZY      # J_v = -R
    bv = -R_ZY.T @ (w * e)
    return cost, Hvv, bv


def _h21_to_full(h):
    H = np.zeros((6, 6))
    q = 0
    for i in range(6):
        for j in range(i, 6):
            H[i, j] = H[j, i] = h[q]; q += 1
    return H


@pytest.fixture(scope="module")
def plane_map(O):
    # a 10 x 10 grid on z = 0.25 inside voxel (0, 0, 0) of a 0.5 m map
    g = np.linspace(0.05, 0.45, 10)
    X, Y = np.meshgrid(g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), np.full(X.size, 0.25)], 1).astype(np.float32)
    m = O.Map(xyz, 0.5, nnf_radius=2, min_points=5, cov_eps=EPS)
    gs = m.gauss()
    assert m.G == 1
    assert np.array_equal(np.abs(gs["normal"][0]), np.float32([0, 0, 1]))
    return m, gs


def _rank1_cov():
    # sigma^2 x x^T + delta I in (xx, xy, xz, yy, yz, zz)
    return np.array([[SIG2 + DELTA, 0, 0, DELTA, 0, DELTA]], np.float32)


def _pose_placing(mu_s, target, d):
    """pose (q = Q_ZY, t) that sends the sensor point mu_s to target + d z;
    t is rounded to FP32, so the residual is recomputed from what is stored"""
    t = (np.asarray(target, np.float64) + np.array([0, 0, d]) - R_ZY @ np.asarray(mu_s, np.float64))
    T8 = np.zeros(8, np.float32)
    T8[:4] = Q_ZY
    T8[4:7] = t
    return T8


@pytest.mark.parametrize("d", [0.1, -0.07, 0.3])
def test_likelihood_omega_rotated_rank1(O, plane_map, d):
    m, gs = plane_map
    mu_m = gs["mu"][0].astype(np.float64)
    eps_n = 1.0 - float(np.float32(1.0 - EPS))   # the eigenvalue along the normal, a = 1 - eps in FP32
    mu_s = np.float32([0.3, -0.2, 0.1])
    T8 = _pose_placing(mu_s, mu_m, d)
    out = O.likelihood(m, mu_s[None], _rank1_cov(), T8[None], dmax=1.0, cmax=1e9, lam_rel=0.0, lam_abs=0.0)
    assert out["ninl"][0] == 1
    e = mu_m - (R_ZY @ mu_s.astype(np.float64) + T8[4:7].astype(np.float64))
    assert abs(e[2] + d) < 1e-6 and np.all(np.abs(e[:2]) < 1e-6)
    cost, Hvv, bv = _closed_form(e, eps_n)
    assert out["loglik"][0] == pytest.approx(-cost, rel=1e-9)
    H = _h21_to_full(out["H21"][0])
    assert np.allclose(H[3:, 3:], Hvv, rtol=1e-9, atol=1e-12)
    assert np.allclose(out["b"][0][3:], bv, rtol=1e-9, atol=1e-12)
    # the transposed rotation R^T Sigma^S R puts the scan variance on map y
    # and leaves the normal direction at eps_n + delta: cost d^2 / (eps_n + delta)
    wrong = d * d / (eps_n + DELTA)
    assert abs(-out["loglik"][0] - wrong) > 0.5 * wrong


@pytest.mark.parametrize("d", [0.1, -0.25])
def test_gicp_terms_omega_rotated_rank1(O, d):
    eps_n = 1e-3
    target = np.float32([[1.5, -0.5, 2.0]])
    tcov = np.float32([[1.0, 0, 0, 1.0, 0, eps_n]])
    mu_s = np.float32([0.3, -0.2, 0.1])
    T8 = _pose_placing(mu_s, target[0], d)
    out = O.gicp_terms(target, tcov, mu_s[None], _rank1_cov(), T8[:7], dmax=1.0)
    assert out["ninl"] == 1 and out["nn"][0] == 0
    e = target[0].astype(np.float64) - (R_ZY @ mu_s.astype(np.float64) + T8[4:7].astype(np.float64))
    cost, Hvv, bv = _closed_form(e, float(np.float32(eps_n)))
    assert out["cost"] == pytest.approx(cost, rel=1e-9)
    H = _h21_to_full(out["H21"])
    assert np.allclose(H[3:, 3:], Hvv, rtol=1e-9, atol=1e-12)
    assert np.allclose(out["b"][3:], bv, rtol=1e-9, atol=1e-12)
    wrong = d * d / (eps_n + DELTA)
    assert abs(out["cost"] - wrong) > 0.5 * wrong


def test_gn_damping_diagonal_scaling(O):
    # diagonal H with entries over four decades: Marquardt's damping divides
    # each b_i by H_ii (1 + lam_rel) + lam_abs; a damping lam_rel tr(H)/6
    # would give b_i / (H_ii + lam_rel tr(H) / 6 + lam_abs) instead
    d = np.array([2.0, 10.0, 0.5, 100.0, 3.0, 0.01])
    H21 = np.array([d[i] if i == j else 0.0 for i in range(6) for j in range(i, 6)])
    b = np.array([1.0, -2.0, 3.0, 0.5, -0.25, -1.0])
    lam_rel, lam_abs = 0.1, 0.01
    psi, rc = O.gn_step(H21, b, lam_rel, lam_abs)
    assert rc == 0
    assert np.allclose(psi, -b / (d * (1 + lam_rel) + lam_abs), rtol=1e-13)
    trace_form = -b / (d + lam_rel * d.sum() / 6 + lam_abs)
    assert np.max(np.abs(psi - trace_form) / np.abs(trace_form)) > 0.5


def test_gn_damping_dense_spd(O):
    rng = np.random.default_rng(5)
    A = rng.normal(size=(6, 6))
    H = A @ A.T + 0.1 * np.eye(6)
    H21 = np.array([H[i, j] for i in range(6) for j in range(i, 6)])
    b = rng.normal(size=6)
    lam_rel, lam_abs = 1e-3, 1e-6
    psi, rc = O.gn_step(H21, b, lam_rel, lam_abs)
    assert rc == 0
    ref = -np.linalg.solve(H + np.diag(lam_rel * np.diag(H) + lam_abs), b)
    assert np.allclose(psi, ref, rtol=1e-10, atol=1e-12)
