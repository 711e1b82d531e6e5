"""Pins of the oracle's likelihood and Gauss-Newton terms (Eq. 2-4), CPU only.

  identity-pose zero residual: scan := voxel means, T = I  =>  every point an
      inlier, c = 0, log-lik = 0, b = 0, psi = 0
  b      central finite differences of the oracle's own log-likelihood under
         T exp(delta) with isotropic scan covariances (Omega then independent
         of delta): d(-loglik)/d delta = 2 b
  H      at a zero-residual configuration the Gauss-Newton matrix is the exact
         Hessian: second differences of -loglik = 2 H
  psi    damping closed form for H = I; Gauss-Newton iterations T <- T exp(psi)
         converge to the true pose on noiseless data (sign and perturbation side)
  outliers  a pose far from the map scores -c_max per point with zero H, b
"""
import numpy as np
import pytest

from _pinutil import M_to_pose8, pose_to_M, se3_exp_ref


def _scene(O, seed=0, r=0.5):
    from paper_2404_16370_amd import synth as S
    sc = S.scene_room(1001)
    xyz = S.sample_map(sc, 60_000, 2000 + seed)
    return O.Map(xyz, r, nnf_radius=2, min_points=5)


def _perturb(T8, xi):
    return M_to_pose8(pose_to_M(T8) @ se3_exp_ref(xi))


def _h21_to_full(h):
    H = np.zeros((6, 6))
    q = 0
    for i in range(6):
        for j in range(i, 6):
            H[i, j] = H[j, i] = h[q]; q += 1
    return H


@pytest.fixture(scope="module")
def room_map(O):
    return _scene(O)


def test_identity_zero_residual(O, room_map):
    m = room_map
    g = m.gauss()
    sel = np.arange(0, m.G, 7)
    scan = g["mu"][sel]
    knn, scov, _ = O.scan_cov(scan, k=10)
    T = np.array([[1, 0, 0, 0, 0, 0, 0, 0]], np.float32)
    out = O.likelihood(m, scan, scov, T, dmax=1.0, cmax=9.0)
    assert out["ninl"][0] == len(scan)
    assert out["loglik"][0] == 0.0
    assert np.all(out["b"][0] == 0.0)
    assert np.all(out["psi"][0] == 0.0)
    H = _h21_to_full(out["H21"][0])
    assert np.all(np.linalg.eigvalsh(H) > 0)


def _iso_setup(O, m, seed):
    rng = np.random.default_rng(seed)
    g = m.gauss()
    sel = rng.choice(m.G, 300, replace=False)
    pts = g["mu"][sel].astype(np.float64) + rng.normal(scale=0.05, size=(300, 3))
    scov = np.tile(np.array([0.3, 0, 0, 0.3, 0, 0.3], np.float32), (300, 1))
    T0 = np.array([1, 0, 0, 0, 0, 0, 0, 0], np.float32)
    T = _perturb(T0, np.array([0.01, -0.02, 0.015, 0.03, -0.02, 0.01]))
    # scan expressed in the sensor frame of T
    M = pose_to_M(T)
    local = ((pts - M[:3, 3]) @ M[:3, :3]).astype(np.float32)
    return T, local, scov


def test_b_is_half_gradient_of_cost(O, room_map):
    m = room_map
    T, scan, scov = _iso_setup(O, m, 3)
    base = O.likelihood(m, scan, scov, T[None], dmax=1.0, cmax=1e9)
    h = 1e-5
    grad = np.zeros(6)
    for a in range(6):
        e = np.zeros(6); e[a] = h
        lp = O.likelihood(m, scan, scov, _perturb(T, e)[None], dmax=1.0, cmax=1e9)
        lm = O.likelihood(m, scan, scov, _perturb(T, -e)[None], dmax=1.0, cmax=1e9)
        assert lp["ninl"][0] == lm["ninl"][0] == base["ninl"][0]
        grad[a] = (-lp["loglik"][0] + lm["loglik"][0]) / (2 * h)
    b = base["b"][0]
    assert np.allclose(grad, 2 * b, rtol=2e-3, atol=1e-3 * np.abs(b).max())


def _interior(mu, r, margin):
    f = mu / r - np.floor(mu / r)
    return np.all((f > margin / r) & (f < 1 - margin / r), axis=1)


def test_H_is_hessian_at_zero_residual(O, room_map):
    m = room_map
    g = m.gauss()
    sel = np.nonzero(_interior(g["mu"].astype(np.float64), 0.5, 0.02))[0][::3]
    scan = g["mu"][sel]
    scov = np.tile(np.array([0.3, 0, 0, 0.3, 0, 0.3], np.float32), (len(sel), 1))
    T = np.array([1, 0, 0, 0, 0, 0, 0, 0], np.float32)
    base = O.likelihood(m, scan, scov, T[None], dmax=1.0, cmax=1e9)
    H = _h21_to_full(base["H21"][0])
    h = 3e-4
    Hfd = np.zeros((6, 6))
    f = lambda xi: -O.likelihood(m, scan, scov, _perturb(T, xi)[None], dmax=1.0, cmax=1e9)["loglik"][0]
    f0 = f(np.zeros(6))
    for a in range(6):
        for b in range(a, 6):
            ea = np.zeros(6); ea[a] = h
            eb = np.zeros(6); eb[b] = h
            Hfd[a, b] = Hfd[b, a] = (f(ea + eb) - f(ea - eb) - f(-ea + eb) + f(-ea - eb)) / (4 * h * h)
    assert np.allclose(Hfd, 2 * H, rtol=2e-2, atol=2e-2 * np.abs(H).max())


def test_gn_damping_closed_form(O):
    H21 = np.array([1 if i == j else 0 for i in range(6) for j in range(i, 6)], np.float64)
    b = np.array([1.0, -2, 3, 0.5, 0, -1])
    psi, rc = O.gn_step(H21, b, 1e-3, 1e-6)
    assert rc == 0
    assert np.allclose(psi, -b / (1 + 1e-3 + 1e-6), rtol=1e-14)


def test_gn_converges_to_truth(O, room_map):
    m = room_map
    g = m.gauss()
    rng = np.random.default_rng(11)
    cand = np.nonzero(_interior(g["mu"].astype(np.float64), 0.5, 0.06))[0]
    sel = rng.choice(cand, min(800, len(cand)), replace=False)
    assert len(sel) > 100
    world = g["mu"][sel].astype(np.float64)
    Ttrue = M_to_pose8(se3_exp_ref(np.array([0.2, -0.1, 0.4, 10.0, 9.5, 1.7])))
    M = pose_to_M(Ttrue)
    scan = ((world - M[:3, 3]) @ M[:3, :3]).astype(np.float32)
    knn, scov, _ = O.scan_cov(scan, k=10)
    T = _perturb(Ttrue, np.array([0.002, -0.001, 0.002, 0.02, 0.015, -0.01]))
    errs = []
    for it in range(8):
        out = O.likelihood(m, scan, scov, T[None], dmax=1.0, cmax=9.0, lam_rel=0.0, lam_abs=0.0)
        T = _perturb(T, out["psi"][0])
        d = np.linalg.inv(pose_to_M(Ttrue)) @ pose_to_M(T)
        errs.append(np.linalg.norm(d[:3, 3]) + np.linalg.norm(d[:3, :3] - np.eye(3)))
    assert errs[-1] < 2e-5, errs   # FP32 pose storage limits the floor
    assert errs[2] < 0.1 * errs[0]


def test_far_pose_all_outliers(O, room_map):
    m = room_map
    scan = np.random.default_rng(1).normal(size=(100, 3)).astype(np.float32)
    scov = np.tile(np.array([1, 0, 0, 1, 0, 1], np.float32), (100, 1))
    T = np.array([[1, 0, 0, 0, 1000, 0, 0, 0]], np.float32)
    out = O.likelihood(m, scan, scov, T, dmax=1.0, cmax=9.0)
    assert out["ninl"][0] == 0 and out["loglik"][0] == -900.0
    assert np.all(out["b"][0] == 0) and np.all(out["psi"][0] == 0)
