"""Pins of the oracle's GICP scan-to-scan odometry (Sec. III-B: the motion
estimate dT and its covariance, GICP after Segal et al. 2009) against facts
that do not depend on the oracle itself:

  * a scan matched against itself at the identity: every point is its own
    nearest neighbour, zero residual, b = 0, cost 0;
  * correspondences equal a brute-force float64 nearest neighbour (random
    points, no near ties) and respect the d_max gate;
  * with isotropic source covariances Omega does not depend on the pose, so
    the cost's directional derivative by central differences is 2 b . delta;
  * a noise-free scan moved by a known transform is matched back to that
    transform (the minimiser of a zero-residual problem);
  * Sigma^dT * H = scale * I.
"""
import numpy as np
import pytest

from paper_2404_16370_amd import synth as S

IDENT = np.array([1, 0, 0, 0, 0, 0, 0], np.float32)


@pytest.fixture(scope="module")
def scans(O):
    w = S.build_workload("room", map_points=200_000, scan_points=800, frames=1)
    sc = w["scans"][0]
    _, cov, _ = O.scan_cov(sc, k=10)
    return sc, cov


def _compose(T, xi, O):
    """T exp(xi) for 7-vectors (FP64)"""
    D = O.se3_exp(np.asarray(xi, np.float64))
    R = S.quat_to_mat(T[:4])
    q = _qmul(T[:4], D[:4])
    return np.concatenate([q / np.linalg.norm(q), T[4:7] + R @ D[4:7]])


def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_self_match_zero_residual(scans, O):
    sc, cov = scans
    r = O.gicp_terms(sc, cov, sc, cov, IDENT)
    assert np.array_equal(r["nn"], np.arange(len(sc)))
    assert r["ninl"] == len(sc) and r["cost"] == 0.0
    assert np.all(r["b"] == 0.0)
    H = np.zeros((6, 6))
    H[np.triu_indices(6)] = r["H21"]
    H = H + H.T - np.diag(np.diag(H))
    assert np.all(np.linalg.eigvalsh(H) > 0)


def test_correspondences_brute_force(O):
    rng = np.random.default_rng(0)
    tgt = rng.uniform(-5, 5, (700, 3)).astype(np.float32)
    src = rng.uniform(-5.5, 5.5, (500, 3)).astype(np.float32)
    cov = np.tile(np.array([1, 0, 0, 1, 0, 1], np.float32), (700, 1))
    scov = np.tile(np.array([1, 0, 0, 1, 0, 1], np.float32), (500, 1))
    for dmax in (0.4, 100.0):
        r = O.gicp_terms(tgt, cov, src, scov, IDENT, dmax=dmax)
        d2 = ((src[:, None, :].astype(np.float64) - tgt[None, :, :]) ** 2).sum(-1)
        ref = np.argmin(d2, axis=1)
        ref = np.where(d2[np.arange(len(src)), ref] <= dmax * dmax, ref, -1)
        assert np.array_equal(r["nn"], ref)


def test_gradient_is_2b(scans, O):
    sc, cov = scans
    iso = np.tile(np.array([0.01, 0, 0, 0.01, 0, 0.01], np.float32), (len(sc), 1))
    # a small motion (under 4 cm at 5 m) keeps every point's match its own
    T = np.array([1.0, 0.002, -0.003, 0.0025, 0.01, -0.008, 0.004])
    T[:4] /= np.linalg.norm(T[:4])
    rng = np.random.default_rng(1)
    for _ in range(3):
        d = rng.normal(size=6)
        d /= np.linalg.norm(d)
        r0 = O.gicp_terms(sc, cov, sc, iso, T.astype(np.float32), dmax=0.5)
        h = 1e-4
        cp = O.gicp_terms(sc, cov, sc, iso, _compose(T, h * d, O).astype(np.float32), dmax=0.5)
        cm = O.gicp_terms(sc, cov, sc, iso, _compose(T, -h * d, O).astype(np.float32), dmax=0.5)
        assert np.array_equal(cp["nn"], r0["nn"]) and np.array_equal(cm["nn"], r0["nn"])
        fd = (cp["cost"] - cm["cost"]) / (2 * h)
        assert abs(fd - 2 * r0["b"] @ d) <= 2e-3 * (abs(fd) + np.abs(2 * r0["b"]).sum() * 1e-2)


def test_recovers_known_motion(scans, O):
    sc, cov = scans
    R = S.rotvec_to_mat(np.array([0.03, -0.02, 0.06]))
    t = np.array([0.25, -0.15, 0.04])
    src = ((sc.astype(np.float64) - t) @ R).astype(np.float32)   # src = R^T (sc - t)
    _, scov, _ = O.scan_cov(src, k=10)
    a = O.gicp_align(sc, cov, src, scov, iters=25)
    q = S.mat_to_quat(R)
    assert a["ok"]
    assert np.abs(a["pose"][4:7] - t).max() < 1e-5
    assert min(np.abs(a["pose"][:4] - q).max(), np.abs(a["pose"][:4] + q).max()) < 1e-5
    assert a["ninl"] == len(sc)


def test_covariance_is_scaled_inverse_hessian(scans, O):
    sc, cov = scans
    for scale in (1.0, 40.0):
        a = O.gicp_align(sc, cov, sc, cov, iters=0, cov_scale=scale)
        H = np.zeros((6, 6))
        H[np.triu_indices(6)] = a["H21"]
        H = H + H.T - np.diag(np.diag(H))
        assert np.allclose(a["cov"] @ H, scale * np.eye(6), atol=1e-9 * scale)
        assert np.allclose(a["cov"], a["cov"].T, rtol=1e-9, atol=0)
