"""GPU GICP scan-to-scan odometry (mp_odometry, Sec. III-B) against the oracle.

  terms at a given dT   correspondences bit-exact (FP32 decisions on both
                        sides), inlier count exact, H within 1e-4 of max|H|,
                        b within 1e-4 of sqrt(H_ii cost), cost 1e-4 relative
                        (FP32 per-point terms against FP64)
  full alignment        dT within 1e-4 rad / 1e-4 m of the oracle's FP64 run
                        (same iterations and damping), and near the true motion
  covariance            within 1e-3 relative of the oracle's; Sigma H = scale I
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2404_16370_amd import megapf as M
from paper_2404_16370_amd import synth as S


@pytest.fixture(scope="module")
def world():
    w = S.build_workload("room", map_points=200_000, scan_points=1000, frames=3)
    m = M.Map(w["map_xyz"], voxel=0.5)
    return dict(w=w, m=m)


def _filter(world, scans, O):
    """a filter holding the scans, and the oracle's (points, covariances) of
    the non-empty ones (asserted equal to the library's scan records)"""
    p = M.mp_filter_default_params(n_particles=64, svgd_iters=1)
    f = M.Filter(world["m"], p)
    recs = []
    for sc in scans:
        sc = np.ascontiguousarray(sc, np.float32)
        f.scan_upload(sc)
        if len(sc):
            _, cov, _ = O.scan_cov(sc, k=10)
            rec = f.debug_get("scan")
            assert np.array_equal(rec[:, :3], sc) and np.array_equal(rec[:, 3:9], cov)
            recs.append((sc, np.ascontiguousarray(cov)))
    return f, recs


def _true_motion(w):
    (R0, t0), (R1, t1) = w["traj"][0], w["traj"][1]
    R = R0.T @ R1
    t = R0.T @ (t1 - t0)
    return S.pose8(R, t)[:7]


def _rot_err(qa, qb):
    qa = qa / np.linalg.norm(qa); qb = qb / np.linalg.norm(qb)
    return 2 * np.arccos(min(1.0, abs(float(np.dot(qa, qb)))))


def test_terms_match_oracle(world, O):
    w = world["w"]
    f, ((p0, c0), (p1, c1)) = _filter(world, w["scans"][:2], O)
    truth = _true_motion(w)
    rng = np.random.default_rng(3)
    for k in range(3):
        init = truth.copy()
        init[4:7] += rng.normal(0, 0.05, 3)
        init[:4] = S.mat_to_quat(S.quat_to_mat(init[:4]) @ S.rotvec_to_mat(rng.normal(0, 0.02, 3)))
        init = init.astype(np.float32)
        res = f.odometry(init=init, iterations=0)
        ref = O.gicp_terms(p0, c0, p1, c1, init, dmax=1.0)
        nn = f.debug_get("odo_nn")
        assert np.array_equal(nn, ref["nn"])
        assert res["inliers"] == ref["ninl"] and ref["ninl"] > 500
        assert abs(res["cost"] - ref["cost"]) <= 1e-4 * ref["cost"]
        hmax = np.abs(ref["H21"]).max()
        assert np.abs(res["H21"] - ref["H21"]).max() <= 1e-4 * hmax
        diag = ref["H21"][[0, 6, 11, 15, 18, 20]]
        assert np.all(np.abs(res["b"] - ref["b"]) <= 1e-4 * np.sqrt(diag * ref["cost"]))
        # iterations 0: dT is the initial one
        assert np.array_equal(res["dT"], init)


def test_alignment_matches_oracle_and_truth(world, O):
    w = world["w"]
    f, ((p0, c0), (p1, c1)) = _filter(world, w["scans"][:2], O)
    res = f.odometry(iterations=20, cov_scale=2.0)
    ref = O.gicp_align(p0, c0, p1, c1, iters=20, dmax=1.0, cov_scale=2.0)
    print("odometry: GPU dT %s, oracle %s, inliers %d" % (np.round(res["dT64"], 6), np.round(ref["pose"], 6),
                                                          res["inliers"]))
    assert _rot_err(res["dT64"][:4], ref["pose"][:4]) <= 1e-4
    assert np.abs(res["dT64"][4:7] - ref["pose"][4:7]).max() <= 1e-4
    truth = _true_motion(w)
    assert _rot_err(res["dT64"][:4], truth[:4]) < np.deg2rad(1.0)
    assert np.abs(res["dT64"][4:7] - truth[4:7]).max() < 0.05
    assert res["cov_ok"] and ref["ok"]
    np.testing.assert_allclose(np.diag(res["cov"]), np.diag(ref["cov"]), rtol=1e-3)
    H = np.zeros((6, 6))
    H[np.triu_indices(6)] = res["H21"]
    H = H + H.T - np.diag(np.diag(H))
    assert np.allclose(res["cov"].astype(np.float64) @ H, 2.0 * np.eye(6), atol=1e-3)
    # the result feeds the prediction step
    f.step(res["dT"], res["cov"])


def test_previous_scan_survives_an_empty_upload(world, O):
    w = world["w"]
    empty = np.zeros((0, 3), np.float32)
    f, _ = _filter(world, [w["scans"][0], empty, w["scans"][1]], O)
    g, _ = _filter(world, w["scans"][:2], O)
    a = f.odometry(iterations=5)
    b = g.odometry(iterations=5)
    assert np.array_equal(a["dT"], b["dT"]) and a["inliers"] == b["inliers"]


def test_odometry_errors(world, O):
    w = world["w"]
    f, _ = _filter(world, w["scans"][:1], O)
    with pytest.raises(M.MegaPFError) as e:
        f.odometry()
    assert e.value.status == M.MP_E_STATE
    f.scan_upload(np.ascontiguousarray(w["scans"][1]))
    for kw in (dict(iterations=-1), dict(d_max=0.0), dict(cov_scale=-1.0), dict(lambda_rel=float("nan"))):
        with pytest.raises(M.MegaPFError) as e:
            f.odometry(**kw)
        assert e.value.status == M.MP_E_ARG
    with pytest.raises(M.MegaPFError):
        f.odometry(init=np.array([0, 0, 0, 0, 0, 0, 0], np.float32))
    with pytest.raises(M.MegaPFError):
        f.odometry(init=np.array([1, 0, 0, 0, np.inf, 0, 0], np.float32))
    f.odometry(iterations=1)
