"""Per-particle parity of the Gauss-Newton displacement psi (Eq. 4) and of one
whole correction iteration (Eq. 2-10 and Alg. 1) against the CPU oracle.

psi = -(H + lambda)^-1 b is compared in the Jacobi-scaled coordinates the
solve works in (x = psi / d, d_i = 1 / sqrt(A_ii), A = H + damping):
  * the solve itself: the GPU's psi against an FP64 solve of the GPU's own
    FP32 sums (H, b), within c kappa u (u = 2^-24 for the FP32 Cholesky,
    2^-53 for the FP64 re-solve taken above a condition estimate of 1e6);
  * the whole stage: the GPU's psi against the oracle's (FP64 throughout),
    within the first-order perturbation bound ||A_o^-1|| (||dA|| ||x|| +
    ||db||) that the differences of the FP32 sums from the oracle's imply,
    plus the solve's own bound.
A near-singular case (lambda_rel = 0, lambda_abs = 1e-6) drives particles
into the FP64 re-solve.  The chained iteration runs LSH, sort, refresh,
likelihood and SVGD on the GPU in one filter step and compares the poses
with the oracle's chain (its lists, its psi, its SVGD update).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2404_16370_amd import megapf as M
from paper_2404_16370_amd import synth as S

U32, U64 = 2.0 ** -24, 2.0 ** -53


@pytest.fixture(scope="module")
def room(O):
    w = S.build_workload("room", map_points=200_000, scan_points=1000)
    m_gpu = M.Map(w["map_xyz"], voxel=0.5, nnf_radius=2, min_points=5, cov_eps=1e-3)
    m_ora = O.Map(w["map_xyz"], 0.5, nnf_radius=2, min_points=5, cov_eps=1e-3)
    return dict(w=w, gpu=m_gpu, ora=m_ora)


def _poses_mixed(w, n, seed):
    """half uniform over the room, half scattered around the ground truth"""
    sc = w["scene"]
    P = S.uniform_particles(n - n // 2, sc.lo, sc.hi, seed)
    R, t = w["traj"][0]
    G = S.gaussian_particles(n // 2, S.pose8(R, t), 0.05, 0.1, seed + 1)
    return np.concatenate([P, G]).astype(np.float32)


def _system(H21, b, lam_rel, lam_abs):
    """damped matrix A = H + diag(lam_rel H_ii + lam_abs), its Jacobi scaling
    d, the scaled matrix and right-hand side, and kappa of the scaled matrix"""
    n = H21.shape[0]
    iu = np.triu_indices(6)
    A = np.zeros((n, 6, 6))
    A[:, iu[0], iu[1]] = H21
    A[:, iu[1], iu[0]] = H21
    dg = A[:, np.arange(6), np.arange(6)].copy()
    A[:, np.arange(6), np.arange(6)] += lam_rel * dg + lam_abs
    d = 1.0 / np.sqrt(A[:, np.arange(6), np.arange(6)])
    As = A * d[:, :, None] * d[:, None, :]
    w = np.linalg.eigvalsh(As)
    kappa = np.where(w[:, 0] > 0, w[:, -1] / np.maximum(w[:, 0], 1e-300), np.inf)
    return A, As, d, -b * d, kappa, w


def _check_psi(psi_gpu, hb, how, ref, lam_rel, lam_abs, label):
    """both psi checks of the module docstring, per particle; returns the
    oracle's kappa and the relative error against the oracle (scaled norm)"""
    Hg, bg = hb[:, :21].astype(np.float64), hb[:, 21:27].astype(np.float64)
    _, Asg, dg, rg, kg, wg = _system(Hg, bg, lam_rel, lam_abs)
    Ao, Aso, do, ro, ko, wo = _system(ref["H21"], ref["b"], lam_rel, lam_abs)
    pd_g = wg[:, 0] > 0
    x_own = np.zeros_like(rg)
    x_own[pd_g] = np.linalg.solve(Asg[pd_g], rg[pd_g][:, :, None])[:, :, 0]
    psi_gpu = psi_gpu.astype(np.float64)
    # (1) the solve: GPU psi against the FP64 solution of the GPU's own sums
    u = np.where(how == 0, U32, U64)
    x_g = psi_gpu / dg
    e1 = np.linalg.norm(x_g - x_own, axis=1)
    b1 = (64.0 * kg * u + 2.0 * U32) * np.linalg.norm(x_own, axis=1) + 1e-30
    ok1 = pd_g & (how < 2)
    bad1 = np.nonzero(ok1 & ~(e1 <= b1))[0]
    assert len(bad1) == 0, "%s: solve of own sums off for %d particles, e.g. %d: err %.3g bound %.3g kappa %.3g how %d" % (
        label, len(bad1), bad1[0], e1[bad1[0]], b1[bad1[0]], kg[bad1[0]], how[bad1[0]])
    # a failed FP64 re-solve writes psi = 0
    assert np.all(psi_gpu[how == 2] == 0.0)
    # (2) against the oracle: the perturbation the FP32 sums' differences imply
    pd_o = wo[:, 0] > 0
    x_o = ref["psi"] / do
    x_gp = psi_gpu / do
    Ag = np.zeros_like(Ao)
    Ag[:] = Asg / (dg[:, :, None] * dg[:, None, :])       # the GPU's damped matrix
    dAs = (Ag - Ao) * do[:, :, None] * do[:, None, :]
    dbs = (bg - ref["b"]) * do
    inv_norm = 1.0 / np.maximum(wo[:, 0], 1e-300)
    pert = inv_norm * (np.linalg.norm(dAs, ord=2, axis=(1, 2)) * np.linalg.norm(x_gp, axis=1)
                       + np.linalg.norm(dbs, axis=1))
    e2 = np.linalg.norm(x_gp - x_o, axis=1)
    # the solve's own bound, carried from the GPU's scaling to the oracle's
    b2 = 1.25 * pert + b1 * (dg / do).max(1) + 1e-12
    ok2 = pd_o & ok1
    bad2 = np.nonzero(ok2 & ~(e2 <= b2))[0]
    assert len(bad2) == 0, "%s: psi vs oracle off for %d particles, e.g. %d: err %.3g bound %.3g kappa %.3g" % (
        label, len(bad2), bad2[0], e2[bad2[0]], b2[bad2[0]], ko[bad2[0]])
    rel = e2 / np.maximum(np.linalg.norm(x_o, axis=1), 1e-30)
    for lo, hi in [(0, 1e3), (1e3, 1e4), (1e4, 1e6), (1e6, np.inf)]:
        sel = ok2 & (ko >= lo) & (ko < hi)
        if sel.any():
            print("%s kappa [%.0e, %.0e): %d particles, rel err max %.3g median %.3g" % (
                label, lo, hi, sel.sum(), rel[sel].max(), np.median(rel[sel])), flush=True)
    return ko, rel, ok2


@pytest.mark.parametrize("layout,n,nscan", [(M.MP_LIK_LAYOUT_GROUPED, 1000, 1000),
                                            (M.MP_LIK_LAYOUT_PARTICLE, 1000, 1000),
                                            (M.MP_LIK_LAYOUT_GROUPED, 300, 700)])
def test_psi_per_particle(room, O, layout, n, nscan):
    w = room["w"]
    scan = np.ascontiguousarray(w["scans"][0][:nscan])
    _, scov, _ = O.scan_cov(scan, k=10)
    poses = _poses_mixed(w, n, 200 + n)
    p = M.mp_filter_default_params(n_particles=n, k=8, lsh_bits=16, svgd_iters=1, window_c=16, d_max=1.0,
                                   c_max=9.0, lik_layout=layout, seed=4001)
    f = M.Filter(room["gpu"], p, poses=poses)
    f.scan_upload(scan, cov6=scov)
    f.debug_set("capture_hb", 1)
    f.debug_stage(M.MP_STAGE_LIK)
    psi, hb, how = f.debug_get("psi"), f.debug_get("hb"), f.debug_get("solve")
    ref = O.likelihood(room["ora"], scan, scov, poses, dmax=1.0, cmax=9.0, lam_rel=1e-3, lam_abs=1e-6)
    ko, rel, ok = _check_psi(psi[:, :6], hb, how, ref, 1e-3, 1e-6, "layout %d" % layout)
    # Marquardt damping keeps the scaled system's condition below about 6 / lam_rel
    assert np.all(ko[ok] < 1e4) and np.all(how == 0)
    # an FP32 solve is good to about kappa x 1e-7 relative; with the FP32
    # sums' own error (a few 1e-6 of the largest entry) 1e-3 covers every particle
    assert rel[ok].max() < 1e-3, rel[ok].max()


def test_psi_fp64_resolve(room, O):
    # a scan of two points: J = [[mu]x, -I] leaves the rotation about the line
    # through them unobserved, so with no relative damping and a tiny
    # absolute one the particles that see both points have a (nearly)
    # singular H and take the FP64 re-solve; particles that see neither keep
    # H = 0 (psi = 0 from the FP32 solve)
    n = 1000
    w = room["w"]
    scan = np.ascontiguousarray(w["scans"][0][[10, 500]])
    _, scov, _ = O.scan_cov(scan, k=10)
    poses = _poses_mixed(w, n, 301)
    p = M.mp_filter_default_params(n_particles=n, k=8, lsh_bits=16, svgd_iters=1, window_c=16, d_max=1.0,
                                   c_max=9.0, lambda_rel=0.0, lambda_abs=1e-6, final_rescore=0, seed=4001)
    f = M.Filter(room["gpu"], p, poses=poses)
    f.scan_upload(scan, cov6=scov)
    f.debug_set("capture_hb", 1)
    f.debug_stage(M.MP_STAGE_LIK)
    psi, hb, how = f.debug_get("psi"), f.debug_get("hb"), f.debug_get("solve")
    ref = O.likelihood(room["ora"], scan, scov, poses, dmax=1.0, cmax=9.0, lam_rel=0.0, lam_abs=1e-6)
    assert np.array_equal(psi[:, 7].astype(np.int64), ref["ninl"].astype(np.int64))
    ko, rel, ok = _check_psi(psi[:, :6], hb, how, ref, 0.0, 1e-6, "two-point scan")
    n64 = int((how >= 1).sum())
    print("FP64 re-solves %d (failed %d) of %d; inliers 2: %d" % (n64, int((how == 2).sum()), n,
                                                                 int((ref["ninl"] == 2).sum())), flush=True)
    assert n64 > 0
    # the branch follows the condition: far above 1e6 always re-solved, far below never
    _, _, _, _, kg, _ = _system(hb[:, :21].astype(np.float64), hb[:, 21:27].astype(np.float64), 0.0, 1e-6)
    assert np.all(how[kg > 1e8] >= 1)
    assert np.all(how[kg < 1e4] == 0)
    # the step's counter equals the per-particle record (one likelihood pass)
    f2 = M.Filter(room["gpu"], p, poses=poses)
    f2.scan_upload(scan, cov6=scov)
    f2.debug_set("capture_hb", 1)
    f2.step()
    assert f2.posterior_query()["fp64_resolves"] == int((f2.debug_get("solve") >= 1).sum()) == n64


def _rot_err(q1, q2):
    """angle of q1^-1 q2, as 2 atan2(|v|, |w|) (well conditioned near 0)"""
    a = q1.astype(np.float64)
    b = q2.astype(np.float64)
    a = a / np.linalg.norm(a, axis=1, keepdims=True)
    b = b / np.linalg.norm(b, axis=1, keepdims=True)
    w = a[:, 0] * b[:, 0] + np.sum(a[:, 1:] * b[:, 1:], axis=1)
    v = a[:, :1] * b[:, 1:] - b[:, :1] * a[:, 1:] - np.cross(a[:, 1:], b[:, 1:])
    return 2.0 * np.arctan2(np.linalg.norm(v, axis=1), np.abs(w))


@pytest.mark.parametrize("n,K,bits,win", [(3000, 8, 12, 16), (2500, 16, 8, 32)])
def test_chained_iteration(room, O, n, K, bits, win):
    # one filter step with one correction iteration and no prediction: every
    # stage on the GPU, fed by the previous one; the oracle chain is fed only
    # by its own results
    w = room["w"]
    scan = np.ascontiguousarray(w["scans"][0][:1000])
    _, scov, _ = O.scan_cov(scan, k=10)
    poses = _poses_mixed(w, n, 400 + n)
    p = M.mp_filter_default_params(n_particles=n, k=K, lsh_bits=bits, svgd_iters=1, window_c=win, post_iters=10,
                                   d_max=1.0, c_max=9.0, final_rescore=0, seed=4001)
    f = M.Filter(room["gpu"], p, poses=poses)
    f.scan_upload(scan, cov6=scov)
    f.step()
    out = f.debug_get("poses")
    nbr_g = f.debug_get("nbr").T
    info = room["gpu"].info()
    lo = np.array(info["box_min"], np.float32)
    hi = np.array(info["box_max"], np.float32)
    codes = O.lsh_codes(poses, O.lsh_frame(4001, 0, 0, lo, hi), 1.0, 5.0, 2.5, 0.3, bits, 4001, 0, 0)
    s, _, _ = O.bucket_sort(codes)
    old = np.full((n, K), -1, np.int32)
    old[:, 0] = np.arange(n)
    nbr, q, _ = O.refresh(poses, s, codes, K, win, 5.0, 2.5, old)
    assert np.array_equal(nbr_g, nbr)
    ref = O.likelihood(room["ora"], scan, scov, poses, dmax=1.0, cmax=9.0, lam_rel=1e-3, lam_abs=1e-6)
    _, new = O.svgd(poses, ref["psi"], nbr, 5.0, 2.5)
    er = _rot_err(out[:, :4], new[:, :4])
    et = np.abs(out[:, 4:7].astype(np.float64) - new[:, 4:7]).max(1)
    # a particle's update mixes the psi of its list: its condition is the
    # worst of theirs
    _, _, _, _, ko, _ = _system(ref["H21"], ref["b"], 1e-3, 1e-6)
    kl = np.where(nbr >= 0, ko[np.maximum(nbr, 0)], 0.0).max(1)
    good = kl <= 1e4
    print("chained n %d K %d: %d of %d particles with kappa <= 1e4; rot err max %.3g, trans err max %.3g; "
          "others: rot %.3g trans %.3g" % (n, K, good.sum(), n, er[good].max(), et[good].max(),
                                           er[~good].max() if (~good).any() else 0.0,
                                           et[~good].max() if (~good).any() else 0.0), flush=True)
    assert good.mean() > 0.99
    assert er[good].max() < 1e-4 and et[good].max() < 1e-4
    # the posterior that closes the step, from the step's own log-likelihoods
    # (within 1e-4 relative of the oracle's, checked above; a relative error
    # of 1e-4 on a log-likelihood of -1000 moves a weight by 10%, so the
    # oracle's propagation is fed the GPU's values) and the oracle's lists
    ll = f.debug_get("psi")[:, 6].astype(np.float64)
    assert np.all(np.abs(ll - ref["loglik"]) <= 1e-4 * np.abs(ref["loglik"]) + 1e-3)
    kv = np.where(nbr >= 0, np.exp(-q.astype(np.float64)), 0.0)
    post = O.posterior(np.full(n, 1.0 / n), ll, nbr, kv, rounds=10)
    wq = f.posterior_query(weights=True)["weights"]
    assert abs(wq.sum() - 1.0) < 1e-6
    assert np.abs(wq - post["post"]).max() < 1e-5


@pytest.mark.parametrize("layout", [M.MP_LIK_LAYOUT_GROUPED, M.MP_LIK_LAYOUT_PARTICLE])
def test_thin_scan_covariances_precision(room, O, layout):
    """Scan covariances from the k-NN of points on walls are thin along the
    wall normal, and particles near the true pose see most points as inliers
    on those walls: the Sherman-Morrison denominator of Omega, the small
    eigenvalue-like term of Sigma^M + R Sigma^S R^T along the normal, is then
    about 1e-3 of its parts.  Formed as lam_n + a u^T D u it keeps FP32
    accuracy (log-likelihood and H within a few 1e-6 of the FP64 oracle);
    formed as 1 - a u^T P u it lost about 10 bits (8e-5).  The bound 2e-5
    separates the two."""
    w = room["w"]
    scan = np.ascontiguousarray(w["scans"][0])
    _, scov, _ = O.scan_cov(scan, k=10)
    R, t = w["traj"][0]
    poses = S.gaussian_particles(1024, S.pose8(R, t), 0.05, 0.1, 7).astype(np.float32)
    p = M.mp_filter_default_params(n_particles=1024, k=8, lsh_bits=16, svgd_iters=1, window_c=16, d_max=1.0,
                                   c_max=9.0, lik_layout=layout, seed=4001)
    f = M.Filter(room["gpu"], p, poses=poses)
    f.scan_upload(scan, cov6=scov)
    f.debug_set("capture_hb", 1)
    f.debug_stage(M.MP_STAGE_LIK)
    psi, hb = f.debug_get("psi"), f.debug_get("hb")
    ref = O.likelihood(room["ora"], scan, scov, poses, dmax=1.0, cmax=9.0)
    assert np.array_equal(psi[:, 7].astype(np.int64), ref["ninl"].astype(np.int64))
    assert np.median(ref["ninl"]) > 0.8 * len(scan)      # mostly inliers, as intended
    ell = np.abs(psi[:, 6].astype(np.float64) - ref["loglik"]) / np.maximum(1.0, np.abs(ref["loglik"]))
    H = hb[:, :21].astype(np.float64)
    eh = np.abs(H - ref["H21"]).max(1) / np.abs(ref["H21"]).max(1)
    print("layout %d: log-likelihood rel err max %.3g, H err max %.3g of max |H|" % (layout, ell.max(), eh.max()),
          flush=True)
    assert ell.max() < 2e-5, ell.max()
    assert eh.max() < 2e-5, eh.max()
