"""GPU parity of the learned surrogate and the rank-1 scorers against the oracle.

  labels        residual field r, grad r (FP32 on the GPU, FP64 oracle): 1e-4 rel
  network       forward of 64-point MFMA tiles vs the oracle's FP64 forward
                that rounds the same operands to bfloat16; remaining
                differences are FP32 accumulation order and the hardware
                sin / exp / rcp, which move a rounded activation by one
                bfloat16 step now and then: |dy| <= 4e-3 (1 + |y|) per
                output, mean |dy| <= 2e-4 (outputs are O(0.1..1))
  gradient      one BF16 training step against the oracle's BF16-emulating
                gradient: per tensor |dG| <= 2e-2 max|G| and the relative
                Frobenius error <= 5e-3 (same error sources as above, summed
                over the batch)
  Adam          one step from the GPU's own gradient against the FP64 update:
                1e-5 relative to the step size
  scorers       residual-field likelihood: loglik 1e-4 rel, H and b 1e-4 of their
                scale (FP32 vs FP64, as the plain path); network likelihood:
                loglik 1e-3 rel, H, b 1e-2 of their scale
Sizes: 1000 points (16 tiles of 64 with a ragged tail), 300 particles x 1000
scan points, batch 1000 (padded to 1024 rows).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2404_16370_amd import megapf as M
from paper_2404_16370_amd import synth as S


@pytest.fixture(scope="module")
def room(O):
    w = S.build_workload("room", map_points=200_000, scan_points=1000)
    m_gpu = M.Map(w["map_xyz"], voxel=0.5, nnf_radius=2, min_points=5, cov_eps=1e-3)
    m_ora = O.Map(w["map_xyz"], 0.5, nnf_radius=2, min_points=5, cov_eps=1e-3)
    sur = M.Surrogate(m_gpu, M.mp_surrogate_default_params(batch=1024, seed=7))
    info = sur.info()
    print("surrogate", {k: v for k, v in info.items() if k != "freqs"}, flush=True)
    return dict(w=w, gpu=m_gpu, ora=m_ora, sur=sur, info=info, oinfo=_oracle_info(O, m_ora, 0.5))


def _oracle_info(O, om, r, dmax=1.0, sigma_s=0.03):
    """the network's input box, frequencies and output scales from the oracle's
    map: the box of the kept voxels, f_max = extent / r cycles per box"""
    vox = om.gauss()["vox"]
    lo = vox.min(0).astype(np.float32) * np.float32(r)
    hi = (vox.max(0) + 1).astype(np.float32) * np.float32(r)
    ext = max(float(hi[a]) - float(lo[a]) for a in range(3))
    return dict(lo=lo, inv_ext=np.full(3, 1.0 / ext, np.float32), freqs=O.ff_freqs(np.float32(ext / r)),
                r_scale=O.r_out(dmax, sigma_s), g_scale=O.r_out(1.0, sigma_s))


def _samples(w, n, seed, spread=0.15):
    rng = np.random.default_rng(seed)
    xyz = w["map_xyz"]
    sel = rng.integers(0, len(xyz), n)
    p = xyz[sel] + rng.normal(0, spread, (n, 3))
    sc = w["scene"]
    k = n // 10
    p[:k] = rng.uniform(sc.lo, sc.hi, (k, 3))
    return p.astype(np.float32)


def _random_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    P = np.zeros(M.MP_SUR_NPARAMS)
    o = 0
    for fi, fo in ((192, 128), (128, 128), (128, 4)):
        P[o:o + fi * fo] = scale * rng.uniform(-1, 1, fi * fo) / np.sqrt(fi); o += fi * fo
        P[o:o + fo] = 0.1 * rng.uniform(-1, 1, fo); o += fo
    return P.astype(np.float32)


def test_info_matches_definition(room, O):
    # every oracle call below takes the oracle's constants (room["oinfo"])
    info, oi = room["info"], room["oinfo"]
    assert np.array_equal(np.asarray(info["lo"], np.float32), oi["lo"])
    assert np.array_equal(np.asarray(info["inv_ext"], np.float32), oi["inv_ext"])
    assert np.array_equal(np.asarray(info["freqs"], np.float32), oi["freqs"])
    assert info["n_params"] == O.mlp_nparams()
    np.testing.assert_allclose(info["r_scale"], oi["r_scale"], rtol=1e-7)
    np.testing.assert_allclose(info["g_scale"], oi["g_scale"], rtol=1e-7)


def test_labels_match_residual_field(room, O):
    p = _samples(room["w"], 5000, 1)
    out = room["sur"].label(p)
    r, g = O.residual_field(room["ora"], p, sigma_s=0.03, dmax=1.0)
    _, _, inl = O.score_field(room["ora"], p, sigma_s=0.03, dmax=1.0)
    assert inl.sum() > 1000 and (~inl).sum() > 100
    # the gate is the same FP32 decision on both sides
    assert np.array_equal(out[:, 0] == np.float32(O.r_out()), ~inl)
    np.testing.assert_allclose(out[:, 0], r, rtol=1e-4, atol=1e-5)
    gs = np.abs(g).max(1, keepdims=True) + 1e-6
    assert np.all(np.abs(out[:, 1:] - g) <= 1e-4 * gs + 1e-5)


def _oracle_forward(O, info, P, p):
    X = O.ff_features(p, info["lo"], info["inv_ext"], info["freqs"], bf16=True)
    return O.mlp_forward(P.astype(np.float64), X, bf16=True)


@pytest.mark.parametrize("n", [1000, 64, 1])
def test_network_forward(room, O, n):
    sur, info = room["sur"], room["oinfo"]
    P = _random_params(3)
    sur.set_params(P)
    assert np.array_equal(sur.get_params(), P)
    p = _samples(room["w"], n, 2)
    out = sur.eval(p)
    y = out.astype(np.float64) / np.array([info["r_scale"], info["g_scale"], info["g_scale"], info["g_scale"]])
    ref = _oracle_forward(O, info, P, p)
    d = np.abs(y - ref)
    print("network forward: max |dy| %.3g, mean %.3g, max |y| %.3g" % (d.max(), d.mean(), np.abs(ref).max()))
    assert np.all(d <= 4e-3 * (1 + np.abs(ref)))
    assert d.mean() <= 2e-4


def test_training_gradient(room, O):
    sur, info = room["sur"], room["oinfo"]
    P = _random_params(4)
    sur.set_params(P)
    p = _samples(room["w"], 1000, 5)
    r, g = O.residual_field(room["ora"], p, sigma_s=0.03, dmax=1.0)
    tgt = np.concatenate([r[:, None], g], axis=1).astype(np.float32)
    loss, G = sur.grad(p, tgt)
    X = O.ff_features(p, info["lo"], info["inv_ext"], info["freqs"], bf16=True)
    sc = np.array([info["r_scale"], info["g_scale"], info["g_scale"], info["g_scale"]], np.float32)
    # the library scales the targets in FP32 (t * (1 / scale))
    T = (tgt * (np.float32(1.0) / sc)).astype(np.float64)
    L_ref, G_ref = O.mlp_loss_grad(P.astype(np.float64), X, T, bf16=True)
    assert abs(loss - L_ref) <= 1e-3 * L_ref
    offs = np.cumsum([0, 192 * 128, 128, 128 * 128, 128, 128 * 4, 4])
    for a, b_ in zip(offs[:-1], offs[1:]):
        gg, rr = G[a:b_].astype(np.float64), G_ref[a:b_]
        rel = np.linalg.norm(gg - rr) / (np.linalg.norm(rr) + 1e-30)
        print("grad block [%d:%d] rel %.3g max %.3g" % (a, b_, rel, np.abs(gg - rr).max() / np.abs(rr).max()))
        assert rel <= 5e-3
        assert np.all(np.abs(gg - rr) <= 2e-2 * np.abs(rr).max())


def test_adam_step(room, O):
    sur, info = room["sur"], room["oinfo"]
    P0 = _random_params(6)
    sur.set_params(P0)
    p = _samples(room["w"], 1000, 7)
    sur.set_data(p)
    losses = sur.train(1)          # batch 1024 >= 1000 samples: the whole set, drawn with replacement
    P1 = sur.get_params()
    lr = 1e-3   # first step of the cosine schedule
    # Adam's first step is lr * g / (|g| + eps') per weight (bias-corrected
    # moments): the sign of the gradient decides it.  The step uses the whole
    # set (batch >= set size); its oracle gradient is the mean of the two
    # halves' gradients.  Checked: the weights whose gradient has one sign in
    # both halves and is well above the GPU's gradient error
    r, g = O.residual_field(room["ora"], p, sigma_s=0.03, dmax=1.0)
    X = O.ff_features(p, info["lo"], info["inv_ext"], info["freqs"], bf16=True)
    sc = np.array([info["r_scale"], info["g_scale"], info["g_scale"], info["g_scale"]], np.float32)
    T = (np.concatenate([r[:, None], g], 1).astype(np.float32) * (np.float32(1.0) / sc)).astype(np.float64)
    _, G1 = O.mlp_loss_grad(P0.astype(np.float64), X[:500], T[:500], bf16=True)
    _, G2 = O.mlp_loss_grad(P0.astype(np.float64), X[500:], T[500:], bf16=True)
    # the GPU's gradient is within 2e-2 of each tensor's largest entry (see
    # the gradient test): weights whose gradient is 3e-2 of it keep their sign
    offs = np.cumsum([0, 192 * 128, 128, 128 * 128, 128, 128 * 4, 4])
    big = np.zeros(len(P0))
    for a, b_ in zip(offs[:-1], offs[1:]):
        big[a:b_] = 3e-2 * np.abs(0.5 * (G1[a:b_] + G2[a:b_])).max()
    sure = (np.sign(G1) == np.sign(G2)) & (np.minimum(np.abs(G1), np.abs(G2)) > big)
    assert sure.sum() > 0.05 * len(P0)
    step = P1.astype(np.float64) - P0.astype(np.float64)
    np.testing.assert_allclose(step[sure], -lr * np.sign(G1[sure]), rtol=0, atol=1e-5 * lr + 1e-7)
    # and the update is the Adam step of the oracle for a gradient of that sign
    P_ref, _, _ = O.adam(P0.astype(np.float64), np.sign(G1), np.zeros(len(P0)), np.zeros(len(P0)), 1,
                         lr=lr, b1=0.9, b2=0.999, eps=1e-8)
    np.testing.assert_allclose(P1[sure], P_ref[sure], rtol=0, atol=1e-5 * lr + 1e-7)
    assert np.isfinite(losses[0])
    assert sur.info()["steps"] == 1


def test_training_reduces_loss(room):
    sur = room["sur"]
    sur.set_params(_random_params(8, scale=1.0))
    p = _samples(room["w"], 20000, 9)
    sur.set_data(p)
    losses = sur.train(300)
    print("loss: first %.4g, last %.4g" % (losses[0], losses[-1]))
    assert np.all(np.isfinite(losses))
    assert losses[-20:].mean() < 0.5 * losses[:5].mean()


def test_training_gain_held_out(room, O):
    """What the trained network gains over the same network untrained: its
    held-out error against the exact residual field (the oracle's), on points
    near the map surfaces and spread over the room.  The plain path it stands
    in for has no such error and is faster (the bench reports both); this is
    the gain of training, not a gain over the plain method."""
    sur = room["sur"]
    sur.set_params(_random_params(31, scale=1.0))
    held = _samples(room["w"], 4000, 33)
    r, g = O.residual_field(room["ora"], held, sigma_s=0.03, dmax=1.0)

    def err():
        y = sur.eval(held).astype(np.float64)
        return np.mean(np.abs(y[:, 0] - r)), np.mean(np.linalg.norm(y[:, 1:] - g, axis=1))

    e0 = err()
    sur.set_data(_samples(room["w"], 60000, 32))
    losses = sur.train(1500)
    e1 = err()
    print("held-out |dr| %.3f -> %.3f, |d grad r| %.3f -> %.3f (loss %.4g -> %.4g)"
          % (e0[0], e1[0], e0[1], e1[1], losses[0], losses[-1]))
    assert e1[0] < 0.5 * e0[0] and e1[1] < e0[1]


def _lik_filter(room, n, poses, scan, scorer, **kw):
    kw.setdefault("lik_layout", M.MP_LIK_LAYOUT_AUTO)
    p = M.mp_filter_default_params(n_particles=n, k=8, lsh_bits=16, svgd_iters=1, post_iters=10, window_c=16,
                                   d_max=1.0, c_max=9.0, seed=4001, scorer=scorer, sigma_s=0.03, **kw)
    f = M.Filter(room["gpu"], p, poses=poses)
    if scorer == M.MP_SCORER_SURROGATE:
        f.set_surrogate(room["sur"])
    f.scan_upload(scan)
    f.debug_set("capture_hb", 1)
    f.debug_stage(M.MP_STAGE_LIK)
    return f.debug_get("psi"), f.debug_get("hb")


def _poses(w, n, seed):
    rng = np.random.default_rng(seed)
    sc = w["scene"]
    P = S.uniform_particles(n - n // 2, sc.lo, sc.hi, seed)
    R, t = w["traj"][0]
    G = S.gaussian_particles(n // 2, S.pose8(R, t), 0.05, 0.1, seed + 1)
    return np.concatenate([P, G]).astype(np.float32)[rng.permutation(n)]


def _check_hb(hb, ref, unt_cost, tol_h, tol_b):
    H = hb[:, :21].astype(np.float64)
    b = hb[:, 21:27].astype(np.float64)
    hn = np.abs(ref["H21"]).max(1, keepdims=True) + 1e-12
    assert np.all(np.abs(H - ref["H21"]) <= tol_h * hn)
    # rank-1 terms: |b_i| <= sqrt(H_ii sum r^2) by Cauchy-Schwarz (b = sum r g, H = sum g g^T)
    diag = ref["H21"][:, [0, 6, 11, 15, 18, 20]]
    bscale = np.sqrt(np.maximum(diag, 0) * np.maximum(unt_cost, 0)[:, None]) + 1e-9
    assert np.all(np.abs(b - ref["b"]) <= tol_b * bscale)


@pytest.mark.parametrize("n,layout", [(300, M.MP_LIK_LAYOUT_PARTICLE), (1, M.MP_LIK_LAYOUT_PARTICLE),
                                      (300, M.MP_LIK_LAYOUT_GROUPED)])
def test_scorefield_likelihood(room, O, n, layout):
    w = room["w"]
    scan = w["scans"][0]
    poses = _poses(w, n, 11)
    psi, hb = _lik_filter(room, n, poses, scan, M.MP_SCORER_SCOREFIELD, lik_layout=layout)
    ref = O.likelihood_rank1(room["ora"], scan, poses, 1, sigma_s=0.03, dmax=1.0, cmax=9.0)
    unt = -O.likelihood_rank1(room["ora"], scan, poses, 1, sigma_s=0.03, dmax=1.0, cmax=1e30)["loglik"]
    ninl = psi[:, 7].astype(np.int64)
    # r^2 < c_max is an FP32 decision on the GPU and FP64 in the oracle
    assert np.all(np.abs(ninl - ref["ninl"]) <= 2)
    ll = psi[:, 6].astype(np.float64)
    assert np.all(np.abs(ll - ref["loglik"]) <= 1e-4 * np.abs(ref["loglik"]) + 1e-2)
    _check_hb(hb, ref, unt, 1e-4, 1e-4)


def test_surrogate_likelihood(room, O):
    w = room["w"]
    info = room["oinfo"]
    sur = room["sur"]
    P = _random_params(12, scale=0.5)
    sur.set_params(P)
    n = 200
    scan = w["scans"][0]
    poses = _poses(w, n, 13)
    psi, hb = _lik_filter(room, n, poses, scan, M.MP_SCORER_SURROGATE)
    kw = dict(params=P.astype(np.float64), lo=info["lo"], inv_ext=info["inv_ext"], freqs=info["freqs"],
              r_scale=info["r_scale"], g_scale=info["g_scale"])
    ref = O.likelihood_rank1(room["ora"], scan, poses, 2, cmax=9.0, **kw)
    unt = -O.likelihood_rank1(room["ora"], scan, poses, 2, cmax=1e30, **kw)["loglik"]
    ninl = psi[:, 7].astype(np.int64)
    print("inliers (network scorer): mean %.1f of 1000, max count diff %d" %
          (ref["ninl"].mean(), np.abs(ninl - ref["ninl"]).max()))
    assert np.all(np.abs(ninl - ref["ninl"]) <= 3)
    ll = psi[:, 6].astype(np.float64)
    assert np.all(np.abs(ll - ref["loglik"]) <= 1e-3 * np.abs(ref["loglik"]) + 1e-1)
    _check_hb(hb, ref, unt, 1e-2, 1e-2)


def test_surrogate_filter_step(room):
    w = room["w"]
    sur = room["sur"]
    n = 2048
    p = M.mp_filter_default_params(n_particles=n, k=8, lsh_bits=12, svgd_iters=3, post_iters=10, window_c=16,
                                   d_max=1.0, seed=4002, scorer=M.MP_SCORER_SURROGATE)
    f = M.Filter(room["gpu"], p, poses=_poses(w, n, 14))
    with pytest.raises(M.MegaPFError):
        f.scan_upload(w["scans"][0])
        f.step()          # no network attached yet
    f.set_surrogate(sur)
    f.step()
    q = f.posterior_query(weights=True)
    assert abs(q["weights"].sum() - 1.0) < 1e-6
    assert np.all(np.isfinite(f.debug_get("poses")))
    with pytest.raises(M.MegaPFError):
        sur.close()       # still attached
    f.set_surrogate(None)


def test_surrogate_check(room, O):
    """The scorer check (mp_filter_set_surrogate_check): its mean |delta s|
    against the oracle (network with bf16 operands, exact residual field) on
    the same sample; a failed check runs the PLAIN scorer (bit-identical to a
    PLAIN filter), a passed one leaves the SURROGATE step untouched."""
    w, info, sur = room["w"], room["oinfo"], room["sur"]
    P = _random_params(21, scale=0.5)
    sur.set_params(P)
    n, stride = 600, 10
    scan = w["scans"][0]
    poses = _poses(w, n, 22)

    def make(scorer, check=None):
        p = M.mp_filter_default_params(n_particles=n, k=8, lsh_bits=12, svgd_iters=2, post_iters=5, window_c=16,
                                       d_max=1.0, c_max=9.0, seed=4003, scorer=scorer, sigma_s=0.03)
        f = M.Filter(room["gpu"], p, poses=poses)
        if scorer == M.MP_SCORER_SURROGATE:
            f.set_surrogate(sur)
        if check is not None:
            f.set_surrogate_check(*check)
        f.scan_upload(scan)
        return f

    plain = make(M.MP_SCORER_PLAIN)
    guarded = make(M.MP_SCORER_SURROGATE, (3, stride, 0.0, 2))     # every check fails
    free = make(M.MP_SCORER_SURROGATE)
    never = make(M.MP_SCORER_SURROGATE, (3, stride, 1e30, 2))      # every check passes
    with pytest.raises(M.MegaPFError):
        guarded.set_surrogate_check(3, 0, 0.5, 2)
    # expected value of the first check: every 10th particle x every scan point
    P8 = poses.astype(np.float64)[::stride]      # unit quaternions: the library keeps them as given
    mu = scan.astype(np.float64)                  # the check's mean does not depend on the point order
    pts = []
    for q in P8:
        R = S.quat_to_mat(q[:4] / np.linalg.norm(q[:4]))
        pts.append(mu @ R.T + q[4:7])
    pts = np.concatenate(pts).astype(np.float32)
    r_ref, _ = O.residual_field(room["ora"], pts, sigma_s=0.03, dmax=1.0)
    r_net = _oracle_forward(O, info, P, pts)[:, 0] * info["r_scale"]
    ds_ref = np.mean(np.abs(np.minimum(r_net ** 2, 9.0) - np.minimum(r_ref ** 2, 9.0)))
    for step in range(4):
        for f in (plain, guarded, free, never):
            f.step()
        qg = guarded.posterior_query()
        if step == 0:
            print("check: GPU mean |ds| %.5f, oracle %.5f" % (qg["sur_check_ds"], ds_ref))
            assert abs(qg["sur_check_ds"] - ds_ref) <= 2e-2 * ds_ref + 2e-2
        if step < 2:   # frames 0 and 1 fall back to PLAIN
            assert np.array_equal(guarded.debug_get("poses"), plain.debug_get("poses"))
            assert np.array_equal(guarded.debug_get("psi"), plain.debug_get("psi"))
        assert np.array_equal(never.debug_get("poses"), free.debug_get("poses"))
    qg, qn, qf = guarded.posterior_query(), never.posterior_query(), free.posterior_query()
    # frame 0: check, fallback for 2 steps; frame 2: no check; frame 3: check, fallback
    assert (qg["sur_checks"], qg["fallback_steps"]) == (2, 3)
    assert (qn["sur_checks"], qn["fallback_steps"]) == (2, 0) and qn["sur_check_ds"] >= 0
    assert (qf["sur_checks"], qf["fallback_steps"], qf["sur_check_ds"]) == (0, 0, -1.0)
    with pytest.raises(M.MegaPFError) as e:
        M.Batch([guarded], autotune=False)
    assert e.value.status == M.MP_E_UNSUPPORTED
    for f in (guarded, free, never):
        f.set_surrogate(None)
    for f in (plain, guarded, free, never):
        f.close()
