"""Pins of the oracle's learned-surrogate functions, CPU only.

  score field   closed form through the eigen-decomposition of Sigma^M (eigen-
                values 1 - a and 1 along / across the normal); central
                differences for its gradient; against the oracle's plain
                likelihood with an isotropic scan covariance sigma_s^2 I at the
                identity pose (one point per call); outliers
  residual field  r = sqrt(s), grad r = grad s / (2 max(r, floor)), r_out and
                zero gradient outside the gate
  bf16 round    torch's float -> bfloat16 conversion (round to nearest even)
  features      numpy sin / cos of 2 pi f x in FP64 (the FP32 fractional part
                only changes the angle by rounding); geometric frequencies
  MLP forward   torch.nn.functional linear + silu in float64
  MLP gradient  torch autograd in float64 and central differences
  BF16 forward  torch float64 forward on bf16-rounded weights and inputs
  Adam          the first step's closed form (m^ = g, v^ = g^2) and torch.optim.Adam
"""
import numpy as np
import pytest
import torch


@pytest.fixture(scope="module")
def room(O):
    from paper_2404_16370_amd import synth as S
    sc = S.scene_room(1001)
    xyz = S.sample_map(sc, 60_000, 2001)
    return O.Map(xyz, 0.5, nnf_radius=2, min_points=5), sc


def _near_surface_points(O, m, n, seed, spread=0.15):
    rng = np.random.default_rng(seed)
    g = m.gauss()
    sel = rng.integers(0, m.G, n)
    return (g["mu"][sel] + rng.normal(0, spread, (n, 3))).astype(np.float32)


def test_score_field_closed_form(O, room):
    m, _ = room
    sig = float(np.float32(0.03))   # the oracle takes sigma_s as FP32
    p = _near_surface_points(O, m, 4000, 1)
    s, g, inl = O.score_field(m, p, sigma_s=sig, dmax=0.3)
    gid = m.lookup(p)
    G = m.gauss()
    a = np.float64(np.float32(1.0) - np.float32(1e-3))
    hit = gid >= 0
    mu = G["mu"][np.maximum(gid, 0)].astype(np.float64)
    nv = G["normal"][np.maximum(gid, 0)].astype(np.float64)
    e = mu - p.astype(np.float64)
    # the stored FP32 normal is unit only to rounding: Sigma^M = I - a n n^T
    # has eigenvalue 1 - a |n|^2 along n and 1 across it
    n2 = np.sum(nv * nv, axis=1)
    nv = nv / np.sqrt(n2)[:, None]
    lam = 1.0 - a * n2 + sig ** 2
    en = np.sum(e * nv, axis=1)
    e2 = np.sum(e * e, axis=1)
    c = en ** 2 / lam + (e2 - en ** 2) / (1.0 + sig ** 2)
    ref_inl = hit & (e2 <= 0.09)
    # the inlier gate is an FP32 decision: skip points within rounding of it
    clear = np.abs(e2 - 0.09) > 1e-5
    assert np.array_equal(inl[clear], ref_inl[clear])
    assert ref_inl.sum() > 1000 and (~ref_inl).sum() > 300 and (ref_inl & (c > 9.0)).sum() > 100
    k = clear & ref_inl
    np.testing.assert_allclose(s[k], c[k], rtol=1e-9, atol=1e-12)
    assert np.all(s[~inl] == 0) and np.all(g[~inl] == 0)
    # gradient of c with respect to p: -2 Omega e (untruncated)
    Oe = en[:, None] * nv / lam[:, None] + (e - en[:, None] * nv) / (1.0 + sig ** 2)
    np.testing.assert_allclose(g[k], -2.0 * Oe[k], rtol=1e-9, atol=1e-9)


def test_score_field_gradient_fd(O, room):
    m, _ = room
    p = _near_surface_points(O, m, 3000, 2, spread=0.05).astype(np.float64)
    s0, g0, i0 = O.score_field(m, p, sigma_s=0.05, dmax=1.0)
    h = 1e-3
    ok = 0
    for a in range(3):
        dp = np.zeros(3); dp[a] = h
        sp, _, ip = O.score_field(m, p + dp, sigma_s=0.05, dmax=1.0)
        sm, _, im = O.score_field(m, p - dp, sigma_s=0.05, dmax=1.0)
        # keep points whose voxel association and inlier state do not change inside the stencil
        same = (m.lookup(p + dp) == m.lookup(p)) & (m.lookup(p - dp) == m.lookup(p)) & i0 & ip & im
        fd = (sp - sm) / (2 * h)
        # the stencil is evaluated at FP32-rounded points: the FD error is
        # O(h^2) curvature plus O(ulp(p) |grad| / h)
        err = np.abs(fd[same] - g0[same, a])
        assert np.all(err <= 1e-3 * (1.0 + np.abs(g0[same, a])) + 4e-4 * np.abs(g0[same, a]) + 2e-3), a
        ok += same.sum()
    assert ok > 1000


def test_residual_field(O, room):
    m, _ = room
    p = _near_surface_points(O, m, 3000, 3, spread=0.6)
    s, g, inl = O.score_field(m, p, sigma_s=0.03, dmax=1.0)
    ro = O.r_out(1.0, 0.03)
    np.testing.assert_allclose(ro, 1.0 / np.sqrt(1e-3 + np.float64(np.float32(0.03)) ** 2))
    r, gr = O.residual_field(m, p, sigma_s=0.03, dmax=1.0, r_floor=1e-2)
    assert inl.sum() > 1000 and (~inl).sum() > 100
    np.testing.assert_allclose(r[inl], np.sqrt(s[inl]), rtol=1e-14)
    d = 2 * np.maximum(np.sqrt(s[inl]), 1e-2)
    np.testing.assert_allclose(gr[inl], g[inl] / d[:, None], rtol=1e-14)
    assert np.all(r[~inl] == ro) and np.all(gr[~inl] == 0)
    # inside the gate r never exceeds r_out (the largest eigenvalue of Omega is 1/(eps + sigma^2))
    assert r[inl].max() <= ro * (1 + 1e-6)


def test_score_field_matches_plain_likelihood(O, room):
    """At the identity pose with scan covariance sigma_s^2 I, the plain
    per-point cost (Eq. 3) of a single-point scan is the score field."""
    m, _ = room
    sig = np.float32(0.2)
    p = _near_surface_points(O, m, 200, 3, spread=0.3)
    s, _, inl = O.score_field(m, p, sigma_s=float(sig), dmax=1.0)
    T = np.array([[1, 0, 0, 0, 0, 0, 0, 0]], np.float32)
    cov = np.array([[sig * sig, 0, 0, sig * sig, 0, sig * sig]], np.float32)
    assert inl.sum() > 100
    for i in range(len(p)):
        out = O.likelihood(m, p[i:i + 1], cov, T, dmax=1.0, cmax=1e9)
        assert out["ninl"][0] == int(inl[i])
        if inl[i]:
            # the plain path builds sigma^2 I in FP32; the score field in FP64
            np.testing.assert_allclose(-out["loglik"][0], s[i], rtol=2e-6, atol=1e-9)


def test_score_field_far_points_are_outliers(O, room):
    m, sc = room
    far = np.array([[500.0, 500.0, 500.0], [-300.0, 0.0, 0.0]], np.float32)
    s, g, inl = O.score_field(m, far)
    assert not inl.any() and np.all(g == 0.0)
    r, gr = O.residual_field(m, far)
    assert np.all(r == O.r_out()) and np.all(gr == 0.0)


def test_bf16_round_matches_torch(O):
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.normal(0, 1, 3000), rng.normal(0, 1e-3, 500), rng.normal(0, 1e4, 500),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, -3.0e-39, 65504.0]])
    # exact ties: values halfway between two bfloat16 numbers
    base = torch.tensor(rng.normal(0, 1, 200), dtype=torch.float32).to(torch.bfloat16).to(torch.float32)
    ulp = torch.abs(base) * 2.0 ** -8
    x = np.concatenate([x, (base + 0.5 * ulp).numpy().astype(np.float64)])
    x32 = x.astype(np.float32).astype(np.float64)
    ref = torch.tensor(x32, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = O.bf16_round(x32)
    np.testing.assert_array_equal(got, ref)


def test_ff_features(O):
    f = O.ff_freqs(100.0, 32)
    assert f[0] == 1.0 and abs(f[-1] - 100.0) < 1e-4
    r = f[1:].astype(np.float64) / f[:-1]
    np.testing.assert_allclose(r, 100.0 ** (1 / 31), rtol=1e-6)
    rng = np.random.default_rng(7)
    lo = np.array([-10.0, -10.0, -1.0], np.float32)
    ext = np.array([20.0, 20.0, 4.0], np.float32)
    inv = (1.0 / ext).astype(np.float32)
    p = (lo + rng.uniform(0, 1, (300, 3)) * ext).astype(np.float32)
    F = O.ff_features(p, lo, inv, f)
    assert F.shape == (300, 192)
    x = ((p - lo) * inv).astype(np.float32).astype(np.float64)
    for a in range(3):
        for l in (0, 5, 17, 31):
            t = f[l].astype(np.float64) * x[:, a]
            col = 2 * (a * 32 + l)
            # FP32 product f*x and fractional part: angle error <= 2 pi (|t| + 1) 2^-23
            tol = 2 * np.pi * (np.abs(t) + 1) * 2.0 ** -22
            assert np.all(np.abs(F[:, col] - np.sin(2 * np.pi * t)) <= tol)
            assert np.all(np.abs(F[:, col + 1] - np.cos(2 * np.pi * t)) <= tol)
    Fb = O.ff_features(p, lo, inv, f, bf16=True)
    np.testing.assert_array_equal(Fb, O.bf16_round(F))


def _torch_mlp(params, dims):
    d0, d1, d2 = dims
    P = torch.as_tensor(params)
    o = 0
    W1 = P[o:o + d0 * d1].view(d0, d1); o += d0 * d1
    b1 = P[o:o + d1]; o += d1
    W2 = P[o:o + d1 * d2].view(d1, d2); o += d1 * d2
    b2 = P[o:o + d2]; o += d2
    W3 = P[o:o + d2 * 4].view(d2, 4); o += d2 * 4
    b3 = P[o:o + 4]
    return W1, b1, W2, b2, W3, b3


def _init(O, dims, seed):
    rng = np.random.default_rng(seed)
    n = O.mlp_nparams(*dims)
    return rng.normal(0, 0.3, n)


def test_mlp_forward_matches_torch(O):
    dims = (24, 16, 12)
    P = _init(O, dims, 11)
    X = np.random.default_rng(12).normal(0, 1, (50, 24))
    Y = O.mlp_forward(P, X, dims)
    W1, b1, W2, b2, W3, b3 = _torch_mlp(P, dims)
    x = torch.as_tensor(X)
    h1 = torch.nn.functional.silu(x @ W1 + b1)
    h2 = torch.nn.functional.silu(h1 @ W2 + b2)
    ref = (h2 @ W3 + b3).numpy()
    np.testing.assert_allclose(Y, ref, rtol=1e-12, atol=1e-12)


def test_mlp_bf16_forward_matches_rounded_torch(O):
    dims = (24, 16, 12)
    P = _init(O, dims, 13)
    X = np.random.default_rng(14).normal(0, 1, (40, 24))
    Y = O.mlp_forward(P, X, dims, bf16=True)

    def rb(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    W1, b1, W2, b2, W3, b3 = _torch_mlp(P, dims)
    x = rb(torch.as_tensor(X))
    h1 = rb(torch.nn.functional.silu(x @ rb(W1) + b1))
    h2 = rb(torch.nn.functional.silu(h1 @ rb(W2) + b2))
    ref = (h2 @ rb(W3) + b3).numpy()
    np.testing.assert_allclose(Y, ref, rtol=1e-10, atol=1e-10)


def test_mlp_gradient_autograd_and_fd(O):
    dims = (18, 10, 8)
    P = _init(O, dims, 15)
    rng = np.random.default_rng(16)
    X = rng.normal(0, 1, (30, 18))
    T = rng.normal(0, 1, (30, 4))
    L, G = O.mlp_loss_grad(P, X, T, dims)
    Pt = torch.tensor(P, requires_grad=True)
    W1, b1, W2, b2, W3, b3 = _torch_mlp(Pt, dims)
    x = torch.as_tensor(X)
    y = torch.nn.functional.silu(torch.nn.functional.silu(x @ W1 + b1) @ W2 + b2) @ W3 + b3
    loss = ((y - torch.as_tensor(T)) ** 2).sum(dim=1).mean()
    loss.backward()
    np.testing.assert_allclose(L, loss.item(), rtol=1e-12)
    np.testing.assert_allclose(G, Pt.grad.numpy(), rtol=1e-9, atol=1e-12)
    h = 1e-6
    for k in rng.choice(len(P), 25, replace=False):
        Pp = P.copy(); Pp[k] += h
        Pm = P.copy(); Pm[k] -= h
        fd = (O.mlp_loss_grad(Pp, X, T, dims)[0] - O.mlp_loss_grad(Pm, X, T, dims)[0]) / (2 * h)
        assert abs(fd - G[k]) <= 1e-6 * (1 + abs(G[k])), k


def test_adam_first_step_closed_form(O):
    rng = np.random.default_rng(17)
    P = rng.normal(0, 1, 100)
    g = rng.normal(0, 1, 100)
    P1, m1, v1 = O.adam(P, g, np.zeros(100), np.zeros(100), 1, lr=1e-2)
    np.testing.assert_allclose(P1, P - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)


def test_adam_matches_torch(O):
    rng = np.random.default_rng(18)
    P = rng.normal(0, 1, 64)
    pt = torch.nn.Parameter(torch.tensor(P))
    opt = torch.optim.Adam([pt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(64); v = np.zeros(64)
    for t in range(1, 8):
        g = rng.normal(0, 1, 64)
        pt.grad = torch.tensor(g)
        opt.step()
        P, m, v = O.adam(P, g, m, v, t, lr=3e-3)
    np.testing.assert_allclose(P, pt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_mlp_bf16_gradient_close_to_exact(O):
    """The BF16-emulating gradient rounds operands to 8 significant bits:
    against the exact FP64 gradient its relative error stays at the level of
    a few bfloat16 ulps (2^-8), with the loss in the forward's tolerance."""
    dims = (192, 128, 128)
    rng = np.random.default_rng(21)
    n = O.mlp_nparams(*dims)
    P = np.zeros(n)
    o = 0
    for fi, fo in ((192, 128), (128, 128), (128, 4)):
        P[o:o + fi * fo] = rng.uniform(-1, 1, fi * fo) / np.sqrt(fi); o += fi * fo
        P[o:o + fo] = rng.uniform(-0.1, 0.1, fo); o += fo
    X = np.sin(rng.uniform(0, 6.3, (64, 192)))
    T = rng.normal(0, 0.3, (64, 4))
    L0, G0 = O.mlp_loss_grad(P, X, T, dims)
    L1, G1 = O.mlp_loss_grad(P, X, T, dims, bf16=True)
    assert abs(L1 - L0) <= 2e-2 * L0
    rel = np.linalg.norm(G1 - G0) / np.linalg.norm(G0)
    assert 1e-5 < rel < 2e-2, rel   # rounded, but only by bfloat16 rounding


def _pose_exp(T8, xi):
    from _pinutil import M_to_pose8, pose_to_M, se3_exp_ref
    return M_to_pose8(pose_to_M(T8) @ se3_exp_ref(xi))


def test_rank1_scorefield_b_and_H_by_differences(O, room):
    """Residual-field scorer, single-point scans below saturation: 2 b =
    d(-loglik)/d delta under T exp(delta) (central differences), and the
    rank-1 H = b b^T / r^2."""
    m, _ = room
    pts = _near_surface_points(O, m, 400, 23, spread=0.04)
    T = np.array([0.9961947, 0.0, 0.0, 0.08715574, 0.05, -0.03, 0.02, 0.0], np.float32)   # 10 deg yaw
    from _pinutil import pose_to_M
    M = pose_to_M(T)
    # scan points in the sensor frame such that R mu + t lands near the surface
    mus = ((pts.astype(np.float64) - M[:3, 3]) @ M[:3, :3]).astype(np.float32)
    checked = 0
    h = 1e-4
    for k in range(len(mus)):
        mu = mus[k:k + 1]
        out = O.likelihood_rank1(m, mu, T[None], 1, sigma_s=0.05, dmax=1.0, cmax=9.0)
        s = -out["loglik"][0]
        if out["ninl"][0] != 1 or s < 0.05 or s > 8.0:
            continue
        b = out["b"][0]
        fd = np.zeros(6)
        stable = True
        for a in range(6):
            xi = np.zeros(6); xi[a] = h
            lp = O.likelihood_rank1(m, mu, _pose_exp(T, xi)[None], 1, sigma_s=0.05, dmax=1.0, cmax=9.0)
            lm = O.likelihood_rank1(m, mu, _pose_exp(T, -xi)[None], 1, sigma_s=0.05, dmax=1.0, cmax=9.0)
            if lp["ninl"][0] != 1 or lm["ninl"][0] != 1:
                stable = False
                break
            fd[a] = (-lp["loglik"][0] + lm["loglik"][0]) / (2 * h)
        if not stable:
            continue
        # FP32 point rounding bounds the difference quotient's accuracy
        assert np.allclose(fd, 2 * b, rtol=2e-2, atol=2e-2 * np.abs(b).max() + 1e-3), (fd, 2 * b)
        H = np.zeros((6, 6))
        q = 0
        for i in range(6):
            for j in range(i, 6):
                H[i, j] = H[j, i] = out["H21"][0][q]; q += 1
        np.testing.assert_allclose(H, np.outer(b, b) / max(s, 1e-4), rtol=1e-9, atol=1e-12)
        checked += 1
        if checked >= 40:
            break
    assert checked >= 20


def test_rank1_untruncated_beyond_saturation(O, room):
    """An inlier above c_max still contributes H and b (as the plain path's
    untruncated terms), its log-likelihood saturates at c_max, and an
    outlier contributes nothing but -c_max."""
    m, _ = room
    g = m.gauss()
    rng = np.random.default_rng(26)
    sel = rng.integers(0, m.G, 200)
    # 0.4 m along the normal: inside the gate, far above c_max for sigma_s = 0.03
    p = (g["mu"][sel] + 0.4 * g["normal"][sel]).astype(np.float32)
    T = np.array([[1, 0, 0, 0, 0, 0, 0, 0]], np.float32)
    seen = 0
    for i in range(len(p)):
        s, _, inl = O.score_field(m, p[i:i + 1], sigma_s=0.03, dmax=1.0)
        out = O.likelihood_rank1(m, p[i:i + 1], T, 1, sigma_s=0.03, dmax=1.0, cmax=9.0)
        if inl[0] and s[0] > 9.0:
            assert out["loglik"][0] == -9.0 and out["ninl"][0] == 0
            assert np.abs(out["b"][0]).max() > 0 and out["H21"][0][0] + out["H21"][0][15] > 0
            seen += 1
        elif inl[0]:
            np.testing.assert_allclose(out["loglik"][0], -s[0], rtol=1e-12)
        else:
            assert out["loglik"][0] == -9.0 and np.all(out["b"][0] == 0) and np.all(out["H21"][0] == 0)
    assert seen > 20


def test_rank1_network_constant_output_closed_form(O, room):
    """Network scorer with W3 = 0: every point gets the bias b3, so
    loglik = -ns min(r0^2, c_max), b = sum r0 g, H = sum g g^T with
    g = [mu x w; w], w = R^T grad r."""
    m, _ = room
    dims = (192, 128, 128)
    n = O.mlp_nparams(*dims)
    rng = np.random.default_rng(24)
    P = rng.normal(0, 0.2, n)
    P[n - 4 - 512:n - 4] = 0.0                    # W3
    r_scale, g_scale = 20.0, 10.0
    r0, gv = 1.5, np.array([0.3, -1.2, 0.5])
    P[n - 4:] = [r0 / r_scale, *(gv / g_scale)]   # b3
    f = O.ff_freqs(40.0)
    lo = np.array([-12, -12, -2], np.float32); inv = np.full(3, 1 / 24.0, np.float32)
    mu = rng.uniform(-3, 3, (50, 3)).astype(np.float32)
    T = np.array([[0.9238795, 0.0, 0.3826834, 0.0, 1.0, 2.0, 0.5, 0.0]], np.float32)
    out = O.likelihood_rank1(m, mu, T, 2, cmax=9.0, params=P, lo=lo, inv_ext=inv, freqs=f, r_scale=r_scale,
                             g_scale=g_scale)
    from _pinutil import pose_to_M
    R = pose_to_M(T[0])[:3, :3]
    gvec = (P[n - 3:] * g_scale)
    w = R.T @ gvec
    mu64 = mu.astype(np.float64)
    gw = np.concatenate([np.cross(mu64, w), np.tile(w, (50, 1))], axis=1)
    r_eff = P[n - 4] * r_scale
    assert out["ninl"][0] == 50
    np.testing.assert_allclose(out["loglik"][0], -50 * r_eff ** 2, rtol=1e-13)
    np.testing.assert_allclose(out["b"][0], r_eff * gw.sum(0), rtol=1e-12, atol=1e-12)
    H = np.zeros((6, 6)); q = 0
    for i in range(6):
        for j in range(i, 6):
            H[i, j] = H[j, i] = out["H21"][0][q]; q += 1
    np.testing.assert_allclose(H, gw.T @ gw, rtol=1e-12, atol=1e-12)


def test_rank1_network_matches_forward_at_identity(O, room):
    m, _ = room
    dims = (192, 128, 128)
    rng = np.random.default_rng(25)
    P = rng.normal(0, 0.1, O.mlp_nparams(*dims))
    f = O.ff_freqs(40.0)
    lo = np.array([-12, -12, -2], np.float32); inv = np.full(3, 1 / 24.0, np.float32)
    p = rng.uniform(-5, 5, (30, 3)).astype(np.float32)
    Y = O.mlp_forward(P, O.ff_features(p, lo, inv, f, bf16=True), dims, bf16=True)
    T = np.array([[1, 0, 0, 0, 0, 0, 0, 0]], np.float32)
    for k in range(len(p)):
        out = O.likelihood_rank1(m, p[k:k + 1], T, 2, cmax=1e6, params=P, lo=lo, inv_ext=inv, freqs=f,
                                 r_scale=3.0, g_scale=1.0)
        np.testing.assert_allclose(-out["loglik"][0], max(Y[k, 0] * 3.0, 0.0) ** 2, rtol=1e-13, atol=1e-15)
