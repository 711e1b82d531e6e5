"""Pins of the oracle's neighbour search, SVGD, posterior and prediction
(CPU only).

  hash6        single-coordinate special cases reduce to the published
               constants (Teschner et al. primes); XOR combination; negative
               coordinates wrap as two's complement
  LSH cells    floor of zeta (Eq. 10) computed in FP64 with scipy rotations
               (decoupled tangent) or scipy logm (coupled SE(3) tangent), away
               from cell boundaries; equal poses without noise share a code
  bucket sort  numpy stable argsort; bucket bounds
  refresh      one bucket (lsh_bits = 0) and window >= N-1 equals brute-force
               K-nearest by FP64 q_ij; persistence of the old list; set semantics
  SVGD         K = 1 gives phi = psi; two-particle translation-only closed form;
               full neighbour sets against a direct O(N^2) sum with scipy logm;
               the exact kernel gradient against finite differences of k through
               expm/logm, the adjoint transport against M xi^ M^-1; J_r^-1 against
               finite differences of log(exp(xi) exp(e)); with W isotropic,
               transport leaves the approximate gradient term unchanged
               (Ad_exp(d) d = d)
  posterior    sums to 1; uniform fixed point; K = 1 identity; two-node closed
               form of one round; shift invariance; long-double softmax
  prediction   zero covariance gives T dT; sample covariance of the noise
  Gaussian init  zero covariance gives the (normalised) mean; sample mean and
               covariance of log(M^-1 T_i); draws distinct from the prediction's
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from _pinutil import between_ref, pose_to_M, random_pose8, se3_exp_ref, se3_log_ref, M_to_pose8, quat_wxyz_to_R

P = [73856093, 19349663, 83492791, 2654435761, 2246822519, 3266489917]


def test_hash6_special_cases(O):
    assert O.hash6([0] * 6) == 0
    for m in range(6):
        c = [0] * 6; c[m] = 1
        assert O.hash6(c) == P[m]
        c[m] = -1
        assert O.hash6(c) == (2 ** 32 - P[m]) % 2 ** 32
        c[m] = 3
        assert O.hash6(c) == (3 * P[m]) % 2 ** 32
    assert O.hash6([1, 1, 0, 0, 0, 0]) == P[0] ^ P[1]
    assert O.hash6([2, 0, 0, 0, 0, -5]) == ((2 * P[0]) % 2 ** 32) ^ ((-5 * P[5]) % 2 ** 32)


def test_lsh_cells_against_fp64(O):
    rng = np.random.default_rng(0)
    n = 3000
    poses = np.stack([random_pose8(rng, tscale=20) for _ in range(n)])
    TL = O.lsh_frame(7, 2, 3, np.array([-30, -30, -5], np.float32), np.array([30, 30, 5], np.float32))
    alpha, sr, st, sl, seed = 1.3, 5.0, 2.5, 0.3, 77
    codes, cells = O.lsh_codes(poses, TL, alpha, sr, st, sl, 20, seed, 2, 3, want_cells=True)
    RL = quat_wxyz_to_R(TL[:4])
    checked = 0
    for i in range(n):
        Ri = quat_wxyz_to_R(poses[i, :4])
        om = Rotation.from_matrix(RL.T @ Ri).as_rotvec()
        u = RL.T @ (poses[i, 4:7].astype(np.float64) - TL[4:7].astype(np.float64))
        z = O.gauss6(seed, i, 2, 3, 2).astype(np.float64)
        zeta = np.concatenate([alpha * sr * om, alpha * st * u]) + sl * z
        frac = zeta - np.floor(zeta)
        if np.all((frac > 1e-4) & (frac < 1 - 1e-4)):
            assert np.array_equal(cells[i], np.floor(zeta).astype(np.int32)), (i, cells[i], zeta)
            checked += 1
        assert codes[i] == (O.hash6(cells[i]) & ((1 << 20) - 1))
    assert checked > 0.99 * n


def test_lsh_coupled_cells_against_fp64(O):
    rng = np.random.default_rng(11)
    n = 2000
    poses = np.stack([random_pose8(rng, tscale=8) for _ in range(n)])
    TL = O.lsh_frame(9, 1, 4, np.array([-10, -10, -2], np.float32), np.array([10, 10, 2], np.float32))
    alpha, sr, st, sl, seed = 0.8, 5.0, 2.5, 0.3, 78
    codes, cells = O.lsh_codes(poses, TL, alpha, sr, st, sl, 20, seed, 1, 4, want_cells=True, tangent=1)
    _, cells_dec = O.lsh_codes(poses, TL, alpha, sr, st, sl, 20, seed, 1, 4, want_cells=True, tangent=0)
    # the rotation part of the tangent is the same program in both forms
    assert np.array_equal(cells[:, :3], cells_dec[:, :3])
    checked = 0
    for i in range(n):
        d = between_ref(TL, poses[i])          # log(T_LSH^-1 T_i) by scipy logm
        if np.linalg.norm(d[:3]) > 3.0:        # logm branch near pi
            continue
        z = O.gauss6(seed, i, 1, 4, 2).astype(np.float64)
        zeta = alpha * np.concatenate([sr * d[:3], st * d[3:]]) + sl * z
        frac = zeta - np.floor(zeta)
        if np.all((frac > 1e-4) & (frac < 1 - 1e-4)):
            assert np.array_equal(cells[i], np.floor(zeta).astype(np.int32)), (i, cells[i], zeta)
            checked += 1
        assert codes[i] == (O.hash6(cells[i]) & ((1 << 20) - 1))
    assert checked > 0.9 * n
    # the coupled translation cells differ from the decoupled ones once rotations differ
    assert not np.array_equal(cells[:, 3:], cells_dec[:, 3:])


def test_lsh_equal_poses_share_code(O):
    T = np.tile(random_pose8(np.random.default_rng(3)), (100, 1))
    TL = O.lsh_frame(1, 0, 0, np.zeros(3, np.float32), np.ones(3, np.float32))
    codes = O.lsh_codes(T, TL, 1.0, 5.0, 2.5, 0.0, 16, 1, 0, 0)
    assert len(np.unique(codes)) == 1
    codes = O.lsh_codes(T, TL, 1.0, 5.0, 2.5, 0.0, 16, 1, 0, 0, tangent=1)
    assert len(np.unique(codes)) == 1


def test_bucket_sort_stable(O):
    rng = np.random.default_rng(4)
    for bits in (1, 4, 16):
        codes = rng.integers(0, 2 ** bits, size=5000).astype(np.uint32)
        s, h, e = O.bucket_sort(codes)
        ref = np.argsort(codes, kind="stable")
        assert np.array_equal(s, ref)
        sc = codes[s]
        for k in range(0, 5000, 37):
            assert np.all(sc[h[k]:e[k]] == sc[k])
            assert h[k] == 0 or sc[h[k] - 1] != sc[k]
            assert e[k] == 5000 or sc[e[k]] != sc[k]


def _q64(Ti, Tj, sr=5.0, st=2.5):
    d = between_ref(Ti, Tj)
    return sr * np.sum(d[:3] ** 2) + st * np.sum(d[3:] ** 2)


def test_refresh_single_bucket_is_bruteforce_knn(O):
    rng = np.random.default_rng(5)
    n, K = 120, 8
    poses = np.stack([random_pose8(rng, tscale=2.0, rot=1.0) for _ in range(n)])
    codes = np.zeros(n, np.uint32)
    s, _, _ = O.bucket_sort(codes)
    nbr, q, cnt = O.refresh(poses, s, codes, K, n - 1, 5.0, 2.5, None)
    Q = np.array([[_q64(poses[i], poses[j]) for j in range(n)] for i in range(n)])
    for i in range(n):
        Q[i, i] = np.inf
        order = np.argsort(Q[i], kind="stable")[:K - 1]
        assert nbr[i, 0] == i and cnt[i] == K
        got = nbr[i, 1:]
        if not np.array_equal(got, order):
            # only allowed when FP64 values are within FP32 resolution
            assert np.allclose(np.sort(Q[i, got]), Q[i, order], rtol=1e-4)
        assert np.all(np.diff(q[i, 1:]) >= 0)


def test_refresh_persistence_and_sets(O):
    rng = np.random.default_rng(6)
    n, K = 200, 6
    poses = np.stack([random_pose8(rng, tscale=1.0, rot=0.5) for _ in range(n)])
    codes = np.arange(n, dtype=np.uint32)           # every particle alone in its bucket
    s, _, _ = O.bucket_sort(codes)
    old = np.full((n, K), -1, np.int32)
    for i in range(n):
        cand = rng.choice(n, 12, replace=False)
        cand = cand[cand != i][:K - 1]
        old[i, 0] = i; old[i, 1:1 + len(cand)] = cand
    nbr, q, cnt = O.refresh(poses, s, codes, K, 32, 5.0, 2.5, old)
    for i in range(n):
        members = [j for j in old[i] if j >= 0 and j != i]
        exp = sorted(members, key=lambda j: (_q64(poses[i], poses[j]), j))[:K - 1]
        got = list(nbr[i, 1:cnt[i]])
        assert nbr[i, 0] == i and cnt[i] == 1 + len(exp)
        assert sorted(got) == sorted(exp)
        assert len(set(nbr[i, :cnt[i]])) == cnt[i]
        assert np.all(nbr[i, cnt[i]:] == -1)


def test_refresh_window_cyclic(O):
    # two buckets; window 3 < bucket size: members at the next 3 sorted positions, cyclic
    rng = np.random.default_rng(7)
    n, K = 10, 10
    poses = np.stack([random_pose8(rng) for _ in range(n)])
    codes = np.array([1, 0, 1, 1, 0, 1, 1, 0, 1, 1], np.uint32)
    s, _, _ = O.bucket_sort(codes)
    nbr, q, cnt = O.refresh(poses, s, codes, K, 3, 5.0, 2.5, None)
    b1 = [0, 2, 3, 5, 6, 8, 9]
    for p, i in enumerate(b1):
        exp = {b1[(p + d) % len(b1)] for d in (1, 2, 3)}
        assert set(nbr[i, 1:cnt[i]]) == exp


def test_svgd_single_neighbour_is_gauss_newton(O):
    rng = np.random.default_rng(8)
    n = 50
    poses = np.stack([random_pose8(rng) for _ in range(n)])
    psi = rng.normal(scale=0.3, size=(n, 6))
    nbr = np.arange(n, dtype=np.int32)[:, None]
    phi, out = O.svgd(poses, psi, nbr, 5.0, 2.5)
    assert np.allclose(phi, psi, atol=1e-12)
    for i in range(n):
        M = pose_to_M(poses[i]) @ se3_exp_ref(psi[i])
        assert np.allclose(pose_to_M(out[i]), M, atol=1e-9)


def test_svgd_two_particle_closed_form(O):
    t1, t2 = np.array([0.1, 0.2, -0.3]), np.array([0.5, -0.1, 0.0])
    poses = np.zeros((2, 8), np.float32)
    poses[:, 0] = 1; poses[0, 4:7] = t1; poses[1, 4:7] = t2
    psi = np.array([[0, 0, 0, 0.05, 0.0, -0.02], [0, 0, 0, -0.01, 0.03, 0.0]])
    nbr = np.array([[0, 1], [1, 0]], np.int32)
    phi, _ = O.svgd(poses, psi, nbr, 5.0, 2.5)
    t1f, t2f = poses[0, 4:7].astype(np.float64), poses[1, 4:7].astype(np.float64)
    k = math.exp(-2.5 * np.sum((t2f - t1f) ** 2))
    exp1 = (psi[0, 3:] + k * psi[1, 3:] + 2 * k * 2.5 * (t1f - t2f)) / (1 + k)
    assert np.allclose(phi[0, :3], 0, atol=1e-15)
    assert np.allclose(phi[0, 3:], exp1, atol=1e-12)


def test_svgd_full_set_direct_sum(O):
    rng = np.random.default_rng(9)
    n = 30
    poses = np.stack([random_pose8(rng, tscale=0.5, rot=0.4) for _ in range(n)])
    psi = rng.normal(scale=0.1, size=(n, 6))
    nbr = np.array([[i] + [j for j in range(n) if j != i] for i in range(n)], np.int32)
    phi, _ = O.svgd(poses, psi, nbr, 5.0, 2.5)
    W = np.array([5.0] * 3 + [2.5] * 3)
    for i in range(n):
        num = np.zeros(6); den = 0.0
        for j in range(n):
            d = between_ref(poses[i], poses[j])
            k = math.exp(-np.sum(W * d * d))
            num += k * psi[j] - 2 * k * W * d
            den += k
        assert np.allclose(phi[i], num / den, atol=2e-6)


def test_posterior_invariants(O):
    rng = np.random.default_rng(10)
    n, K = 400, 6
    ll = rng.normal(scale=5, size=n)
    prior = np.full(n, 1.0 / n)
    nbr = np.stack([np.concatenate([[i], rng.choice(n, K - 1, replace=False)]) for i in range(n)]).astype(np.int32)
    kval = np.concatenate([np.ones((n, 1)), rng.uniform(0.1, 1, (n, K - 1))], 1)
    r = O.posterior(prior, ll, nbr, kval, rounds=10)
    assert abs(r["post"].sum() - 1) < 1e-12
    # long-double softmax
    l = ll.astype(np.longdouble)
    e = np.exp(l - l.max())
    assert np.allclose(r["p0"], (e / e.sum()).astype(np.float64), rtol=1e-12, atol=1e-300)
    # shift invariance
    r2 = O.posterior(prior, ll + 1234.5, nbr, kval, rounds=10)
    assert np.allclose(r2["post"], r["post"], rtol=1e-9)
    assert r["map_index"] == int(np.argmax(r["post"]))
    assert abs(r["n_eff"] - 1 / np.sum(r["post"] ** 2)) < 1e-9 * r["n_eff"]
    # uniform is a fixed point
    ru = O.posterior(prior, np.zeros(n), nbr, kval, rounds=10)
    assert np.allclose(ru["post"], 1.0 / n, rtol=1e-12)
    # K = 1: no smoothing
    r1 = O.posterior(prior, ll, np.arange(n, dtype=np.int32)[:, None], np.ones((n, 1)), rounds=10)
    assert np.allclose(r1["post"], r1["p0"], rtol=1e-12)


def test_posterior_two_nodes_one_round(O):
    k = 0.37
    ll = np.array([0.0, math.log(3.0)])
    nbr = np.array([[0, 1], [1, 0]], np.int32)
    kval = np.array([[1, k], [1, k]])
    r = O.posterior(np.array([0.5, 0.5]), ll, nbr, kval, rounds=1)
    p = np.array([0.25, 0.75])
    exp = np.array([(p[0] + k * p[1]) / (1 + k), (p[1] + k * p[0]) / (1 + k)])
    assert np.allclose(r["post"], exp / exp.sum(), rtol=1e-14)
    # prior enters multiplicatively; the floor keeps log(0) finite
    r0 = O.posterior(np.array([0.0, 1.0]), np.zeros(2), nbr, kval, rounds=0, prior_floor=1e-30)
    assert r0["post"][0] == pytest.approx(1e-30, rel=1e-6)


def test_predict_no_noise_and_noise_covariance(O):
    rng = np.random.default_rng(11)
    n = 20000
    poses = np.stack([random_pose8(rng) for _ in range(50)])
    dT = np.array([0.9, 0.1, -0.3, 0.2, 0.5, -0.2, 0.1], np.float32)
    dT[:4] /= np.linalg.norm(dT[:4])
    out = O.predict(poses, dT, None, 1, 3)
    D = pose_to_M(dT)
    for i in range(len(poses)):
        assert np.allclose(pose_to_M(out[i]), pose_to_M(poses[i]) @ D, atol=1e-6)
    A = rng.normal(size=(6, 6)) * 0.05
    cov = (A @ A.T).astype(np.float32)
    base = np.tile(poses[0], (n, 1))
    out = O.predict(base, dT, cov, 9, 4)
    TD = pose_to_M(poses[0]) @ D
    deltas = np.stack([se3_log_ref(np.linalg.inv(TD) @ pose_to_M(out[i])) for i in range(0, n, 4)])
    C = np.cov(deltas.T)
    assert np.allclose(C, cov, atol=0.1 * np.abs(cov).max())


def test_init_gauss_covariance_and_zero(O):
    rng = np.random.default_rng(15)
    mean = random_pose8(rng)[:7].copy()
    mean[:4] *= 1.7                        # not unit: normalised on input
    Z = O.init_gauss(3, 10, mean, np.zeros(36, np.float32))
    M0 = pose_to_M(np.r_[mean[:4] / np.linalg.norm(mean[:4].astype(np.float64)), mean[4:]])
    for i in range(10):
        assert np.allclose(pose_to_M(Z[i]), M0, atol=1e-6)
    A = rng.normal(size=(6, 6)) * 0.08
    cov = (A @ A.T).astype(np.float32)
    n = 20000
    out = O.init_gauss(5, n, mean, cov)
    Minv = np.linalg.inv(M0)
    deltas = np.stack([se3_log_ref(Minv @ pose_to_M(out[i])) for i in range(0, n, 4)])
    assert np.abs(deltas.mean(0)).max() < 0.05 * np.sqrt(np.diag(cov)).max()
    assert np.allclose(np.cov(deltas.T), cov, atol=0.1 * np.abs(cov).max())
    # its draws are not the prediction's (another purpose of the generator)
    mean8 = np.r_[mean[:4] / np.linalg.norm(mean[:4]), mean[4:], 0].astype(np.float32)
    pred = O.predict(np.tile(mean8, (4, 1)), np.array([1, 0, 0, 0, 0, 0, 0], np.float32), cov, 5, 0)
    assert not np.allclose(pred[:4], out[:4])


def _vee(M):
    return np.array([M[2, 1], M[0, 2], M[1, 0], M[0, 3], M[1, 3], M[2, 3]])


def test_jr_inv_against_finite_differences(O):
    rng = np.random.default_rng(12)
    h = 1e-5
    for trial in range(12):
        xi = np.concatenate([rng.normal(size=3) * (0.3 + 0.2 * trial), rng.normal(size=3) * 2.0])
        if np.linalg.norm(xi[:3]) > 2.8:
            xi[:3] *= 2.8 / np.linalg.norm(xi[:3])
        J = O.se3_jr_inv(xi)
        E = se3_exp_ref(xi)
        Jfd = np.zeros((6, 6))
        for c in range(6):
            e = np.zeros(6); e[c] = h
            Jfd[:, c] = (se3_log_ref(E @ se3_exp_ref(e)) - se3_log_ref(E @ se3_exp_ref(-e))) / (2 * h)
        assert np.abs(J - Jfd).max() < 1e-6 * (1 + np.abs(J).max()), (trial, np.abs(J - Jfd).max())
    # small argument: J_r^-1 = I + ad/2 + O(|xi|^2)
    xi = np.array([1e-4, -2e-4, 1.5e-4, 3e-4, 1e-4, -2e-4])
    ad = np.zeros((6, 6))
    from _pinutil import hat
    ad[:3, :3] = hat(xi[:3]); ad[3:, :3] = hat(xi[3:]); ad[3:, 3:] = hat(xi[:3])
    assert np.abs(O.se3_jr_inv(xi) - (np.eye(6) + 0.5 * ad)).max() < 1e-7


def _svgd_direct(poses, psi, sr, st, grad_exact, transport):
    """phi of every particle over the full set, each term from scipy expm/logm:
    the kernel gradient by central differences of k(T_i, T_j exp(e)), the
    transport as vee(M_ij (v^) M_ij^-1)"""
    from _pinutil import twist_M
    n = len(poses)
    W = np.array([sr] * 3 + [st] * 3)
    h = 1e-5
    Ms = [pose_to_M(p) for p in poses]
    phi = np.zeros((n, 6))
    for i in range(n):
        num = np.zeros(6); den = 0.0
        Mi_inv = np.linalg.inv(Ms[i])
        for j in range(n):
            Mij = Mi_inv @ Ms[j]
            d = se3_log_ref(Mij)
            k = math.exp(-np.sum(W * d * d))
            if grad_exact:
                g = np.zeros(6)
                for c in range(6):
                    e = np.zeros(6); e[c] = h
                    dp = se3_log_ref(Mij @ se3_exp_ref(e)); dm = se3_log_ref(Mij @ se3_exp_ref(-e))
                    g[c] = (math.exp(-np.sum(W * dp * dp)) - math.exp(-np.sum(W * dm * dm))) / (2 * h)
            else:
                g = -2 * k * W * d
            v = k * psi[j] + g
            if transport:
                v = _vee(Mij @ twist_M(v) @ np.linalg.inv(Mij))
            num += v
            den += k
        phi[i] = num / den
    return phi


@pytest.mark.parametrize("grad_exact,transport", [(True, False), (False, True), (True, True)])
def test_svgd_variants_direct_sum(O, grad_exact, transport):
    rng = np.random.default_rng(13)
    n = 16
    poses = np.stack([random_pose8(rng, tscale=0.4, rot=0.8) for _ in range(n)])
    psi = rng.normal(scale=0.1, size=(n, 6))
    nbr = np.array([[i] + [j for j in range(n) if j != i] for i in range(n)], np.int32)
    phi, _ = O.svgd(poses, psi, nbr, 5.0, 2.5, grad_exact=grad_exact, transport=transport)
    ref = _svgd_direct(poses, psi, 5.0, 2.5, grad_exact, transport)
    assert np.abs(phi - ref).max() < 2e-6, np.abs(phi - ref).max()
    # the variant changes the result at this spread
    phi0, _ = O.svgd(poses, psi, nbr, 5.0, 2.5)
    assert np.abs(phi - phi0).max() > 1e-3


def test_svgd_transport_keeps_gradient_term(O):
    # Ad_{exp(d)} d = d: with psi = 0, the approximate gradient and an isotropic
    # W (sigma_r = sigma_t), transport is the identity
    rng = np.random.default_rng(14)
    n = 40
    poses = np.stack([random_pose8(rng, tscale=1.0, rot=1.0) for _ in range(n)])
    nbr = np.array([[i] + list(rng.choice([j for j in range(n) if j != i], 7, replace=False)) for i in range(n)],
                   np.int32)
    psi = np.zeros((n, 6))
    a, _ = O.svgd(poses, psi, nbr, 3.0, 3.0)
    b, _ = O.svgd(poses, psi, nbr, 3.0, 3.0, transport=True)
    assert np.abs(a - b).max() < 1e-12
    # with W anisotropic it is not (the translation row mixes in t x omega)
    a, _ = O.svgd(poses, psi, nbr, 5.0, 2.5)
    b, _ = O.svgd(poses, psi, nbr, 5.0, 2.5, transport=True)
    assert np.abs(a - b).max() > 1e-3
