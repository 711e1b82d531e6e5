"""Pins of the oracle's map side (CPU only).

  eig3            numpy.linalg.eigh (eigenvalues, eigenvector directions)
  map Gaussians   numpy mean / (1/n) covariance / eigh on tiny voxel sets;
                  GICP normalisation I - (1-eps) n n^T: eigenvalues (eps,1,1),
                  planar patch -> plane normal; min_points filter; id order
  NNF             brute force over all occupied voxels (Chebyshev radius R,
                  smallest integer squared distance, ties to the smaller id)
  scan covariances  numpy k-NN by squared distance (ties to lower index),
                  numpy covariance of the point and its neighbours
  per-point map   neighbour lists against scipy cKDTree (search block covering
                  the map) and numpy brute force within the Chebyshev voxel
                  block; covariances against numpy; a plane's normal;
                  the field against a KD-tree nearest kept point of every
                  cell centre within R r; ids in (vz, vy, vx, index) order
"""
import numpy as np
import pytest


def test_eig3_against_numpy(O):
    rng = np.random.default_rng(0)
    for _ in range(300):
        A = rng.normal(size=(3, 3)) * rng.choice([1e-3, 1, 1e3])
        S = A @ A.T
        if rng.random() < 0.2:   # repeated eigenvalue
            U, _, _ = np.linalg.svd(A)
            S = U @ np.diag([1.0, 1.0, 3.0]) @ U.T
        w, V = O.eig3(S)
        wr, Vr = np.linalg.eigh(S)
        assert np.allclose(w, wr, rtol=1e-12, atol=1e-12 * np.abs(wr).max())
        assert np.allclose(V @ np.diag(w) @ V.T, S, atol=1e-11 * np.abs(wr).max())
        assert np.allclose(V.T @ V, np.eye(3), atol=1e-12)
        if wr[1] - wr[0] > 1e-6 * wr[2]:
            assert abs(abs(V[:, 0] @ Vr[:, 0]) - 1) < 1e-9


def _voxel_sets(rng, r=0.5):
    vox = rng.integers(-4, 5, size=(12, 3))
    vox = np.unique(vox, axis=0)
    pts, owner = [], []
    for k, v in enumerate(vox):
        n = int(rng.integers(2, 30))
        p = (v + rng.uniform(0.02, 0.98, size=(n, 3))) * r
        pts.append(p); owner += [k] * n
    P = np.concatenate(pts).astype(np.float32)
    perm = rng.permutation(len(P))
    return P[perm], vox, np.array(owner)[perm]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_map_gaussians_against_numpy(O, seed):
    rng = np.random.default_rng(seed)
    r, eps, minp = 0.5, 1e-3, 5
    P, vox, owner = _voxel_sets(rng, r)
    m = O.Map(P, r, nnf_radius=1, min_points=minp, cov_eps=eps)
    g = m.gauss()
    # expected kept voxels, ascending (z, y, x)
    keep = []
    for k, v in enumerate(vox):
        pts = P[owner == k].astype(np.float64)
        if len(pts) >= minp:
            keep.append((v[2], v[1], v[0], k))
    keep.sort()
    assert m.G == len(keep)
    for gid, (_, _, _, k) in enumerate(keep):
        pts = P[owner == k].astype(np.float64)
        assert np.array_equal(g["vox"][gid], vox[k])
        assert g["npts"][gid] == len(pts)
        mu = pts.mean(axis=0)
        assert np.allclose(g["mu64"][gid], mu, atol=1e-13)
        S = np.cov(pts.T, bias=True)
        w, V = np.linalg.eigh(S)
        n = V[:, 0]
        ref = np.eye(3) - (1 - eps) * np.outer(n, n)
        got = g["cov64"][gid]
        Sg = np.array([[got[0], got[1], got[2]], [got[1], got[3], got[4]], [got[2], got[4], got[5]]])
        if w[1] - w[0] > 1e-9:
            assert np.allclose(Sg, ref, atol=1e-9)
        assert np.allclose(np.linalg.eigvalsh(Sg), [eps, 1, 1], atol=1e-12)


def test_planar_voxel_normal(O):
    rng = np.random.default_rng(5)
    nrm = np.array([0.3, -0.4, 0.866]); nrm /= np.linalg.norm(nrm)
    a = np.cross(nrm, [1, 0, 0]); a /= np.linalg.norm(a); b = np.cross(nrm, a)
    c = np.array([0.25, 0.25, 0.25])
    P = c + 0.1 * rng.uniform(-1, 1, (200, 1)) * a + 0.1 * rng.uniform(-1, 1, (200, 1)) * b
    m = O.Map(P.astype(np.float32), 0.5, nnf_radius=0, min_points=5, cov_eps=1e-3)
    g = m.gauss()
    assert m.G == 1
    s = g["cov64"][0]
    Sg = np.array([[s[0], s[1], s[2]], [s[1], s[3], s[4]], [s[2], s[4], s[5]]])
    # the normal is the eigenvector of eigenvalue eps (up to the FP32 rounding of the points)
    assert abs(nrm @ Sg @ nrm - 1e-3) < 1e-5


@pytest.mark.parametrize("R", [0, 1, 2, 3])
def test_nnf_bruteforce(O, R):
    rng = np.random.default_rng(10 + R)
    r = 0.25
    occ = np.unique(rng.integers(-5, 6, size=(25, 3)), axis=0)
    pts = np.repeat((occ + 0.5) * r, 6, axis=0) + rng.uniform(-0.05, 0.05, (6 * len(occ), 3)) * r
    m = O.Map(pts.astype(np.float32), r, nnf_radius=R, min_points=5)
    g = m.gauss()
    assert m.G == len(occ)
    gv = g["vox"]
    org, dim = m.grid()
    assert np.array_equal(org, gv.min(axis=0) - R) and np.array_equal(dim, gv.max(axis=0) - gv.min(axis=0) + 1 + 2 * R)
    # every voxel of the grid plus a margin outside it
    rngv = [np.arange(org[a] - 2, org[a] + dim[a] + 2) for a in range(3)]
    V = np.stack(np.meshgrid(*rngv, indexing="ij"), -1).reshape(-1, 3)
    q = ((V + 0.5) * r).astype(np.float32)
    got = m.lookup(q)
    d = V[:, None, :] - gv[None, :, :]
    cheb = np.abs(d).max(-1)
    d2 = (d * d).sum(-1)
    key = np.where(cheb <= R, d2 * 100000 + np.arange(len(gv))[None, :], np.iinfo(np.int64).max)
    best = key.argmin(1)
    exp = np.where(key.min(1) == np.iinfo(np.int64).max, -1, best)
    assert np.array_equal(got, exp)
    assert m.nb == int((exp >= 0).sum())


def test_map_empty_and_min_points(O):
    m = O.Map(np.zeros((3, 3), np.float32), 0.5, min_points=5)
    assert m.G == 0 and m.nb == 0
    assert np.all(m.lookup(np.zeros((4, 3), np.float32)) == -1)


def test_scan_cov_against_numpy(O):
    rng = np.random.default_rng(7)
    P = rng.normal(size=(300, 3)).astype(np.float32)
    k = 10
    knn, cov, cov64 = O.scan_cov(P, k=k, eps=1e-3)
    P64 = P.astype(np.float64)
    for i in range(len(P)):
        d2 = ((P64 - P64[i]) ** 2).sum(1)
        d2[i] = np.inf
        order = np.lexsort((np.arange(len(P)), d2))[:k]
        assert np.array_equal(np.sort(knn[i]), np.sort(order)) or np.allclose(np.sort(d2[knn[i]]), np.sort(d2[order]), rtol=1e-6)
        nb = P64[np.concatenate([[i], knn[i]])]
        S = np.cov(nb.T, bias=True)
        w, V = np.linalg.eigh(S)
        n = V[:, 0]
        ref = np.eye(3) - (1 - 1e-3) * np.outer(n, n)
        c = cov64[i]
        Sg = np.array([[c[0], c[1], c[2]], [c[1], c[3], c[4]], [c[2], c[4], c[5]]])
        assert np.allclose(Sg, ref, atol=1e-9)


def test_scan_cov_planar_and_tiny(O):
    rng = np.random.default_rng(8)
    xy = rng.uniform(-1, 1, (50, 2))
    P = np.concatenate([xy, np.full((50, 1), 0.7)], 1).astype(np.float32)
    _, _, cov64 = O.scan_cov(P, k=10)
    assert np.allclose(cov64[:, 5], 1e-3, atol=1e-12)      # zz = eps
    assert np.allclose(cov64[:, [0, 3]], 1.0, atol=1e-12)
    _, cov, _ = O.scan_cov(P[:4], k=10)                   # fewer than 5 points -> identity
    assert np.allclose(cov, [1, 0, 0, 1, 0, 1])


def _surface_points(rng, n, r):
    """points on two perpendicular planes and a sphere cap, spacing ~ r / 3"""
    a = rng.uniform(0, 3, size=(n // 3, 2))
    p1 = np.c_[a, np.zeros(n // 3)]
    b = rng.uniform(0, 3, size=(n // 3, 2))
    p2 = np.c_[b[:, 0], np.zeros(n // 3) + 0.01, b[:, 1]]
    m = n - 2 * (n // 3)
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    p3 = np.array([1.5, 1.5, 1.5]) + 0.8 * u
    return np.concatenate([p1, p2, p3]).astype(np.float32) + rng.normal(scale=0.002, size=(n, 3)).astype(np.float32)


def test_point_map_knn_against_kdtree(O):
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(20)
    P = _surface_points(rng, 3000, 0.2)
    k = 10
    m = O.Map(P, 0.2, nnf_radius=2, min_points=5, per_point=True, point_k=k, point_search=1000, want_knn=True)
    d, j = cKDTree(P.astype(np.float64)).query(P.astype(np.float64), k=k + 2)
    checked = 0
    for i in range(len(P)):
        # the query returns the point itself first (distance 0)
        nb = [x for x in j[i] if x != i][:k]
        dd = [dx for dx, x in zip(d[i], j[i]) if x != i]
        if dd[k] - dd[k - 1] > 1e-5 and np.all(np.diff(dd[:k]) > 1e-5):
            assert list(m.knn[i]) == nb, i
            checked += 1
    assert checked > 0.9 * len(P)


def test_point_map_voxel_block_bruteforce(O):
    rng = np.random.default_rng(21)
    P = _surface_points(rng, 1500, 0.25)
    r, k, S = 0.25, 8, 1
    m = O.Map(P, r, nnf_radius=2, min_points=5, per_point=True, point_k=k, point_search=S, want_knn=True)
    P64 = P.astype(np.float64)
    V = np.floor(P * np.float32(1.0 / r)).astype(np.int64)
    for i in range(0, len(P), 7):
        inblk = np.all(np.abs(V - V[i]) <= S, axis=1)
        inblk[i] = False
        cand = np.nonzero(inblk)[0]
        dd = np.sum((P64[cand] - P64[i]) ** 2, axis=1)
        order = cand[np.lexsort((cand, dd))]
        want = list(order[:k]) + [-1] * max(0, k - len(order))
        ds = np.sort(dd)
        if len(ds) <= k or ds[k] - ds[k - 1] > 1e-9:
            assert list(m.knn[i]) == want, i


def test_point_map_gaussians_against_numpy(O):
    rng = np.random.default_rng(22)
    P = _surface_points(rng, 2000, 0.2)
    m = O.Map(P, 0.2, nnf_radius=2, min_points=6, per_point=True, point_k=9, point_search=2, want_knn=True)
    g = m.gauss()
    V = np.floor(P * np.float32(1.0 / 0.2)).astype(np.int64)
    kept = [i for i in range(len(P)) if np.sum(m.knn[i] >= 0) + 1 >= 6]
    order = sorted(kept, key=lambda i: (V[i, 2], V[i, 1], V[i, 0], i))
    assert m.G == len(order)
    assert np.array_equal(g["mu"], P[order])
    assert np.array_equal(g["vox"], V[order].astype(np.int32))
    for gi in range(0, m.G, 11):
        i = order[gi]
        nb = m.knn[i][m.knn[i] >= 0]
        X = np.concatenate([P[i:i + 1], P[nb]]).astype(np.float64)
        C = np.cov(X.T, bias=True)
        w, U = np.linalg.eigh(C)
        n = U[:, 0]
        assert g["npts"][gi] == len(X)
        if w[1] - w[0] > 1e-6 * max(w[2], 1e-12):
            assert abs(abs(float(g["normal"][gi] @ n)) - 1) < 1e-6
            a = 1 - 1e-3
            ref = np.eye(3) - a * np.outer(n, n)
            cov = g["cov64"][gi]
            full = np.array([[cov[0], cov[1], cov[2]], [cov[1], cov[3], cov[4]], [cov[2], cov[4], cov[5]]])
            assert np.allclose(full, ref, atol=1e-9)


def test_point_map_plane_normal(O):
    rng = np.random.default_rng(23)
    P = np.c_[rng.uniform(0, 2, size=(800, 2)), np.full(800, 0.3)].astype(np.float32)
    m = O.Map(P, 0.2, nnf_radius=1, min_points=5, per_point=True, point_k=10, point_search=2)
    g = m.gauss()
    assert m.G == 800
    assert np.allclose(np.abs(g["normal"][:, 2]), 1.0, atol=1e-6)


def test_point_map_field_against_kdtree(O):
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(24)
    r, R = 0.2, 2
    P = _surface_points(rng, 2500, r)
    m = O.Map(P, r, nnf_radius=R, min_points=5, per_point=True, point_k=10, point_search=2)
    g = m.gauss()
    org, dim = m.grid()
    keys, gids = m.band()
    tree = cKDTree(g["mu"].astype(np.float64))
    zz, yy, xx = np.meshgrid(np.arange(dim[2]), np.arange(dim[1]), np.arange(dim[0]), indexing="ij")
    lin = ((zz * dim[1] + yy) * dim[0] + xx).ravel()
    cells = np.stack([xx.ravel() + org[0], yy.ravel() + org[1], zz.ravel() + org[2]], 1)
    centres = (cells.astype(np.float64) + 0.5) * r
    d, j = tree.query(centres, k=2)
    field = np.full(lin.size, -1, np.int64)
    field[keys] = gids
    lim = R * r
    clear = (np.abs(d[:, 0] - lim) > 1e-5) & (d[:, 1] - d[:, 0] > 1e-6)
    want = np.where(d[:, 0] <= lim, j[:, 0], -1)
    assert np.array_equal(field[clear], want[clear])
    assert clear.mean() > 0.99
    # lookups go through the same field
    q = rng.uniform(P.min(0) - 0.5, P.max(0) + 0.5, size=(5000, 3)).astype(np.float32)
    cq = np.floor(q * np.float32(1.0 / r)).astype(np.int64) - org
    inside = np.all((cq >= 0) & (cq < dim), axis=1)
    lq = (cq[:, 2] * dim[1] + cq[:, 1]) * dim[0] + cq[:, 0]
    exp = np.where(inside, field[np.where(inside, lq, 0)], -1)
    assert np.array_equal(m.lookup(q), exp)
