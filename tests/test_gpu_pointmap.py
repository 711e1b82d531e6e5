"""GPU parity of the map of per-point Gaussians (gauss_mode POINT, the
paper's nearest-point field) against the CPU oracle, through the C-ABI.

  bit-exact   Gaussian count, points, voxels, neighbourhood sizes and FP32
              normals (same neighbour ranking and FP64 Jacobi on both sides);
              band size, grid; field lookups (random points and points on
              cell faces); every neighbour-list capacity (k = 3, 10, 32) and
              search radius (1, 4)
  1e-4 rel    log-likelihoods, H and b of the likelihood on this map (both
              launch layouts), as for the per-voxel map
  ties        a lattice (exactly equal distances), in scan and shuffled order:
              an open gap, marked xfail (normals of about half the points differ)
  errors      HASH backend and out-of-range point_k / point_search rejected
The map: the room scene subsampled to 40,000 points, 0.2 m cells, R = 2.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2404_16370_amd import megapf as M
from paper_2404_16370_amd import synth as S

R_CELL, RAD = 0.2, 2


@pytest.fixture(scope="module")
def pm(O):
    w = S.build_workload("room", map_points=200_000, scan_points=1000)
    rng = np.random.default_rng(7)
    xyz = np.ascontiguousarray(w["map_xyz"][rng.choice(len(w["map_xyz"]), 40_000, replace=False)])
    g = M.Map(xyz, voxel=R_CELL, nnf_radius=RAD, min_points=5, gauss_mode=M.MP_GAUSS_POINT, point_k=10,
              point_search=2)
    o = O.Map(xyz, R_CELL, nnf_radius=RAD, min_points=5, per_point=True, point_k=10, point_search=2)
    print("point map", g.info(), flush=True)
    return dict(w=w, xyz=xyz, gpu=g, ora=o)


def _same_gauss(gm, om):
    info = gm.info()
    assert info["num_gauss"] == om.G
    g, o = gm.gauss(), om.gauss()
    assert np.array_equal(g["mu"], o["mu"])
    assert np.array_equal(g["vox"], o["vox"])
    assert np.array_equal(g["count"], o["npts"])
    assert np.array_equal(g["normal"], o["normal"])
    assert info["num_band"] == om.nb
    org, dim = om.grid()
    assert list(info["grid_origin"]) == list(org) and list(info["grid_dim"]) == list(dim)


def test_point_map_bitexact(pm):
    _same_gauss(pm["gpu"], pm["ora"])
    assert pm["gpu"].info()["backend"] == M.MP_NNF_DENSE
    rng = np.random.default_rng(3)
    sc = pm["w"]["scene"]
    q = rng.uniform(sc.lo - 1, sc.hi + 1, size=(300_000, 3)).astype(np.float32)
    q[:30000] = (np.round(q[:30000] / R_CELL) * R_CELL).astype(np.float32)
    q[30000:40000] = pm["xyz"][rng.choice(len(pm["xyz"]), 10000)]
    assert np.array_equal(pm["gpu"].lookup(q), pm["ora"].lookup(q))


@pytest.mark.parametrize("k,search,minp", [(3, 1, 3), (32, 1, 20), (10, 4, 5), (16, 2, 12)])
def test_point_map_variants_bitexact(pm, O, k, search, minp):
    xyz = np.ascontiguousarray(pm["xyz"][:15000])
    g = M.Map(xyz, voxel=0.15, nnf_radius=1, min_points=minp, gauss_mode=M.MP_GAUSS_POINT, point_k=k,
              point_search=search)
    o = O.Map(xyz, 0.15, nnf_radius=1, min_points=minp, per_point=True, point_k=k, point_search=search)
    _same_gauss(g, o)
    rng = np.random.default_rng(k)
    q = xyz[rng.choice(len(xyz), 20000)] + rng.normal(scale=0.1, size=(20000, 3)).astype(np.float32)
    assert np.array_equal(g.lookup(q), o.lookup(q))


def _tied_lattice(shuffle):
    # a lattice with spacing and offsets exact in FP32: every point has many
    # neighbours at exactly equal distances, and half the lattice planes lie
    # exactly on cell faces; both sides break ties by the lower index
    g = np.stack(np.meshgrid(np.arange(30), np.arange(26), np.arange(6), indexing="ij"), -1).reshape(-1, 3)
    xyz = (0.125 * g + np.array([1.0, -2.0, 0.25])).astype(np.float32)
    if shuffle:
        xyz = xyz[np.random.default_rng(5).permutation(len(xyz))]
    return np.ascontiguousarray(xyz)


@pytest.mark.parametrize("shuffle", [False, True])
def test_point_map_lattice_lists_bitexact(O, shuffle):
    # the ranked neighbour list of every point, as the device build forms it,
    # against the oracle's (brute force over the voxel cube)
    xyz = _tied_lattice(shuffle)
    print("lattice lists", len(xyz), "shuffled", shuffle, flush=True)
    dev = M.debug_map_point_knn(xyz, 0.25, point_k=10, point_search=2, nnf_radius=2, min_points=5)
    om = O.Map(xyz, 0.25, nnf_radius=2, min_points=5, per_point=True, point_k=10, point_search=2, want_knn=True)
    bad = np.nonzero((dev != om.knn).any(1))[0]
    if len(bad):
        i = int(bad[0])
        print("first differing point", i, xyz[i], "device", dev[i], "oracle", om.knn[i], flush=True)
    assert len(bad) == 0, "%d of %d lists differ" % (len(bad), len(xyz))


@pytest.mark.parametrize("shuffle", [False, True])
def test_point_map_lattice_ties_bitexact(O, shuffle):
    # the whole per-point map of the tied lattice: Gaussians, normals, field
    xyz = _tied_lattice(shuffle)
    print("lattice point map", len(xyz), "shuffled", shuffle, flush=True)
    gm = M.Map(xyz, voxel=0.25, nnf_radius=2, min_points=5, gauss_mode=M.MP_GAUSS_POINT, point_k=10, point_search=2)
    om = O.Map(xyz, 0.25, nnf_radius=2, min_points=5, per_point=True, point_k=10, point_search=2)
    _same_gauss(gm, om)
    rng = np.random.default_rng(9)
    q = rng.uniform(xyz.min(0) - 0.6, xyz.max(0) + 0.6, size=(50000, 3)).astype(np.float32)
    q[:20000] = (np.round(q[:20000] / 0.125) * 0.125).astype(np.float32)
    assert np.array_equal(gm.lookup(q), om.lookup(q))


def _poses_near(w, n, seed):
    R, t = w["traj"][0]
    gt = S.pose8(R, t)
    P = S.uniform_particles(n - n // 2, w["scene"].lo, w["scene"].hi, seed)
    G = S.gaussian_particles(n // 2, gt, 0.05, 0.1, seed + 1)
    return np.concatenate([P, G]).astype(np.float32)


@pytest.mark.parametrize("layout,n", [(M.MP_LIK_LAYOUT_GROUPED, 600), (M.MP_LIK_LAYOUT_PARTICLE, 257)])
def test_point_map_likelihood_parity(pm, O, layout, n):
    w = pm["w"]
    scan = np.ascontiguousarray(w["scans"][0][:1000])
    _, scov, _ = O.scan_cov(scan, k=10)
    poses = _poses_near(w, n, 60 + n)
    p = M.mp_filter_default_params(n_particles=n, k=8, lsh_bits=8, svgd_iters=1, post_iters=1, window_c=8,
                                   d_max=0.5, c_max=9.0, lik_layout=layout, seed=4001)
    f = M.Filter(pm["gpu"], p, poses=poses)
    f.scan_upload(scan, cov6=scov)
    f.debug_set("capture_hb", 1)
    f.debug_stage(M.MP_STAGE_LIK)
    psi = f.debug_get("psi")
    hb = f.debug_get("hb")
    ref = O.likelihood(pm["ora"], scan, scov, poses, dmax=0.5, cmax=9.0, lam_rel=1e-3, lam_abs=1e-6)
    assert np.array_equal(psi[:, 7].astype(np.int64), ref["ninl"].astype(np.int64))
    assert ref["ninl"][n // 2:].mean() > 0.5 * len(scan)     # particles near the truth see the map
    ll = psi[:, 6].astype(np.float64)
    assert np.all(np.abs(ll - ref["loglik"]) <= 1e-4 * np.abs(ref["loglik"]) + 1e-3)
    H = hb[:, :21].astype(np.float64)
    hn = np.abs(ref["H21"]).max(1, keepdims=True) + 1e-12
    assert np.all(np.abs(H - ref["H21"]) <= 1e-4 * hn)
    b = hb[:, 21:27].astype(np.float64)
    diag = ref["H21"][:, [0, 6, 11, 15, 18, 20]]
    big = 1e9
    unt = O.likelihood(pm["ora"], scan, scov, poses, dmax=0.5, cmax=big)
    cost = (-unt["loglik"] - big * (scan.shape[0] - unt["ninl"]))[:, None]
    bscale = np.sqrt(np.maximum(diag, 0) * np.maximum(cost, 0)) + 1e-9
    assert np.all(np.abs(b - ref["b"]) <= 1e-4 * bscale)


def test_point_map_errors(pm):
    xyz = pm["xyz"][:1000]
    with pytest.raises(M.MegaPFError) as e:
        M.Map(xyz, voxel=0.2, gauss_mode=M.MP_GAUSS_POINT, backend=M.MP_NNF_HASH)
    assert e.value.status == M.MP_E_UNSUPPORTED
    for kw in (dict(point_k=2), dict(point_k=33), dict(point_search=0), dict(point_search=5), dict(gauss_mode=7),
               dict(nnf_radius=0)):
        with pytest.raises(M.MegaPFError) as e:
            M.Map(xyz, voxel=0.2, **{"gauss_mode": M.MP_GAUSS_POINT, **kw})
        assert e.value.status == M.MP_E_ARG
    # an empty map and a map too sparse for any neighbourhood
    m0 = M.Map(np.zeros((0, 3), np.float32), voxel=0.2, gauss_mode=M.MP_GAUSS_POINT)
    assert m0.info()["num_gauss"] == 0
    sparse = np.zeros((30, 3), np.float32)
    sparse[:, 0] = np.arange(30, dtype=np.float32) * np.float32(5.0)   # 5 m apart on a line
    m1 = M.Map(sparse, voxel=0.2, gauss_mode=M.MP_GAUSS_POINT)
    assert m1.info()["num_gauss"] == 0
    assert np.all(m1.lookup(sparse) == -1)
    # the box of all map voxels beyond 2^28 cells (145 m diagonal at 0.2 m: 725^3)
    diag = (np.arange(30, dtype=np.float32)[:, None] * np.float32(5.0)) * np.ones((1, 3), np.float32)
    with pytest.raises(M.MegaPFError) as e:
        M.Map(diag, voxel=0.2, gauss_mode=M.MP_GAUSS_POINT)
    assert e.value.status == M.MP_E_UNSUPPORTED
