"""Parity at the full benchmark size: 1,048,576 particles x 8192 scan points
on the 20M-point campus map, in the launch configuration bench.py times
(dense NNF, one scan chunk, default batch), on outputs the oracle can compute
one by one:
  bit-exact   map Gaussians (ids, voxels, means, normals), LSH codes of all
              particles, the complete bucket order and bounds, neighbour lists
              of 2048 sampled particles
  1e-4 rel    log-likelihoods of 256 sampled particles (inlier counts exact);
              H within 1e-4 of max|H| and b within 1e-4 of sqrt(H_ii sum c)
              per particle: the plain FP32 sums over all 8192 points of a
              lane (one chunk) against the FP64 oracle
  property    posterior weights sum to 1 and the MAP weight is the largest
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2404_16370_amd import megapf as M
from paper_2404_16370_amd import synth as S

N = 1_048_576
NS = 8192


@pytest.fixture(scope="module")
def campus(O):
    w = S.build_workload("campus", map_points=20_000_000, scan_points=NS, frames=2)
    print("campus generated", flush=True)
    m = M.Map(w["map_xyz"], voxel=1.0, nnf_radius=2, min_points=5)
    om = O.Map(w["map_xyz"], 1.0, nnf_radius=2, min_points=5)
    print("maps built", m.info(), flush=True)
    return dict(w=w, gpu=m, ora=om)


def test_campus_map_bitexact(campus):
    g = campus["gpu"].gauss()
    o = campus["ora"].gauss()
    assert len(g["mu"]) == campus["ora"].G
    assert np.array_equal(g["vox"], o["vox"]) and np.array_equal(g["mu"], o["mu"])
    assert np.array_equal(g["normal"], o["normal"]) and np.array_equal(g["count"], o["npts"])


def test_campus_stages(campus, O):
    w = campus["w"]
    info = campus["gpu"].info()
    p = M.mp_filter_default_params(n_particles=N, k=16, lsh_bits=24, svgd_iters=10, post_iters=10, window_c=32,
                                   d_max=2.0, seed=4003)
    f = M.Filter(campus["gpu"], p, box=(info["box_min"], info["box_max"]))
    scan = w["scans"][0]
    f.scan_upload(scan)
    poses = f.debug_get("poses")
    lo = np.array(info["box_min"], np.float32); hi = np.array(info["box_max"], np.float32)
    assert np.array_equal(poses, O.init_uniform(4003, N, lo, hi))
    # LSH codes, sort and bounds for all particles
    f.debug_stage(M.MP_STAGE_LSH, 0)
    codes = f.debug_get("codes")
    ref = O.lsh_codes(poses, O.lsh_frame(4003, 0, 0, lo, hi), 1.0, 5.0, 2.5, 0.3, 24, 4003, 0, 0)
    assert np.array_equal(codes, ref)
    f.debug_stage(M.MP_STAGE_SORT)
    s, h, e = O.bucket_sort(ref)
    assert np.array_equal(f.debug_get("sorted"), s)
    assert np.array_equal(f.debug_get("head"), h) and np.array_equal(f.debug_get("end"), e)
    # neighbour refresh: compare 2048 sampled particles (the oracle refreshes all, cheaply)
    f.debug_stage(M.MP_STAGE_REFRESH)
    nbr = f.debug_get("nbr").T
    nref, _, cref = O.refresh(poses, s, ref, 16, 32, 5.0, 2.5, None)
    rng = np.random.default_rng(0)
    pick = rng.choice(N, 2048, replace=False)
    assert np.array_equal(nbr[pick], nref[pick])
    assert np.array_equal(f.debug_get("cnt")[pick], cref[pick])
    # likelihood of 256 sampled particles, scan covariances as the library computed them from the scan
    f.debug_set("capture_hb", 1)
    f.debug_stage(M.MP_STAGE_LIK)
    psi = f.debug_get("psi")
    hb = f.debug_get("hb")
    _, scov, _ = O.scan_cov(scan, k=10)
    pick = rng.choice(N, 256, replace=False)
    lk = O.likelihood(campus["ora"], scan, scov, poses[pick], dmax=2.0, cmax=9.0)
    assert np.array_equal(psi[pick, 7].astype(np.int64), lk["ninl"].astype(np.int64))
    assert np.all(np.abs(psi[pick, 6] - lk["loglik"]) <= 1e-4 * np.abs(lk["loglik"]) + 1e-3)
    H = hb[pick, :21].astype(np.float64)
    b = hb[pick, 21:27].astype(np.float64)
    hn = np.abs(lk["H21"]).max(1, keepdims=True) + 1e-12
    herr = np.abs(H - lk["H21"]) / hn
    unt = O.likelihood(campus["ora"], scan, scov, poses[pick], dmax=2.0, cmax=1e9)
    cost = (-unt["loglik"] - 1e9 * (NS - unt["ninl"]))[:, None]
    diag = lk["H21"][:, [0, 6, 11, 15, 18, 20]]
    berr = np.abs(b - lk["b"]) / (np.sqrt(np.maximum(diag, 0) * np.maximum(cost, 0)) + 1e-9)
    print("full size, FP32 sums over 8192 points: max H error %.2e of max|H|, max b error %.2e of its scale"
          % (herr.max(), berr.max()), flush=True)
    assert herr.max() <= 1e-4 and berr.max() <= 1e-4
    # full step: posterior is a distribution with its MAP on top
    f.step()
    q = f.posterior_query(weights=True)
    wts = q["weights"]
    assert abs(wts.sum() - 1) < 1e-4 and q["map_weight"] >= wts.max() * (1 - 1e-6)
