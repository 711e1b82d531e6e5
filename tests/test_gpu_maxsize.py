"""The largest filter the library takes: 2^26 = 67,108,864 particles (K = 8,
24 LSH bits, a 512-point scan), one stage at a time, against the oracle on
samples at the head, the middle and the tail of the index range, and by
properties over all particles:
  bit-exact   uniform initial poses and LSH codes of the sampled particles
  1e-4 rel    log-likelihoods of the sampled particles (inlier counts exact)
  property    the sort is a permutation, codes ascend, equal codes keep
              ascending particle order; every list starts with its particle
              (kernel value 1) and holds distinct valid indices with kernel
              values in [0, 1] (exp(-q) underflows for distant particles);
              updated poses finite; posterior weights sum to 1
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2404_16370_amd import megapf as M
from paper_2404_16370_amd import synth as S

N = 1 << 26
SEED = 4005
BLOCKS = [(0, 512), (N // 2 - 256, 512), (N - 512, 512)]


def test_max_particles(O):
    w = S.build_workload("room", map_points=200_000, scan_points=512)
    m = M.Map(w["map_xyz"], voxel=0.5)
    om = O.Map(w["map_xyz"], 0.5)
    info = m.info()
    lo = np.array(info["box_min"], np.float32); hi = np.array(info["box_max"], np.float32)
    scan = np.ascontiguousarray(w["scans"][0])
    _, scov, _ = O.scan_cov(scan, k=10)
    p = M.mp_filter_default_params(n_particles=N, k=8, lsh_bits=24, svgd_iters=1, post_iters=2, window_c=8,
                                   d_max=1.0, c_max=9.0, seed=SEED)
    f = M.Filter(m, p, box=(lo, hi))
    f.scan_upload(scan, cov6=scov)
    print("filter of %d particles created" % N, flush=True)
    ref = {a: O.init_uniform_range(SEED, a, n, lo, hi) for a, n in BLOCKS}
    poses = f.debug_get("poses")
    for a, n in BLOCKS:
        assert np.array_equal(poses[a:a + n], ref[a]), a
    del poses
    # LSH codes
    f.debug_stage(M.MP_STAGE_LSH, 0)
    codes = f.debug_get("codes")
    TL = O.lsh_frame(SEED, 0, 0, lo, hi)
    assert np.array_equal(f.debug_get("tlsh"), TL)
    for a, n in BLOCKS:
        assert np.array_equal(codes[a:a + n], O.lsh_codes(ref[a], TL, 1.0, 5.0, 2.5, 0.3, 24, SEED, 0, 0,
                                                          first_index=a)), a
    # sort: a stable permutation
    f.debug_stage(M.MP_STAGE_SORT)
    srt = f.debug_get("sorted").astype(np.int64)
    sc = f.debug_get("scodes")
    assert np.array_equal(np.bincount(srt, minlength=N), np.ones(N, np.int64))
    assert np.array_equal(sc, codes[srt])
    assert np.all(sc[1:] >= sc[:-1])
    same = sc[1:] == sc[:-1]
    assert np.all(srt[1:][same] > srt[:-1][same])
    del srt, sc, same, codes
    print("codes and sort checked", flush=True)
    # refresh: list invariants on a sample of particles
    f.debug_stage(M.MP_STAGE_REFRESH)
    nbr = f.debug_get("nbr")
    kv = f.debug_get("kval")
    pick = np.r_[0:4096, N - 4096:N, np.random.default_rng(1).integers(0, N, 8192)]
    L = nbr[:, pick]
    assert np.array_equal(L[0], pick)
    assert np.all((L >= -1) & (L < N))
    for c in range(L.shape[1]):
        v = L[:, c][L[:, c] >= 0]
        assert len(np.unique(v)) == len(v)
    K = kv[:, pick]
    # exp(-q) of a neighbour far away in pose space underflows to 0 in FP32
    assert np.all(np.where(L >= 0, (K >= 0) & (K <= 1), K == 0))
    assert np.all(K[0] == 1.0)
    del nbr, kv
    # likelihood of the sampled particles
    f.debug_stage(M.MP_STAGE_LIK)
    psi = f.debug_get("psi")
    for a, n in BLOCKS:
        lk = O.likelihood(om, scan, scov, ref[a], dmax=1.0, cmax=9.0)
        assert np.array_equal(psi[a:a + n, 7].astype(np.int64), lk["ninl"].astype(np.int64)), a
        assert np.all(np.abs(psi[a:a + n, 6] - lk["loglik"]) <= 1e-4 * np.abs(lk["loglik"]) + 1e-3), a
    del psi
    print("likelihood checked", flush=True)
    f.debug_stage(M.MP_STAGE_SVGD)
    assert np.all(np.isfinite(f.debug_get("poses")))
    f.debug_stage(M.MP_STAGE_POSTERIOR)
    q = f.posterior_query(weights=True)
    assert abs(q["weights"].sum() - 1.0) < 1e-4
    assert q["map_weight"] == pytest.approx(q["weights"].max(), rel=1e-6)
    f.close()


def test_min_particles(O):
    # the smallest filter: one particle, K = 1, one bucket; a step is a
    # Gauss-Newton update of that particle and its weight is 1
    w = S.build_workload("room", map_points=50_000, scan_points=300)
    m = M.Map(w["map_xyz"], voxel=0.5)
    R, t = w["traj"][0]
    pose = S.pose8(R, t)[None, :].astype(np.float32)
    p = M.mp_filter_default_params(n_particles=1, k=1, lsh_bits=0, svgd_iters=3, post_iters=2, window_c=0,
                                   d_max=1.0, seed=3)
    f = M.Filter(m, p, poses=pose)
    f.scan_upload(np.ascontiguousarray(w["scans"][0]))
    f.step()
    q = f.posterior_query(poses=True, weights=True)
    assert q["weights"].shape == (1,) and q["weights"][0] == pytest.approx(1.0)
    assert q["map_index"] == 0 and np.all(np.isfinite(q["poses"]))
    # started at the truth, the Gauss-Newton steps stay within a few cm of it
    assert np.linalg.norm(q["poses"][0, 4:7] - pose[0, 4:7]) < 0.05
    assert np.array_equal(f.debug_get("nbr"), np.zeros((1, 1), np.int32))
    f.close()


def test_out_of_memory_leaves_filter_usable():
    # 2^26 particles and a 65,536-point scan: the likelihood's partial sums
    # alone (64 chunks x 29 floats per particle) need 498 GB, more than the
    # device holds; the step fails with MP_E_OOM before launching anything,
    # and the same filter then steps with a small scan
    w = S.build_workload("room", map_points=200_000, scan_points=1000)
    m = M.Map(w["map_xyz"], voxel=0.5)
    info = m.info()
    p = M.mp_filter_default_params(n_particles=N, k=8, lsh_bits=24, svgd_iters=1, post_iters=1, window_c=8,
                                   d_max=1.0, seed=SEED)
    f = M.Filter(m, p, box=(info["box_min"], info["box_max"]))
    reps = 66
    big = np.concatenate([w["scans"][0] + np.float32(0.01 * r) for r in range(reps)])[:65536]
    f.scan_upload(np.ascontiguousarray(big.astype(np.float32)))
    head = f.debug_get("poses")[:4096].copy()
    print("stepping %d particles with a %d-point scan (expecting MP_E_OOM)" % (N, len(big)), flush=True)
    with pytest.raises(M.MegaPFError) as e:
        f.step()
    assert e.value.status == M.MP_E_OOM
    assert np.array_equal(f.debug_get("poses")[:4096], head)
    f.scan_upload(np.ascontiguousarray(w["scans"][0][:256]))
    f.step()
    q = f.posterior_query()
    assert q["frame"] == 1 and np.isfinite(q["map_weight"])
    f.close()
