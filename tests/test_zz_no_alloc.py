"""mp_odometry_noalloc (the allocation-free odometry) against mp_odometry,
through the C-ABI: identical outputs on two calls in a row, the second on
smaller scans, and the size limit of its fixed work area."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2404_16370_amd import megapf as M
from paper_2404_16370_amd import synth as S


def _same(a, b):
    assert np.array_equal(a["dT"], b["dT"]) and np.array_equal(a["cov"], b["cov"])
    for k in ("H21", "b", "dT64"):
        assert np.array_equal(a[k], b[k]), k
    assert a["cost"] == b["cost"] and a["inliers"] == b["inliers"] and a["cov_ok"] == b["cov_ok"]


def test_odometry_noalloc_matches_odometry():
    w = S.build_workload("room", map_points=200_000, scan_points=8000, frames=3)
    m = M.Map(w["map_xyz"], voxel=0.5)
    f = M.Filter(m, M.mp_filter_default_params(n_particles=64, svgd_iters=1))
    init = np.array([1, 0, 0, 0, 0.05, -0.02, 0.01], np.float32)
    results = []
    for n0, n1 in [(8000, 6000), (1500, 900)]:   # the second call on smaller scans
        print("odometry noalloc: scans of %d and %d points" % (n0, n1), flush=True)
        f.scan_upload(np.ascontiguousarray(w["scans"][0][:n0]))
        f.scan_upload(np.ascontiguousarray(w["scans"][1][:n1]))
        ref = f.odometry(init=init, iterations=10)
        got = f.odometry(init=init, iterations=10, noalloc=True)
        _same(got, ref)
        assert got["inliers"] > 0.5 * n1
        results.append(got)
    assert not np.array_equal(results[0]["H21"], results[1]["H21"])
    # the existing entry point still works after the fixed-area calls
    _same(f.odometry(init=init, iterations=10), results[1])


def test_odometry_noalloc_size_limit():
    w = S.build_workload("room", map_points=200_000, scan_points=8000, frames=2)
    m = M.Map(w["map_xyz"], voxel=0.5)
    f = M.Filter(m, M.mp_filter_default_params(n_particles=64, svgd_iters=1))
    big = np.concatenate([w["scans"][1]] * 3)[:20000] + np.float32(0.001)
    f.scan_upload(np.ascontiguousarray(w["scans"][0]))
    f.scan_upload(np.ascontiguousarray(big.astype(np.float32)))
    with pytest.raises(M.MegaPFError) as e:
        f.odometry(noalloc=True)
    assert e.value.status == M.MP_E_ARG and "16384" in str(e.value)
    # the allocating entry point takes the same scans
    assert f.odometry(iterations=2)["inliers"] > 0
