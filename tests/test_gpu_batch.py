"""Batched multi-instance step (one HIP graph replay per step) against the
same filters stepped one by one with mp_filter_step, through the C-ABI.

Each instance has a twin built with identical parameters, initial poses and
scans.  The batch replays its graph; the twins run eagerly; between replays
the test reads state back (eager work on the same stream).  The graph runs the
same kernels on the same inputs, so poses, psi, neighbour lists and posterior
weights must agree bit for bit, for steps without prediction, with prediction
and noise (step values uploaded to the device before each replay), with an
odd SVGD iteration count (pose buffer copied back), with the residual-field
scorer, with the network scorer (its likelihood kernel captured in the
graph), on a hashed map, on a map of per-point Gaussians, with the coupled
LSH tangent, two hash tables, the exact kernel gradient, adjoint transport and
the final re-score, and after a scan of another size forces a new capture.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2404_16370_amd import megapf as M
from paper_2404_16370_amd import synth as S


@pytest.fixture(scope="module")
def world():
    w = S.build_workload("room", map_points=200_000, scan_points=1000, frames=4)
    dense = M.Map(w["map_xyz"], voxel=0.5)
    hashed = M.Map(w["map_xyz"], voxel=0.5, backend=M.MP_NNF_HASH)
    sur = M.Surrogate(dense, M.mp_surrogate_default_params(seed=11))
    point = M.Map(w["map_xyz"], voxel=0.2, nnf_radius=3, gauss_mode=M.MP_GAUSS_POINT)
    return dict(w=w, dense=dense, hashed=hashed, sur=sur, point=point)


def _poses(w, n, seed):
    sc = w["scene"]
    R, t = w["traj"][0]
    P = S.uniform_particles(n - n // 2, sc.lo, sc.hi, seed)
    G = S.gaussian_particles(n // 2, S.pose8(R, t), 0.05, 0.1, seed + 1)
    return np.concatenate([P, G]).astype(np.float32)


VARIANTS = dict(lsh_tangent=M.MP_LSH_TANGENT_SE3, lsh_tables=2, svgd_grad=M.MP_SVGD_GRAD_EXACT,
                svgd_transport=M.MP_SVGD_TRANSPORT_ADJOINT, final_rescore=1)

SPECS = [
    # (map, n, svgd_iters, k, scorer, scan slice[, further filter parameters])
    ("dense", 1000, 3, 8, M.MP_SCORER_PLAIN, slice(0, 1000)),
    ("dense", 4096, 2, 16, M.MP_SCORER_PLAIN, slice(0, 700)),
    ("hashed", 300, 1, 8, M.MP_SCORER_SCOREFIELD, slice(100, 900)),
    ("dense", 500, 2, 8, M.MP_SCORER_SURROGATE, slice(0, 300)),
    ("dense", 800, 3, 8, M.MP_SCORER_PLAIN, slice(0, 900), VARIANTS),
    ("point", 600, 2, 8, M.MP_SCORER_PLAIN, slice(0, 800), dict(d_max=0.6)),
]


def _make(world, spec, seed, **kw):
    mp, n, iters, k, scorer, sl = spec[:6]
    extra = dict(d_max=1.0)
    if len(spec) > 6:
        extra.update(spec[6])
    extra.update(kw)
    p = M.mp_filter_default_params(n_particles=n, k=k, lsh_bits=12, svgd_iters=iters, post_iters=10, window_c=16,
                                   seed=seed, scorer=scorer, **extra)
    f = M.Filter(world[mp], p, poses=_poses(world["w"], n, seed))
    if scorer == M.MP_SCORER_SURROGATE:
        f.set_surrogate(world["sur"])
    f.scan_upload(np.ascontiguousarray(world["w"]["scans"][0][sl]))
    return f


def _state(f):
    return {k: f.debug_get(k) for k in ("poses", "psi", "nbr", "post", "prior")}


def _assert_same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k]), "%s: %s differs" % (what, k)


def test_batch_replay_matches_eager(world):
    batch_f = [_make(world, s, 900 + i) for i, s in enumerate(SPECS)]
    b = M.Batch(batch_f, autotune=True)
    info = b.info()
    assert info["n_instances"] == len(SPECS)
    assert set(info["lik_batch"]).issubset({2, 4, 8, 16, 0})
    print("autotuned (layout, batch):", list(zip(info["lik_layout"], info["lik_batch"])))
    # twins with the layout the tuner picked (the gather batch does not change
    # the order of the arithmetic; the layout does)
    twins = [_make(world, s, 900 + i, lik_layout=info["lik_layout"][i]) for i, s in enumerate(SPECS)]
    rng = np.random.default_rng(5)
    odo = world["w"]["odometry"]
    for step in range(4):
        if step == 0:
            dT = cov = None
        else:
            dT = np.stack([odo[1][0] for _ in SPECS]).astype(np.float32)
            cov = np.stack([np.diag(rng.uniform(1e-5, 1e-3, 6)) for _ in SPECS]).astype(np.float32)
        b.step(dT, cov)
        for i, t in enumerate(twins):
            t.step(None if dT is None else dT[i], None if cov is None else cov[i])
        for i, (f, t) in enumerate(zip(batch_f, twins)):
            _assert_same(_state(f), _state(t), "step %d instance %d" % (step, i))
            qa, qb = f.posterior_query(), t.posterior_query()
            assert qa["map_index"] == qb["map_index"] and qa["frame"] == qb["frame"] == step + 1
    assert b.info()["captures"] == 1
    # a scan of another size forces a new capture
    new_scan = np.ascontiguousarray(world["w"]["scans"][1][:850])
    batch_f[1].scan_upload(new_scan)
    twins[1].scan_upload(new_scan)
    b.step(None, None)
    for t in twins:
        t.step()
    assert b.info()["captures"] == 2
    for i, (f, t) in enumerate(zip(batch_f, twins)):
        _assert_same(_state(f), _state(t), "after recapture, instance %d" % i)
    # filters stay usable alone and cannot be destroyed while batched
    batch_f[0].step()
    with pytest.raises(M.MegaPFError):
        batch_f[0].close()
    b.close()
    batch_f[0].close()
    for f in batch_f[1:] + twins:
        f.set_surrogate(None)
        f.close()


def test_batch_errors(world):
    f = M.Filter(world["dense"], M.mp_filter_default_params(n_particles=64, svgd_iters=1))
    with pytest.raises(M.MegaPFError):
        M.Batch([f])            # no scan yet
    f.scan_upload(world["w"]["scans"][0][:100])
    with pytest.raises(M.MegaPFError):
        M.Batch([f, f])         # the same filter twice
    b = M.Batch([f], autotune=False)
    with pytest.raises(M.MegaPFError):
        b.step(np.array([[1, 0, 0, 0, np.nan, 0, 0]], np.float32), None)
    b.step(None, None)
    b.close()
