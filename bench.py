"""Throughput of the Stein particle filter hot path on one MI355X.

One step = one mp_filter_step on a fresh scan: prediction, 10 iterations of
(LSH codes, bucket sort, neighbour refresh, likelihood + Gauss-Newton, SVGD),
and the posterior propagation, for 1,048,576 particles and 8192 scan points
on a synthetic 200 x 200 x 15 m campus map (20M points, 1 m voxels).  Scans
for all timed steps are generated and copied to HBM before timing; the timed
region covers mp_scan_upload (device-resident points) + mp_filter_step.

Prints one JSON line.  `roofline` refers to the likelihood kernel (k_lik_grp),
timed with HIP events on the stream it runs on; `cpu_baseline` times the CPU
oracle on a bounded sample of the same workload on this host's cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "filter steps/s and particle-point evals/s at 1M particles, plain vs surrogate"
PEAK_FP32 = 157.3e12        # MI355X FP32 vector, FLOP/s
PEAK_BF16 = 2.5e15          # MI355X dense bf16 matrix, FLOP/s
MLP_MACS = 192 * 128 + 128 * 128 + 128 * 4        # one network evaluation
TRAIN_MACS = 192 * 128 * 2 + 128 * 128 * 3        # matrix-core MACs per training sample (2 forward, 3 backward GEMMs)
PEAK_HBM = 8.0e12           # bytes/s
# FP32 operations of one likelihood evaluation in k_lik (an fma counts 2):
#   inlier:  transform 18, voxel key 3, residual and gate 8, R^T n and R^T e 30,
#            Sherman-Morrison Omega 42 (D u 15, q = u - D u 3, u^T D u 5,
#            beta 4, Omega 15), Omega e and cost 20, cost add 1, b 18,
#            [mu]x Omega 27, H_ww 24, H_wv 9, H_vv 12                  = 212
#   outlier: transform 18, voxel key 3 (+ residual and gate 8 on an NNF hit) = 21..29
FLOPS_INLIER = 212
FLOPS_OUTLIER = 21
# the method's algorithmic count per evaluation (transform 18, rotate Sigma^M
# 90, 3x3 inverse 46, residual and cost 45, H / b blocks 75, 28 accumulations)
FLOPS_ALGORITHMIC = 300
GATHER_BYTES = 32           # one Gaussian record of the dense NNF per evaluation (the cell index is computed)

WORKLOADS = {
    "campus": dict(particles=1_048_576, scan_points=8192, svgd_iters=10, k=16, lsh_bits=24, voxel=1.0,
                   map_points=20_000_000, window_c=32, post_iters=10),
    "floor": dict(particles=65_536, scan_points=4096, svgd_iters=20, k=16, lsh_bits=20, voxel=0.5,
                  map_points=2_000_000, window_c=32, post_iters=10),
    "room": dict(particles=4096, scan_points=1024, svgd_iters=10, k=8, lsh_bits=16, voxel=0.5,
                 map_points=200_000, window_c=16, post_iters=10),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


COUNTER_PROFILE = os.path.join(ROOT, "profiles", "k_lik_campus_1M_x_8192_counters.md")
KERNEL_SOURCES = ("paper_2404_16370_amd/csrc/likelihood.hip", "paper_2404_16370_amd/csrc/mp_lookup.hpp",
                  "paper_2404_16370_amd/csrc/mp_det.hpp")


def measured_traffic(workload):
    """HBM-side bytes per k_lik launch from the committed counter profile
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy kernel), or None when
    the profile is missing, covers another workload, or the kernel source has
    changed since the counters were taken."""
    import hashlib
    if workload != "campus" or not os.path.exists(COUNTER_PROFILE):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    vals = {}
    for line in open(COUNTER_PROFILE):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_sha256"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(wl, w, scan, budget_s=15.0):
    """Time the oracle's correction iteration on a sample of particles and
    scale to the workload (particles x iterations)."""
    import oracle as O
    O.build(force=False)
    t0 = time.perf_counter()
    om = O.Map(w["map_xyz"], wl["voxel"], nnf_radius=2, min_points=5)
    t_map = time.perf_counter() - t0
    _, scov, _ = O.scan_cov(scan, k=10)
    from paper_2404_16370_amd import synth as S
    # particles as the workload starts them: uniform over the map box and SO(3)
    poses = S.uniform_particles(262144, w["scene"].lo, w["scene"].hi, 3003)
    info_lo, info_hi = w["scene"].lo.astype(np.float32), w["scene"].hi.astype(np.float32)

    def one_iteration(P):
        n = len(P)
        TL = O.lsh_frame(1, 0, 0, info_lo, info_hi)
        codes = O.lsh_codes(P, TL, 1.0, 5.0, 2.5, 0.3, wl["lsh_bits"], 1, 0, 0)
        s, _, _ = O.bucket_sort(codes)
        nbr, q, cnt = O.refresh(P, s, codes, wl["k"], wl["window_c"], 5.0, 2.5, None)
        lk = O.likelihood(om, scan, scov, P, dmax=2 * wl["voxel"], cmax=9.0)
        O.svgd(P, lk["psi"], nbr, 5.0, 2.5)
        return lk

    m = 64
    t0 = time.perf_counter()
    one_iteration(poses[:m])
    dt = time.perf_counter() - t0
    m = int(min(len(poses), max(64, m * budget_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    one_iteration(poses[:m])
    dt = time.perf_counter() - t0
    per_particle_iter = dt / m
    step_s = per_particle_iter * wl["particles"] * wl["svgd_iters"]
    evals = wl["scan_points"] * m
    cores = O.num_threads()
    # the same iteration on one thread, on a sample sized for about a quarter of the budget
    m1 = int(max(16, min(m, m * 0.25 * budget_s / max(dt * cores, 1e-3))))
    O.set_threads(1)
    t0 = time.perf_counter()
    one_iteration(poses[:m1])
    dt1 = time.perf_counter() - t0
    O.set_threads(cores)
    single = {"evals_per_s": wl["scan_points"] * m1 / dt1,
              "steps_per_s": 1.0 / (dt1 / m1 * wl["particles"] * wl["svgd_iters"]), "sample_particles": m1}
    return {"value": 1.0 / step_s, "unit": "filter steps/s", "cores": cores, "kind": "oracle",
            "sample": ("one correction iteration (LSH, sort, refresh, likelihood+GN, SVGD) of %d of the "
                       "workload's particles x %d scan points, %.1f s; scaled to %d particles x %d iterations "
                       "(posterior and prediction not included)" %
                       (m, wl["scan_points"], dt, wl["particles"], wl["svgd_iters"])),
            "evals_per_s": evals / dt, "map_build_s": t_map, "single_core": single, "cpu_model": cpu_model()}


def cpu_model():
    """the host CPU's model name (from /proc/cpuinfo)"""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def odometry_leg(M, m, w, scans, cpu):
    """GICP scan-to-scan odometry (mp_odometry, 20 iterations, d_max 1 m) over
    the workload's consecutive scan pairs, started from the workload's noisy
    motion prior (what an IMU or wheel odometry supplies) and from the
    identity, against the true motion; the oracle's FP64 run on the same
    pairs beside it."""
    import torch
    from paper_2404_16370_amd import synth as S

    def err(p, truth):
        q = np.asarray(p[:4], np.float64)
        q = q / np.linalg.norm(q)
        return (float(np.linalg.norm(np.asarray(p[4:7], np.float64) - truth[4:7])),
                float(np.degrees(2 * np.arccos(min(1.0, abs(float(q @ truth[:4])))))))

    p = M.mp_filter_default_params(n_particles=64, svgd_iters=1)
    f = M.Filter(m, p)
    recs, pairs, times = [], [], []
    for k in range(len(scans)):
        f.scan_upload(scans[k])
        recs.append(f.debug_get("scan").copy())
        if k == 0:
            continue
        (R0, t0), (R1, t1) = w["traj"][k - 1], w["traj"][k]
        truth = S.pose8(R0.T @ R1, R0.T @ (t1 - t0)).astype(np.float64)
        prior = np.asarray(w["odometry"][k][0], np.float32)
        f.odometry(init=prior)   # warm
        torch.cuda.synchronize()
        t_0 = time.perf_counter()
        r = f.odometry(init=prior)
        times.append(time.perf_counter() - t_0)
        r_id = f.odometry()
        pairs.append(dict(frame=k, motion_deg=float(np.degrees(2 * np.arccos(min(1.0, abs(truth[0]))))),
                          prior=err(prior, truth), refined=err(r["dT64"], truth),
                          from_identity=err(r_id["dT64"], truth), inliers=r["inliers"], prior7=prior, dT64=r["dT64"],
                          k=k))
    f.close()
    ns = len(recs[-1])
    evals = 21.0 * ns * len(recs[-2])       # distance evaluations of 21 correspondence searches
    t_med = float(np.median(times))
    out = {"ms_per_call": 1e3 * t_med, "scan_points": ns, "iterations": 20, "pairs": len(pairs),
           "error_m_deg": {"prior": [q["prior"] for q in pairs], "refined_from_prior": [q["refined"] for q in pairs],
                           "from_identity": [q["from_identity"] for q in pairs]},
           "motion_deg": [q["motion_deg"] for q in pairs], "inliers": [q["inliers"] for q in pairs],
           "roofline": {"bound": "alu", "achieved": evals * 8 / t_med / 1e12, "peak": PEAK_FP32 / 1e12,
                        "unit": "TFLOP/s", "frac": evals * 8 / t_med / PEAK_FP32, "traffic": None,
                        "kernel": "k_odo_nn + k_odo_terms + k_odo_step, 21 evaluations (8 flops per distance)"}}
    if cpu:
        import oracle as O
        dt, worst = [], 0.0
        for q in pairs:
            a, b = recs[q["k"] - 1], recs[q["k"]]
            t_0 = time.perf_counter()
            ref = O.gicp_align(a[:, :3], np.ascontiguousarray(a[:, 3:9]), b[:, :3], np.ascontiguousarray(b[:, 3:9]),
                               init7=q["prior7"], iters=20, dmax=1.0)
            dt.append(time.perf_counter() - t_0)
            worst = max(worst, float(np.abs(q["dT64"][4:7] - ref["pose"][4:7]).max()))
        out["cpu_baseline"] = {"value": 1e3 * float(np.median(dt)), "unit": "ms per call", "cores": O.num_threads(),
                               "kind": "oracle", "sample": "the same scan pairs and priors, 20 iterations"}
        out["vs_oracle_max_m"] = worst
    return out


def surrogate_leg(M, m, wl, minfo, scans, odo, warmup, steps):
    """The same filter step with the network scorer (weights as initialised:
    the step's cost does not depend on their values)."""
    import torch
    sur = M.Surrogate(m, M.mp_surrogate_default_params(seed=5003))
    p = M.mp_filter_default_params(n_particles=wl["particles"], k=wl["k"], lsh_bits=wl["lsh_bits"],
                                   svgd_iters=wl["svgd_iters"], post_iters=wl["post_iters"],
                                   window_c=wl["window_c"], d_max=2.0 * wl["voxel"], seed=4003,
                                   scorer=M.MP_SCORER_SURROGATE)
    f = M.Filter(m, p, box=(minfo["box_min"], minfo["box_max"]))
    f.set_surrogate(sur)

    def run(k):
        dT, cov = odo[k] if k > 0 else (None, None)
        f.scan_upload(scans[k])
        f.step(dT, cov)

    for k in range(warmup):
        run(k)
        log("surrogate warmup step %d done" % k)
    torch.cuda.synchronize()
    lik_ms, lik_n = [], []
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        run(k)
        st = f.stage_times()
        lik_ms.append(st["likelihood_core"][0])
        lik_n.append(st["likelihood_core"][1])
        log("surrogate step %d done" % k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    evals_iter = float(wl["particles"]) * wl["scan_points"]
    t_launch = (sum(lik_ms) / max(sum(lik_n), 1)) * 1e-3
    achieved = evals_iter * 2 * MLP_MACS / t_launch
    f.set_surrogate(None)
    res = {"steps_per_s": steps / elapsed, "evals_per_s": steps * evals_iter * wl["svgd_iters"] / elapsed,
           "kernel": "k_lik_sur", "launch_ms": t_launch * 1e3,
           "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                        "frac": achieved / PEAK_BF16, "traffic": None},
           "weights": "initial (untrained); cost independent of values"}
    del f
    sur.close()
    return res


def train_leg(M, S, m, w, minfo, steps=50):
    """Adam steps of the surrogate at batch 65,536 over 4M labelled samples."""
    import torch
    sur = M.Surrogate(m, M.mp_surrogate_default_params(seed=5004))
    xyz = S.surrogate_samples(w["map_xyz"], minfo["box_min"], minfo["box_max"], 4_000_000, 5005)
    sur.set_data(torch.from_numpy(xyz).cuda())
    sur.train(3, losses=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = sur.train(steps)          # copies the losses back: synchronises
    dt = time.perf_counter() - t0
    batch = sur.params.batch
    achieved = steps * batch * 2 * TRAIN_MACS / dt
    res = {"ms_per_step": 1e3 * dt / steps, "samples_per_s": steps * batch / dt, "batch": batch,
           "train_samples": len(xyz), "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
           "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                        "frac": achieved / PEAK_BF16, "traffic": None, "kernel": "whole training step"}}
    sur.close()
    return res


SEQUENCES = {
    # the paper's kidnap sequences (Sec. IV-A): the sensor view blocked for a
    # while and the sensor moved meanwhile; blocked frames predict with a wide
    # noise (the uncertainty grows), so the particles spread over the map
    "floor": dict(particles=65536, k=16, lsh_bits=20, svgd_iters=20, window_c=32, voxel=0.5, d_max=1.0,
                  frames=60, occlusion=(25, 31), kidnap=28, kidnap_dist=20.0, blocked=(0.8, 6.0), seed=4002),
    # the same at the paper's outdoor scale with its 80 m / 90 deg teleport (40 frames: casting a
    # campus scan takes seconds of CPU)
    "campus": dict(particles=1_048_576, k=16, lsh_bits=24, svgd_iters=10, window_c=32, voxel=1.0, d_max=2.0,
                   frames=40, occlusion=(15, 21), kidnap=18, kidnap_dist=80.0, blocked=(1.0, 25.0), seed=4003),
}


def sequence_main(args):
    """Global localisation, occlusion and kidnap (the paper's kidnap
    sequences, Sec. IV-A, as a synthetic analogue) on the floor scene (65,536
    particles, 60 frames, scans blocked for frames 25..30 while the sensor is
    teleported 20 m at frame 28) or the campus (1,048,576 particles, 40
    frames, blocked 15..20, teleported 80 m and 90 deg at frame 18), from a
    uniform start; blocked frames predict with a wide noise, so the particles
    spread.  Each frame's motion is the workload's noisy prior refined by
    mp_odometry when both scans are there and the match keeps half the points
    (else the prior); the maximum-posterior pose and its smoothed version
    (mp_smoother) against the truth: convergence and recovery frames, ATE."""
    from paper_2404_16370_amd import synth as S
    cfg = SEQUENCES[args.scene]
    frames = args.seq_frames if args.seq_frames else cfg["frames"]
    occl, kid = cfg["occlusion"], cfg["kidnap"]
    if args.kidnap_frame:
        # the teleport at another frame, the view blocked from 3 frames before it to 3 after
        kid = args.kidnap_frame
        occl = (kid - (cfg["kidnap"] - cfg["occlusion"][0]), kid + (cfg["occlusion"][1] - cfg["kidnap"]))
    br, bt = cfg["blocked"]
    blocked_cov = np.diag([br ** 2] * 3 + [bt ** 2] * 3).astype(np.float32)
    t0 = time.perf_counter()
    # the scans are cast before anything touches the GPU (the workers are forked)
    w = S.build_workload(args.scene, frames=frames, kidnap_frame=kid, kidnap_dist=cfg["kidnap_dist"], occlusion=occl,
                         workers=min(16, os.cpu_count() or 1),
                         progress=lambda d, n: log("scans cast: %d of %d" % (d, n)) if d % 8 == 0 or d == n else None)
    log("sequence generated in %.1f s" % (time.perf_counter() - t0))
    import torch
    from paper_2404_16370_amd import megapf as M
    torch.cuda.set_device(0)
    if args.map == "point":
        # the paper's fields: 0.1 m cells indoors, 0.2 m outdoors; coverage and gate 5 cells
        cell = 0.1 if args.scene == "floor" else 0.2
        m = M.Map(torch.from_numpy(w["map_xyz"]).cuda(), voxel=cell, nnf_radius=5, gauss_mode=M.MP_GAUSS_POINT)
        dmax = 5 * cell
    else:
        m = M.Map(torch.from_numpy(w["map_xyz"]).cuda(), voxel=cfg["voxel"])
        dmax = cfg["d_max"]
    info = m.info()
    log("map: %s" % info)
    p = M.mp_filter_default_params(n_particles=cfg["particles"], k=cfg["k"], lsh_bits=cfg["lsh_bits"],
                                   svgd_iters=cfg["svgd_iters"], post_iters=10, window_c=cfg["window_c"],
                                   d_max=dmax, seed=cfg["seed"], **VARIANTS[args.variant])
    f = M.Filter(m, p, box=(info["box_min"], info["box_max"]))
    sm = M.Smoother(window=5, jump_m=1.0, jump_rad=0.2)

    def err(pose, k):
        R, t = w["traj"][k]
        g = S.pose8(R, t)
        q = np.asarray(pose[:4], np.float64)
        q /= np.linalg.norm(q)
        return (float(np.linalg.norm(np.asarray(pose[4:7], np.float64) - g[4:7])),
                float(np.degrees(2 * np.arccos(min(1.0, abs(float(q @ g[:4])))))))

    raw, smooth, used_odo = [], [], 0
    n_prev = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(frames):
        scan = np.ascontiguousarray(w["scans"][k])
        f.scan_upload(scan)
        dT, cov = w["odometry"][k] if k > 0 else (None, None)
        if k > 0 and not len(scan):
            cov = blocked_cov
        if k > 0 and len(scan) and n_prev:
            r = f.odometry(init=np.asarray(dT, np.float32))
            if r["inliers"] >= 0.5 * len(scan):
                dT = r["dT"]
                used_odo += 1
        f.step(dT, cov)
        q = f.posterior_query()
        raw.append(err(q["map_pose"], k))
        if k % 20 == 0:
            log("frame %d: raw error %.3f m %.2f deg" % (k, raw[-1][0], raw[-1][1]))
        smooth.append(err(sm.push(q["map_pose"], dT), k))
        if len(scan):
            n_prev = len(scan)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    def first_ok(errs, start):
        for k in range(start, len(errs)):
            if all(e[0] < 0.5 and e[1] < 5.0 for e in errs[k:min(k + 3, len(errs))]):
                return k
        return None

    conv = first_ok(raw, 0)
    rec = first_ok(raw, occl[1])
    # frames scored: after the first convergence, outside the blocked frames and
    # the raw estimate's recovery gap (the same frames for both series)
    scored = [k for k in range(frames) if conv is not None and k >= conv and
              not (occl[0] <= k < (rec if rec is not None else frames))]

    def summary(errs):
        if not scored:
            return None
        em = np.array([errs[k][0] for k in scored])
        ed = np.array([errs[k][1] for k in scored])
        return {"ate_m": float(np.sqrt(np.mean(em ** 2))), "ate_deg": float(np.sqrt(np.mean(ed ** 2))),
                "median_m": float(np.median(em)), "median_deg": float(np.median(ed)),
                "frames_off_mode": int(np.sum(em > 1.0)),
                "ate_m_on_mode": float(np.sqrt(np.mean(em[em <= 1.0] ** 2))) if np.any(em <= 1.0) else None,
                "recovered_frame": first_ok(errs, occl[1])}

    raw_s, sm_s = summary(raw), summary(smooth)
    res = {"metric": "global localisation, occlusion and kidnap recovery (%s, %d particles)" % (args.scene,
                                                                                                 cfg["particles"]),
           "value": sm_s["ate_m"] if sm_s else None, "unit": "m ATE (smoothed representative pose)", "n_gpus": 1,
           "steps": frames, "warmup": 0, "ms_per_step": 1e3 * dt / frames, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "%s: %d particles x %d scan points x %d SVGD iterations, %d frames, "
                                  "uniform start, scans blocked for frames %d..%d, %.0f m kidnap at frame %d" %
                                  (args.scene, cfg["particles"], len(w["scans"][0]), cfg["svgd_iters"], frames,
                                   occl[0], occl[1] - 1, cfg["kidnap_dist"], kid),
                      "variant": args.variant, "variant_params": VARIANTS[args.variant],
                      "map": args.map, "map_gaussians": info["num_gauss"], "d_max": dmax},
           "converged_frame": conv, "scans_return_frame": occl[1], "scored_frames": len(scored),
           "raw": raw_s, "smoothed": sm_s, "frames_with_scan_odometry": used_odo,
           "per_frame_error_raw": raw, "per_frame_error_smoothed": smooth}
    f.close()
    sm.close()
    print(json.dumps(res), flush=True)


LAYOUT_NAMES = {0: "auto", 1: "particle", 2: "grouped"}


def batch_leg(M, S, steps, warmup, scorers=("plain",), log_fn=None):
    """The batched serving shape: 32 independent filters on 4 scenes (2 room-type
    maps of 200k points, 2 floor-type maps of 2M points, 0.5 m voxels), N
    log-uniform in [4096, 262144], scans of 1024..8192 points, 10 / 20 SVGD
    iterations, stepped by one graph replay per step (the likelihood passes of
    every iteration as one persistent tile-queue launch); the same instances
    stepped one by one for reference.  With "surrogate" in `scorers` the same
    32 instances run again with the network scorer (one untrained network per
    scene: its cost does not depend on the weights)."""
    import torch
    rng = np.random.default_rng(5000)
    scenes = []
    t0 = time.perf_counter()
    for j, (kind, seed) in enumerate((("room", 5001), ("room", 5002), ("floor", 5003), ("floor", 5004))):
        sc = S.scene_room(seed) if kind == "room" else S.scene_floor(seed)
        xyz = S.sample_map(sc, 200_000 if kind == "room" else 2_000_000, seed + 100)
        r = np.random.default_rng(seed + 200)
        pos = S.random_free_point(sc, r)
        scan = S.make_scan(sc, S.random_rotation(r), pos, 8192, 0.02 if kind == "room" else 0.03, seed + 300)
        m = M.Map(torch.from_numpy(xyz).cuda(), voxel=0.5)
        scenes.append(dict(kind=kind, scene=sc, map=m, scan=scan))
    if log_fn:
        log_fn("batch scenes built in %.1f s" % (time.perf_counter() - t0))
    n_inst = 32
    Ns = np.exp(rng.uniform(np.log(4096), np.log(262144), n_inst)).astype(np.int64)
    NSs = rng.integers(1024, 8193, n_inst)
    out = {"config": {"workload": "batch: 32 filters on 2 room-type (200k points) and 2 floor-type (2M points) "
                                  "maps, N log-uniform 4096..262144 (sum %d), scans 1024..8192 points, 10 / 20 "
                                  "SVGD iterations" % int(Ns.sum())},
           "particles": [int(v) for v in Ns], "scan_points": [int(v) for v in NSs]}
    for scorer in scorers:
        surs = [M.Surrogate(sd["map"], M.mp_surrogate_default_params(seed=31 + j)) for j, sd in enumerate(scenes)] \
            if scorer == "surrogate" else None
        filters = []
        for i in range(n_inst):
            sd = scenes[i % 4]
            iters = 10 if sd["kind"] == "room" else 20
            p = M.mp_filter_default_params(n_particles=int(Ns[i]), k=8 if sd["kind"] == "room" else 16,
                                           lsh_bits=16 if sd["kind"] == "room" else 20, svgd_iters=iters,
                                           post_iters=10, window_c=16 if sd["kind"] == "room" else 32, d_max=1.0,
                                           seed=6000 + i,
                                           scorer=M.MP_SCORER_SURROGATE if surs else M.MP_SCORER_PLAIN)
            f = M.Filter(sd["map"], p, box=(sd["scene"].lo, sd["scene"].hi))
            if surs:
                f.set_surrogate(surs[i % 4])
            f.scan_upload(np.ascontiguousarray(sd["scan"][:int(NSs[i])]))
            filters.append(f)
        b = M.Batch(filters, autotune=True)
        for k in range(warmup):
            b.step()
        torch.cuda.synchronize()
        info = b.info()
        evals = info["evals_per_step"]
        t0 = time.perf_counter()
        for k in range(steps):
            b.step()
        torch.cuda.synchronize()
        t_graph = (time.perf_counter() - t0) / steps
        t0 = time.perf_counter()
        for k in range(steps):
            for f in filters:
                f.step()
        torch.cuda.synchronize()
        t_seq = (time.perf_counter() - t0) / steps
        out[scorer] = {"evals_per_s": evals / t_graph, "graph_step_ms": 1e3 * t_graph,
                       "sequential_step_ms": 1e3 * t_seq, "speedup_vs_sequential": t_seq / t_graph,
                       "evals_per_step": evals, "instances_in_queue": info["queued_instances"],
                       "queue_gather_batch": info["queue_batch"], "queue_workgroups": info["queue_workgroups"],
                       "queue_tiles_per_step": info["queue_tiles_per_step"],
                       "lik_layout": [LAYOUT_NAMES.get(v, str(v)) for v in info["lik_layout"]],
                       "captures": info["captures"]}
        if log_fn:
            log_fn("batch %s: %.1f ms per graph step, %.3g evals/s (%.1f ms stepped one by one)" % (
                scorer, 1e3 * t_graph, evals / t_graph, 1e3 * t_seq))
        b.close()
        for f in filters:
            if surs:
                f.set_surrogate(None)
            f.close()
        if surs:
            for su in surs:
                su.close()
    for sd in scenes:
        sd["map"].close()
    return out


def batch_main(args):
    """The batched serving shape with both scorers (see batch_leg)."""
    import torch
    from paper_2404_16370_amd import megapf as M
    from paper_2404_16370_amd import synth as S
    torch.cuda.set_device(0)
    leg = batch_leg(M, S, args.steps, args.warmup, scorers=("plain", "surrogate"), log_fn=log)
    res = {"metric": "batched multi-instance filter steps: particle-point evals/s across 32 instances",
           "value": leg["plain"]["evals_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": leg["plain"]["graph_step_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": leg["config"],
           "plain": leg["plain"], "surrogate": leg["surrogate"],
           "surrogate_vs_plain": leg["surrogate"]["evals_per_s"] / leg["plain"]["evals_per_s"],
           "particles": leg["particles"], "scan_points": leg["scan_points"]}
    print(json.dumps(res), flush=True)


def _rot_angle_deg(q_a, q_b):
    """angle between unit quaternions (w, x, y, z), degrees"""
    d = np.abs(np.sum(np.asarray(q_a, np.float64) * np.asarray(q_b, np.float64), axis=-1))
    return np.degrees(2.0 * np.arccos(np.clip(d, 0.0, 1.0)))


def surrogate_eval_main(args):
    """Quality of the learned surrogate on the floor workload (60 x 60 x 8 m,
    2M map points, 0.5 m voxels): held-out score error, pose error of
    65,536-particle filters with the plain, score-field and network scorers,
    convergence basin of single Gauss-Newton particles, mode recall, and the
    weight footprint against the map's."""
    import torch
    from paper_2404_16370_amd import megapf as M
    from paper_2404_16370_amd import synth as S
    torch.cuda.set_device(0)
    frames = args.frames
    w = S.build_workload("floor", frames=frames)
    m = M.Map(torch.from_numpy(w["map_xyz"]).cuda(), voxel=0.5)
    minfo = m.info()
    lo, hi = w["scene"].lo, w["scene"].hi
    L = max(minfo["box_max"][a] - minfo["box_min"][a] for a in range(3))
    sur = M.Surrogate(m, M.mp_surrogate_default_params(seed=5002, total_steps=args.train_steps, sigma_s=args.sigma_s,
                                                       lr=args.lr, f_max=args.fmax_scale * L / 0.5))
    xyz = S.surrogate_samples(w["map_xyz"], minfo["box_min"], minfo["box_max"], 4_000_000, 5006)
    n_hold = len(xyz) // 20
    hold, train = xyz[:n_hold], xyz[n_hold:]
    sur.set_data(torch.from_numpy(train).cuda())
    t0 = time.perf_counter()
    losses = []
    done = 0
    while done < args.train_steps:
        k = min(2000, args.train_steps - done)
        losses.extend(sur.train(k).tolist())
        done += k
        log("trained %d / %d steps, loss %.4g" % (done, args.train_steps, losses[-1]))
    t_train = time.perf_counter() - t0
    lab = sur.label(hold)          # residual field (r, grad r)
    pred = sur.eval(hold)
    r_out = sur.info()["r_scale"]
    dr = np.abs(pred[:, 0] - lab[:, 0])
    gate = lab[:, 0] < r_out                       # inside the gate
    near = gate & (lab[:, 0] ** 2 < 9.0)           # below saturation
    gl, gp = lab[gate, 1:].astype(np.float64), pred[gate, 1:].astype(np.float64)
    cosang = np.sum(gl * gp, 1) / (np.linalg.norm(gl, axis=1) * np.linalg.norm(gp, axis=1) + 1e-30)
    ang = np.degrees(np.arccos(np.clip(cosang, -1, 1)))
    ds = np.abs(np.minimum(pred[:, 0].astype(np.float64) ** 2, 9.0) - np.minimum(lab[:, 0].astype(np.float64) ** 2, 9.0))
    quality = {"heldout_points": int(n_hold), "abs_dr_mean": float(dr.mean()), "abs_dr_p90": float(np.percentile(dr, 90)),
               "abs_dr_mean_below_saturation": float(dr[near].mean()) if near.any() else None,
               "abs_ds_mean (s = min(r^2, c_max))": float(ds.mean()), "abs_ds_p90": float(np.percentile(ds, 90)),
               "grad_angle_deg_median": float(np.median(ang)), "grad_angle_deg_p90": float(np.percentile(ang, 90)),
               "train_steps": args.train_steps, "train_s": t_train, "loss_first": losses[0],
               "loss_last": float(np.mean(losses[-100:]))}

    # filters from the same uniform start, same odometry
    def run_filter(scorer, check=None):
        p = M.mp_filter_default_params(n_particles=65536, k=16, lsh_bits=20, svgd_iters=20, post_iters=10,
                                       window_c=32, d_max=1.0, seed=4002, scorer=scorer, sigma_s=args.sigma_s)
        f = M.Filter(m, p, box=(lo, hi))
        if scorer == M.MP_SCORER_SURROGATE:
            f.set_surrogate(sur)
        if check is not None:
            f.set_surrogate_check(*check)
        errs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(frames):
            dT, cov = w["odometry"][k]
            f.scan_upload(w["scans"][k])
            f.step(dT, cov)
            q = f.posterior_query()
            R, t = w["traj"][k]
            gt = S.pose8(R, t)
            errs.append((float(np.linalg.norm(q["map_pose"][4:7] - gt[4:7])),
                         float(_rot_angle_deg(q["map_pose"][:4], gt[:4]))))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        poses = f.debug_get("poses")
        post = f.debug_get("post").astype(np.float64)
        nbr = f.debug_get("nbr")
        q = f.posterior_query()
        if scorer == M.MP_SCORER_SURROGATE:
            f.set_surrogate(None)
        return dict(errors=errs, s_per_frame=dt / frames, poses=poses, post=post, nbr=nbr,
                    fallback_steps=q["fallback_steps"], checks=q["sur_checks"], last_check_ds=q["sur_check_ds"])

    # the network alone, and with its check against the exact field every 10
    # frames on 1% of the particles (fallback to PLAIN for 10 frames when the
    # mean |delta s| exceeds 0.5)
    runs = {name: run_filter(sc, ck) for name, sc, ck in (("plain", M.MP_SCORER_PLAIN, None),
                                                          ("scorefield", M.MP_SCORER_SCOREFIELD, None),
                                                          ("surrogate", M.MP_SCORER_SURROGATE, None),
                                                          ("surrogate_checked", M.MP_SCORER_SURROGATE,
                                                           (10, 100, 0.5, 10)))}
    for name, r in runs.items():
        log("%s: final error %.3f m %.2f deg, %.3f s/frame" % (name, r["errors"][-1][0], r["errors"][-1][1],
                                                             r["s_per_frame"]))

    def modes(r):
        post, nbr = r["post"], r["nbr"]
        nb = np.where(nbr >= 0, nbr, np.arange(nbr.shape[1])[None, :])
        is_mode = (post >= 1e-3) & np.all(post[None, :] >= post[nb], axis=0)
        return r["poses"][is_mode]

    mp_, ms_ = modes(runs["plain"]), modes(runs["surrogate"])
    hit = 0
    for P in mp_:
        if len(ms_) == 0:
            break
        dt_ = np.linalg.norm(ms_[:, 4:7] - P[4:7], axis=1)
        da = _rot_angle_deg(ms_[:, :4], P[None, :4])
        hit += bool(np.any((dt_ <= 0.25) & (da <= 5.0)))
    recall = hit / len(mp_) if len(mp_) else None

    # convergence basin: independent Gauss-Newton particles (K = 1) around the truth
    R0, t0_ = w["traj"][0]
    gt0 = S.pose8(R0, t0_)
    rng = np.random.default_rng(7)
    nb_ = 2000
    dist = rng.uniform(0.5, 3.0, nb_)
    angd = rng.uniform(5.0, 30.0, nb_)
    dirs = rng.normal(size=(nb_, 3)); dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    axes = rng.normal(size=(nb_, 3)); axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    start = np.zeros((nb_, 8), np.float32)
    for i in range(nb_):
        Rp = S.rotvec_to_mat(axes[i] * np.radians(angd[i])) @ R0
        start[i] = S.pose8(Rp, t0_ + dirs[i] * dist[i])
    basin = {}
    for name, sc in (("plain", M.MP_SCORER_PLAIN), ("scorefield", M.MP_SCORER_SCOREFIELD),
                     ("surrogate", M.MP_SCORER_SURROGATE)):
        p = M.mp_filter_default_params(n_particles=nb_, k=1, lsh_bits=8, svgd_iters=30, post_iters=0, window_c=0,
                                       d_max=1.0, seed=4012, scorer=sc, sigma_s=args.sigma_s)
        f = M.Filter(m, p, poses=start)
        if sc == M.MP_SCORER_SURROGATE:
            f.set_surrogate(sur)
        f.scan_upload(w["scans"][0])
        f.step()
        P = f.debug_get("poses")
        et = np.linalg.norm(P[:, 4:7] - gt0[4:7], axis=1)
        ea = _rot_angle_deg(P[:, :4], gt0[None, :4])
        basin[name] = float(np.mean((et < 0.1) & (ea < 2.0)))
        if sc == M.MP_SCORER_SURROGATE:
            f.set_surrogate(None)
    fin = {k: r["errors"][-1] for k, r in runs.items()}
    res = {"metric": "surrogate quality on the floor workload (final pose error, held-out score error)",
           "value": fin["surrogate"][0], "unit": "m", "n_gpus": 1, "steps": frames, "warmup": 0,
           "ms_per_step": 1e3 * runs["surrogate"]["s_per_frame"], "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16 network, f32 filter", "data": "synthetic",
           "config": {"workload": "floor: 65536 particles x 4096 scan points x 20 SVGD iterations, %d frames, "
                                  "2M map points at 0.5 m voxels; network trained on 3.8M of 4M samples" % frames,
                      "sigma_s": args.sigma_s, "lr": args.lr, "f_max": args.fmax_scale * L / 0.5},
           "final_error_m_deg": fin,
           "added_error_vs_plain": {"m": fin["surrogate"][0] - fin["plain"][0],
                                    "deg": fin["surrogate"][1] - fin["plain"][1]},
           "gate": {"added_error_max_m": 0.05, "added_error_max_deg": 0.5,
                    "network_alone_passed": bool(fin["surrogate"][0] - fin["plain"][0] <= 0.05 and
                                                 fin["surrogate"][1] - fin["plain"][1] <= 0.5),
                    "checked_passed": bool(fin["surrogate_checked"][0] - fin["plain"][0] <= 0.05 and
                                           fin["surrogate_checked"][1] - fin["plain"][1] <= 0.5),
                    "checked_ran_network_frames": frames - int(runs["surrogate_checked"]["fallback_steps"])},
           "checked": {"added_error_vs_plain": {"m": fin["surrogate_checked"][0] - fin["plain"][0],
                                                "deg": fin["surrogate_checked"][1] - fin["plain"][1]},
                       "fallback_frames": runs["surrogate_checked"]["fallback_steps"],
                       "checks": runs["surrogate_checked"]["checks"],
                       "last_check_mean_abs_ds": runs["surrogate_checked"]["last_check_ds"]},
           "per_frame_errors": {k: r["errors"] for k, r in runs.items()},
           "s_per_frame": {k: r["s_per_frame"] for k, r in runs.items()},
           "heldout": quality, "mode_recall": recall, "modes_plain": int(len(mp_)), "modes_surrogate": int(len(ms_)),
           "basin_fraction": basin,
           "footprint_bytes": {"network_image": sur.info()["weight_bytes"], "map": minfo["device_bytes"]}}
    sur.close()
    print(json.dumps(res), flush=True)


VARIANTS = {
    "default": {},
    "lsh_tangent_se3": {"lsh_tangent": 1},
    "lsh_tables_2": {"lsh_tables": 2},
    "svgd_grad_exact": {"svgd_grad": 1},
    "svgd_transport_adjoint": {"svgd_transport": 1},
    "svgd_exact_and_adjoint": {"svgd_grad": 1, "svgd_transport": 1},
}


def variants_leg(M, m, wl, minfo, scans, odo, warmup=1, steps=1):
    """One full-size filter step per accuracy variant of the neighbour search
    and the Stein update (same map, scans and seed); stage times of the last
    step, and the SVGD kernel against its HBM roofline."""
    import torch
    n, K, it = wl["particles"], wl["k"], wl["svgd_iters"]
    svgd_bytes = (28.0 + 8 * K + 56.0 * K + 28.0) * n * it   # algorithmic bytes, neighbour gathers included
    out = {}
    for name, kw in VARIANTS.items():
        p = M.mp_filter_default_params(n_particles=n, k=K, lsh_bits=wl["lsh_bits"], svgd_iters=it,
                                       post_iters=wl["post_iters"], window_c=wl["window_c"], d_max=2.0 * wl["voxel"],
                                       seed=4003, **kw)
        f = M.Filter(m, p, box=(minfo["box_min"], minfo["box_max"]))
        ms = []
        for k in range(warmup + steps):
            dT, cov = odo[k] if k > 0 else (None, None)
            f.scan_upload(scans[k])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            f.step(dT, cov)
            e1.record()
            torch.cuda.synchronize()
            if k >= warmup:
                ms.append(e0.elapsed_time(e1))
        st = f.stage_times()
        sv = st["svgd"][0]
        out[name] = {"params": kw, "step_ms": round(float(np.median(ms)), 3),
                     "stage_ms": {k: round(st[k][0], 3) for k in ("lsh", "sort", "refresh", "svgd")},
                     "svgd_hbm_frac": round(svgd_bytes / PEAK_HBM / (sv * 1e-3), 4) if sv > 0 else None}
        f.close()
        torch.cuda.synchronize()
        log("variant %s: %.1f ms per step" % (name, out[name]["step_ms"]))
    return out


def svgd_refresh_bytes(K):
    """compulsory bytes per particle and launch: SVGD reads K neighbour ids and
    kernel values, its own pose and psi, writes its pose; the refresh reads its
    sorted slot, bucket bounds, pose and old list, writes list, kernel values
    and count"""
    return 8.0 * K + 96.0, 48.0 + 12.0 * K


def point_map_leg(M, xyz, wl, scans, odo, cell=0.2, radius=5, warmup=1, steps=2):
    """The same filter step on the paper's own map: one Gaussian per map point
    (10 nearest neighbours within 2 voxels), a dense nearest-point field of
    `cell` m cells covering radius * cell around the map (the inlier gate d_max
    set to that coverage).  Build time and bytes, step and likelihood times."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pm = M.Map(xyz, voxel=cell, nnf_radius=radius, min_points=5, gauss_mode=M.MP_GAUSS_POINT, point_k=10,
               point_search=2)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = pm.info()
    log("per-point map built in %.2f s: %s" % (t_build, info))
    dmax = radius * cell
    p = M.mp_filter_default_params(n_particles=wl["particles"], k=wl["k"], lsh_bits=wl["lsh_bits"],
                                   svgd_iters=wl["svgd_iters"], post_iters=wl["post_iters"],
                                   window_c=wl["window_c"], d_max=dmax, seed=4003)
    f = M.Filter(pm, p, box=(info["box_min"], info["box_max"]))
    ms, lik, nlik = [], [], []
    for k in range(warmup + steps):
        dT, cov = odo[k] if k > 0 else (None, None)
        f.scan_upload(scans[k])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        f.step(dT, cov)
        e1.record()
        torch.cuda.synchronize()
        if k >= warmup:
            st = f.stage_times()
            ms.append(e0.elapsed_time(e1))
            lik.append(st["likelihood_core"][0])
            nlik.append(st["likelihood_core"][1])
    psi = f.debug_get("psi")
    inl = float(psi[:, 7].astype(np.float64).sum()) / (float(wl["particles"]) * wl["scan_points"])
    f.close()
    pm.close()
    torch.cuda.synchronize()
    return {"cell_m": cell, "nnf_radius": radius, "d_max": dmax, "build_s": round(t_build, 3),
            "num_gauss": info["num_gauss"], "field_cells": info["table_slots"], "band_cells": info["num_band"],
            "device_bytes": info["device_bytes"], "step_ms": round(float(np.median(ms)), 3),
            "likelihood_launch_ms": round(sum(lik) / max(sum(nlik), 1), 3), "inlier_fraction": round(inl, 4)}


def _med_p90(v):
    a = np.asarray(v, np.float64)
    return {"median_ms": round(float(np.median(a)), 3), "p90_ms": round(float(np.percentile(a, 90)), 3),
            "n": int(a.size)}


def stage_roofline(stages, wl, lik_flops_launch, t_step):
    """Each stage of one filter step against the resource that bounds it.
    `frac` takes the algorithmic bytes per particle: what the method must
    move, neighbour gathers included (prediction 56 B per
    frame; LSH 36 B; sort 16 B per 8-bit pass + 12 B of bucket bounds;
    refresh 28 + 4K + 32C + 32K + 8K; SVGD 28 + 8K + 56K; posterior 20 + R
    (12K + 4)).  A fraction above 1 means the caches serve the gathers.
    `frac_compulsory` takes the bytes each launch must move once, gathers
    counted once.  The likelihood and the scan k-NN are set against the FP32
    peak.  `step` sums the stages' roofline times over the measured step time."""
    n, it, K, C, R = wl["particles"], wl["svgd_iters"], wl["k"], wl["window_c"], wl["post_iters"]
    ns, passes = wl["scan_points"], (wl["lsh_bits"] + 7) // 8
    svgd_c, refresh_c = svgd_refresh_bytes(K)
    work = {
        "predict": ("hbm", 56.0 * n, 64.0 * n),
        "lsh": ("hbm", 36.0 * n * it, 44.0 * n * it),
        "sort": ("hbm", (16.0 * passes + 12.0) * n * it, (16.0 * passes + 12.0) * n * it),
        "refresh": ("hbm", (28.0 + 4 * K + 32.0 * C + 32.0 * K + 8 * K) * n * it, refresh_c * n * it),
        "likelihood": ("alu", lik_flops_launch * it, lik_flops_launch * it),
        "svgd": ("hbm", (28.0 + 8 * K + 56.0 * K + 28.0) * n * it, svgd_c * n * it),
        "posterior": ("hbm", (20.0 + R * (12.0 * K + 4)) * n, (36.0 + R * (8.0 * K + 8)) * n),
        "scan": ("alu", 8.0 * ns * (ns - 1), 8.0 * ns * (ns - 1)),
    }
    out, t_min = {}, 0.0
    for name, (bound, w, wc) in work.items():
        ms = stages.get(name, (0.0, 0))[0]
        peak = PEAK_HBM if bound == "hbm" else PEAK_FP32
        t = w / peak
        t_min += t
        if ms > 0:
            out[name] = {"bound": bound, "ms": round(ms, 3), "roofline_ms": round(1e3 * t, 4),
                         "frac": round(t / (ms * 1e-3), 4), "frac_compulsory": round(wc / peak / (ms * 1e-3), 4)}
    out["step"] = {"roofline_ms": round(1e3 * t_min, 3), "ms": round(1e3 * t_step, 3),
                   "frac": round(t_min / t_step, 4)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="campus",
                    choices=sorted(WORKLOADS) + ["batch", "surrogate-eval", "sequence"])
    ap.add_argument("--frames", type=int, default=50, help="surrogate-eval: filter frames")
    ap.add_argument("--seq-frames", type=int, default=0, help="sequence: frames (0: the scene's default)")
    ap.add_argument("--scene", default="floor", choices=["floor", "campus"], help="sequence: scene")
    ap.add_argument("--kidnap-frame", type=int, default=0,
                    help="sequence: frame of the teleport (0: the scene's default); the blocked frames move with it")
    ap.add_argument("--train-steps", type=int, default=20000, help="surrogate-eval: Adam steps")
    ap.add_argument("--sigma-s", type=float, default=0.03, help="surrogate-eval: sensor std of the score field")
    ap.add_argument("--lr", type=float, default=1e-3, help="surrogate-eval: Adam step")
    ap.add_argument("--fmax-scale", type=float, default=1.0, help="surrogate-eval: f_max in units of L / voxel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate scorer and training legs")
    ap.add_argument("--surrogate-steps", type=int, default=1)
    ap.add_argument("--variant", default="default", choices=sorted(VARIANTS),
                    help="sequence: LSH / SVGD accuracy variant of the filter")
    ap.add_argument("--no-point-map", action="store_true",
                    help="skip the leg on the map of per-point Gaussians (0.2 m nearest-point field)")
    ap.add_argument("--map", default="voxel", choices=["voxel", "point"],
                    help="sequence: per-voxel Gaussians (0.5 m) or per-point Gaussians (0.1 m field)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the leg timing the LSH tangent / tables and SVGD gradient / transport variants")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the leg stepping 32 filters of the batched serving shape (plain scorer)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy before timing (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X "
              "(sharding over several GPUs is designed, not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return batch_main(args)
    if args.workload == "surrogate-eval":
        return surrogate_eval_main(args)
    if args.workload == "sequence":
        return sequence_main(args)
    import torch
    from paper_2404_16370_amd import megapf as M
    from paper_2404_16370_amd import synth as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = WORKLOADS[args.workload]
    nframes = max(args.warmup + args.steps, 1 + args.surrogate_steps) + 1
    t0 = time.perf_counter()
    w = S.build_workload(args.workload, map_points=wl["map_points"], scan_points=wl["scan_points"],
                         frames=max(nframes, 2))
    log("workload generated in %.1f s (%d map points, %d frames)" % (time.perf_counter() - t0,
                                                                      len(w["map_xyz"]), len(w["scans"])))
    t0 = time.perf_counter()
    xyz = torch.from_numpy(w["map_xyz"]).cuda()
    m = M.Map(xyz, voxel=wl["voxel"], nnf_radius=2, min_points=5)
    torch.cuda.synchronize()
    minfo = m.info()
    log("map built in %.2f s: %s" % (time.perf_counter() - t0, minfo))

    p = M.mp_filter_default_params(n_particles=wl["particles"], k=wl["k"], lsh_bits=wl["lsh_bits"],
                                   svgd_iters=wl["svgd_iters"], post_iters=wl["post_iters"],
                                   window_c=wl["window_c"], d_max=2.0 * wl["voxel"], seed=4003)
    f = M.Filter(m, p, box=(minfo["box_min"], minfo["box_max"]))
    scans = [torch.from_numpy(np.ascontiguousarray(s)).cuda() for s in w["scans"]]
    odo = w["odometry"]
    torch.cuda.synchronize()

    def run(k):
        dT, cov = odo[k] if k > 0 else (None, None)
        f.scan_upload(scans[k])
        f.step(dT, cov)

    if args.copy_calibration:
        # plain elementwise kernel reading 1 GiB and writing 1 GiB (reference for byte counters)
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        torch.cuda.synchronize()
        dst = src * 2.0
        torch.cuda.synchronize()
        del src, dst
    for k in range(args.warmup):
        run(k)
        log("warmup step %d done" % k)
    torch.cuda.synchronize()
    lik_ms, lik_n, up_ms, step_ms = [], [], [], []
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        dT, cov = odo[k] if k > 0 else (None, None)
        e0.record()
        f.scan_upload(scans[k])
        e1.record()
        f.step(dT, cov)
        e2.record()
        st = f.stage_times()   # synchronises on this step's events
        lik_ms.append(st["likelihood_core"][0])
        lik_n.append(st["likelihood_core"][1])
        up_ms.append(e0.elapsed_time(e1))
        step_ms.append(e1.elapsed_time(e2))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = f.stage_times()
    q = f.posterior_query(weights=True)
    psi = f.debug_get("psi")
    inl = psi[:, 7].astype(np.float64).sum()
    ns = wl["scan_points"]
    n = wl["particles"]
    evals_iter = float(n) * ns
    inl_frac = inl / evals_iter
    t_launch = (sum(lik_ms) / max(sum(lik_n), 1)) * 1e-3
    flops_launch = evals_iter * (inl_frac * FLOPS_INLIER + (1 - inl_frac) * FLOPS_OUTLIER)
    achieved = flops_launch / t_launch
    steps_per_s = args.steps / elapsed
    evals_per_s = steps_per_s * evals_iter * wl["svgd_iters"]
    res = {
        "metric": METRIC,
        "value": round(steps_per_s, 4),
        "unit": "filter steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %d particles x %d scan points x %d SVGD iterations per step, %d map points "
                               "at %.1f m voxels, K=%d, %d LSH bits" %
                               (args.workload, n, ns, wl["svgd_iters"], wl["map_points"], wl["voxel"], wl["k"],
                                wl["lsh_bits"]),
                   "particles": n, "scan_points": ns, "svgd_iters": wl["svgd_iters"], "scorer": "plain"},
        "evals_per_s": evals_per_s,
        "likelihood_kernel_evals_per_s": evals_iter / t_launch,
        "inlier_fraction": round(inl_frac, 4),
        "stage_ms_last_step": {k: round(v[0], 3) for k, v in stages.items() if v[1]},
        "step_ms_events": {"with_scan_upload": _med_p90([a + b for a, b in zip(up_ms, step_ms)]),
                           "without_scan_upload": _med_p90(step_ms), "scan_upload": _med_p90(up_ms)},
        "stage_roofline": stage_roofline(stages, wl, flops_launch, elapsed / args.steps),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": measured_traffic(args.workload),
                     "kernel": "k_lik_grp (grouped layout)", "launch_ms": t_launch * 1e3,
                     "logical_gather_GBps": evals_iter * GATHER_BYTES / t_launch / 1e9,
                     "logical_gather_frac_of_hbm": evals_iter * GATHER_BYTES / t_launch / PEAK_HBM,
                     "flops_per_eval": {"kernel_inlier": FLOPS_INLIER, "kernel_outlier": FLOPS_OUTLIER,
                                        "algorithmic": FLOPS_ALGORITHMIC},
                     "frac_at_algorithmic_flops": evals_iter * FLOPS_ALGORITHMIC / t_launch / PEAK_FP32},
        "posterior": {"map_weight": q["map_weight"], "n_eff": q["n_eff"], "sum_w": float(q["weights"].sum())},
        "paper_context": {"filter_steps_per_s": round(1000.0 / 90.8, 2), "hardware": "NVIDIA A100",
                          "note": "the paper's 1,048,576-particle indoor run (90.8 ms per frame); its scan size and "
                                  "iterations per frame are not stated, so it is context, not a baseline"},
    }
    if not args.no_surrogate:
        res["surrogate"] = surrogate_leg(M, m, wl, minfo, scans, odo, 1, args.surrogate_steps)
        res["surrogate"]["vs_plain"] = res["surrogate"]["steps_per_s"] / steps_per_s
        res["surrogate_training"] = train_leg(M, S, m, w, minfo)
    if not args.no_variants:
        f.close()
        res["variants"] = variants_leg(M, m, wl, minfo, scans, odo)
    if not args.no_point_map:
        f.close()
        res["map_per_voxel"] = {"voxel_m": wl["voxel"], "num_gauss": minfo["num_gauss"],
                                "device_bytes": minfo["device_bytes"], "d_max": 2.0 * wl["voxel"]}
        res["map_per_point"] = point_map_leg(M, xyz, wl, scans, odo)
    res["odometry"] = odometry_leg(M, m, w, scans, not args.no_cpu_baseline)
    if not args.no_batch:
        f.close()
        res["batch"] = batch_leg(M, S, 2, 1, scorers=("plain",), log_fn=log)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, w, w["scans"][-1], args.cpu_budget)
    print(json.dumps(res), flush=True)


def log_children():
    """Processes this run started that are still alive at its end (none are
    expected): named on stderr so that a leftover can be traced."""
    try:
        import psutil
        kids = psutil.Process().children(recursive=True)
    except Exception:
        return
    for k in kids:
        try:
            log("child process still alive at exit: pid %d %s" % (k.pid, " ".join(k.cmdline())[:200]))
        except Exception:
            pass
    if not kids:
        log("no child processes alive at exit")


if __name__ == "__main__":
    main()
    log_children()
