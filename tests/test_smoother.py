"""Smoothing of the representative pose (mp_smoother_*, Sec. IV-A): host
logic, exercised through the C-ABI without a GPU.

  * a constant pose is returned unchanged;
  * on an exact constant-velocity path with the true increments every
    carried pose equals the newest, so the output is the newest pose;
  * noisy poses along a path (true increments) come out closer to the truth
    than they went in, by about the square root of the window;
  * poses beyond the jump thresholds are held back (the output stays on the
    track) until switch_frames of them in a row agree, which then take over;
  * argument errors.
"""
import numpy as np
import pytest

from paper_2404_16370_amd import megapf as M
from paper_2404_16370_amd import synth as S


def _pose(R, t):
    return S.pose8(R, t)[:7].astype(np.float32)


def _compose(a, b):
    Ra, Rb = S.quat_to_mat(a[:4]), S.quat_to_mat(b[:4])
    return _pose(Ra @ Rb, a[4:7] + Ra @ b[4:7])


def _err(a, b):
    qa = a[:4] / np.linalg.norm(a[:4]); qb = b[:4] / np.linalg.norm(b[:4])
    return np.linalg.norm(a[4:7].astype(np.float64) - b[4:7]), 2 * np.arccos(min(1.0, abs(float(qa @ qb))))


def test_constant_pose():
    s = M.Smoother(window=5)
    P = _pose(S.rotvec_to_mat(np.array([0.1, -0.2, 0.3])), np.array([1.0, 2.0, 3.0]))
    I = np.array([1, 0, 0, 0, 0, 0, 0], np.float32)
    for _ in range(8):
        out = s.push(P, I)
        e = _err(out, P)
        assert e[0] < 1e-6 and e[1] < 1e-6


def test_constant_velocity_path_is_unchanged():
    s = M.Smoother(window=6)
    D = _pose(S.rotvec_to_mat(np.array([0.0, 0.0, 0.08])), np.array([0.5, 0.02, 0.0]))
    P = _pose(np.eye(3), np.array([3.0, -1.0, 0.5]))
    for k in range(12):
        if k:
            P = _compose(P, D)
        out = s.push(P, D if k else None)
        e = _err(out, P)
        assert e[0] < 1e-5 and e[1] < 1e-5


def test_noisy_path_is_smoothed():
    rng = np.random.default_rng(0)
    W = 9
    s = M.Smoother(window=W, jump_m=1.0, jump_rad=0.3)
    D = _pose(S.rotvec_to_mat(np.array([0.0, 0.01, 0.05])), np.array([0.4, 0.0, 0.01]))
    T = _pose(np.eye(3), np.zeros(3))
    raw, smooth = [], []
    for k in range(200):
        if k:
            T = _compose(T, D)
        noisy = _compose(T, _pose(S.rotvec_to_mat(rng.normal(0, 0.01, 3)), rng.normal(0, 0.05, 3)))
        out = s.push(noisy, D if k else None)
        if k >= W:
            raw.append(_err(noisy, T)[0])
            smooth.append(_err(out, T)[0])
    ratio = np.sqrt(np.mean(np.square(smooth)) / np.mean(np.square(raw)))
    assert ratio < 1.5 / np.sqrt(W)


def test_far_poses_are_held_back_until_they_persist():
    s = M.Smoother(window=5, jump_m=1.0, jump_rad=0.2, switch_frames=3)
    I = np.array([1, 0, 0, 0, 0, 0, 0], np.float32)
    A = _pose(np.eye(3), np.zeros(3))
    for _ in range(5):
        s.push(A, I)
    # single frames on other modes (far from the track and from each other) are held back
    for x in (20.0, -15.0, 20.0):
        assert _err(s.push(_pose(np.eye(3), np.array([x, 0.0, 0.0])), I), A)[0] < 1e-6
    # a persistent new location (a kidnap recovery) takes over on its third frame
    B = _pose(np.eye(3), np.array([20.0, 5.0, 0.0]))
    assert _err(s.push(B, I), A)[0] < 1e-6
    assert _err(s.push(B, I), A)[0] < 1e-6
    assert _err(s.push(B, I), B)[0] < 1e-6
    # a rotation jump counts as far too
    C = _pose(S.rotvec_to_mat(np.array([0.0, 0.0, 0.5])), np.array([20.0, 5.0, 0.0]))
    assert _err(s.push(C, I), B)[1] < 1e-6
    s1 = M.Smoother(window=5, switch_frames=1)   # switch_frames 1: every far pose restarts the track
    s1.push(A, I)
    assert _err(s1.push(C, I), C)[1] < 1e-6


def test_errors():
    with pytest.raises(M.MegaPFError):
        M.Smoother(window=0)
    with pytest.raises(M.MegaPFError):
        M.Smoother(jump_m=-1.0)
    with pytest.raises(M.MegaPFError):
        M.Smoother(switch_frames=0)
    s = M.Smoother()
    with pytest.raises(M.MegaPFError):
        s.push(np.array([0, 0, 0, 0, 0, 0, 0], np.float32))
    with pytest.raises(M.MegaPFError):
        s.push(np.array([1, 0, 0, 0, np.nan, 0, 0], np.float32))
    s.close()
