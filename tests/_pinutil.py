"""Independent FP64 references used only to pin the oracle: matrix
exponential/logarithm from scipy, plain numpy statistics.  None of this is
shared with the oracle or the GPU path."""
import numpy as np
from scipy.linalg import expm, logm
from scipy.spatial.transform import Rotation


def quat_wxyz_to_R(q):
    q = np.asarray(q, np.float64)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def pose_to_M(T):
    M = np.eye(4)
    M[:3, :3] = quat_wxyz_to_R(T[:4])
    M[:3, 3] = np.asarray(T[4:7], np.float64)
    return M


def hat(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0.0]])


def twist_M(xi):
    M = np.zeros((4, 4))
    M[:3, :3] = hat(xi[:3])
    M[:3, 3] = xi[3:]
    return M


def se3_log_ref(M):
    L = np.real(logm(M))
    return np.array([L[2, 1], L[0, 2], L[1, 0], L[0, 3], L[1, 3], L[2, 3]])


def se3_exp_ref(xi):
    return expm(twist_M(np.asarray(xi, np.float64)))


def between_ref(Ti, Tj):
    return se3_log_ref(np.linalg.inv(pose_to_M(Ti)) @ pose_to_M(Tj))


def M_to_pose8(M):
    q = Rotation.from_matrix(M[:3, :3]).as_quat()
    out = np.zeros(8, np.float32)
    out[:4] = [q[3], q[0], q[1], q[2]]
    if out[0] < 0:
        out[:4] *= -1
    out[4:7] = M[:3, 3]
    return out


def random_pose8(rng, tscale=5.0, rot=np.pi):
    R = Rotation.from_rotvec(rng.normal(size=3) * rot / 2).as_matrix()
    M = np.eye(4)
    M[:3, :3] = R
    M[:3, 3] = rng.normal(size=3) * tscale
    return M_to_pose8(M)
