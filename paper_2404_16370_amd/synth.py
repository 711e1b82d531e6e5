"""Seeded synthetic scenes, scans, trajectories and particle sets.

Stand-ins for the range data the paper evaluates on (indoor Azure Kinect and
outdoor Livox sequences, Sec. IV), which are not available: analytic scenes
made of triangles, vertical cylinders and an optional heightfield ground; map
points sampled uniformly by area; scans by ray casting from a ground-truth
pose with Gaussian range noise.

This module only generates inputs.  It holds none of the filter's arithmetic,
is used both by the tests (for the GPU path and the CPU oracle alike) and by
the benchmark, and imports neither.

Workloads (sizes follow the five benchmark configurations):
  room    20x20x4 m room, 6 faces + 40 axis-aligned boxes, 200k map points,
          voxel 0.5 m, 1024-point scans (noise 0.02 m), 4096 particles
  floor   60x60x8 m floor, 30 polygonal rooms with door gaps, 300 boxes,
          50 cylinders, ~2M map points, voxel 0.5 m, 4096-point scans
          (noise 0.03 m), 65,536 particles, 0.5 m + 5 deg per frame
  campus  200x200x15 m, 120 extruded polygon buildings, Perlin ground
          (0.2 m amplitude), 2000 poles, ~20M map points, voxel 1.0 m,
          8192-point scans (noise 0.03 m), 1,048,576 particles, kidnap
          (80 m, 90 deg) at frame 100
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


# ---------------------------------------------------------------- rotations (input generation only)
def quat_to_mat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def mat_to_quat(R):
    tr = R[0, 0] + R[1, 1] + R[2, 2]
    if tr > 0:
        s = math.sqrt(tr + 1.0) * 2
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = math.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif R[1, 1] > R[2, 2]:
        s = math.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = math.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    q = np.array(q)
    q /= np.linalg.norm(q)
    if q[0] < 0:
        q = -q
    return q


def rotvec_to_mat(v):
    th = float(np.linalg.norm(v))
    if th < 1e-12:
        return np.eye(3)
    k = np.asarray(v) / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K


def rpy_to_mat(roll, pitch, yaw):
    cr, sr, cp, sp, cy, sy = (math.cos(roll), math.sin(roll), math.cos(pitch), math.sin(pitch),
                              math.cos(yaw), math.sin(yaw))
    Rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1]])
    Ry = np.array([[cp, 0, sp], [0, 1, 0], [-sp, 0, cp]])
    Rx = np.array([[1, 0, 0], [0, cr, -sr], [0, sr, cr]])
    return Rz @ Ry @ Rx


def random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    return quat_to_mat(q)


def pose8(R, t) -> np.ndarray:
    """(qw,qx,qy,qz,tx,ty,tz,0) float32 record."""
    out = np.zeros(8, np.float32)
    out[:4] = mat_to_quat(R)
    out[4:7] = t
    return out


def uniform_particles(n, lo, hi, seed) -> np.ndarray:
    """n poses with translation uniform in the box and rotation uniform on SO(3)."""
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    out = np.zeros((n, 8), np.float32)
    out[:, :4] = q
    out[:, 4:7] = rng.uniform(lo, hi, size=(n, 3))
    # renormalise in float32 so that |q| is as close to 1 as float32 allows
    qq = out[:, :4].astype(np.float64)
    out[:, :4] = (qq / np.linalg.norm(qq, axis=1, keepdims=True)).astype(np.float32)
    return out


def gaussian_particles(n, center8, sig_rot, sig_trans, seed) -> np.ndarray:
    """n poses scattered around a pose (right-perturbed by isotropic noise)."""
    rng = np.random.default_rng(seed)
    R0 = quat_to_mat(center8[:4].astype(np.float64))
    t0 = center8[4:7].astype(np.float64)
    out = np.zeros((n, 8), np.float32)
    for i in range(n):
        R = R0 @ rotvec_to_mat(rng.normal(scale=sig_rot, size=3))
        out[i] = pose8(R, t0 + rng.normal(scale=sig_trans, size=3))
    return out


# ---------------------------------------------------------------- Perlin noise (Perlin 2002, "Improving Noise")
class Perlin2D:
    def __init__(self, seed):
        rng = np.random.default_rng(seed)
        p = rng.permutation(256)
        self.p = np.concatenate([p, p]).astype(np.int64)

    @staticmethod
    def _fade(t):
        return t * t * t * (t * (t * 6 - 15) + 10)

    @staticmethod
    def _grad(h, x, y):
        # eight gradient directions
        g = h & 7
        u = np.where(g < 4, x, y)
        v = np.where(g < 4, y, x)
        return np.where(g & 1, -u, u) + np.where(g & 2, -2.0 * v, 2.0 * v) * 0.5

    def __call__(self, x, y):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        xi = np.floor(x).astype(np.int64)
        yi = np.floor(y).astype(np.int64)
        xf = x - xi
        yf = y - yi
        X = xi & 255
        Y = yi & 255
        u = self._fade(xf)
        v = self._fade(yf)
        p = self.p
        aa = p[p[X] + Y]
        ab = p[p[X] + Y + 1]
        ba = p[p[X + 1] + Y]
        bb = p[p[X + 1] + Y + 1]
        x1 = (1 - u) * self._grad(aa, xf, yf) + u * self._grad(ba, xf - 1, yf)
        x2 = (1 - u) * self._grad(ab, xf, yf - 1) + u * self._grad(bb, xf - 1, yf - 1)
        return (1 - v) * x1 + v * x2


# ---------------------------------------------------------------- scenes
@dataclass
class Scene:
    name: str
    lo: np.ndarray
    hi: np.ndarray
    tris: np.ndarray                       # (T,3,3)
    cyl: np.ndarray                        # (C,5): cx, cy, r, z0, z1
    polys: List[np.ndarray] = field(default_factory=list)   # solid footprints (buildings)
    poly_h: List[float] = field(default_factory=list)
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))  # solid boxes lo(3), hi(3)
    ground_amp: float = 0.0
    ground_scale: float = 10.0
    perlin: Optional[Perlin2D] = None
    sensor_z: tuple = (0.5, 3.5)

    def ground(self, x, y):
        if self.perlin is None:
            return np.zeros_like(np.asarray(x, np.float64))
        return self.ground_amp * self.perlin(np.asarray(x) / self.ground_scale, np.asarray(y) / self.ground_scale)


def _rect(p0, e1, e2):
    """two triangles of the parallelogram p0, p0+e1, p0+e1+e2, p0+e2"""
    p0 = np.asarray(p0, np.float64); e1 = np.asarray(e1, np.float64); e2 = np.asarray(e2, np.float64)
    a, b, c, d = p0, p0 + e1, p0 + e1 + e2, p0 + e2
    return [np.stack([a, b, c]), np.stack([a, c, d])]


def _box_tris(lo, hi):
    lo = np.asarray(lo, np.float64); hi = np.asarray(hi, np.float64)
    dx, dy, dz = hi - lo
    X, Y, Z = np.array([dx, 0, 0]), np.array([0, dy, 0]), np.array([0, 0, dz])
    t = []
    t += _rect(lo, X, Y) + _rect(lo + Z, X, Y)
    t += _rect(lo, X, Z) + _rect(lo + Y, X, Z)
    t += _rect(lo, Y, Z) + _rect(lo + X, Y, Z)
    return t


def _wall(a, b, z0, z1):
    a = np.array([a[0], a[1], z0]); b = np.array([b[0], b[1], z0])
    return _rect(a, b - a, np.array([0, 0, z1 - z0]))


def scene_room(seed=1001) -> Scene:
    rng = np.random.default_rng(seed)
    W, D, H = 20.0, 20.0, 4.0
    tris = _box_tris([0, 0, 0], [W, D, H])
    boxes = []
    for _ in range(40):
        s = rng.uniform(0.3, 2.0, size=3)
        c = rng.uniform([0.5, 0.5], [W - 0.5 - s[0], D - 0.5 - s[1]])
        lo = np.array([c[0], c[1], 0.0]); hi = lo + s
        boxes.append(np.concatenate([lo, hi]))
        tris += _box_tris(lo, hi)
    return Scene("room", np.array([0, 0, 0.0]), np.array([W, D, H]), np.array(tris), np.zeros((0, 5)),
                 boxes=np.array(boxes), sensor_z=(0.5, 3.5))


def _random_polygon(rng, center, rmin, rmax, nv):
    ang = np.sort(rng.uniform(0, 2 * np.pi, nv))
    # spread the angles so that no sector is degenerate
    ang = np.sort((ang + np.linspace(0, 2 * np.pi, nv, endpoint=False)) / 2.0 % (2 * np.pi))
    rad = rng.uniform(rmin, rmax, nv)
    return np.stack([center[0] + rad * np.cos(ang), center[1] + rad * np.sin(ang)], axis=1)


def scene_floor(seed=1002) -> Scene:
    rng = np.random.default_rng(seed)
    W, D, H = 60.0, 60.0, 8.0
    tris = _box_tris([0, 0, 0], [W, D, H])
    # 30 rooms on a jittered 6x5 grid, 4-6 walls each, one door gap per room
    for k in range(30):
        gx, gy = k % 6, k // 6
        c = np.array([(gx + 0.5) * W / 6, (gy + 0.5) * D / 5]) + rng.uniform(-1.5, 1.5, 2)
        poly = _random_polygon(rng, c, 3.0, 4.5, int(rng.integers(4, 7)))
        door = int(rng.integers(len(poly)))
        for e in range(len(poly)):
            a, b = poly[e], poly[(e + 1) % len(poly)]
            if e == door:
                L = np.linalg.norm(b - a)
                if L > 1.5:
                    m0 = a + (b - a) * (0.5 - 0.5 / L)
                    m1 = a + (b - a) * (0.5 + 0.5 / L)
                    tris += _wall(a, m0, 0, H) + _wall(m1, b, 0, H)
                    continue
            tris += _wall(a, b, 0, H)
    boxes = []
    for _ in range(300):
        s = rng.uniform(0.3, 2.0, size=3)
        c = rng.uniform([0.5, 0.5], [W - 0.5 - s[0], D - 0.5 - s[1]])
        lo = np.array([c[0], c[1], 0.0]); hi = lo + s
        boxes.append(np.concatenate([lo, hi]))
        tris += _box_tris(lo, hi)
    cyl = []
    for _ in range(50):
        r = rng.uniform(0.1, 0.5)
        cxy = rng.uniform(1, W - 1, 2)
        cyl.append([cxy[0], cxy[1], r, 0.0, rng.uniform(1, 8)])
    return Scene("floor", np.array([0, 0, 0.0]), np.array([W, D, H]), np.array(tris), np.array(cyl),
                 boxes=np.array(boxes), sensor_z=(1.2, 1.8))


def scene_campus(seed=1003) -> Scene:
    rng = np.random.default_rng(seed)
    W, D, H = 200.0, 200.0, 15.0
    tris = []
    polys, hs = [], []
    for k in range(120):
        gx, gy = k % 11, k // 11
        c = np.array([(gx + 0.5) * W / 11, (gy + 0.5) * D / 11]) + rng.uniform(-3, 3, 2)
        nv = int(rng.integers(4, 9))
        diam = rng.uniform(8, 30)
        poly = _random_polygon(rng, c, 0.3 * diam, 0.5 * diam, nv)
        h = rng.uniform(4, 15)
        polys.append(poly); hs.append(h)
        for e in range(nv):
            tris += _wall(poly[e], poly[(e + 1) % nv], -0.5, h)
        cz = np.array([c[0], c[1], h])
        for e in range(nv):
            a, b = poly[e], poly[(e + 1) % nv]
            tris.append(np.stack([cz, [a[0], a[1], h], [b[0], b[1], h]]))
    cyl = []
    while len(cyl) < 2000:
        cxy = rng.uniform(1, W - 1, (4000, 2))
        inside = np.zeros(len(cxy), bool)
        for p in polys:
            inside |= _points_in_poly(cxy, p)
        for q in cxy[~inside][:2000 - len(cyl)]:
            cyl.append([q[0], q[1], rng.uniform(0.1, 0.5), -0.5, rng.uniform(3, 10)])
    sc = Scene("campus", np.array([0, 0, -0.5]), np.array([W, D, H]), np.array(tris), np.array(cyl),
               polys=polys, poly_h=hs, ground_amp=0.2, ground_scale=8.0, perlin=Perlin2D(seed + 7),
               sensor_z=(1.6, 2.0))
    return sc


def _points_in_poly(pts, poly):
    x = pts[:, 0]; y = pts[:, 1]
    inside = np.zeros(len(pts), bool)
    n = len(poly)
    for i in range(n):
        x1, y1 = poly[i]; x2, y2 = poly[(i + 1) % n]
        if y1 == y2:
            continue
        cond = (y1 > y) != (y2 > y)
        xc = x1 + (y - y1) * (x2 - x1) / (y2 - y1)
        inside ^= cond & (x < xc)
    return inside


def _point_in_poly(p, poly):
    x, y = p
    inside = False
    n = len(poly)
    for i in range(n):
        x1, y1 = poly[i]; x2, y2 = poly[(i + 1) % n]
        if (y1 > y) != (y2 > y):
            xc = x1 + (y - y1) * (x2 - x1) / (y2 - y1)
            if x < xc:
                inside = not inside
    return inside


# ---------------------------------------------------------------- sampling map points
def sample_map(scene: Scene, n: int, seed: int) -> np.ndarray:
    """n points uniform by area over all surfaces (float32, (n,3))."""
    rng = np.random.default_rng(seed)
    T = scene.tris
    tri_area = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)
    cyl = scene.cyl
    cyl_area = 2 * np.pi * cyl[:, 2] * (cyl[:, 4] - cyl[:, 3]) if len(cyl) else np.zeros(0)
    g_area = np.array([(scene.hi[0] - scene.lo[0]) * (scene.hi[1] - scene.lo[1])]) if scene.perlin is not None \
        else np.zeros(0)
    areas = np.concatenate([tri_area, cyl_area, g_area])
    counts = rng.multinomial(n, areas / areas.sum())
    out = np.empty((n, 3), np.float64)
    o = 0
    nt = len(T)
    tc = counts[:nt]
    idx = np.repeat(np.arange(nt), tc)
    m = len(idx)
    if m:
        u = rng.random(m); v = rng.random(m)
        flip = u + v > 1
        u[flip] = 1 - u[flip]; v[flip] = 1 - v[flip]
        A, B, Cc = T[idx, 0], T[idx, 1], T[idx, 2]
        out[o:o + m] = A + u[:, None] * (B - A) + v[:, None] * (Cc - A)
        o += m
    cc = counts[nt:nt + len(cyl)]
    idx = np.repeat(np.arange(len(cyl)), cc)
    m = len(idx)
    if m:
        th = rng.uniform(0, 2 * np.pi, m)
        z = rng.uniform(cyl[idx, 3], cyl[idx, 4])
        out[o:o + m, 0] = cyl[idx, 0] + cyl[idx, 2] * np.cos(th)
        out[o:o + m, 1] = cyl[idx, 1] + cyl[idx, 2] * np.sin(th)
        out[o:o + m, 2] = z
        o += m
    if scene.perlin is not None:
        m = int(counts[-1])
        x = rng.uniform(scene.lo[0], scene.hi[0], m)
        y = rng.uniform(scene.lo[1], scene.hi[1], m)
        out[o:o + m, 0] = x; out[o:o + m, 1] = y; out[o:o + m, 2] = scene.ground(x, y)
        o += m
    assert o == n
    return out.astype(np.float32)


# ---------------------------------------------------------------- ray casting
def raycast(scene: Scene, origin, dirs, max_range=80.0) -> np.ndarray:
    """first-hit distance along each unit direction from one origin (inf = miss)."""
    o = np.asarray(origin, np.float64)
    d = np.asarray(dirs, np.float64)
    nr = d.shape[0]
    best = np.full(nr, np.inf)
    T = scene.tris
    if len(T):
        A = T[:, 0]
        e1 = T[:, 1] - A
        e2 = T[:, 2] - A
        nrm = np.cross(e1, e2)
        nn = np.einsum("tk,tk->t", nrm, nrm)
        good = nn > 1e-18
        A, e1, e2, nrm, nn = A[good], e1[good], e2[good], nrm[good], nn[good]
        f1 = np.cross(e2, nrm) / nn[:, None]
        f2 = np.cross(nrm, e1) / nn[:, None]
        oa = o[None, :] - A
        c_t = -np.einsum("tk,tk->t", nrm, oa)      # n.(A - o)
        c_u = np.einsum("tk,tk->t", f1, oa)
        c_v = np.einsum("tk,tk->t", f2, oa)
        M = np.concatenate([nrm, f1, f2], axis=0).T  # (3, 3T)
        nt = len(A)
        for c0 in range(0, nr, 4096):
            dd = d[c0:c0 + 4096]
            P = dd @ M
            nd, fd1, fd2 = P[:, :nt], P[:, nt:2 * nt], P[:, 2 * nt:]
            with np.errstate(divide="ignore", invalid="ignore"):
                t = c_t[None, :] / nd
                u = c_u[None, :] + t * fd1
                v = c_v[None, :] + t * fd2
                ok = (np.abs(nd) > 1e-12) & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 1e-6)
            t = np.where(ok, t, np.inf)
            best[c0:c0 + 4096] = np.minimum(best[c0:c0 + 4096], t.min(axis=1))
    if len(scene.cyl):
        cy = scene.cyl
        dx = d[:, None, 0]; dy = d[:, None, 1]
        ox = o[0] - cy[None, :, 0]; oy = o[1] - cy[None, :, 1]
        a = dx * dx + dy * dy
        b = 2 * (ox * dx + oy * dy)
        c = ox * ox + oy * oy - cy[None, :, 2] ** 2
        disc = b * b - 4 * a * c
        with np.errstate(invalid="ignore", divide="ignore"):
            sq = np.sqrt(np.maximum(disc, 0))
            t1 = (-b - sq) / (2 * a)
            t2 = (-b + sq) / (2 * a)
        for tt in (t1, t2):
            z = o[2] + tt * d[:, None, 2]
            ok = (disc > 0) & (a > 1e-12) & (tt > 1e-6) & (z >= cy[None, :, 3]) & (z <= cy[None, :, 4])
            best = np.minimum(best, np.where(ok, tt, np.inf).min(axis=1))
    if scene.perlin is not None:
        # the ground lies within +-amp of z = 0: march only between the two
        # bounding planes, then bisect the first sign change
        amp = scene.ground_amp + 1e-3
        dz = d[:, 2]
        down = dz < -1e-9
        hit = np.full(nr, np.inf)
        if down.any():
            dd = d[down]
            t_in = np.maximum((o[2] - amp) / -dd[:, 2], 0.0)
            t_out = np.minimum((o[2] + amp) / -dd[:, 2], max_range)
            t_in = np.minimum(t_in, t_out)
            ns = 48
            prev_t = t_in.copy()
            p = o[None, :] + prev_t[:, None] * dd
            prev_f = p[:, 2] - scene.ground(p[:, 0], p[:, 1])
            h = np.full(len(dd), np.inf)
            for s in range(1, ns + 1):
                t = t_in + (t_out - t_in) * (s / ns)
                p = o[None, :] + t[:, None] * dd
                f = p[:, 2] - scene.ground(p[:, 0], p[:, 1])
                cross = (prev_f > 0) & (f <= 0) & ~np.isfinite(h)
                if cross.any():
                    lo_t = prev_t[cross].copy(); hi_t = t[cross].copy(); dc = dd[cross]
                    for _ in range(30):
                        mid = 0.5 * (lo_t + hi_t)
                        pm = o[None, :] + mid[:, None] * dc
                        fm = pm[:, 2] - scene.ground(pm[:, 0], pm[:, 1])
                        above = fm > 0
                        lo_t = np.where(above, mid, lo_t); hi_t = np.where(above, hi_t, mid)
                    h[cross] = 0.5 * (lo_t + hi_t)
                prev_t = t; prev_f = f
            hit[down] = h
        best = np.minimum(best, hit)
    best[best > max_range] = np.inf
    return best


def is_free(scene: Scene, p, margin=0.3) -> bool:
    p = np.asarray(p, np.float64)
    if np.any(p < scene.lo + margin) or np.any(p > scene.hi - margin):
        return False
    for b in scene.boxes:
        if np.all(p > b[:3] - margin) and np.all(p < b[3:] + margin):
            return False
    for c in scene.cyl:
        if (p[0] - c[0]) ** 2 + (p[1] - c[1]) ** 2 < (c[2] + margin) ** 2 and c[3] - margin < p[2] < c[4] + margin:
            return False
    for poly, h in zip(scene.polys, scene.poly_h):
        if p[2] < h + margin and _point_in_poly(p[:2], poly):
            return False
    # keep clear of walls: no hit closer than the margin in 26 directions
    dirs = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1) if (i, j, k) != (0, 0, 0)],
                    np.float64)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    return bool(np.all(raycast(scene, p, dirs, max_range=3 * margin) > margin))


def random_free_point(scene: Scene, rng, zmode="box"):
    for _ in range(10000):
        x = rng.uniform(scene.lo[0] + 1, scene.hi[0] - 1)
        y = rng.uniform(scene.lo[1] + 1, scene.hi[1] - 1)
        z = rng.uniform(*scene.sensor_z) + (scene.ground(x, y) if scene.perlin is not None else 0.0)
        p = np.array([x, y, float(z)])
        if is_free(scene, p):
            return p
    raise RuntimeError("no free space found")


def make_scan(scene: Scene, R, t, n_points, sigma, seed, max_range=80.0, oversample=3) -> np.ndarray:
    """n_points hits of rays uniform on the sphere, expressed in the sensor
    frame, with N(0, sigma^2) noise per axis.  Fewer points if the scene is
    mostly out of range."""
    rng = np.random.default_rng(seed)
    pts = []
    have = 0
    for _ in range(8):
        m = int(max(n_points - have, 1) * oversample)
        d = rng.normal(size=(m, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = raycast(scene, t, d, max_range)
        ok = np.isfinite(r)
        hit = t[None, :] + r[ok, None] * d[ok]
        pts.append(hit)
        have += int(ok.sum())
        if have >= n_points:
            break
    P = np.concatenate(pts)[:n_points]
    local = (P - t[None, :]) @ np.asarray(R)  # R^T (p - t)
    local += rng.normal(scale=sigma, size=local.shape)
    return local.astype(np.float32)


# ---------------------------------------------------------------- trajectories and odometry
def trajectory(scene: Scene, n_frames, step, yaw_step_deg, seed, kidnap_frame=None, kidnap_dist=80.0,
               kidnap_yaw_deg=90.0):
    """ground-truth sensor poses (list of (R, t)) moving `step` m and
    `yaw_step_deg` deg per frame through free space, with a small random tilt."""
    rng = np.random.default_rng(seed)
    p = random_free_point(scene, rng)
    yaw = rng.uniform(-np.pi, np.pi)
    turn = 1.0
    out = []
    for f in range(n_frames):
        if kidnap_frame is not None and f == kidnap_frame:
            for _ in range(200):
                a = rng.uniform(-np.pi, np.pi)
                q = p + kidnap_dist * np.array([math.cos(a), math.sin(a), 0.0])
                if scene.perlin is not None:
                    q[2] = scene.ground(q[0], q[1]) + np.mean(scene.sensor_z)
                if is_free(scene, q):
                    p = q
                    yaw += math.radians(kidnap_yaw_deg)
                    break
        if f > 0 and not (kidnap_frame is not None and f == kidnap_frame):
            if rng.random() < 0.1:
                turn = -turn
            moved = False
            for attempt in range(24):
                yaw_c = yaw + turn * math.radians(yaw_step_deg) + attempt * math.radians(15.0) * (1 if attempt % 2 else -1)
                d = np.array([math.cos(yaw_c), math.sin(yaw_c), 0.0])
                q = p + step * d
                if scene.perlin is not None:
                    q[2] = scene.ground(q[0], q[1]) + np.mean(scene.sensor_z)
                if is_free(scene, q) and raycast(scene, p, d[None, :], 2.0)[0] > 1.0:
                    p, yaw, moved = q, yaw_c, True
                    break
            if not moved:
                yaw += math.pi
        tilt = rng.normal(scale=math.radians(2.0), size=2)
        out.append((rpy_to_mat(tilt[0], tilt[1], yaw), p.copy()))
    return out


def odometry(prev, cur, seed, sig_rot=0.01, sig_trans=0.02, teleported=False, step_hint=None):
    """relative motion prev^-1 cur, right-perturbed by noise; returns
    (dT as (qw,qx,qy,qz,tx,ty,tz) float32, 6x6 covariance over [omega; v])."""
    rng = np.random.default_rng(seed)
    R0, t0 = prev
    R1, t1 = cur
    if teleported and step_hint is not None:
        R1, t1 = step_hint
    dR = R0.T @ R1
    dt = R0.T @ (t1 - t0)
    nR = rotvec_to_mat(rng.normal(scale=sig_rot, size=3))
    nt = rng.normal(scale=sig_trans, size=3)
    dRn = dR @ nR
    dtn = dt + dR @ nt
    out = np.zeros(7, np.float32)
    out[:4] = mat_to_quat(dRn)
    out[4:7] = dtn
    cov = np.diag([sig_rot ** 2] * 3 + [sig_trans ** 2] * 3).astype(np.float32)
    return out, cov


# ---------------------------------------------------------------- workloads
WORKLOADS = {
    "room": dict(scene=scene_room, map_points=200_000, voxel=0.5, scan_points=1024, scan_sigma=0.02,
                 particles=4096, k=8, lsh_bits=16, svgd_iters=10, frames=1, step=0.0, yaw_deg=0.0),
    "floor": dict(scene=scene_floor, map_points=2_000_000, voxel=0.5, scan_points=4096, scan_sigma=0.03,
                  particles=65_536, k=16, lsh_bits=20, svgd_iters=20, frames=50, step=0.5, yaw_deg=5.0),
    "campus": dict(scene=scene_campus, map_points=20_000_000, voxel=1.0, scan_points=8192, scan_sigma=0.03,
                   particles=1_048_576, k=16, lsh_bits=24, svgd_iters=10, frames=200, step=0.5, yaw_deg=5.0,
                   kidnap_frame=100),
    # a short sequence in the room scene (moving sensor, 5 m teleport at frame 10)
    "room_seq": dict(scene=scene_room, map_points=200_000, voxel=0.5, scan_points=1024, scan_sigma=0.02,
                     particles=4096, k=8, lsh_bits=16, svgd_iters=10, frames=20, step=0.3, yaw_deg=5.0,
                     kidnap_frame=10, kidnap_dist=5.0),
}

SEEDS = {"room": 1, "floor": 2, "campus": 3, "room_seq": 11}


def surrogate_samples(map_xyz, lo, hi, n, seed, sigma=0.25, uniform_frac=0.1) -> np.ndarray:
    """Training positions for the score-field surrogate: map points displaced
    by N(0, sigma^2 I) and a fraction drawn uniformly in the box [lo, hi]."""
    rng = np.random.default_rng(seed)
    k = int(round(n * uniform_frac))
    sel = rng.integers(0, len(map_xyz), n - k)
    near = map_xyz[sel].astype(np.float64) + rng.normal(0.0, sigma, (n - k, 3))
    far = rng.uniform(np.asarray(lo, np.float64), np.asarray(hi, np.float64), (k, 3))
    out = np.concatenate([near, far]).astype(np.float32)
    return out[rng.permutation(n)]


def _scan_job(args):
    return make_scan(*args)


def build_workload(name, map_points=None, scan_points=None, frames=None, seed_offset=0, kidnap_frame=None,
                   kidnap_dist=None, occlusion=None, workers=1, progress=None):
    """Scene, map points, ground-truth trajectory, scans and odometry of a workload.

    kidnap_frame / kidnap_dist override the workload's teleport (the odometry
    keeps reporting an ordinary step there); occlusion = (first, end) blanks
    the scans of frames first .. end - 1 (the sensor view is blocked, the
    odometry keeps reporting the motion).  workers > 1 casts the scans in
    that many processes (each scan depends only on its own seed, so the
    result is the same); progress(done, total) is called as scans finish."""
    w = dict(WORKLOADS[name])
    if kidnap_frame is not None:
        w["kidnap_frame"] = kidnap_frame
    if kidnap_dist is not None:
        w["kidnap_dist"] = kidnap_dist
    c = SEEDS[name] + seed_offset
    scene = w["scene"](1000 + c)
    n_map = map_points or w["map_points"]
    n_scan = scan_points or w["scan_points"]
    n_frames = frames or w["frames"]
    xyz = sample_map(scene, n_map, 2000 + c)
    rng = np.random.default_rng(2100 + c)
    if n_frames == 1 and w["step"] == 0.0:
        p = random_free_point(scene, rng)
        traj = [(random_rotation(rng), p)]
    else:
        traj = trajectory(scene, n_frames, w["step"], w["yaw_deg"], 2200 + c, w.get("kidnap_frame"),
                          kidnap_dist=w.get("kidnap_dist", 80.0))
    jobs = {f: (scene, R, t, n_scan, w["scan_sigma"], 2300 + c + 7919 * f) for f, (R, t) in enumerate(traj)
            if not (occlusion is not None and occlusion[0] <= f < occlusion[1])}
    cast = {}
    if workers > 1 and len(jobs) > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            for k, (f, sc) in enumerate(zip(jobs, ex.map(_scan_job, jobs.values()))):
                cast[f] = sc
                if progress:
                    progress(k + 1, len(jobs))
    else:
        for k, (f, a) in enumerate(jobs.items()):
            cast[f] = _scan_job(a)
            if progress:
                progress(k + 1, len(jobs))
    scans, odo = [], []
    for f, (R, t) in enumerate(traj):
        scans.append(cast[f] if f in cast else np.zeros((0, 3), np.float32))
        if f > 0:
            kid = w.get("kidnap_frame") is not None and f == w.get("kidnap_frame")
            hint = None
            if kid:  # odometry keeps reporting an ordinary step
                R0, t0 = traj[f - 1]
                yaw_d = math.radians(w["yaw_deg"])
                hint = (R0 @ rpy_to_mat(0, 0, yaw_d), t0 + R0 @ np.array([w["step"], 0, 0]))
            odo.append(odometry(traj[f - 1], traj[f], 2400 + c + f, teleported=kid, step_hint=hint))
        else:
            odo.append((None, None))
    return dict(scene=scene, map_xyz=xyz, traj=traj, scans=scans, odometry=odo, params=w)
