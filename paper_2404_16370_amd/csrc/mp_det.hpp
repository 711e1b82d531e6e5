// mp_det.hpp -- deterministic FP32 device programs.
//
// Every discrete decision of the filter (voxel of a transformed point, inlier
// gate, LSH cell and hash, neighbour ranking key, scan k-NN order, uniform
// initial poses) is taken by one of these programs.  They use only IEEE
// single-precision +, -, *, /, sqrt and explicit fma in a fixed order, and
// this translation unit is compiled with -ffp-contract=off, so the result is
// a function of the inputs alone.  Their definitions (operation order,
// polynomial degrees, constants) are part of the library's specification.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpdet {

// ------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC 2011: ten rounds of two 32x32->64 multiplies with key bumps.
struct u32x4 { uint32_t v[4]; };

__host__ __device__ inline u32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t a = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        const uint32_t b = (uint32_t)m1;
        const uint32_t c = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        const uint32_t d = (uint32_t)m0;
        c0 = a; c1 = b; c2 = c; c3 = d;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    u32x4 r;
    r.v[0] = c0; r.v[1] = c1; r.v[2] = c2; r.v[3] = c3;
    return r;
}

enum : uint32_t { PURPOSE_PRED = 1, PURPOSE_LSH = 2, PURPOSE_TLSH = 3, PURPOSE_INIT = 4, PURPOSE_WINIT = 5, PURPOSE_BATCH = 6,
                  PURPOSE_INIT_GAUSS = 7 };

// counter = (a, b, c, purpose << 16 | block), key = seed
__device__ inline u32x4 rng(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t purpose, uint32_t block) {
    return philox(a, b, c, (purpose << 16) | block, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ inline float unit_co(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }         // [0, 1)
__device__ inline float unit_oc(uint32_t x) { return (float)((x >> 8) + 1u) * 0x1p-24f; }  // (0, 1]

// ------------------------------------------------------------ elementary functions
// ln x for positive normal x:  x = m 2^e, m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s) with s = (m-1)/(m+1), series through s^11.
__device__ inline float ln(float x) {
    const uint32_t bits = __float_as_uint(x);
    int e = (int)(bits >> 23) - 127;
    float m = __uint_as_float((bits & 0x007FFFFFu) | 0x3F800000u);
    if (m > 1.41421356237309505f) {
        m = m * 0.5f;
        e = e + 1;
    }
    const float s = (m - 1.0f) / (m + 1.0f);
    const float z = s * s;
    float p = 1.0f / 11.0f;
    p = p * z + 1.0f / 9.0f;
    p = p * z + 1.0f / 7.0f;
    p = p * z + 1.0f / 5.0f;
    p = p * z + 1.0f / 3.0f;
    p = p * z + 1.0f;
    const float lm = (2.0f * s) * p;
    return (float)e * 0.693147180559945309f + lm;
}

// sin and cos of 2 pi u, u in [0, 1): quadrant q = floor(4u), x = (4u - q) pi/2,
// Taylor polynomials through x^13 (sin) and x^12 (cos).
__device__ inline void sincos_2pi(float u, float& s_out, float& c_out) {
    const float t = u * 4.0f;
    const float qf = floorf(t);
    const int q = (int)qf;
    const float x = (t - qf) * 1.57079632679489662f;
    const float x2 = x * x;
    float ps = -1.0f / 6227020800.0f;
    ps = ps * x2 + 1.0f / 39916800.0f;
    ps = ps * x2 - 1.0f / 362880.0f;
    ps = ps * x2 + 1.0f / 5040.0f;
    ps = ps * x2 - 1.0f / 120.0f;
    ps = ps * x2 + 1.0f / 6.0f;
    const float sx = x - (x * x2) * ps;
    float pc = 1.0f / 479001600.0f;
    pc = pc * x2 - 1.0f / 3628800.0f;
    pc = pc * x2 + 1.0f / 40320.0f;
    pc = pc * x2 - 1.0f / 720.0f;
    pc = pc * x2 + 1.0f / 24.0f;
    pc = pc * x2 - 0.5f;
    const float cx = 1.0f + x2 * pc;
    switch (q & 3) {
        case 0: s_out = sx; c_out = cx; break;
        case 1: s_out = cx; c_out = -sx; break;
        case 2: s_out = -sx; c_out = -cx; break;
        default: s_out = -cx; c_out = sx; break;
    }
}

// P(s) = sum_{k=0..7} (-1)^k s^k / (2k+1), so atan z = z P(z^2) for |z| <= tan(pi/12)
__device__ inline float atan_series(float s) {
    float p = -1.0f / 15.0f;
    p = p * s + 1.0f / 13.0f;
    p = p * s - 1.0f / 11.0f;
    p = p * s + 1.0f / 9.0f;
    p = p * s - 1.0f / 7.0f;
    p = p * s + 1.0f / 5.0f;
    p = p * s - 1.0f / 3.0f;
    p = p * s + 1.0f;
    return p;
}

constexpr float kTanPi12 = 0.267949192431122706f;
constexpr float kSqrt3 = 1.73205080756887729f;
constexpr float kPi6 = 0.523598775598298873f;
constexpr float kPi2 = 1.57079632679489662f;

// atan z for z in [0, 1]; above tan(pi/12) reduce with atan z = pi/6 + atan((sqrt3 z - 1)/(z + sqrt3))
__device__ inline float atan01(float z) {
    if (z <= kTanPi12) return z * atan_series(z * z);
    const float r = (z * kSqrt3 - 1.0f) / (z + kSqrt3);
    return kPi6 + r * atan_series(r * r);
}

// theta / n with theta = 2 atan2(n, w), n >= 0, w >= 0: rotation vector = (theta/n) * (qx, qy, qz)
__device__ inline float rotvec_scale(float n, float w) {
    if (n <= w * kTanPi12) {
        const float z = n / w;
        return (2.0f * atan_series(z * z)) / w;
    }
    const float a = (n <= w) ? atan01(n / w) : (kPi2 - atan01(w / n));
    return (2.0f * a) / n;
}

// ------------------------------------------------------------ pose algebra
struct quat { float w, x, y, z; };

// Hamilton product; the terms are paired so that conj(q) (x) q has an exactly zero vector part
__device__ inline quat qmul(const quat a, const quat b) {
    quat r;
    r.w = ((a.w * b.w - a.x * b.x) - a.y * b.y) - a.z * b.z;
    r.x = (a.w * b.x + a.x * b.w) + (a.y * b.z - a.z * b.y);
    r.y = (a.w * b.y + a.y * b.w) + (a.z * b.x - a.x * b.z);
    r.z = (a.w * b.z + a.z * b.w) + (a.x * b.y - a.y * b.x);
    return r;
}
__device__ inline quat qconj(const quat a) { return quat{a.w, -a.x, -a.y, -a.z}; }

// rotation matrix (row-major) of a unit quaternion
struct mat3 { float m[9]; };
__device__ inline mat3 qmat(const quat q) {
    const float xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
    const float xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z;
    const float wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z;
    mat3 R;
    R.m[0] = 1.0f - 2.0f * (yy + zz);
    R.m[1] = 2.0f * (xy - wz);
    R.m[2] = 2.0f * (xz + wy);
    R.m[3] = 2.0f * (xy + wz);
    R.m[4] = 1.0f - 2.0f * (xx + zz);
    R.m[5] = 2.0f * (yz - wx);
    R.m[6] = 2.0f * (xz - wy);
    R.m[7] = 2.0f * (yz + wx);
    R.m[8] = 1.0f - 2.0f * (xx + yy);
    return R;
}

// R^T v
__device__ inline float3 rot_t(const mat3& R, const float3 v) {
    float3 o;
    o.x = __builtin_fmaf(R.m[0], v.x, __builtin_fmaf(R.m[3], v.y, R.m[6] * v.z));
    o.y = __builtin_fmaf(R.m[1], v.x, __builtin_fmaf(R.m[4], v.y, R.m[7] * v.z));
    o.z = __builtin_fmaf(R.m[2], v.x, __builtin_fmaf(R.m[5], v.y, R.m[8] * v.z));
    return o;
}

// R mu + t: the transform whose result picks the voxel of a scan point
__device__ inline float3 xform(const float* R, const float3 t, const float3 mu) {
    float3 p;
    p.x = __builtin_fmaf(R[0], mu.x, __builtin_fmaf(R[1], mu.y, __builtin_fmaf(R[2], mu.z, t.x)));
    p.y = __builtin_fmaf(R[3], mu.x, __builtin_fmaf(R[4], mu.y, __builtin_fmaf(R[5], mu.z, t.y)));
    p.z = __builtin_fmaf(R[6], mu.x, __builtin_fmaf(R[7], mu.y, __builtin_fmaf(R[8], mu.z, t.z)));
    return p;
}

// floor to int32, clamped to [-2^30, 2^30] (a single med3 for finite input)
__device__ inline int32_t floor_i32(float z) {
    const float f = __builtin_fminf(__builtin_fmaxf(floorf(z), -1073741824.0f), 1073741824.0f);
    return (int32_t)f;
}

// log map of a quaternion (canonical w >= 0); also returns w and theta/n
__device__ inline float3 qlog(quat q, float& w_out, float& scale_out) {
    if (q.w < 0.0f) q = quat{-q.w, -q.x, -q.y, -q.z};
    const float n = sqrtf((q.x * q.x + q.y * q.y) + q.z * q.z);
    const float sc = rotvec_scale(n, q.w);
    w_out = q.w;
    scale_out = sc;
    return float3{sc * q.x, sc * q.y, sc * q.z};
}

// d = log(T_i^-1 T_j) with the coupled SE(3) logarithm: rotation vector
// omega of qr = conj(q_i) q_j and rho = V(omega)^-1 tr, tr = R_i^T (t_j - t_i).
// Also hands back qr, tr and beta, the coefficient of V^-1 = I - 1/2 omega^ +
// beta omega^2.
__device__ inline void se3_between_ex(const quat qi, const float3 ti, const quat qj, const float3 tj, float3& om,
                                      float3& rho, quat& qr, float3& tr, float& beta) {
    qr = qmul(qconj(qi), qj);
    const mat3 Ri = qmat(qi);
    const float3 dt = float3{tj.x - ti.x, tj.y - ti.y, tj.z - ti.z};
    tr = rot_t(Ri, dt);
    float w, sc;
    om = qlog(qr, w, sc);
    const float th2 = (om.x * om.x + om.y * om.y) + om.z * om.z;
    if (th2 < 0.0025f) {
        beta = 1.0f / 30240.0f;
        beta = beta * th2 + 1.0f / 720.0f;
        beta = beta * th2 + 1.0f / 12.0f;
    } else {
        beta = (1.0f - (0.5f * sc) * w) / th2;
    }
    const float c1x = om.y * tr.z - om.z * tr.y, c1y = om.z * tr.x - om.x * tr.z, c1z = om.x * tr.y - om.y * tr.x;
    const float c2x = om.y * c1z - om.z * c1y, c2y = om.z * c1x - om.x * c1z, c2z = om.x * c1y - om.y * c1x;
    rho.x = (tr.x - 0.5f * c1x) + beta * c2x;
    rho.y = (tr.y - 0.5f * c1y) + beta * c2y;
    rho.z = (tr.z - 0.5f * c1z) + beta * c2z;
}

__device__ inline void se3_between(const quat qi, const float3 ti, const quat qj, const float3 tj, float3& om,
                                   float3& rho) {
    quat qr;
    float3 tr;
    float beta;
    se3_between_ex(qi, ti, qj, tj, om, rho, qr, tr, beta);
}

// q_ij = d^T W d with W = diag(sigma_r I3, sigma_t I3) (Eq. 7-8): ranks neighbours
__device__ inline float qdist(const quat qi, const float3 ti, const quat qj, const float3 tj, float sigma_r,
                              float sigma_t) {
    float3 om, rho;
    se3_between(qi, ti, qj, tj, om, rho);
    const float th2 = (om.x * om.x + om.y * om.y) + om.z * om.z;
    const float rr = (rho.x * rho.x + rho.y * rho.y) + rho.z * rho.z;
    return sigma_r * th2 + sigma_t * rr;
}

// six standard normals by Box-Muller from two Philox blocks
__device__ inline void gauss6(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t purpose, float z[6]) {
    const u32x4 w0 = rng(seed, a, b, c, purpose, 0);
    const u32x4 w1 = rng(seed, a, b, c, purpose, 1);
    const uint32_t w[8] = {w0.v[0], w0.v[1], w0.v[2], w0.v[3], w1.v[0], w1.v[1], w1.v[2], w1.v[3]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float u1 = unit_oc(w[2 * k]);
        const float u2 = unit_co(w[2 * k + 1]);
        const float r = sqrtf(-2.0f * ln(u1));
        float s, c2;
        sincos_2pi(u2, s, c2);
        z[2 * k] = r * c2;
        z[2 * k + 1] = r * s;
    }
}

// uniform rotation from three uniforms (Shoemake, Graphics Gems III, 1992)
__device__ inline quat shoemake(float u1, float u2, float u3) {
    const float a = sqrtf(1.0f - u1), b = sqrtf(u1);
    float s2, c2, s3, c3;
    sincos_2pi(u2, s2, c2);
    sincos_2pi(u3, s3, c3);
    return quat{b * c3, a * s2, a * c2, b * s3};
}

// pose with uniform rotation and translation uniform in [lo, hi)
__device__ inline void random_pose(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t purpose,
                                   const float lo[3], const float hi[3], quat& q, float3& t) {
    const u32x4 r0 = rng(seed, a, b, c, purpose, 0);
    const u32x4 r1 = rng(seed, a, b, c, purpose, 1);
    q = shoemake(unit_co(r0.v[0]), unit_co(r0.v[1]), unit_co(r0.v[2]));
    t.x = lo[0] + unit_co(r1.v[0]) * (hi[0] - lo[0]);
    t.y = lo[1] + unit_co(r1.v[1]) * (hi[1] - lo[1]);
    t.z = lo[2] + unit_co(r1.v[2]) * (hi[2] - lo[2]);
}

// XOR of products of the cell coordinates with three primes of Teschner et
// al. (2003) and three further odd constants
__device__ inline uint32_t hash6(const int32_t c[6]) {
    return ((uint32_t)c[0] * 73856093u) ^ ((uint32_t)c[1] * 19349663u) ^ ((uint32_t)c[2] * 83492791u) ^
           ((uint32_t)c[3] * 2654435761u) ^ ((uint32_t)c[4] * 2246822519u) ^ ((uint32_t)c[5] * 3266489917u);
}

}  // namespace mpdet
