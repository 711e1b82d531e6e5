/*
 * mpo.c -- plain, slow CPU oracle for the Gauss-Newton Stein particle filter
 * of Koide et al., "MegaParticles: Range-based 6-DoF Monte Carlo Localization
 * with GPU-Accelerated Stein Particle Filter" (ICRA 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * Precision rules
 *   - Every floating-point result (log-likelihood, H, b, psi, SVGD update,
 *     posterior, prediction) is computed in FP64 from the FP32 inputs the GPU
 *     sees.
 *   - Every discrete decision (voxel key, NNF hit, inlier test, LSH cell and
 *     hash, bucket order, neighbour ranking key q_ij, scan k-NN order) is taken
 *     by a deterministic FP32 program: plain IEEE single-precision +,-,*,/,sqrt
 *     and explicit fmaf() in a fixed order, no library transcendental, no
 *     contraction (built with -ffp-contract=off).  The GPU takes the same
 *     decision with the same FP32 program, so the integer outputs must agree
 *     bit for bit.
 *   - Random numbers come from Philox4x32-10 (Salmon et al., SC'11), written
 *     here from its published definition, keyed by (seed) with a counter of
 *     (index, frame, iteration, purpose<<16 | block).
 *
 * Parity status of every function is stated in its comment: "pinned by"
 * lists what the CPU tests check it against.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MPO_API __attribute__((visibility("default")))

/* ======================================================================= */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:     */
/* as easy as 1, 2, 3", SC 2011).  Pinned by the published known-answer     */
/* vectors.                                                                 */
/* ======================================================================= */
MPO_API void mpo_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

enum { MPO_PURPOSE_PRED = 1, MPO_PURPOSE_LSH = 2, MPO_PURPOSE_TLSH = 3, MPO_PURPOSE_INIT = 4, MPO_PURPOSE_INITG = 7 };

static void rng_block(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t purpose, uint32_t blk,
                      uint32_t out[4]) {
    uint32_t ctr[4] = {a, b, c, (purpose << 16) | blk};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    mpo_philox(ctr, key, out);
}

/* uniform in [0,1): top 24 bits scaled by 2^-24 (exact) */
static float u01_co(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }
/* uniform in (0,1]: for the logarithm of Box-Muller */
static float u01_oc(uint32_t x) { return (float)((x >> 8) + 1u) * 0x1p-24f; }

/* ======================================================================= */
/* Deterministic FP32 elementary functions.  Only +,-,*,/ in a fixed order. */
/* Pinned against libm (accuracy) in the CPU tests.                         */
/* ======================================================================= */

/* natural log for x in (0, 1] (also valid for any positive normal x):
 * x = m * 2^e with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(s),
 * s = (m-1)/(m+1), atanh series to s^11. */
MPO_API float mpo_det_log(float x) {
    uint32_t bits;
    memcpy(&bits, &x, 4);
    int e = (int)(bits >> 23) - 127;
    uint32_t mb = (bits & 0x007FFFFFu) | 0x3F800000u;
    float m;
    memcpy(&m, &mb, 4);
    if (m > 1.41421356237309505f) { m = m * 0.5f; e = e + 1; }
    float s = (m - 1.0f) / (m + 1.0f);
    float z = s * s;
    float p = (1.0f / 11.0f);
    p = p * z + (1.0f / 9.0f);
    p = p * z + (1.0f / 7.0f);
    p = p * z + (1.0f / 5.0f);
    p = p * z + (1.0f / 3.0f);
    p = p * z + 1.0f;
    float lm = (2.0f * s) * p;
    float le = (float)e * 0.693147180559945309f;
    return le + lm;
}

/* sin and cos of 2*pi*u for u in [0,1): quadrant from floor(4u) (exact),
 * x = f*pi/2 with f in [0,1), Taylor series to x^13 / x^12. */
MPO_API void mpo_det_sincos2pi(float u, float* s_out, float* c_out) {
    float t = u * 4.0f;
    float qf = floorf(t);
    int q = (int)qf;
    float f = t - qf;
    float x = f * 1.57079632679489662f;
    float x2 = x * x;
    float sp = -(1.0f / 6227020800.0f);
    sp = sp * x2 + (1.0f / 39916800.0f);
    sp = sp * x2 - (1.0f / 362880.0f);
    sp = sp * x2 + (1.0f / 5040.0f);
    sp = sp * x2 - (1.0f / 120.0f);
    sp = sp * x2 + (1.0f / 6.0f);
    /* sin x = x - x^3/6 + ... : the polynomial above holds the alternating
     * coefficients with the sign of x^3 folded in below */
    float sn = x - (x * x2) * sp;
    float cp = (1.0f / 479001600.0f);
    cp = cp * x2 - (1.0f / 3628800.0f);
    cp = cp * x2 + (1.0f / 40320.0f);
    cp = cp * x2 - (1.0f / 720.0f);
    cp = cp * x2 + (1.0f / 24.0f);
    cp = cp * x2 - 0.5f;
    float cs = 1.0f + x2 * cp;
    float s, c;
    switch (q & 3) {
        case 0: s = sn; c = cs; break;
        case 1: s = cs; c = -sn; break;
        case 2: s = -sn; c = -cs; break;
        default: s = -cs; c = sn; break;
    }
    *s_out = s;
    *c_out = c;
}

/* atan series z*P(z^2) for |z| <= tan(pi/12):  P(s) = sum_k (-1)^k s^k/(2k+1) */
static float atan_poly(float s) {
    float p = -(1.0f / 15.0f);
    p = p * s + (1.0f / 13.0f);
    p = p * s - (1.0f / 11.0f);
    p = p * s + (1.0f / 9.0f);
    p = p * s - (1.0f / 7.0f);
    p = p * s + (1.0f / 5.0f);
    p = p * s - (1.0f / 3.0f);
    p = p * s + 1.0f;
    return p;
}

#define MPO_TAN_PI12 0.267949192431122706f
#define MPO_SQRT3 1.73205080756887729f
#define MPO_PI_6 0.523598775598298873f
#define MPO_PI_2 1.57079632679489662f

/* atan(z) for z in [0, 1] */
static float atan_unit(float z) {
    if (z <= MPO_TAN_PI12) return z * atan_poly(z * z);
    float zr = (z * MPO_SQRT3 - 1.0f) / (z + MPO_SQRT3);
    return MPO_PI_6 + zr * atan_poly(zr * zr);
}

/* theta/n where theta = 2*atan2(n, w), for n >= 0, w >= 0, (n,w) != 0.
 * This is the scale from the vector part of a unit quaternion to the
 * rotation vector, with no singularity at n = 0. */
MPO_API float mpo_det_rotvec_scale(float n, float w) {
    if (n <= w * MPO_TAN_PI12) {
        float z = n / w;
        return (2.0f * atan_poly(z * z)) / w;
    }
    float a;
    if (n <= w) a = atan_unit(n / w);
    else a = MPO_PI_2 - atan_unit(w / n);
    return (2.0f * a) / n;
}

/* ======================================================================= */
/* Deterministic FP32 pose algebra (quaternion (w,x,y,z) + translation).    */
/* ======================================================================= */
typedef struct { float w, x, y, z; } q32;

/* Hamilton product a (x) b, fixed evaluation order */
static q32 q32_mul(q32 a, q32 b) {
    q32 r;
    /* terms paired so that conj(q) (x) q has an exactly zero vector part */
    r.w = ((a.w * b.w - a.x * b.x) - a.y * b.y) - a.z * b.z;
    r.x = (a.w * b.x + a.x * b.w) + (a.y * b.z - a.z * b.y);
    r.y = (a.w * b.y + a.y * b.w) + (a.z * b.x - a.x * b.z);
    r.z = (a.w * b.z + a.z * b.w) + (a.x * b.y - a.y * b.x);
    return r;
}
static q32 q32_conj(q32 a) { q32 r = {a.w, -a.x, -a.y, -a.z}; return r; }

/* rotation matrix of a (unit) quaternion, row-major R[9] */
static void q32_to_R(q32 q, float R[9]) {
    float xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
    float xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z;
    float wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z;
    R[0] = 1.0f - 2.0f * (yy + zz); R[1] = 2.0f * (xy - wz);        R[2] = 2.0f * (xz + wy);
    R[3] = 2.0f * (xy + wz);        R[4] = 1.0f - 2.0f * (xx + zz); R[5] = 2.0f * (yz - wx);
    R[6] = 2.0f * (xz - wy);        R[7] = 2.0f * (yz + wx);        R[8] = 1.0f - 2.0f * (xx + yy);
}

/* p = R mu + t, the transform that decides the NNF voxel */
static void xform32(const float R[9], const float t[3], const float mu[3], float p[3]) {
    p[0] = fmaf(R[0], mu[0], fmaf(R[1], mu[1], fmaf(R[2], mu[2], t[0])));
    p[1] = fmaf(R[3], mu[0], fmaf(R[4], mu[1], fmaf(R[5], mu[2], t[1])));
    p[2] = fmaf(R[6], mu[0], fmaf(R[7], mu[1], fmaf(R[8], mu[2], t[2])));
}

/* v' = R^T v */
static void rotT32(const float R[9], const float v[3], float o[3]) {
    o[0] = fmaf(R[0], v[0], fmaf(R[3], v[1], R[6] * v[2]));
    o[1] = fmaf(R[1], v[0], fmaf(R[4], v[1], R[7] * v[2]));
    o[2] = fmaf(R[2], v[0], fmaf(R[5], v[1], R[8] * v[2]));
}

/* rotation vector of a quaternion (log map of SO(3)); canonical w >= 0 */
static void q32_log(q32 q, float om[3], float* w_out, float* scale_out) {
    if (q.w < 0.0f) { q.w = -q.w; q.x = -q.x; q.y = -q.y; q.z = -q.z; }
    float n = sqrtf((q.x * q.x + q.y * q.y) + q.z * q.z);
    float sc = mpo_det_rotvec_scale(n, q.w);
    om[0] = sc * q.x; om[1] = sc * q.y; om[2] = sc * q.z;
    if (w_out) *w_out = q.w;
    if (scale_out) *scale_out = sc;
}

/* d = log(T_i^-1 T_j) with the coupled SE(3) logarithm (Eq. 8): the
 * rotation vector om of conj(q_i) q_j and rho = V(om)^-1 R_i^T (t_j - t_i).
 * Deterministic FP32: it decides neighbour ranks and, in the coupled LSH
 * tangent, cells. */
static void se3_between32(const float* Ti, const float* Tj, float om[3], float rho[3]) {
    q32 qi = {Ti[0], Ti[1], Ti[2], Ti[3]}, qj = {Tj[0], Tj[1], Tj[2], Tj[3]};
    q32 qr = q32_mul(q32_conj(qi), qj);
    float R[9];
    q32_to_R(qi, R);
    float dt[3] = {Tj[4] - Ti[4], Tj[5] - Ti[5], Tj[6] - Ti[6]};
    float tr[3];
    rotT32(R, dt, tr);
    float w, sc;
    q32_log(qr, om, &w, &sc);
    float th2 = (om[0] * om[0] + om[1] * om[1]) + om[2] * om[2];
    float beta;
    if (th2 < 0.0025f) {
        beta = (1.0f / 30240.0f);
        beta = beta * th2 + (1.0f / 720.0f);
        beta = beta * th2 + (1.0f / 12.0f);
    } else {
        beta = (1.0f - (0.5f * sc) * w) / th2;
    }
    /* rho = V^-1 t = t - 1/2 om x t + beta om x (om x t) */
    float c1[3] = {om[1] * tr[2] - om[2] * tr[1], om[2] * tr[0] - om[0] * tr[2], om[0] * tr[1] - om[1] * tr[0]};
    float c2[3] = {om[1] * c1[2] - om[2] * c1[1], om[2] * c1[0] - om[0] * c1[2], om[0] * c1[1] - om[1] * c1[0]};
    for (int k = 0; k < 3; ++k) rho[k] = (tr[k] - 0.5f * c1[k]) + beta * c2[k];
}

/* Kernel distance key q_ij = d^T W d with d = log(T_i^-1 T_j) (Eq. 7-8).
 * Deterministic FP32: it ranks neighbours (Alg. 1). */
MPO_API float mpo_det_qdist(const float* Ti, const float* Tj, float sigma_r, float sigma_t) {
    float om[3], rho[3];
    se3_between32(Ti, Tj, om, rho);
    float th2 = (om[0] * om[0] + om[1] * om[1]) + om[2] * om[2];
    float rr = (rho[0] * rho[0] + rho[1] * rho[1]) + rho[2] * rho[2];
    return sigma_r * th2 + sigma_t * rr;
}

/* six N(0,1) samples by Box-Muller from two Philox blocks */
MPO_API void mpo_gauss6(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t purpose, float z[6]) {
    uint32_t w[8];
    rng_block(seed, a, b, c, purpose, 0, w);
    rng_block(seed, a, b, c, purpose, 1, w + 4);
    for (int k = 0; k < 3; ++k) {
        float u1 = u01_oc(w[2 * k]);
        float u2 = u01_co(w[2 * k + 1]);
        float r = sqrtf(-2.0f * mpo_det_log(u1));
        float s, cc;
        mpo_det_sincos2pi(u2, &s, &cc);
        z[2 * k] = r * cc;
        z[2 * k + 1] = r * s;
    }
}

/* uniform rotation (Shoemake, Graphics Gems III, 1992) from three uniforms */
static q32 shoemake(float u1, float u2, float u3) {
    float a = sqrtf(1.0f - u1), b = sqrtf(u1);
    float s2, c2, s3, c3;
    mpo_det_sincos2pi(u2, &s2, &c2);
    mpo_det_sincos2pi(u3, &s3, &c3);
    q32 q = {b * c3, a * s2, a * c2, b * s3};
    return q;
}

/* random SE(3) pose: rotation uniform on SO(3), translation uniform in the box */
static void random_pose(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t purpose,
                        const float lo[3], const float hi[3], float T[8]) {
    uint32_t w0[4], w1[4];
    rng_block(seed, a, b, c, purpose, 0, w0);
    rng_block(seed, a, b, c, purpose, 1, w1);
    q32 q = shoemake(u01_co(w0[0]), u01_co(w0[1]), u01_co(w0[2]));
    T[0] = q.w; T[1] = q.x; T[2] = q.y; T[3] = q.z;
    for (int k = 0; k < 3; ++k) T[4 + k] = lo[k] + u01_co(w1[k]) * (hi[k] - lo[k]);
    T[7] = 0.0f;
}

/* T^LSH of (frame, iteration): Alg. 1 first step */
MPO_API void mpo_lsh_frame(uint64_t seed, uint32_t frame, uint32_t it, const float lo[3], const float hi[3],
                           float T[8]) {
    random_pose(seed, 0u, frame, it, MPO_PURPOSE_TLSH, lo, hi, T);
}

/* uniform initial particle i */
MPO_API void mpo_init_uniform(uint64_t seed, int64_t n, const float lo[3], const float hi[3], float* poses) {
    for (int64_t i = 0; i < n; ++i) random_pose(seed, (uint32_t)i, 0u, 0u, MPO_PURPOSE_INIT, lo, hi, poses + 8 * i);
}

/* uniform initial particles i0 .. i0 + n - 1 (a sample of a large set) */
MPO_API void mpo_init_uniform_range(uint64_t seed, int64_t i0, int64_t n, const float lo[3], const float hi[3],
                                    float* poses) {
    for (int64_t k = 0; k < n; ++k)
        random_pose(seed, (uint32_t)(i0 + k), 0u, 0u, MPO_PURPOSE_INIT, lo, hi, poses + 8 * k);
}

/* 6-D integer hash of the LSH cell (Teschner et al. 2003 style XOR of
 * products; three Teschner primes plus three fixed odd constants) */
static const uint32_t HASH_P[6] = {73856093u, 19349663u, 83492791u, 2654435761u, 2246822519u, 3266489917u};
MPO_API uint32_t mpo_hash6(const int32_t c[6]) {
    uint32_t h = 0;
    for (int m = 0; m < 6; ++m) h ^= (uint32_t)c[m] * HASH_P[m];
    return h;
}

static int32_t floor_to_i32(float z) {
    float f = floorf(z);
    if (f > 1073741824.0f) f = 1073741824.0f;
    if (f < -1073741824.0f) f = -1073741824.0f;
    return (int32_t)f;
}

/* LSH code of Eq. (9)-(10):
 *   zeta = alpha * W^K x_i + delta_i,  delta_i = sigma_lsh * N(0, I6) drawn
 *   per particle,  cell = floor(zeta),  code = hash6(cell) & (2^bits - 1),
 * with the tangent x_i of T_i at T^LSH either
 *   tangent 0 (decoupled)  [log(R_L^T R_i); R_L^T (t_i - t_L)]
 *   tangent 1 (coupled)    log(T_LSH^-1 T_i), the SE(3) logarithm of Eq. (8).
 * Deterministic FP32.  Pinned by cells of zeta computed in FP64 (rotation
 * vectors, matrix logarithm) away from cell boundaries. */
MPO_API void mpo_lsh_codes_range(const float* poses, int64_t i0, int64_t n, const float TL[8], float alpha,
                                 float sigma_r, float sigma_t, float sigma_lsh, int bits, uint64_t seed, uint32_t frame,
                                 uint32_t it, int32_t tangent, uint32_t* codes, int32_t* cells);

MPO_API void mpo_lsh_codes(const float* poses, int64_t n, const float TL[8], float alpha, float sigma_r,
                           float sigma_t, float sigma_lsh, int bits, uint64_t seed, uint32_t frame, uint32_t it,
                           int32_t tangent, uint32_t* codes, int32_t* cells /* nullable n*6 */) {
    mpo_lsh_codes_range(poses, 0, n, TL, alpha, sigma_r, sigma_t, sigma_lsh, bits, seed, frame, it, tangent, codes,
                        cells);
}

/* the same for particles i0 .. i0 + n - 1 (poses[k] is particle i0 + k) */
MPO_API void mpo_lsh_codes_range(const float* poses, int64_t i0, int64_t n, const float TL[8], float alpha,
                                 float sigma_r, float sigma_t, float sigma_lsh, int bits, uint64_t seed, uint32_t frame,
                                 uint32_t it, int32_t tangent, uint32_t* codes, int32_t* cells /* nullable n*6 */) {
    uint32_t mask = bits >= 32 ? 0xFFFFFFFFu : ((1u << bits) - 1u);
    float ar = alpha * sigma_r, at = alpha * sigma_t;
    q32 qL = {TL[0], TL[1], TL[2], TL[3]};
    float RL[9];
    q32_to_R(qL, RL);
    q32 qLc = q32_conj(qL);
    for (int64_t i = 0; i < n; ++i) {
        const float* T = poses + 8 * i;
        float om[3], u[3];
        if (tangent == 1) {
            se3_between32(TL, T, om, u);
        } else {
            q32 qi = {T[0], T[1], T[2], T[3]};
            q32 qr = q32_mul(qLc, qi);
            q32_log(qr, om, NULL, NULL);
            float dt[3] = {T[4] - TL[4], T[5] - TL[5], T[6] - TL[6]};
            rotT32(RL, dt, u);
        }
        float z6[6];
        mpo_gauss6(seed, (uint32_t)(i0 + i), frame, it, MPO_PURPOSE_LSH, z6);
        int32_t c[6];
        for (int k = 0; k < 3; ++k) {
            c[k] = floor_to_i32(ar * om[k] + sigma_lsh * z6[k]);
            c[3 + k] = floor_to_i32(at * u[k] + sigma_lsh * z6[3 + k]);
        }
        codes[i] = mpo_hash6(c) & mask;
        if (cells) memcpy(cells + 6 * i, c, sizeof(c));
    }
}

/* ======================================================================= */
/* FP64 helpers                                                             */
/* ======================================================================= */
static void qd_to_R(const double q_in[4], double R[9]) {
    double nq = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    double w = q_in[0] / nq, x = q_in[1] / nq, y = q_in[2] / nq, z = q_in[3] / nq;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void qd_mul(const double a[4], const double b[4], double r[4]) {
    r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    r[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    r[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    r[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

/* sym 3x3 stored (xx, xy, xz, yy, yz, zz) -> full */
static void sym6_full(const double s[6], double A[9]) {
    A[0] = s[0]; A[1] = s[1]; A[2] = s[2];
    A[3] = s[1]; A[4] = s[3]; A[5] = s[4];
    A[6] = s[2]; A[7] = s[4]; A[8] = s[5];
}

static void mat3_mul(const double A[9], const double B[9], double C[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

static void mat3_T(const double A[9], double B[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[3 * j + i] = A[3 * i + j];
}

/* inverse of a 3x3 by the adjugate; returns determinant */
static double mat3_inv(const double A[9], double B[9]) {
    double c00 = A[4] * A[8] - A[5] * A[7];
    double c01 = A[5] * A[6] - A[3] * A[8];
    double c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    double id = 1.0 / det;
    B[0] = c00 * id; B[1] = (A[2] * A[7] - A[1] * A[8]) * id; B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    B[3] = c01 * id; B[4] = (A[0] * A[8] - A[2] * A[6]) * id; B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    B[6] = c02 * id; B[7] = (A[1] * A[6] - A[0] * A[7]) * id; B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    return det;
}

/* Cyclic Jacobi eigen-decomposition of a symmetric 3x3 (Golub & Van Loan,
 * Matrix Computations, sec. 8.5).  Eigenvalues ascending in w, eigenvectors
 * in the columns of V.  Pinned against numpy.linalg.eigh. */
MPO_API void mpo_eig3(const double S_in[9], double w[3], double V[9]) {
    double A[9];
    memcpy(A, S_in, sizeof(A));
    for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        double diag = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-300 || off <= 1e-34 * diag) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                double apq = A[3 * p + q];
                if (apq == 0.0) continue;
                double app = A[3 * p + p], aqq = A[3 * q + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J with J the rotation in the (p,q) plane */
                for (int k = 0; k < 3; ++k) {
                    double akp = A[3 * k + p], akq = A[3 * k + q];
                    A[3 * k + p] = c * akp - s * akq;
                    A[3 * k + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = A[3 * p + k], aqk = A[3 * q + k];
                    A[3 * p + k] = c * apk - s * aqk;
                    A[3 * q + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    double vkp = V[3 * k + p], vkq = V[3 * k + q];
                    V[3 * k + p] = c * vkp - s * vkq;
                    V[3 * k + q] = s * vkp + c * vkq;
                }
            }
    }
    double ev[3] = {A[0], A[4], A[8]};
    int ord[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (ev[ord[j]] < ev[ord[i]]) { int t = ord[i]; ord[i] = ord[j]; ord[j] = t; }
    double Vs[9];
    for (int c = 0; c < 3; ++c) {
        w[c] = ev[ord[c]];
        for (int r = 0; r < 3; ++r) Vs[3 * r + c] = V[3 * r + ord[c]];
    }
    memcpy(V, Vs, sizeof(Vs));
}

/* GICP plane normalisation (Segal et al. 2009): covariance S of a point
 * neighbourhood -> I - (1-eps) n n^T with n the eigenvector of the smallest
 * eigenvalue.  Output (xx, xy, xz, yy, yz, zz). */
static void gicp_normalise(const double S[9], double eps, double out6[6], double n_out[3]) {
    double w[3], V[9];
    mpo_eig3(S, w, V);
    double n[3] = {V[0], V[3], V[6]};
    if (n_out) { n_out[0] = n[0]; n_out[1] = n[1]; n_out[2] = n[2]; }
    double a = 1.0 - eps;
    out6[0] = 1.0 - a * n[0] * n[0];
    out6[1] = -a * n[0] * n[1];
    out6[2] = -a * n[0] * n[2];
    out6[3] = 1.0 - a * n[1] * n[1];
    out6[4] = -a * n[1] * n[2];
    out6[5] = 1.0 - a * n[2] * n[2];
}

/* ======================================================================= */
/* Map: per-voxel Gaussians and the nearest-neighbour field (Sec. III-C,   */
/* "Likelihood evaluation").  The NNF is the band of Chebyshev radius R    */
/* voxels around the occupied voxels; each band voxel v maps to the        */
/* occupied voxel u minimising (|v-u|^2 integer, gid(u)).                  */
/* gid order is ascending (vz, vy, vx).                                    */
/* ======================================================================= */
typedef struct {
    float r, inv_r, eps;
    float a32;     /* 1 - eps as the FP32 value the GPU uses */
    int R, min_pts;
    int32_t org[3], dim[3]; /* band grid: voxel v -> linear index of v - org */
    int64_t G;
    int32_t* vox;  /* G*3 voxel coordinates */
    float* mu;     /* G*3 FP32 (rounded from FP64) */
    float* cov;    /* G*6 FP32 */
    float* nrm;    /* G*3 FP32 unit normals: the map covariance is I - a32 n n^T */
    double* mu64;  /* G*3 */
    double* cov64; /* G*6 */
    int32_t* npts; /* G */
    int64_t nb;
    int64_t* bkey; /* nb, ascending linear index */
    int32_t* bgid; /* nb */
} mpo_map;

typedef struct { int32_t v[3]; int64_t idx; } vrec;

static int cmp_vrec(const void* a, const void* b) {
    const vrec* x = (const vrec*)a;
    const vrec* y = (const vrec*)b;
    for (int k = 2; k >= 0; --k) {
        if (x->v[k] != y->v[k]) return x->v[k] < y->v[k] ? -1 : 1;
    }
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

typedef struct { int64_t key; int32_t d2; int32_t gid; } brec;
static int cmp_brec(const void* a, const void* b) {
    const brec* x = (const brec*)a;
    const brec* y = (const brec*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->d2 != y->d2) return x->d2 < y->d2 ? -1 : 1;
    return (x->gid > y->gid) - (x->gid < y->gid);
}

/* voxel coordinate of a point: floor(x * (1/r)), FP32 */
MPO_API void mpo_voxel_of(const float* p, int64_t n, float r, int32_t* out) {
    float inv_r = 1.0f / r;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) out[3 * i + k] = floor_to_i32(p[3 * i + k] * inv_r);
}

static int64_t grid_key(const mpo_map* m, const int32_t v[3]) {
    int64_t x = (int64_t)v[0] - m->org[0], y = (int64_t)v[1] - m->org[1], z = (int64_t)v[2] - m->org[2];
    if (x < 0 || y < 0 || z < 0 || x >= m->dim[0] || y >= m->dim[1] || z >= m->dim[2]) return -1;
    return (z * m->dim[1] + y) * m->dim[0] + x;
}

MPO_API mpo_map* mpo_map_build(const float* xyz, int64_t n, float r, int R, int min_pts, float eps) {
    mpo_map* m = (mpo_map*)calloc(1, sizeof(mpo_map));
    m->r = r; m->inv_r = 1.0f / r; m->R = R; m->min_pts = min_pts; m->eps = eps;
    m->a32 = 1.0f - eps;
    vrec* recs = (vrec*)malloc(sizeof(vrec) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) recs[i].v[k] = floor_to_i32(xyz[3 * i + k] * m->inv_r);
        recs[i].idx = i;
    }
    qsort(recs, (size_t)n, sizeof(vrec), cmp_vrec);
    /* count kept voxels */
    int64_t G = 0;
    for (int64_t s = 0; s < n;) {
        int64_t e = s + 1;
        while (e < n && memcmp(recs[e].v, recs[s].v, sizeof(recs[s].v)) == 0) ++e;
        if (e - s >= min_pts) ++G;
        s = e;
    }
    m->G = G;
    m->vox = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)(G ? G : 1));
    m->mu = (float*)malloc(sizeof(float) * 3 * (size_t)(G ? G : 1));
    m->cov = (float*)malloc(sizeof(float) * 6 * (size_t)(G ? G : 1));
    m->nrm = (float*)malloc(sizeof(float) * 3 * (size_t)(G ? G : 1));
    m->mu64 = (double*)malloc(sizeof(double) * 3 * (size_t)(G ? G : 1));
    m->cov64 = (double*)malloc(sizeof(double) * 6 * (size_t)(G ? G : 1));
    m->npts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(G ? G : 1));
    int64_t g = 0;
    for (int64_t s = 0; s < n;) {
        int64_t e = s + 1;
        while (e < n && memcmp(recs[e].v, recs[s].v, sizeof(recs[s].v)) == 0) ++e;
        int64_t cnt = e - s;
        if (cnt >= min_pts) {
            /* mean: sequential FP64 sum in ascending point index */
            double sm[3] = {0, 0, 0};
            for (int64_t k = s; k < e; ++k)
                for (int a = 0; a < 3; ++a) sm[a] = sm[a] + (double)xyz[3 * recs[k].idx + a];
            double mu[3];
            for (int a = 0; a < 3; ++a) mu[a] = sm[a] / (double)cnt;
            /* maximum-likelihood covariance (1/n), centred */
            double S6[6] = {0, 0, 0, 0, 0, 0};
            for (int64_t k = s; k < e; ++k) {
                double d[3];
                for (int a = 0; a < 3; ++a) d[a] = (double)xyz[3 * recs[k].idx + a] - mu[a];
                S6[0] += d[0] * d[0]; S6[1] += d[0] * d[1]; S6[2] += d[0] * d[2];
                S6[3] += d[1] * d[1]; S6[4] += d[1] * d[2]; S6[5] += d[2] * d[2];
            }
            double S[9];
            for (int a = 0; a < 6; ++a) S6[a] /= (double)cnt;
            sym6_full(S6, S);
            double c6[6], nv[3];
            gicp_normalise(S, (double)eps, c6, nv);
            for (int a = 0; a < 3; ++a) m->nrm[3 * g + a] = (float)nv[a];
            for (int a = 0; a < 3; ++a) {
                m->vox[3 * g + a] = recs[s].v[a];
                m->mu64[3 * g + a] = mu[a];
                m->mu[3 * g + a] = (float)mu[a];
            }
            for (int a = 0; a < 6; ++a) { m->cov64[6 * g + a] = c6[a]; m->cov[6 * g + a] = (float)c6[a]; }
            m->npts[g] = (int32_t)cnt;
            ++g;
        }
        s = e;
    }
    free(recs);
    /* band grid */
    if (G > 0) {
        int32_t lo[3], hi[3];
        for (int a = 0; a < 3; ++a) { lo[a] = m->vox[a]; hi[a] = m->vox[a]; }
        for (int64_t k = 0; k < G; ++k)
            for (int a = 0; a < 3; ++a) {
                if (m->vox[3 * k + a] < lo[a]) lo[a] = m->vox[3 * k + a];
                if (m->vox[3 * k + a] > hi[a]) hi[a] = m->vox[3 * k + a];
            }
        for (int a = 0; a < 3; ++a) { m->org[a] = lo[a] - R; m->dim[a] = hi[a] - lo[a] + 1 + 2 * R; }
        int side = 2 * R + 1;
        int64_t ne = G * (int64_t)side * side * side;
        brec* br = (brec*)malloc(sizeof(brec) * (size_t)ne);
        int64_t q = 0;
        for (int64_t k = 0; k < G; ++k)
            for (int dz = -R; dz <= R; ++dz)
                for (int dy = -R; dy <= R; ++dy)
                    for (int dx = -R; dx <= R; ++dx) {
                        int32_t v[3] = {m->vox[3 * k] + dx, m->vox[3 * k + 1] + dy, m->vox[3 * k + 2] + dz};
                        br[q].key = grid_key(m, v);
                        br[q].d2 = dx * dx + dy * dy + dz * dz;
                        br[q].gid = (int32_t)k;
                        ++q;
                    }
        qsort(br, (size_t)ne, sizeof(brec), cmp_brec);
        int64_t nb = 0;
        for (int64_t k = 0; k < ne; ++k)
            if (k == 0 || br[k].key != br[k - 1].key) ++nb;
        m->nb = nb;
        m->bkey = (int64_t*)malloc(sizeof(int64_t) * (size_t)nb);
        m->bgid = (int32_t*)malloc(sizeof(int32_t) * (size_t)nb);
        int64_t j = 0;
        for (int64_t k = 0; k < ne; ++k)
            if (k == 0 || br[k].key != br[k - 1].key) { m->bkey[j] = br[k].key; m->bgid[j] = br[k].gid; ++j; }
        free(br);
    } else {
        m->nb = 0;
        m->bkey = (int64_t*)malloc(sizeof(int64_t));
        m->bgid = (int32_t*)malloc(sizeof(int32_t));
    }
    return m;
}

/* ======================================================================= */
/* Map of per-point Gaussians and its nearest-neighbour field, the paper's */
/* own construction (Sec. III-C): every map point p_k is a Gaussian        */
/* N(p_k, Sigma_k), Sigma_k from the point's neighbourhood (GICP, Segal et */
/* al. 2009), and the field, a grid of cell edge r, stores for each cell   */
/* the map point nearest to the cell's centre.                             */
/*   neighbourhood  the k nearest other points j, by the FP32 program       */
/*                  d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz)), dx = x_j - x_i */
/*                  (the scan covariances' program), ties to the lower      */
/*                  index, among the points whose voxel floor(p / r) lies   */
/*                  within Chebyshev distance S of the point's voxel        */
/*   Gaussian       FP64 mean and 1/(m) covariance of {p_i} U neighbours    */
/*                  (m = count, summed self first then in list order),      */
/*                  GICP-normalised: I - (1 - eps) n n^T; mu = p_i itself;  */
/*                  the point is kept when m >= min_pts                     */
/*   ids            kept points in ascending (vz, vy, vx, index)            */
/*   field          cell c (voxel coordinates) maps to the kept point       */
/*                  minimising (d2, id) with d2 = (ex*ex + ey*ey) + ez*ez,  */
/*                  e = p - ((float)c + 0.5) r (FP32), over points with     */
/*                  d2 <= (R r)^2; a point within R r of the centre has its */
/*                  voxel within Chebyshev R of c, so each kept point       */
/*                  proposes to the cells of that block only               */
/* Band keys carry d2 as its IEEE bit pattern (monotone for d2 >= 0).      */
/* ======================================================================= */
MPO_API mpo_map* mpo_map_build_points(const float* xyz, int64_t n, float r, int R, int k, int S, int min_pts,
                                      float eps, int32_t* knn_out /* n*k nullable, -1 pads */) {
    mpo_map* m = (mpo_map*)calloc(1, sizeof(mpo_map));
    m->r = r; m->inv_r = 1.0f / r; m->R = R; m->min_pts = min_pts; m->eps = eps;
    m->a32 = 1.0f - eps;
    int32_t* vx = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) vx[3 * i + a] = floor_to_i32(xyz[3 * i + a] * m->inv_r);
    double* c64 = (double*)malloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1));
    double* nv64 = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel
    {
        float* bd = (float*)malloc(sizeof(float) * (size_t)(k > 0 ? k : 1));
        int64_t* bj = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int32_t c = 0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                int far = 0;
                for (int a = 0; a < 3; ++a) {
                    int64_t dv = (int64_t)vx[3 * j + a] - vx[3 * i + a];
                    if (dv > S || dv < -S) far = 1;
                }
                if (far) continue;
                float dx = xyz[3 * j] - xyz[3 * i], dy = xyz[3 * j + 1] - xyz[3 * i + 1];
                float dz = xyz[3 * j + 2] - xyz[3 * i + 2];
                float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                int32_t p;
                if (c < k) p = c++;
                else if (d2 < bd[k - 1] || (d2 == bd[k - 1] && j < bj[k - 1])) p = k - 1;
                else continue;
                while (p > 0 && (bd[p - 1] > d2 || (bd[p - 1] == d2 && bj[p - 1] > j))) {
                    bd[p] = bd[p - 1]; bj[p] = bj[p - 1]; --p;
                }
                bd[p] = d2; bj[p] = j;
            }
            if (knn_out)
                for (int32_t a = 0; a < k; ++a) knn_out[i * k + a] = a < c ? (int32_t)bj[a] : -1;
            cnt[i] = c + 1;
            if (c + 1 < min_pts) continue;
            double sm[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
            for (int32_t a = 0; a < c; ++a)
                for (int q = 0; q < 3; ++q) sm[q] = sm[q] + (double)xyz[3 * bj[a] + q];
            double mu[3];
            for (int q = 0; q < 3; ++q) mu[q] = sm[q] / (double)(c + 1);
            double S6[6] = {0, 0, 0, 0, 0, 0};
            for (int32_t a = -1; a < c; ++a) {
                int64_t j = a < 0 ? i : bj[a];
                double d[3];
                for (int q = 0; q < 3; ++q) d[q] = (double)xyz[3 * j + q] - mu[q];
                S6[0] += d[0] * d[0]; S6[1] += d[0] * d[1]; S6[2] += d[0] * d[2];
                S6[3] += d[1] * d[1]; S6[4] += d[1] * d[2]; S6[5] += d[2] * d[2];
            }
            for (int q = 0; q < 6; ++q) S6[q] /= (double)(c + 1);
            double Sf[9];
            sym6_full(S6, Sf);
            gicp_normalise(Sf, (double)eps, c64 + 6 * i, nv64 + 3 * i);
        }
        free(bd);
        free(bj);
    }
    /* ids: kept points in ascending (vz, vy, vx, index) */
    vrec* recs = (vrec*)malloc(sizeof(vrec) * (size_t)(n > 0 ? n : 1));
    int64_t G = 0;
    for (int64_t i = 0; i < n; ++i)
        if (cnt[i] >= min_pts) {
            memcpy(recs[G].v, vx + 3 * i, sizeof(recs[G].v));
            recs[G].idx = i;
            ++G;
        }
    qsort(recs, (size_t)G, sizeof(vrec), cmp_vrec);
    m->G = G;
    size_t Ga = (size_t)(G ? G : 1);
    m->vox = (int32_t*)malloc(sizeof(int32_t) * 3 * Ga);
    m->mu = (float*)malloc(sizeof(float) * 3 * Ga);
    m->cov = (float*)malloc(sizeof(float) * 6 * Ga);
    m->nrm = (float*)malloc(sizeof(float) * 3 * Ga);
    m->mu64 = (double*)malloc(sizeof(double) * 3 * Ga);
    m->cov64 = (double*)malloc(sizeof(double) * 6 * Ga);
    m->npts = (int32_t*)malloc(sizeof(int32_t) * Ga);
    for (int64_t g = 0; g < G; ++g) {
        int64_t i = recs[g].idx;
        for (int a = 0; a < 3; ++a) {
            m->vox[3 * g + a] = recs[g].v[a];
            m->mu[3 * g + a] = xyz[3 * i + a];
            m->mu64[3 * g + a] = (double)xyz[3 * i + a];
            m->nrm[3 * g + a] = (float)nv64[3 * i + a];
        }
        for (int a = 0; a < 6; ++a) { m->cov64[6 * g + a] = c64[6 * i + a]; m->cov[6 * g + a] = (float)c64[6 * i + a]; }
        m->npts[g] = cnt[i];
    }
    free(c64); free(nv64); free(cnt); free(vx);
    /* field */
    if (G > 0) {
        int32_t lo[3], hi[3];
        for (int a = 0; a < 3; ++a) { lo[a] = m->vox[a]; hi[a] = m->vox[a]; }
        for (int64_t g = 0; g < G; ++g)
            for (int a = 0; a < 3; ++a) {
                if (m->vox[3 * g + a] < lo[a]) lo[a] = m->vox[3 * g + a];
                if (m->vox[3 * g + a] > hi[a]) hi[a] = m->vox[3 * g + a];
            }
        for (int a = 0; a < 3; ++a) { m->org[a] = lo[a] - R; m->dim[a] = hi[a] - lo[a] + 1 + 2 * R; }
        float lim = (float)R * r;
        float lim2 = lim * lim;
        int side = 2 * R + 1;
        int64_t ne = G * (int64_t)side * side * side;
        brec* br = (brec*)malloc(sizeof(brec) * (size_t)(ne > 0 ? ne : 1));
        int64_t q = 0;
        for (int64_t g = 0; g < G; ++g)
            for (int dz = -R; dz <= R; ++dz)
                for (int dy = -R; dy <= R; ++dy)
                    for (int dx = -R; dx <= R; ++dx) {
                        int32_t v[3] = {m->vox[3 * g] + dx, m->vox[3 * g + 1] + dy, m->vox[3 * g + 2] + dz};
                        float e[3];
                        for (int a = 0; a < 3; ++a) e[a] = m->mu[3 * g + a] - ((float)v[a] + 0.5f) * r;
                        float d2 = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2];
                        if (!(d2 <= lim2)) continue;
                        uint32_t bits;
                        memcpy(&bits, &d2, 4);
                        br[q].key = grid_key(m, v);
                        br[q].d2 = (int32_t)bits;
                        br[q].gid = (int32_t)g;
                        ++q;
                    }
        qsort(br, (size_t)q, sizeof(brec), cmp_brec);
        int64_t nb = 0;
        for (int64_t t = 0; t < q; ++t)
            if (t == 0 || br[t].key != br[t - 1].key) ++nb;
        m->nb = nb;
        m->bkey = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nb ? nb : 1));
        m->bgid = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nb ? nb : 1));
        int64_t j = 0;
        for (int64_t t = 0; t < q; ++t)
            if (t == 0 || br[t].key != br[t - 1].key) { m->bkey[j] = br[t].key; m->bgid[j] = br[t].gid; ++j; }
        free(br);
    } else {
        m->nb = 0;
        m->bkey = (int64_t*)malloc(sizeof(int64_t));
        m->bgid = (int32_t*)malloc(sizeof(int32_t));
    }
    free(recs);
    return m;
}

MPO_API void mpo_map_free(mpo_map* m) {
    if (!m) return;
    free(m->vox); free(m->mu); free(m->cov); free(m->nrm); free(m->mu64); free(m->cov64); free(m->npts);
    free(m->bkey); free(m->bgid); free(m);
}

MPO_API int64_t mpo_map_num_gauss(const mpo_map* m) { return m->G; }
MPO_API int64_t mpo_map_num_band(const mpo_map* m) { return m->nb; }
MPO_API void mpo_map_grid(const mpo_map* m, int32_t org[3], int32_t dim[3]) {
    memcpy(org, m->org, sizeof(m->org));
    memcpy(dim, m->dim, sizeof(m->dim));
}
MPO_API void mpo_map_gauss(const mpo_map* m, int32_t* vox, float* mu, float* cov, double* mu64, double* cov64,
                           int32_t* npts, float* nrm) {
    size_t G = (size_t)m->G;
    if (nrm) memcpy(nrm, m->nrm, sizeof(float) * 3 * G);
    if (vox) memcpy(vox, m->vox, sizeof(int32_t) * 3 * G);
    if (mu) memcpy(mu, m->mu, sizeof(float) * 3 * G);
    if (cov) memcpy(cov, m->cov, sizeof(float) * 6 * G);
    if (mu64) memcpy(mu64, m->mu64, sizeof(double) * 3 * G);
    if (cov64) memcpy(cov64, m->cov64, sizeof(double) * 6 * G);
    if (npts) memcpy(npts, m->npts, sizeof(int32_t) * G);
}
MPO_API void mpo_map_band(const mpo_map* m, int64_t* keys, int32_t* gids) {
    memcpy(keys, m->bkey, sizeof(int64_t) * (size_t)m->nb);
    memcpy(gids, m->bgid, sizeof(int32_t) * (size_t)m->nb);
}

/* NNF lookup of a voxel: gid or -1 */
static int32_t nnf_voxel(const mpo_map* m, const int32_t v[3]) {
    int64_t key = grid_key(m, v);
    if (key < 0 || m->nb == 0) return -1;
    int64_t lo = 0, hi = m->nb - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (m->bkey[mid] == key) return m->bgid[mid];
        if (m->bkey[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

MPO_API void mpo_map_lookup(const mpo_map* m, const float* p, int64_t n, int32_t* gid) {
    for (int64_t i = 0; i < n; ++i) {
        int32_t v[3];
        for (int k = 0; k < 3; ++k) v[k] = floor_to_i32(p[3 * i + k] * m->inv_r);
        gid[i] = nnf_voxel(m, v);
    }
}

/* ======================================================================= */
/* Scan covariances: k nearest other scan points by FP32 squared distance, */
/* ties by index; covariance of {self} U kNN (1/(k+1)), GICP-normalised.   */
/* ======================================================================= */
MPO_API void mpo_scan_cov(const float* xyz, int32_t n, int32_t k, float eps, int32_t* knn /* n*k, nullable */,
                          float* cov6 /* n*6 */, double* cov6_64 /* nullable */) {
    int32_t kk = k < n - 1 ? k : n - 1;
    float* bd = (float*)malloc(sizeof(float) * (size_t)(k > 0 ? k : 1));
    int32_t* bj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
    for (int32_t i = 0; i < n; ++i) {
        int32_t cnt = 0;
        for (int32_t j = 0; j < n; ++j) {
            if (j == i) continue;
            float dx = xyz[3 * j] - xyz[3 * i], dy = xyz[3 * j + 1] - xyz[3 * i + 1], dz = xyz[3 * j + 2] - xyz[3 * i + 2];
            float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            /* insert (d2, j) into the sorted list of the kk best */
            if (cnt < kk) {
                int32_t p = cnt++;
                while (p > 0 && (bd[p - 1] > d2 || (bd[p - 1] == d2 && bj[p - 1] > j))) { bd[p] = bd[p - 1]; bj[p] = bj[p - 1]; --p; }
                bd[p] = d2; bj[p] = j;
            } else if (kk > 0 && (d2 < bd[kk - 1] || (d2 == bd[kk - 1] && j < bj[kk - 1]))) {
                int32_t p = kk - 1;
                while (p > 0 && (bd[p - 1] > d2 || (bd[p - 1] == d2 && bj[p - 1] > j))) { bd[p] = bd[p - 1]; bj[p] = bj[p - 1]; --p; }
                bd[p] = d2; bj[p] = j;
            }
        }
        if (knn) for (int32_t a = 0; a < k; ++a) knn[(int64_t)i * k + a] = a < kk ? bj[a] : -1;
        double c6[6];
        if (kk + 1 < 5) {
            c6[0] = 1; c6[1] = 0; c6[2] = 0; c6[3] = 1; c6[4] = 0; c6[5] = 1;
        } else {
            double sm[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
            for (int32_t a = 0; a < kk; ++a)
                for (int c = 0; c < 3; ++c) sm[c] = sm[c] + (double)xyz[3 * bj[a] + c];
            double mu[3];
            for (int c = 0; c < 3; ++c) mu[c] = sm[c] / (double)(kk + 1);
            double S6[6] = {0, 0, 0, 0, 0, 0};
            for (int32_t a = -1; a < kk; ++a) {
                int32_t j = a < 0 ? i : bj[a];
                double d[3];
                for (int c = 0; c < 3; ++c) d[c] = (double)xyz[3 * j + c] - mu[c];
                S6[0] += d[0] * d[0]; S6[1] += d[0] * d[1]; S6[2] += d[0] * d[2];
                S6[3] += d[1] * d[1]; S6[4] += d[1] * d[2]; S6[5] += d[2] * d[2];
            }
            for (int c = 0; c < 6; ++c) S6[c] /= (double)(kk + 1);
            double S[9];
            sym6_full(S6, S);
            gicp_normalise(S, (double)eps, c6, NULL);
        }
        for (int c = 0; c < 6; ++c) {
            cov6[6 * (int64_t)i + c] = (float)c6[c];
            if (cov6_64) cov6_64[6 * (int64_t)i + c] = c6[c];
        }
    }
    free(bd);
    free(bj);
}

/* ======================================================================= */
/* Likelihood and Gauss-Newton displacement (Eq. 2-4).                      */
/*   e_k = mu^M - T mu^S,  Omega_k = (Sigma^M + R Sigma^S R^T)^-1,          */
/*   c_k = e_k^T Omega_k e_k; log-lik = -sum_k min(c_k, c_max) over inliers */
/*   and -c_max per outlier;  J_k = de_k/d delta for T exp(delta),          */
/*   delta = [omega; v]  =>  J_k = [R [mu^S]x , -R];                        */
/*   H = sum J^T Omega J, b = sum J^T Omega e (inliers, Omega held fixed);   */
/*   psi = -(H + diag(lam_rel H_ii + lam_abs))^-1 b.                       */
/* ======================================================================= */
static int chol6_solve(const double A_in[36], const double b[6], double x[6]) {
    double L[36];
    memset(L, 0, sizeof(L));
    for (int j = 0; j < 6; ++j) {
        double s = A_in[6 * j + j];
        for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
        if (!(s > 0.0)) return -1;
        L[6 * j + j] = sqrt(s);
        for (int i = j + 1; i < 6; ++i) {
            double t = A_in[6 * i + j];
            for (int k = 0; k < j; ++k) t -= L[6 * i + k] * L[6 * j + k];
            L[6 * i + j] = t / L[6 * j + j];
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= L[6 * i + k] * y[k];
        y[i] = t / L[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < 6; ++k) t -= L[6 * k + i] * x[k];
        x[i] = t / L[6 * i + i];
    }
    return 0;
}

/* Gauss-Newton step from H (21 upper entries) and b */
MPO_API int mpo_gn_step(const double H21[21], const double b[6], double lam_rel, double lam_abs, double psi[6]) {
    double A[36];
    int q = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) { A[6 * i + j] = H21[q]; A[6 * j + i] = H21[q]; ++q; }
    /* Levenberg-Marquardt damping scaled by the diagonal (Marquardt 1963) */
    for (int i = 0; i < 6; ++i) A[6 * i + i] += lam_rel * A[6 * i + i] + lam_abs;
    double nb[6];
    for (int i = 0; i < 6; ++i) nb[i] = -b[i];
    int rc = chol6_solve(A, nb, psi);
    if (rc != 0) for (int i = 0; i < 6; ++i) psi[i] = 0.0;
    return rc;
}

MPO_API void mpo_likelihood(const mpo_map* m, const float* sxyz, const float* scov, int32_t ns, const float* poses,
                            int64_t n, float dmax, float cmax, double lam_rel, double lam_abs, double* loglik,
                            double* H21, double* b6, double* psi6, int32_t* ninl) {
    float dmax2 = dmax * dmax;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        const float* T = poses + 8 * i;
        q32 q = {T[0], T[1], T[2], T[3]};
        float R32[9];
        q32_to_R(q, R32);
        float t32[3] = {T[4], T[5], T[6]};
        double qd[4] = {T[0], T[1], T[2], T[3]}, R[9], Rt[9];
        qd_to_R(qd, R);
        mat3_T(R, Rt);
        double t[3] = {T[4], T[5], T[6]};
        double ll = 0.0, H[36], b[6];
        memset(H, 0, sizeof(H));
        memset(b, 0, sizeof(b));
        int32_t ni = 0;
        for (int32_t k = 0; k < ns; ++k) {
            const float* ms = sxyz + 3 * (int64_t)k;
            float p32[3];
            xform32(R32, t32, ms, p32);
            int32_t v[3];
            for (int a = 0; a < 3; ++a) v[a] = floor_to_i32(p32[a] * m->inv_r);
            int32_t g = nnf_voxel(m, v);
            if (g < 0) { ll -= (double)cmax; continue; }
            const float* mm = m->mu + 3 * (int64_t)g;
            float e32[3] = {mm[0] - p32[0], mm[1] - p32[1], mm[2] - p32[2]};
            float d2 = fmaf(e32[0], e32[0], fmaf(e32[1], e32[1], e32[2] * e32[2]));
            if (!(d2 <= dmax2)) { ll -= (double)cmax; continue; }
            ++ni;
            /* FP64 from here */
            double mu[3] = {ms[0], ms[1], ms[2]};
            double p[3], e[3];
            for (int a = 0; a < 3; ++a) p[a] = R[3 * a] * mu[0] + R[3 * a + 1] * mu[1] + R[3 * a + 2] * mu[2] + t[a];
            for (int a = 0; a < 3; ++a) e[a] = (double)mm[a] - p[a];
            /* map covariance from the FP32 normal and a = 1 - eps (FP32), in FP64 */
            double SS6[6], SM[9], SS[9], tmp[9], RSR[9], C[9], Om[9];
            const float* nv = m->nrm + 3 * (int64_t)g;
            for (int r2 = 0; r2 < 3; ++r2)
                for (int c2 = 0; c2 < 3; ++c2)
                    SM[3 * r2 + c2] = (r2 == c2 ? 1.0 : 0.0) - (double)m->a32 * (double)nv[r2] * (double)nv[c2];
            for (int a = 0; a < 6; ++a) SS6[a] = scov[6 * (int64_t)k + a];
            sym6_full(SS6, SS);
            mat3_mul(R, SS, tmp);
            mat3_mul(tmp, Rt, RSR);
            for (int a = 0; a < 9; ++a) C[a] = SM[a] + RSR[a];
            mat3_inv(C, Om);
            double Oe[3];
            for (int a = 0; a < 3; ++a) Oe[a] = Om[3 * a] * e[0] + Om[3 * a + 1] * e[1] + Om[3 * a + 2] * e[2];
            double c = e[0] * Oe[0] + e[1] * Oe[1] + e[2] * Oe[2];
            ll -= (c < (double)cmax) ? c : (double)cmax;
            /* J = [R [mu]x , -R]  (3x6) */
            double Sk[9] = {0, -mu[2], mu[1], mu[2], 0, -mu[0], -mu[1], mu[0], 0};
            double RS[9];
            mat3_mul(R, Sk, RS);
            double J[18];
            for (int a = 0; a < 3; ++a)
                for (int cc = 0; cc < 3; ++cc) { J[6 * a + cc] = RS[3 * a + cc]; J[6 * a + 3 + cc] = -R[3 * a + cc]; }
            double OJ[18];
            for (int a = 0; a < 3; ++a)
                for (int cc = 0; cc < 6; ++cc)
                    OJ[6 * a + cc] = Om[3 * a] * J[cc] + Om[3 * a + 1] * J[6 + cc] + Om[3 * a + 2] * J[12 + cc];
            for (int r = 0; r < 6; ++r) {
                for (int cc = 0; cc < 6; ++cc)
                    H[6 * r + cc] += J[r] * OJ[cc] + J[6 + r] * OJ[6 + cc] + J[12 + r] * OJ[12 + cc];
                b[r] += J[r] * Oe[0] + J[6 + r] * Oe[1] + J[12 + r] * Oe[2];
            }
        }
        double h21[21];
        int q2 = 0;
        for (int r = 0; r < 6; ++r)
            for (int cc = r; cc < 6; ++cc) h21[q2++] = H[6 * r + cc];
        if (loglik) loglik[i] = ll;
        if (H21) memcpy(H21 + 21 * i, h21, sizeof(h21));
        if (b6) memcpy(b6 + 6 * i, b, sizeof(b));
        if (ninl) ninl[i] = ni;
        if (psi6) mpo_gn_step(h21, b, lam_rel, lam_abs, psi6 + 6 * i);
    }
}

/* ======================================================================= */
/* Alg. 1 lines 2-5: distribute particles into buckets.  Stable order by   */
/* (code, index); head/end of each run.  Pinned by numpy stable argsort.    */
/* ======================================================================= */
typedef struct { uint32_t code; int32_t idx; } crec;
static int cmp_crec(const void* a, const void* b) {
    const crec* x = (const crec*)a;
    const crec* y = (const crec*)b;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

MPO_API void mpo_bucket_sort(const uint32_t* codes, int64_t n, int32_t* sorted_idx, int32_t* head, int32_t* end) {
    crec* r = (crec*)malloc(sizeof(crec) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { r[i].code = codes[i]; r[i].idx = (int32_t)i; }
    qsort(r, (size_t)n, sizeof(crec), cmp_crec);
    for (int64_t s = 0; s < n; ++s) sorted_idx[s] = r[s].idx;
    for (int64_t s = 0; s < n;) {
        int64_t e = s + 1;
        while (e < n && r[e].code == r[s].code) ++e;
        for (int64_t k = s; k < e; ++k) { if (head) head[k] = (int32_t)s; if (end) end[k] = (int32_t)e; }
        s = e;
    }
    free(r);
}

/* ======================================================================= */
/* Alg. 1 lines 6-12: refresh the neighbour list of each particle.          */
/* Candidates: previous list, self, and the window of up to C bucket-mates */
/* following the particle in sorted order (cyclic within the bucket).  The */
/* list keeps self first, then the K-1 others with the smallest (q_ij, j). */
/* ======================================================================= */
MPO_API void mpo_refresh(const float* poses, int64_t n, const int32_t* sorted_idx, const uint32_t* codes, int32_t K,
                         int32_t C, float sigma_r, float sigma_t, const int32_t* old_nbr /* n*K row per particle */,
                         int32_t* nbr_out /* n*K */, float* q_out /* n*K */, int32_t* cnt_out) {
    int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t s = 0; s < n; ++s) pos[sorted_idx[s]] = (int32_t)s;
#pragma omp parallel
    {
        int32_t cap = K + C + 1;
        int32_t* cj = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
        float* cq = (float*)malloc(sizeof(float) * (size_t)cap);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int32_t nc = 0;
            /* bucket of i */
            int64_t s = pos[i];
            int64_t h = s, e = s + 1;
            while (h > 0 && codes[sorted_idx[h - 1]] == codes[i]) --h;
            while (e < n && codes[sorted_idx[e]] == codes[i]) ++e;
            int64_t msz = e - h;
            int64_t w = msz - 1 < C ? msz - 1 : C;
            for (int64_t d = 1; d <= w; ++d) cj[nc++] = sorted_idx[h + ((s - h + d) % msz)];
            for (int32_t a = 0; a < K; ++a) {
                int32_t j = old_nbr ? old_nbr[i * K + a] : -1;
                if (j >= 0 && j != (int32_t)i) cj[nc++] = j;
            }
            /* dedupe */
            int32_t m2 = 0;
            for (int32_t a = 0; a < nc; ++a) {
                int dup = 0;
                for (int32_t b2 = 0; b2 < m2; ++b2)
                    if (cj[b2] == cj[a]) { dup = 1; break; }
                if (!dup) cj[m2++] = cj[a];
            }
            for (int32_t a = 0; a < m2; ++a) cq[a] = mpo_det_qdist(poses + 8 * i, poses + 8 * (int64_t)cj[a], sigma_r, sigma_t);
            /* selection sort by (q, j) of the K-1 best */
            int32_t keep = m2 < K - 1 ? m2 : K - 1;
            for (int32_t a = 0; a < keep; ++a) {
                int32_t best = a;
                for (int32_t b2 = a + 1; b2 < m2; ++b2)
                    if (cq[b2] < cq[best] || (cq[b2] == cq[best] && cj[b2] < cj[best])) best = b2;
                int32_t tj = cj[a]; cj[a] = cj[best]; cj[best] = tj;
                float tq = cq[a]; cq[a] = cq[best]; cq[best] = tq;
            }
            nbr_out[i * K] = (int32_t)i;
            if (q_out) q_out[i * K] = 0.0f;
            for (int32_t a = 0; a < K - 1; ++a) {
                nbr_out[i * K + 1 + a] = a < keep ? cj[a] : -1;
                if (q_out) q_out[i * K + 1 + a] = a < keep ? cq[a] : INFINITY;
            }
            cnt_out[i] = 1 + keep;
        }
        free(cj);
        free(cq);
    }
    free(pos);
}

/* ======================================================================= */
/* FP64 SE(3): exp, log (coupled), composition.  Pinned against scipy's    */
/* expm/logm of the 4x4 homogeneous matrix.                                 */
/* ======================================================================= */
/* T (q,t) as 7 doubles */
MPO_API void mpo_se3_exp(const double xi[6], double T[7]) {
    const double* w = xi;
    const double* v = xi + 3;
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2);
    double A, B, hs, hc;
    if (th < 1e-5) {
        A = 0.5 - th2 / 24.0;
        B = 1.0 / 6.0 - th2 / 120.0;
        hs = 0.5 - th2 / 48.0; /* sin(th/2)/th */
        hc = 1.0 - th2 / 8.0;
    } else {
        A = (1.0 - cos(th)) / th2;
        B = (th - sin(th)) / (th2 * th);
        hs = sin(0.5 * th) / th;
        hc = cos(0.5 * th);
    }
    T[0] = hc; T[1] = hs * w[0]; T[2] = hs * w[1]; T[3] = hs * w[2];
    double c1[3] = {w[1] * v[2] - w[2] * v[1], w[2] * v[0] - w[0] * v[2], w[0] * v[1] - w[1] * v[0]};
    double c2[3] = {w[1] * c1[2] - w[2] * c1[1], w[2] * c1[0] - w[0] * c1[2], w[0] * c1[1] - w[1] * c1[0]};
    for (int k = 0; k < 3; ++k) T[4 + k] = v[k] + A * c1[k] + B * c2[k];
}

MPO_API void mpo_se3_log(const double T[7], double xi[6]) {
    double q[4] = {T[0], T[1], T[2], T[3]};
    double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) q[k] /= nq;
    if (q[0] < 0) for (int k = 0; k < 4; ++k) q[k] = -q[k];
    double n = sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double th = 2.0 * atan2(n, q[0]);
    double sc = (n < 1e-12) ? 2.0 / q[0] : th / n;
    double w[3] = {sc * q[1], sc * q[2], sc * q[3]};
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double beta;
    if (th2 < 1e-6) beta = 1.0 / 12.0 + th2 / 720.0;
    else beta = (1.0 - 0.5 * th * cos(0.5 * th) / sin(0.5 * th)) / th2;
    const double* t = T + 4;
    double c1[3] = {w[1] * t[2] - w[2] * t[1], w[2] * t[0] - w[0] * t[2], w[0] * t[1] - w[1] * t[0]};
    double c2[3] = {w[1] * c1[2] - w[2] * c1[1], w[2] * c1[0] - w[0] * c1[2], w[0] * c1[1] - w[1] * c1[0]};
    for (int k = 0; k < 3; ++k) { xi[k] = w[k]; xi[3 + k] = t[k] - 0.5 * c1[k] + beta * c2[k]; }
}

static void se3_compose(const double A[7], const double B[7], double C[7]) {
    double R[9];
    qd_to_R(A, R);
    double q[4];
    qd_mul(A, B, q);
    for (int k = 0; k < 4; ++k) C[k] = q[k];
    for (int a = 0; a < 3; ++a) C[4 + a] = A[4 + a] + R[3 * a] * B[4] + R[3 * a + 1] * B[5] + R[3 * a + 2] * B[6];
}

static void se3_inv(const double A[7], double B[7]) {
    double R[9];
    qd_to_R(A, R);
    B[0] = A[0]; B[1] = -A[1]; B[2] = -A[2]; B[3] = -A[3];
    for (int a = 0; a < 3; ++a) B[4 + a] = -(R[a] * A[4] + R[3 + a] * A[5] + R[6 + a] * A[6]);
}

static void pose_to_d(const float* p, double T[7]) { for (int k = 0; k < 7; ++k) T[k] = (double)p[k]; }

/* T_i^-1 T_j in FP64 */
static void se3_rel(const float* Ti, const float* Tj, double C[7]) {
    double A[7], B[7], Ai[7];
    pose_to_d(Ti, A);
    pose_to_d(Tj, B);
    se3_inv(A, Ai);
    se3_compose(Ai, B, C);
}

/* d_ij = log(T_i^-1 T_j) in FP64 (Eq. 8) */
MPO_API void mpo_se3_between(const float* Ti, const float* Tj, double d[6]) {
    double C[7];
    se3_rel(Ti, Tj, C);
    mpo_se3_log(C, d);
}

/* ad of xi = [om; rho] in the tangent order [rotation; translation]:
 * [[om^, 0], [rho^, om^]], row-major 6x6 */
static void se3_ad(const double xi[6], double A[36]) {
    memset(A, 0, sizeof(double) * 36);
    for (int blk = 0; blk < 3; ++blk) {
        const double* v = blk == 1 ? xi + 3 : xi;
        int r0 = blk == 0 ? 0 : 3, c0 = blk == 2 ? 3 : 0;
        A[6 * (r0 + 0) + c0 + 1] = -v[2]; A[6 * (r0 + 0) + c0 + 2] = v[1];
        A[6 * (r0 + 1) + c0 + 0] = v[2];  A[6 * (r0 + 1) + c0 + 2] = -v[0];
        A[6 * (r0 + 2) + c0 + 0] = -v[1]; A[6 * (r0 + 2) + c0 + 1] = v[0];
    }
}

/* inverse of a 6x6 matrix by Gauss-Jordan elimination with partial pivoting;
 * returns 0 when a pivot vanishes */
static int inv6(const double A_in[36], double X[36]) {
    double A[36];
    memcpy(A, A_in, sizeof(A));
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) X[6 * r + c] = r == c ? 1.0 : 0.0;
    for (int c = 0; c < 6; ++c) {
        int piv = c;
        for (int r = c + 1; r < 6; ++r)
            if (fabs(A[6 * r + c]) > fabs(A[6 * piv + c])) piv = r;
        if (A[6 * piv + c] == 0.0) return 0;
        for (int k = 0; k < 6; ++k) {
            double t = A[6 * c + k]; A[6 * c + k] = A[6 * piv + k]; A[6 * piv + k] = t;
            t = X[6 * c + k]; X[6 * c + k] = X[6 * piv + k]; X[6 * piv + k] = t;
        }
        double ip = 1.0 / A[6 * c + c];
        for (int k = 0; k < 6; ++k) { A[6 * c + k] *= ip; X[6 * c + k] *= ip; }
        for (int r = 0; r < 6; ++r) {
            if (r == c) continue;
            double f = A[6 * r + c];
            if (f == 0.0) continue;
            for (int k = 0; k < 6; ++k) { A[6 * r + k] -= f * A[6 * c + k]; X[6 * r + k] -= f * X[6 * c + k]; }
        }
    }
    return 1;
}

/* Inverse right Jacobian of SE(3): J_r(xi) = sum_{n >= 0} (-ad_xi)^n / (n+1)!
 * is the derivative of exp(xi + e) against exp(xi) exp(J_r e); its inverse
 * gives log(exp(xi) exp(e)) = xi + J_r^-1(xi) e + O(e^2).  The series is
 * summed until its terms vanish in FP64, then inverted (|om| < 2 pi).
 * Pinned by central differences of log(exp(xi) exp(e)) through matrix
 * exponential and logarithm, and by I + ad/2 for small xi. */
MPO_API int32_t mpo_se3_jr_inv(const double xi[6], double Ji[36]) {
    double ad[36], term[36], Jr[36], nxt[36];
    se3_ad(xi, ad);
    for (int k = 0; k < 36; ++k) { term[k] = (k % 7 == 0) ? 1.0 : 0.0; Jr[k] = term[k]; }
    for (int n = 1; n <= 200; ++n) {
        double mx = 0.0;
        for (int r = 0; r < 6; ++r)
            for (int c = 0; c < 6; ++c) {
                double s = 0.0;
                for (int m = 0; m < 6; ++m) s += term[6 * r + m] * ad[6 * m + c];
                nxt[6 * r + c] = -s / (double)(n + 1);
            }
        for (int k = 0; k < 36; ++k) {
            term[k] = nxt[k];
            Jr[k] += term[k];
            if (fabs(term[k]) > mx) mx = fabs(term[k]);
        }
        if (mx < 1e-300 || (n > 6 && mx < 1e-18)) break;
    }
    return inv6(Jr, Ji) ? 0 : -1;
}

/* Adjoint of T = (R, t) in the tangent order [rotation; translation]:
 * T exp(xi) T^-1 = exp(Ad_T xi),  Ad_T = [[R, 0], [t^ R, R]] */
static void se3_Ad(const double T[7], double Ad[36]) {
    double R[9];
    qd_to_R(T, R);
    const double* t = T + 4;
    double tx[9] = {0, -t[2], t[1], t[2], 0, -t[0], -t[1], t[0], 0};
    memset(Ad, 0, sizeof(double) * 36);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            Ad[6 * r + c] = R[3 * r + c];
            Ad[6 * (r + 3) + c + 3] = R[3 * r + c];
            double s = 0.0;
            for (int m = 0; m < 3; ++m) s += tx[3 * r + m] * R[3 * m + c];
            Ad[6 * (r + 3) + c] = s;
        }
}

/* ======================================================================= */
/* Modified SVGD update (Eq. 5-8):                                          */
/*   phi_i = sum_j (k_ij psi_j + grad_{T_j} k_ij) / sum_j k_ij,             */
/*   k_ij = exp(-d_ij^T W d_ij),  d_ij = log(T_i^-1 T_j),                    */
/*   T_i <- T_i exp(phi_i), all neighbours at the pre-update poses.          */
/* The kernel gradient with respect to a right perturbation of T_j is       */
/*   grad_exact 0:  -2 k_ij W d_ij            (J_r^-1(d_ij) taken as I)     */
/*   grad_exact 1:  -2 k_ij J_r^-1(d_ij)^T W d_ij                           */
/* and with transport 1 each neighbour's vector k_ij psi_j + grad, which    */
/* lives in the tangent at T_j, is carried to the tangent at T_i by         */
/* Ad_{T_i^-1 T_j} before the sum.                                          */
/* Pinned by: K = 1 gives psi; two-particle closed form; full-set direct    */
/* sums whose gradient is a finite difference of k and whose transport is   */
/* M_ij xi^ M_ij^-1, all through matrix exponential and logarithm.          */
/* ======================================================================= */
MPO_API void mpo_svgd(const float* poses, int64_t n, const double* psi /* n*6 */, const int32_t* nbr, int32_t K,
                      float sigma_r, float sigma_t, int32_t grad_exact, int32_t transport,
                      double* phi_out /* n*6 nullable */, double* poses_out /* n*7 */) {
    double W[6] = {sigma_r, sigma_r, sigma_r, sigma_t, sigma_t, sigma_t};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double num[6] = {0, 0, 0, 0, 0, 0}, den = 0.0;
        for (int32_t a = 0; a < K; ++a) {
            int32_t j = nbr[i * K + a];
            if (j < 0) continue;
            double Tij[7], d[6];
            se3_rel(poses + 8 * i, poses + 8 * (int64_t)j, Tij);
            mpo_se3_log(Tij, d);
            double qv = 0.0;
            for (int c = 0; c < 6; ++c) qv += W[c] * d[c] * d[c];
            double kij = exp(-qv);
            den += kij;
            double wd[6], g[6], v[6];
            for (int c = 0; c < 6; ++c) wd[c] = W[c] * d[c];
            if (grad_exact) {
                double Ji[36];
                mpo_se3_jr_inv(d, Ji);
                for (int c = 0; c < 6; ++c) {
                    double s = 0.0;
                    for (int m = 0; m < 6; ++m) s += Ji[6 * m + c] * wd[m];
                    g[c] = -2.0 * kij * s;
                }
            } else {
                for (int c = 0; c < 6; ++c) g[c] = -2.0 * kij * wd[c];
            }
            for (int c = 0; c < 6; ++c) v[c] = kij * psi[6 * (int64_t)j + c] + g[c];
            if (transport) {
                double Ad[36], u[6];
                se3_Ad(Tij, Ad);
                for (int r = 0; r < 6; ++r) {
                    double s = 0.0;
                    for (int m = 0; m < 6; ++m) s += Ad[6 * r + m] * v[m];
                    u[r] = s;
                }
                memcpy(v, u, sizeof(v));
            }
            for (int c = 0; c < 6; ++c) num[c] += v[c];
        }
        double phi[6];
        for (int c = 0; c < 6; ++c) phi[c] = den > 0 ? num[c] / den : 0.0;
        if (phi_out) memcpy(phi_out + 6 * i, phi, sizeof(phi));
        double T[7], E[7], Tn[7];
        pose_to_d(poses + 8 * i, T);
        mpo_se3_exp(phi, E);
        se3_compose(T, E, Tn);
        double nq = sqrt(Tn[0] * Tn[0] + Tn[1] * Tn[1] + Tn[2] * Tn[2] + Tn[3] * Tn[3]);
        for (int k = 0; k < 4; ++k) Tn[k] /= nq;
        memcpy(poses_out + 7 * i, Tn, sizeof(Tn));
    }
}

/* ======================================================================= */
/* Posterior on the neighbour graph (Sec. III-D, Eq. 11).                   */
/*   l_i = log max(pi_i, floor) + loglik_i / tau;  p = softmax(l) (FP64     */
/*   log-sum-exp);  R rounds of p'_i = sum_j k_ij p_j / sum_j k_ij with      */
/*   k_ij = exp(-q_ij) of the neighbour lists; renormalise; MAP = argmax,    */
/*   ties to the smallest index.                                            */
/* ======================================================================= */
MPO_API int64_t mpo_posterior(const double* prior, const double* loglik, int64_t n, const int32_t* nbr,
                              const double* kval /* n*K kernel values k_ij */, int32_t K, int32_t rounds, double tau,
                              double prior_floor, double* p0_out /* n nullable */, double* post_out /* n */,
                              double* neff_out) {
    double* l = (double*)malloc(sizeof(double) * (size_t)n);
    double* a = (double*)malloc(sizeof(double) * (size_t)n);
    double* b = (double*)malloc(sizeof(double) * (size_t)n);
    double mx = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double pr = prior[i] > prior_floor ? prior[i] : prior_floor;
        l[i] = log(pr) + loglik[i] / tau;
        if (l[i] > mx) mx = l[i];
    }
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += exp(l[i] - mx);
    double ls = log(s);
    for (int64_t i = 0; i < n; ++i) a[i] = exp(l[i] - mx - ls);
    if (p0_out) memcpy(p0_out, a, sizeof(double) * (size_t)n);
    for (int32_t r = 0; r < rounds; ++r) {
        for (int64_t i = 0; i < n; ++i) {
            double num = 0.0, den = 0.0;
            for (int32_t c = 0; c < K; ++c) {
                int32_t j = nbr[i * K + c];
                if (j < 0) continue;
                num += kval[i * K + c] * a[j];
                den += kval[i * K + c];
            }
            b[i] = den > 0 ? num / den : a[i];
        }
        double* t = a; a = b; b = t;
    }
    double z = 0.0;
    for (int64_t i = 0; i < n; ++i) z += a[i];
    int64_t best = 0;
    double e2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        post_out[i] = a[i] / z;
        e2 += post_out[i] * post_out[i];
        if (post_out[i] > post_out[best]) best = i;
    }
    if (neff_out) *neff_out = 1.0 / e2;
    free(l); free(a); free(b);
    return best;
}

/* ======================================================================= */
/* Prediction step (Eq. 1):  T_i <- T_i dT exp(delta_i),                    */
/* delta_i = L z_i with L the Cholesky factor of Sigma^dT (FP64).          */
/* ======================================================================= */
MPO_API int mpo_chol6(const double A[36], double L[36]) {
    memset(L, 0, sizeof(double) * 36);
    for (int j = 0; j < 6; ++j) {
        double s = A[6 * j + j];
        for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
        if (s < 0.0) return -1;
        L[6 * j + j] = sqrt(s);
        for (int i = j + 1; i < 6; ++i) {
            double t = A[6 * i + j];
            for (int k = 0; k < j; ++k) t -= L[6 * i + k] * L[6 * j + k];
            L[6 * i + j] = L[6 * j + j] > 0 ? t / L[6 * j + j] : 0.0;
        }
    }
    return 0;
}

/* T_i dT exp(L z_i), z_i ~ N(0, I6) drawn for (i, frame) under `purpose` */
static void predict_purpose(const float* poses, int64_t n, const float dT[7], const float cov[36], uint64_t seed,
                            uint32_t frame, uint32_t purpose, double* poses_out);

MPO_API void mpo_predict(const float* poses, int64_t n, const float dT[7], const float cov[36] /* nullable */,
                         uint64_t seed, uint32_t frame, double* poses_out /* n*7 */) {
    predict_purpose(poses, n, dT, cov, seed, frame, MPO_PURPOSE_PRED, poses_out);
}

/* Gaussian initial particles around a pose (tracking start): T_i = M exp(L z_i)
 * with L L^T = cov, the draw of Eq. (1)'s prediction noise taken about M
 * (purpose 7, frame 0).  Pinned by the sample covariance of log(M^-1 T_i) and
 * by a zero covariance. */
MPO_API void mpo_init_gauss(uint64_t seed, int64_t n, const float mean[7], const float cov[36],
                            double* poses_out /* n*7 */) {
    float* P = (float*)malloc(sizeof(float) * 8 * (size_t)(n > 0 ? n : 1));
    double nq = 0.0;
    for (int k = 0; k < 4; ++k) nq += (double)mean[k] * (double)mean[k];
    nq = sqrt(nq);
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 4; ++k) P[8 * i + k] = (float)((double)mean[k] / nq);
        for (int k = 4; k < 7; ++k) P[8 * i + k] = mean[k];
        P[8 * i + 7] = 0.0f;
    }
    const float ident[7] = {1, 0, 0, 0, 0, 0, 0};
    predict_purpose(P, n, ident, cov, seed, 0u, MPO_PURPOSE_INITG, poses_out);
    free(P);
}

static void predict_purpose(const float* poses, int64_t n, const float dT[7], const float cov[36], uint64_t seed,
                            uint32_t frame, uint32_t purpose, double* poses_out) {
    double L[36];
    int noise = 0;
    if (cov) {
        double A[36];
        for (int k = 0; k < 36; ++k) A[k] = cov[k];
        noise = (mpo_chol6(A, L) == 0);
    }
    double D[7];
    for (int k = 0; k < 7; ++k) D[k] = dT[k];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double T[7], TD[7], out[7];
        pose_to_d(poses + 8 * i, T);
        se3_compose(T, D, TD);
        if (noise) {
            float z[6];
            mpo_gauss6(seed, (uint32_t)i, frame, 0u, purpose, z);
            double dl[6];
            for (int r = 0; r < 6; ++r) {
                double s = 0.0;
                for (int c = 0; c <= r; ++c) s += L[6 * r + c] * (double)z[c];
                dl[r] = s;
            }
            double E[7];
            mpo_se3_exp(dl, E);
            se3_compose(TD, E, out);
        } else {
            memcpy(out, TD, sizeof(out));
        }
        double nq = sqrt(out[0] * out[0] + out[1] * out[1] + out[2] * out[2] + out[3] * out[3]);
        for (int k = 0; k < 4; ++k) out[k] /= nq;
        memcpy(poses_out + 7 * i, out, sizeof(out));
    }
}

MPO_API int mpo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the timing loops (results do not depend on it) */
MPO_API void mpo_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ======================================================================= */
/* Learned surrogate of the map's per-point score.                          */
/*                                                                          */
/* Score field: the per-point GICP cost with the scan covariance replaced   */
/* by sigma_s^2 I, so it depends on position only.  For an inlier (NNF hit  */
/* and |e| <= d_max, e = mu_g - p): s = e^T (Sigma^M_g + sigma_s^2 I)^-1 e,  */
/* grad s = -2 Omega e, untruncated, as the plain path's H and b are.       */
/* Residual field (the surrogate's target): r = sqrt(s),                    */
/* grad r = grad s / (2 max(r, r_floor)) for an inlier; r = r_out, grad r = */
/* 0 otherwise (r_out = d_max / sqrt(eps + sigma_s^2), the largest r inside */
/* the gate).                                                               */
/* Network: x~ = (p - lo) * inv_ext (FP32), 32 geometric frequencies per    */
/* axis, features sin/cos(2 pi frac(f_l x~_a)) ordered (axis, frequency,   */
/* sin|cos) -> 192 -> 128 -> 128 -> 4 with SiLU; outputs (r, grad r) scaled.*/
/* ======================================================================= */

/* score field at one FP32 point; returns 1 for an inlier (s, grad s set) */
static int sf_point(const mpo_map* m, const float q[3], float sigma_s, float dmax2, double* s_out, double g_out[3]) {
    double beta = 1.0 + (double)sigma_s * (double)sigma_s;
    int32_t v[3];
    for (int a = 0; a < 3; ++a) v[a] = floor_to_i32(q[a] * m->inv_r);
    int32_t g = nnf_voxel(m, v);
    *s_out = 0.0;
    g_out[0] = g_out[1] = g_out[2] = 0.0;
    if (g < 0) return 0;
    const float* mm = m->mu + 3 * (int64_t)g;
    float e32[3] = {mm[0] - q[0], mm[1] - q[1], mm[2] - q[2]};
    float d2 = fmaf(e32[0], e32[0], fmaf(e32[1], e32[1], e32[2] * e32[2]));
    if (!(d2 <= dmax2)) return 0;
    double e[3] = {(double)mm[0] - q[0], (double)mm[1] - q[1], (double)mm[2] - q[2]};
    const float* nv = m->nrm + 3 * (int64_t)g;
    double C[9], Om[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            C[3 * r + c] = (r == c ? beta : 0.0) - (double)m->a32 * (double)nv[r] * (double)nv[c];
    mat3_inv(C, Om);
    double Oe[3];
    for (int a = 0; a < 3; ++a) Oe[a] = Om[3 * a] * e[0] + Om[3 * a + 1] * e[1] + Om[3 * a + 2] * e[2];
    *s_out = e[0] * Oe[0] + e[1] * Oe[1] + e[2] * Oe[2];
    for (int a = 0; a < 3; ++a) g_out[a] = -2.0 * Oe[a];
    return 1;
}

/* residual field at one FP32 point */
static int rf_point(const mpo_map* m, const float q[3], float sigma_s, float dmax2, double r_floor, double r_out,
                    double* r_ret, double g_ret[3]) {
    double s, gs[3];
    int inl = sf_point(m, q, sigma_s, dmax2, &s, gs);
    if (!inl) {
        *r_ret = r_out;
        g_ret[0] = g_ret[1] = g_ret[2] = 0.0;
        return 0;
    }
    double r = sqrt(s);
    double d = 2.0 * (r > r_floor ? r : r_floor);
    *r_ret = r;
    for (int a = 0; a < 3; ++a) g_ret[a] = gs[a] / d;
    return 1;
}

MPO_API void mpo_score_field(const mpo_map* m, const float* p, int64_t n, float sigma_s, float dmax, double* s_out,
                             double* g_out, int32_t* inl_out) {
    float dmax2 = dmax * dmax;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double gr[3];
        int inl = sf_point(m, p + 3 * i, sigma_s, dmax2, &s_out[i], gr);
        if (g_out) for (int a = 0; a < 3; ++a) g_out[3 * i + a] = gr[a];
        if (inl_out) inl_out[i] = inl;
    }
}

MPO_API void mpo_residual_field(const mpo_map* m, const float* p, int64_t n, float sigma_s, float dmax,
                                double r_floor, double r_out, double* r_ret, double* g_ret) {
    float dmax2 = dmax * dmax;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double gr[3];
        rf_point(m, p + 3 * i, sigma_s, dmax2, r_floor, r_out, &r_ret[i], gr);
        for (int a = 0; a < 3; ++a) g_ret[3 * i + a] = gr[a];
    }
}

/* round a double to the nearest bfloat16 (ties to even), returned as double */
MPO_API double mpo_bf16_round(double x) {
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (double)f;
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* geometric frequencies, cycles per unit of the normalised coordinate */
MPO_API void mpo_ff_freqs(float fmax, int nf, float* f) {
    for (int l = 0; l < nf; ++l) f[l] = (float)pow((double)fmax, nf > 1 ? (double)l / (double)(nf - 1) : 0.0);
}

static void ff_point(const float p[3], const float lo[3], const float inv_ext[3], const float* freqs, int nf,
                     int bf16, double* o) {
    const double tau = 6.283185307179586476925;
    for (int a = 0; a < 3; ++a) {
        float x = (p[a] - lo[a]) * inv_ext[a];
        for (int l = 0; l < nf; ++l) {
            float t = freqs[l] * x;
            float fr = t - floorf(t);
            double ang = tau * (double)fr;
            double sv = sin(ang), cv = cos(ang);
            o[2 * (a * nf + l)] = bf16 ? mpo_bf16_round(sv) : sv;
            o[2 * (a * nf + l) + 1] = bf16 ? mpo_bf16_round(cv) : cv;
        }
    }
}

MPO_API void mpo_ff_features(const float* p, int64_t n, const float lo[3], const float inv_ext[3], const float* freqs,
                             int nf, int bf16, double* feat /* n x 6 nf */) {
    for (int64_t i = 0; i < n; ++i) ff_point(p + 3 * i, lo, inv_ext, freqs, nf, bf16, feat + (size_t)i * 6 * nf);
}

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double silu_d(double z) {
    double sg = 1.0 / (1.0 + exp(-z));
    return sg * (1.0 + z * (1.0 - sg));
}

/* parameter vector layout (all FP64 here, FP32 master copies on the GPU):
 * W1 [D0][D1] (input-major), b1 [D1], W2 [D1][D2], b2 [D2], W3 [D2][4], b3 [4] */
MPO_API int64_t mpo_mlp_nparams(int d0, int d1, int d2) {
    return (int64_t)d0 * d1 + d1 + (int64_t)d1 * d2 + d2 + (int64_t)d2 * 4 + 4;
}

static double rnd(double x, int bf16) { return bf16 ? mpo_bf16_round(x) : x; }

/* one sample; bf16 != 0 rounds the GEMM operands (weights and the layer
 * inputs x, h1, h2) to bfloat16 as the GPU does, accumulating in FP64 */
static void mlp_fwd1(const double* P, int d0, int d1, int d2, const double* x, int bf16, double* z1, double* h1,
                     double* z2, double* h2, double y[4]) {
    const double* W1 = P;
    const double* b1 = W1 + (size_t)d0 * d1;
    const double* W2 = b1 + d1;
    const double* b2 = W2 + (size_t)d1 * d2;
    const double* W3 = b2 + d2;
    const double* b3 = W3 + (size_t)d2 * 4;
    for (int j = 0; j < d1; ++j) {
        double z = 0.0;
        for (int k = 0; k < d0; ++k) z += rnd(x[k], bf16) * rnd(W1[(size_t)k * d1 + j], bf16);
        z1[j] = z + b1[j];
        h1[j] = rnd(silu(z1[j]), bf16);
    }
    for (int j = 0; j < d2; ++j) {
        double z = 0.0;
        for (int k = 0; k < d1; ++k) z += h1[k] * rnd(W2[(size_t)k * d2 + j], bf16);
        z2[j] = z + b2[j];
        h2[j] = rnd(silu(z2[j]), bf16);
    }
    for (int j = 0; j < 4; ++j) {
        double z = 0.0;
        for (int k = 0; k < d2; ++k) z += h2[k] * rnd(W3[(size_t)k * 4 + j], bf16);
        y[j] = z + b3[j];
    }
}

MPO_API void mpo_mlp_forward(const double* P, int d0, int d1, int d2, const double* X, int64_t n, int bf16,
                             double* Y /* n x 4 */) {
#pragma omp parallel
    {
        double* buf = (double*)malloc(sizeof(double) * (size_t)(2 * d1 + 2 * d2));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            mlp_fwd1(P, d0, d1, d2, X + (size_t)i * d0, bf16, buf, buf + d1, buf + 2 * d1, buf + 2 * d1 + d2,
                     Y + (size_t)i * 4);
        free(buf);
    }
}

/* mean squared error over the 4 outputs, L = (1/n) sum_i |y_i - t_i|^2, and
 * its gradient with respect to every parameter.  bf16 != 0 follows the GPU
 * training step: the forward of mlp_fwd1 with rounding, dL/dy and the
 * layer-3 backward unrounded, and the hidden-layer gradients dz2, dz1
 * rounded to bfloat16 wherever they enter a product or a bias sum. */
MPO_API double mpo_mlp_loss_grad(const double* P, int d0, int d1, int d2, const double* X, const double* T, int64_t n,
                                 int bf16, double* G /* nparams, nullable */) {
    const double* W1 = P;
    const double* b1 = W1 + (size_t)d0 * d1;
    const double* W2 = b1 + d1;
    const double* b2 = W2 + (size_t)d1 * d2;
    const double* W3 = b2 + d2;
    int64_t np = mpo_mlp_nparams(d0, d1, d2);
    if (G) memset(G, 0, sizeof(double) * (size_t)np);
    double* gW1 = G;
    double* gb1 = G ? gW1 + (size_t)d0 * d1 : NULL;
    double* gW2 = G ? gb1 + d1 : NULL;
    double* gb2 = G ? gW2 + (size_t)d1 * d2 : NULL;
    double* gW3 = G ? gb2 + d2 : NULL;
    double* gb3 = G ? gW3 + (size_t)d2 * 4 : NULL;
    double* z1 = (double*)malloc(sizeof(double) * (size_t)d1);
    double* h1 = (double*)malloc(sizeof(double) * (size_t)d1);
    double* z2 = (double*)malloc(sizeof(double) * (size_t)d2);
    double* h2 = (double*)malloc(sizeof(double) * (size_t)d2);
    double* dz2 = (double*)malloc(sizeof(double) * (size_t)d2);
    double* dz1 = (double*)malloc(sizeof(double) * (size_t)d1);
    double loss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double* x = X + (size_t)i * d0;
        double y[4], dy[4];
        mlp_fwd1(P, d0, d1, d2, x, bf16, z1, h1, z2, h2, y);
        for (int j = 0; j < 4; ++j) {
            double r = y[j] - T[(size_t)i * 4 + j];
            loss += r * r;
            dy[j] = 2.0 * r / (double)n;
        }
        if (!G) continue;
        for (int j = 0; j < 4; ++j) {
            gb3[j] += dy[j];
            for (int k = 0; k < d2; ++k) gW3[(size_t)k * 4 + j] += h2[k] * dy[j];
        }
        for (int k = 0; k < d2; ++k) {
            double s = 0.0;
            for (int j = 0; j < 4; ++j) s += rnd(W3[(size_t)k * 4 + j], bf16) * dy[j];
            dz2[k] = rnd(s * silu_d(z2[k]), bf16);
        }
        for (int j = 0; j < d2; ++j) {
            gb2[j] += dz2[j];
            for (int k = 0; k < d1; ++k) gW2[(size_t)k * d2 + j] += h1[k] * dz2[j];
        }
        for (int k = 0; k < d1; ++k) {
            double s = 0.0;
            for (int j = 0; j < d2; ++j) s += rnd(W2[(size_t)k * d2 + j], bf16) * dz2[j];
            dz1[k] = rnd(s * silu_d(z1[k]), bf16);
        }
        for (int j = 0; j < d1; ++j) {
            gb1[j] += dz1[j];
            for (int k = 0; k < d0; ++k) gW1[(size_t)k * d1 + j] += rnd(x[k], bf16) * dz1[j];
        }
    }
    free(z1); free(h1); free(z2); free(h2); free(dz2); free(dz1);
    return loss / (double)n;
}

/* one Adam step (Kingma & Ba 2015) with bias correction, t >= 1 */
MPO_API void mpo_adam(double* P, const double* G, double* Mv, double* Vv, int64_t np, int t, double lr, double b1,
                      double b2, double eps) {
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t k = 0; k < np; ++k) {
        Mv[k] = b1 * Mv[k] + (1.0 - b1) * G[k];
        Vv[k] = b2 * Vv[k] + (1.0 - b2) * G[k] * G[k];
        double mh = Mv[k] / c1, vh = Vv[k] / c2;
        P[k] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* Likelihood with a scalar residual r(p') per point in place of the GICP
 * term (rank-1 Gauss-Newton).  mode 1: the residual field; mode 2: the
 * network (features of the FP32 point, bf16-emulating forward, outputs
 * scaled by r_scale and g_scale, r clamped at 0).  In FP64 with R from the
 * quaternion: w = R^T grad r, g = [mu x w; w], H += g g^T, b += r g
 * (= J_p^T grad s / 2), loglik -= min(r^2, c_max); points with r^2 < c_max
 * are counted as inliers. */
MPO_API void mpo_likelihood_rank1(const mpo_map* m, const float* sxyz, int32_t ns, const float* poses, int64_t n,
                                  int mode, float sigma_s, float dmax, float cmax, const double* P, const float lo[3],
                                  const float inv_ext[3], const float* freqs, int nf, double r_scale, double g_scale,
                                  double r_floor, double r_out, double lam_rel, double lam_abs, double* loglik,
                                  double* H21, double* b6, double* psi6, int32_t* ninl) {
    float dmax2 = dmax * dmax;
    const int d0 = 6 * nf, d1 = 128, d2 = 128;
#pragma omp parallel
    {
        double* buf = (double*)malloc(sizeof(double) * (size_t)(d0 + 2 * d1 + 2 * d2));
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            const float* T = poses + 8 * i;
            q32 q = {T[0], T[1], T[2], T[3]};
            float R32[9];
            q32_to_R(q, R32);
            float t32[3] = {T[4], T[5], T[6]};
            double qd[4] = {T[0], T[1], T[2], T[3]}, R[9];
            qd_to_R(qd, R);
            double ll = 0.0, H[36], b[6];
            memset(H, 0, sizeof(H));
            memset(b, 0, sizeof(b));
            int32_t ni = 0;
            for (int32_t k = 0; k < ns; ++k) {
                const float* ms = sxyz + 3 * (int64_t)k;
                float p32[3];
                xform32(R32, t32, ms, p32);
                double r, gr[3];
                if (mode == 1) {
                    rf_point(m, p32, sigma_s, dmax2, r_floor, r_out, &r, gr);
                } else {
                    double* x = buf;
                    double y[4];
                    ff_point(p32, lo, inv_ext, freqs, nf, 1, x);
                    mlp_fwd1(P, d0, d1, d2, x, 1, buf + d0, buf + d0 + d1, buf + d0 + 2 * d1,
                             buf + d0 + 2 * d1 + d2, y);
                    r = y[0] * r_scale;
                    if (r < 0.0) r = 0.0;
                    for (int a = 0; a < 3; ++a) gr[a] = y[1 + a] * g_scale;
                }
                double s = r * r;
                ll -= s < (double)cmax ? s : (double)cmax;
                if (s < (double)cmax) ++ni;
                double w[3], mu[3] = {ms[0], ms[1], ms[2]};
                for (int a = 0; a < 3; ++a) w[a] = R[a] * gr[0] + R[3 + a] * gr[1] + R[6 + a] * gr[2];
                double gw[6] = {mu[1] * w[2] - mu[2] * w[1], mu[2] * w[0] - mu[0] * w[2], mu[0] * w[1] - mu[1] * w[0],
                                w[0], w[1], w[2]};
                for (int r1 = 0; r1 < 6; ++r1) {
                    b[r1] += r * gw[r1];
                    for (int c1 = 0; c1 < 6; ++c1) H[6 * r1 + c1] += gw[r1] * gw[c1];
                }
            }
            double h21[21];
            int q2 = 0;
            for (int r1 = 0; r1 < 6; ++r1)
                for (int c1 = r1; c1 < 6; ++c1) h21[q2++] = H[6 * r1 + c1];
            if (loglik) loglik[i] = ll;
            if (H21) memcpy(H21 + 21 * i, h21, sizeof(h21));
            if (b6) memcpy(b6 + 6 * i, b, sizeof(b));
            if (ninl) ninl[i] = ni;
            if (psi6) mpo_gn_step(h21, b, lam_rel, lam_abs, psi6 + 6 * i);
        }
        free(buf);
    }
}

/* ======================================================================= */
/* GICP scan-to-scan odometry (Sec. III-B: the motion estimate dT and its  */
/* covariance that feed Eq. (1); GICP after Segal et al. 2009).            */
/* Source = the current scan (points mu_k, covariances S_k), target = the  */
/* previous scan (points q_j, covariances T_j); dT maps current-frame      */
/* points into the previous frame.  For pose (R, t):                       */
/*   p_k = R mu_k + t (FP32, the filter's transform program);              */
/*   j(k) = argmin_j |q_j - p_k|^2 in FP32 with the fma order of the        */
/*          likelihood's residual gate, ties to the lower index;           */
/*   inlier iff that distance^2 <= d_max^2;                                 */
/*   then in FP64: e = q_j - p, C = T_j + R S_k R^T, Omega = C^-1,          */
/*   J = [R [mu]x, -R], H += J^T Omega J, b += J^T Omega e,                 */
/*   cost += e^T Omega e.                                                   */
/* Gauss-Newton: psi from the damped system of the filter, dT <- dT exp(psi)*/
/* for a fixed number of iterations; Sigma^dT = scale * H^-1 at the final   */
/* pose (the covariance "based on the Hessian").                            */
/* ======================================================================= */
static int32_t gicp_nn(const float* txyz, int32_t nt, const float p[3], float* d2_out) {
    int32_t best = -1;
    float bd = INFINITY;
    for (int32_t j = 0; j < nt; ++j) {
        const float dx = txyz[3 * (int64_t)j] - p[0], dy = txyz[3 * (int64_t)j + 1] - p[1],
                    dz = txyz[3 * (int64_t)j + 2] - p[2];
        const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        if (d2 < bd) { bd = d2; best = j; }
    }
    *d2_out = bd;
    return best;
}

MPO_API void mpo_gicp_terms(const float* txyz, const float* tcov, int32_t nt, const float* sxyz, const float* scov,
                            int32_t ns, const float pose[7], float dmax, int32_t* nn, double H21[21], double b6[6],
                            double* cost, int32_t* ninl) {
    const float dmax2 = dmax * dmax;
    q32 q = {pose[0], pose[1], pose[2], pose[3]};
    float R32[9];
    q32_to_R(q, R32);
    const float t32[3] = {pose[4], pose[5], pose[6]};
    double qd[4] = {pose[0], pose[1], pose[2], pose[3]}, R[9], Rt[9];
    qd_to_R(qd, R);
    mat3_T(R, Rt);
    const double t[3] = {pose[4], pose[5], pose[6]};
    double H[36], b[6], c = 0.0;
    memset(H, 0, sizeof(H));
    memset(b, 0, sizeof(b));
    int32_t ni = 0;
    /* correspondences (independent per point), then the sums in point order */
    int32_t* jj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ns > 0 ? ns : 1));
#pragma omp parallel for schedule(static)
    for (int32_t k = 0; k < ns; ++k) {
        float p32[3], d2;
        xform32(R32, t32, sxyz + 3 * (int64_t)k, p32);
        const int32_t j = gicp_nn(txyz, nt, p32, &d2);
        jj[k] = (j >= 0 && d2 <= dmax2) ? j : -1;
    }
    for (int32_t k = 0; k < ns; ++k) {
        const float* ms = sxyz + 3 * (int64_t)k;
        const int32_t j = jj[k];
        if (nn) nn[k] = j;
        if (j < 0) continue;
        ++ni;
        const double mu[3] = {ms[0], ms[1], ms[2]};
        double p[3], e[3];
        for (int a = 0; a < 3; ++a) p[a] = R[3 * a] * mu[0] + R[3 * a + 1] * mu[1] + R[3 * a + 2] * mu[2] + t[a];
        for (int a = 0; a < 3; ++a) e[a] = (double)txyz[3 * (int64_t)j + a] - p[a];
        double T6[6], S6[6], TT[9], SS[9], tmp[9], RSR[9], C[9], Om[9];
        for (int a = 0; a < 6; ++a) { T6[a] = tcov[6 * (int64_t)j + a]; S6[a] = scov[6 * (int64_t)k + a]; }
        sym6_full(T6, TT);
        sym6_full(S6, SS);
        mat3_mul(R, SS, tmp);
        mat3_mul(tmp, Rt, RSR);
        for (int a = 0; a < 9; ++a) C[a] = TT[a] + RSR[a];
        mat3_inv(C, Om);
        double Oe[3];
        for (int a = 0; a < 3; ++a) Oe[a] = Om[3 * a] * e[0] + Om[3 * a + 1] * e[1] + Om[3 * a + 2] * e[2];
        c += e[0] * Oe[0] + e[1] * Oe[1] + e[2] * Oe[2];
        const double Sk[9] = {0, -mu[2], mu[1], mu[2], 0, -mu[0], -mu[1], mu[0], 0};
        double RS[9], J[18], OJ[18];
        mat3_mul(R, Sk, RS);
        for (int a = 0; a < 3; ++a)
            for (int cc = 0; cc < 3; ++cc) { J[6 * a + cc] = RS[3 * a + cc]; J[6 * a + 3 + cc] = -R[3 * a + cc]; }
        for (int a = 0; a < 3; ++a)
            for (int cc = 0; cc < 6; ++cc)
                OJ[6 * a + cc] = Om[3 * a] * J[cc] + Om[3 * a + 1] * J[6 + cc] + Om[3 * a + 2] * J[12 + cc];
        for (int r = 0; r < 6; ++r) {
            for (int cc = 0; cc < 6; ++cc) H[6 * r + cc] += J[r] * OJ[cc] + J[6 + r] * OJ[6 + cc] + J[12 + r] * OJ[12 + cc];
            b[r] += J[r] * Oe[0] + J[6 + r] * Oe[1] + J[12 + r] * Oe[2];
        }
    }
    free(jj);
    int q2 = 0;
    for (int r = 0; r < 6; ++r)
        for (int cc = r; cc < 6; ++cc) H21[q2++] = H[6 * r + cc];
    memcpy(b6, b, sizeof(b));
    *cost = c;
    *ninl = ni;
}

/* pose_io: in = initial dT (7), out = final dT (FP64, normalised quaternion);
   decisions of every iteration use the pose rounded to FP32 */
MPO_API int mpo_gicp_align(const float* txyz, const float* tcov, int32_t nt, const float* sxyz, const float* scov,
                           int32_t ns, double pose_io[7], int32_t iters, float dmax, double lam_rel, double lam_abs,
                           double cov_scale, double cov36[36], double H21_out[21], double* cost_out, int32_t* ninl_out) {
    double H21[21], b6[6], c = 0.0;
    int32_t ni = 0;
    for (int it = 0; it <= iters; ++it) {
        float p32[7];
        for (int k = 0; k < 7; ++k) p32[k] = (float)pose_io[k];
        mpo_gicp_terms(txyz, tcov, nt, sxyz, scov, ns, p32, dmax, NULL, H21, b6, &c, &ni);
        if (it == iters) break;
        double psi[6], D[7], T[7];
        mpo_gn_step(H21, b6, lam_rel, lam_abs, psi);
        mpo_se3_exp(psi, D);
        se3_compose(pose_io, D, T);
        const double nq = sqrt(T[0] * T[0] + T[1] * T[1] + T[2] * T[2] + T[3] * T[3]);
        for (int k = 0; k < 4; ++k) T[k] /= nq;
        memcpy(pose_io, T, sizeof(T));
    }
    if (H21_out) memcpy(H21_out, H21, sizeof(H21));
    if (cost_out) *cost_out = c;
    if (ninl_out) *ninl_out = ni;
    /* Sigma = scale * H^-1 (columns by Cholesky solves) */
    double A[36], e[6], col[6];
    int q = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) { A[6 * i + j] = H21[q]; A[6 * j + i] = H21[q]; ++q; }
    int rc = 0;
    for (int jcol = 0; jcol < 6; ++jcol) {
        for (int i = 0; i < 6; ++i) e[i] = (i == jcol) ? 1.0 : 0.0;
        if (chol6_solve(A, e, col) != 0) { rc = -1; memset(col, 0, sizeof(col)); }
        for (int i = 0; i < 6; ++i) cov36[6 * i + jcol] = cov_scale * col[i];
    }
    return rc;
}
