// likelihood.hip -- per-particle GICP log-likelihood, Gauss-Newton H, b and
// the displacement psi (Eq. 2-4).
//
// For particle T = (R, t) and scan point k with Gaussian N(mu_k, Sigma^S_k):
//   p = R mu + t  (FP32, fixed fma order: it decides the voxel)
//   g = m^nnf(floor(p / r)),  e = mu^M_g - p,  inlier iff g exists and
//   |e|^2 <= d_max^2 (both FP32 decisions)
//   Omega = (Sigma^M_g + R Sigma^S R^T)^-1,  c = e^T Omega e
//   log-lik = -(sum_inliers min(c, c_max) + c_max * outliers)
//   J = de/d delta for T exp(delta), delta = [omega; v]:  J = R [[mu]x, -I]
//   H = sum J^T Omega J,  b = sum J^T Omega e  (inliers, Omega held fixed)
// Everything is evaluated in the body frame of the particle:
//   e_b = R^T e, Omega_b = R^T Omega R = (Sigma^S + R^T Sigma^M R)^-1 and
//   J_b = [[mu]x, -I], so H_vv = Omega_b, H_wv = [mu]x Omega_b,
//   H_ww = -[mu]x Omega_b [mu]x, b_w = (Omega_b e_b) x mu, b_v = -Omega_b e_b.
// Map Gaussians are GICP-normalised, Sigma^M = I - a n n^T with a = 1 - eps,
// so R^T Sigma^M R = I - a u u^T with u = R^T n (no 3x3 rotation of Sigma^M).
//
// Launch shape: one lane per particle, particles taken in LSH-sorted order so
// that similar poses share a wavefront (their transformed points hit the same
// voxels and cache lines); 256 lanes per workgroup; scan points streamed
// through LDS in tiles of 256 records and read as wave-uniform broadcasts;
// scan points split into chunks over extra workgroups when N is small, with
// FP32 partial sums per chunk combined by compensated (Kahan) summation in the
// solve kernel.  Workgroup ids are remapped so that each of the 8 XCDs (each
// with its own L2) takes a contiguous range of sorted particles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "mp_det.hpp"
#include "mp_internal.hpp"
#include "mp_lookup.hpp"
#include "mp_solve.hpp"

namespace {

constexpr int kLanes = 256;   // particles per workgroup
constexpr int kTile = 256;    // scan records per LDS tile
constexpr int kNumPartial = 29;  // H 21, b 6, inlier cost, outlier count

struct LikArgs {
    MapView map;
    const float4* __restrict__ poses;   // N x 2 float4 (q; t, 0)
    const int32_t* __restrict__ order;  // sorted position -> particle (or null)
    const float4* __restrict__ scan;    // ns x 3 float4 records
    float* __restrict__ partial;        // [chunk][29][N]
    int32_t n, ns, chunk_len, nchunks, nbx;
    float dmax2, cmax;
    float sig2, ib, r_floor, r_out;   // residual-field scorer: sigma_s^2, 1 / (1 + sigma_s^2), floor of r, r outside the gate
};

__device__ inline int remap_xcd(int bid, int nb) {
    // dispatch places workgroup bid on XCD bid % 8; give each XCD a contiguous range
    const int x = bid & 7, k = bid >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + min(x, r) + k;
}

// One scan point against the lane's particle, given the (possibly missed)
// Gaussian record; accumulates into the lane's sums.  Outliers add nothing to
// the cost sum, H or b and are not counted as inliers (each costs c_max in the
// solve: outliers = points - inliers).  Nothing is branched: an outlier's mean
// is replaced by 0 in the Jacobian and its Omega, cost and b terms are
// multiplied or selected by the inlier flag.  Every record is finite (cells
// outside the band carry a far sentinel mean), so the masked terms are finite.
// KAHAN: compensated cost sum, for lanes that sum long runs of points.
struct Acc {
    float h[21];
    float bw0, bw1, bw2, oe0, oe1, oe2;
    float cost, comp;   // comp: compensation of the (optional) Kahan cost sum
    int32_t nin;        // inliers (plain) / points below c_max (residual field)
};

__device__ __forceinline__ void acc_zero(Acc& S) {
#pragma unroll
    for (int m = 0; m < 21; ++m) S.h[m] = 0.0f;
    S.bw0 = S.bw1 = S.bw2 = S.oe0 = S.oe1 = S.oe2 = 0.0f;
    S.cost = S.comp = 0.0f;
    S.nin = 0;
}

template <bool KAHAN>
__device__ __forceinline__ void add_cost(Acc& S, float y) {
    if (KAHAN) {
        const float yy = y - S.comp;
        const float tt = S.cost + yy;
        S.comp = (tt - S.cost) - yy;
        S.cost = tt;
    } else {
        S.cost += y;
    }
}

// Staged scan record: r0 = (mu, P00), r1 = (P01, P02, P11, P12),
// r2 = (P22, D00, D11, D22) with P = (Sigma^S + I)^-1 and D = I - P =
// Sigma^S P (its off-diagonal entries are -P_ij).  In the body frame
// C = Sigma^S + I - a u u^T (u = R^T n), so Omega = C^-1 = P + beta q q^T with
// q = P u = u - D u and beta = a / (1 - a u^T P u) (Sherman-Morrison).  The
// denominator is the small eigenvalue-like term of C along u: formed as
// 1 - a u^T P u it loses about 10 bits to cancellation when Sigma^S is thin
// along u, so it is taken as lam_n + a u^T D u with lam_n = 1 - a |n|^2 from
// the map record (the same quantity for |u| = |n|, both terms non-negative).
template <bool KAHAN>
__device__ __forceinline__ void accumulate(Acc& S, const mpdet::mat3& Rm, const float a, const float dmax2,
                                           const float cmax, const float4 r0, const float4 r1, const float4 r2,
                                           const float3 p, const bool hit, const float4 gm, const float4 gn) {
    const float ex = gm.x - p.x, ey = gm.y - p.y, ez = gm.z - p.z;
    const float d2 = __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez));
    const bool inl = hit && (d2 <= dmax2);
    const float m = inl ? 1.0f : 0.0f;
    const float3 mu = make_float3(inl ? r0.x : 0.0f, inl ? r0.y : 0.0f, inl ? r0.z : 0.0f);
    const float3 u = mpdet::rot_t(Rm, make_float3(gn.x, gn.y, gn.z));
    const float3 eb = mpdet::rot_t(Rm, make_float3(ex, ey, ez));
    const float p00 = r0.w, p01 = r1.x, p02 = r1.y, p11 = r1.z, p12 = r1.w, p22 = r2.x;
    const float du0 = __builtin_fmaf(r2.y, u.x, __builtin_fmaf(-p01, u.y, -p02 * u.z));
    const float du1 = __builtin_fmaf(-p01, u.x, __builtin_fmaf(r2.z, u.y, -p12 * u.z));
    const float du2 = __builtin_fmaf(-p02, u.x, __builtin_fmaf(-p12, u.y, r2.w * u.z));
    const float q0 = u.x - du0, q1 = u.y - du1, q2 = u.z - du2;
    const float udu = __builtin_fmaf(u.x, du0, __builtin_fmaf(u.y, du1, u.z * du2));
    const float beta = a * __builtin_amdgcn_rcpf(__builtin_fmaf(a, udu, gn.w));
    const float v0 = beta * q0, v1 = beta * q1, v2 = beta * q2;
    const float o00 = __builtin_fmaf(v0, q0, p00), o01 = __builtin_fmaf(v0, q1, p01);
    const float o02 = __builtin_fmaf(v0, q2, p02), o11 = __builtin_fmaf(v1, q1, p11);
    const float o12 = __builtin_fmaf(v1, q2, p12), o22 = __builtin_fmaf(v2, q2, p22);
    const float w0 = __builtin_fmaf(o00, eb.x, __builtin_fmaf(o01, eb.y, o02 * eb.z));
    const float w1 = __builtin_fmaf(o01, eb.x, __builtin_fmaf(o11, eb.y, o12 * eb.z));
    const float w2 = __builtin_fmaf(o02, eb.x, __builtin_fmaf(o12, eb.y, o22 * eb.z));
    const float cst = __builtin_fmaf(eb.x, w0, __builtin_fmaf(eb.y, w1, eb.z * w2));
    add_cost<KAHAN>(S, inl ? fminf(cst, cmax) : 0.0f);
    S.nin += inl ? 1 : 0;
    S.oe0 = __builtin_fmaf(m, w0, S.oe0);
    S.oe1 = __builtin_fmaf(m, w1, S.oe1);
    S.oe2 = __builtin_fmaf(m, w2, S.oe2);
    S.bw0 = __builtin_fmaf(w1, mu.z, __builtin_fmaf(-w2, mu.y, S.bw0));
    S.bw1 = __builtin_fmaf(w2, mu.x, __builtin_fmaf(-w0, mu.z, S.bw1));
    S.bw2 = __builtin_fmaf(w0, mu.y, __builtin_fmaf(-w1, mu.x, S.bw2));
    // B = [mu]x Omega: row0 = -mu_z O_1 + mu_y O_2, row1 = mu_z O_0 - mu_x O_2, row2 = -mu_y O_0 + mu_x O_1
    const float B00 = __builtin_fmaf(-mu.z, o01, mu.y * o02);
    const float B01 = __builtin_fmaf(-mu.z, o11, mu.y * o12);
    const float B02 = __builtin_fmaf(-mu.z, o12, mu.y * o22);
    const float B10 = __builtin_fmaf(mu.z, o00, -mu.x * o02);
    const float B11 = __builtin_fmaf(mu.z, o01, -mu.x * o12);
    const float B12 = __builtin_fmaf(mu.z, o02, -mu.x * o22);
    const float B20 = __builtin_fmaf(-mu.y, o00, mu.x * o01);
    const float B21 = __builtin_fmaf(-mu.y, o01, mu.x * o11);
    const float B22 = __builtin_fmaf(-mu.y, o02, mu.x * o12);
    // H_ww = -B [mu]x
    S.h[0] = __builtin_fmaf(-B01, mu.z, __builtin_fmaf(B02, mu.y, S.h[0]));
    S.h[1] = __builtin_fmaf(-B02, mu.x, __builtin_fmaf(B00, mu.z, S.h[1]));
    S.h[2] = __builtin_fmaf(-B00, mu.y, __builtin_fmaf(B01, mu.x, S.h[2]));
    S.h[6] = __builtin_fmaf(-B12, mu.x, __builtin_fmaf(B10, mu.z, S.h[6]));
    S.h[7] = __builtin_fmaf(-B10, mu.y, __builtin_fmaf(B11, mu.x, S.h[7]));
    S.h[11] = __builtin_fmaf(-B20, mu.y, __builtin_fmaf(B21, mu.x, S.h[11]));
    // H_wv = B (zero for outliers: mu was replaced by 0)
    S.h[3] += B00; S.h[4] += B01; S.h[5] += B02;
    S.h[8] += B10; S.h[9] += B11; S.h[10] += B12;
    S.h[12] += B20; S.h[13] += B21; S.h[14] += B22;
    // H_vv = Omega (inliers)
    S.h[15] = __builtin_fmaf(m, o00, S.h[15]); S.h[16] = __builtin_fmaf(m, o01, S.h[16]);
    S.h[17] = __builtin_fmaf(m, o02, S.h[17]); S.h[18] = __builtin_fmaf(m, o11, S.h[18]);
    S.h[19] = __builtin_fmaf(m, o12, S.h[19]); S.h[20] = __builtin_fmaf(m, o22, S.h[20]);
}

// P = (Sigma^S + I)^-1 of a raw scan record r0 = (mu, S00), r1 = (S01, S02,
// S11, S12), r2 = (S22, ..), written back into the same slots (adjugate / det;
// the eigenvalues of Sigma^S + I are >= 1 for a positive semi-definite
// Sigma^S), and the diagonal of D = Sigma^S P into r2.yzw (formed from
// Sigma^S, not as 1 - P_ii).
__device__ __forceinline__ void stage_inverse(float4& r0, float4& r1, float4& r2) {
    const float s00 = r0.w, s01 = r1.x, s02 = r1.y, s11 = r1.z, s12 = r1.w, s22 = r2.x;
    const float c00 = r0.w + 1.0f, c01 = r1.x, c02 = r1.y, c11 = r1.z + 1.0f, c12 = r1.w, c22 = r2.x + 1.0f;
    const float i00 = __builtin_fmaf(c11, c22, -c12 * c12);
    const float i01 = __builtin_fmaf(c02, c12, -c01 * c22);
    const float i02 = __builtin_fmaf(c01, c12, -c02 * c11);
    const float i11 = __builtin_fmaf(c00, c22, -c02 * c02);
    const float i12 = __builtin_fmaf(c01, c02, -c00 * c12);
    const float i22 = __builtin_fmaf(c00, c11, -c01 * c01);
    const float rd = 1.0f / __builtin_fmaf(c00, i00, __builtin_fmaf(c01, i01, c02 * i02));
    const float p00 = i00 * rd, p01 = i01 * rd, p02 = i02 * rd, p11 = i11 * rd, p12 = i12 * rd, p22 = i22 * rd;
    r0.w = p00;
    r1 = make_float4(p01, p02, p11, p12);
    r2 = make_float4(p22, __builtin_fmaf(s00, p00, __builtin_fmaf(s01, p01, s02 * p02)),
                     __builtin_fmaf(s01, p01, __builtin_fmaf(s11, p11, s12 * p12)),
                     __builtin_fmaf(s02, p02, __builtin_fmaf(s12, p12, s22 * p22)));
}

// Residual-field scorer (rank-1 Gauss-Newton on r = sqrt(s)):
//   inside the gate (NNF hit, |e| <= d_max): s = e^T Omega e with
//   Omega = I / beta + kappa n n^T (beta = 1 + sigma_s^2, kappa =
//   a / (beta (lam_n + sigma_s^2)), lam_n = 1 - a |n|^2 from the record),
//   r = sqrt(s), grad r = -Omega e / max(r, r_floor) (map frame);
//   outside: r = r_out, grad r = 0.
// Every point: w = R^T grad r, g = [mu x w; w], H += g g^T, b += r g,
// log-lik -min(r^2, c_max); r^2 >= c_max counts as an outlier (cost c_max).
template <bool KAHAN>
__device__ __forceinline__ void accumulate_sf(Acc& S, const mpdet::mat3& Rm, const float a, const float dmax2,
                                              const float cmax, const float sig2, const float ib,
                                              const float r_floor, const float r_out, const float4 r0,
                                              const float3 p, const bool hit, const float4 gm, const float4 gn,
                                              const bool valid) {
    const float3 mu = make_float3(r0.x, r0.y, r0.z);
    const float ex = gm.x - p.x, ey = gm.y - p.y, ez = gm.z - p.z;   // finite (far sentinel outside the band)
    const float d2 = __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez));
    const bool gate = hit && (d2 <= dmax2);
    const float kap = a / ((1.0f + sig2) * (gn.w + sig2));
    const float ne = __builtin_fmaf(gn.x, ex, __builtin_fmaf(gn.y, ey, gn.z * ez));
    const float c = __builtin_fmaf(kap * ne, ne, d2 * ib);
    const float r = gate ? __builtin_sqrtf(c) : r_out;
    const float id = gate ? 1.0f / fmaxf(r, r_floor) : 0.0f;     // grad r = -Omega e / max(r, floor)
    const float kn = kap * ne;
    const float gx = -id * __builtin_fmaf(kn, gn.x, ex * ib);
    const float gy = -id * __builtin_fmaf(kn, gn.y, ey * ib);
    const float gz = -id * __builtin_fmaf(kn, gn.z, ez * ib);
    const float3 w = mpdet::rot_t(Rm, make_float3(gx, gy, gz));
    const float g6[6] = {mu.y * w.z - mu.z * w.y, mu.z * w.x - mu.x * w.z, mu.x * w.y - mu.y * w.x, w.x, w.y, w.z};
    int q = 0;
#pragma unroll
    for (int rr = 0; rr < 6; ++rr)
#pragma unroll
        for (int cc = rr; cc < 6; ++cc) {
            S.h[q] = __builtin_fmaf(g6[rr], g6[cc], S.h[q]);
            ++q;
        }
    // b_w is kept in bw*, b_v in -oe* (the solve's partial layout stores -oe)
    S.bw0 = __builtin_fmaf(r, g6[0], S.bw0);
    S.bw1 = __builtin_fmaf(r, g6[1], S.bw1);
    S.bw2 = __builtin_fmaf(r, g6[2], S.bw2);
    S.oe0 = __builtin_fmaf(-r, g6[3], S.oe0);
    S.oe1 = __builtin_fmaf(-r, g6[4], S.oe1);
    S.oe2 = __builtin_fmaf(-r, g6[5], S.oe2);
    const float sq = r * r;
    const bool below = valid && sq < cmax;
    add_cost<KAHAN>(S, below ? sq : 0.0f);
    S.nin += below ? 1 : 0;
}

// Map access of the likelihood kernels.  DENSE: g is a record index of the
// band grid, points outside the grid take the miss record (far sentinel mean,
// so every point "hits" and the residual gate rejects); HASH: g is a Gaussian
// id or -1.
template <int BACKEND>
__device__ __forceinline__ int32_t lik_cell(const MapView& v, const float3 p) {
    return BACKEND == MP_NNF_DENSE ? (int32_t)mp_nnf_cell_or(v, p.x, p.y, p.z, v.dmiss)
                                   : mp_nnf_lookup<BACKEND>(v, p.x, p.y, p.z);
}

template <int BACKEND>
__device__ __forceinline__ int32_t lik_none(const MapView& v) {
    return BACKEND == MP_NNF_DENSE ? (int32_t)v.dmiss : -1;
}

template <int BACKEND>
__device__ __forceinline__ bool lik_hit(int32_t g) {
    return BACKEND == MP_NNF_DENSE || g >= 0;
}

template <int BACKEND>
__device__ __forceinline__ void lik_record(const MapView& v, int32_t g, float4& m, float4& n) {
    if (BACKEND == MP_NNF_DENSE) {
        mp_dense_record(v, (uint32_t)g, m, n);
    } else {
        const float4* r = v.gauss + 2 * (size_t)max(g, 0);
        m = r[0];
        n = r[1];
    }
}

// Scan points are walked in batches of BATCH per lane: first the NNF cells of
// the whole batch are requested back to back (BATCH independent gathers in
// flight), then the batch is evaluated with each Gaussian record fetched two
// points ahead; the transformed points of the batch stay in registers.
template <int BACKEND, int BATCH, int SC = MP_SCORER_PLAIN>
__global__ __launch_bounds__(kLanes) void k_lik(LikArgs A) {
    __shared__ float4 tile[kTile * 3];
    const int nb = A.nbx * A.nchunks;
    const int logical = remap_xcd(blockIdx.x, nb);
    const int chunk = logical / A.nbx;
    const int pblk = logical - chunk * A.nbx;
    const int s = pblk * kLanes + threadIdx.x;
    int i = s < A.n ? (A.order ? A.order[s] : s) : 0;
    const bool active = s < A.n && i >= 0 && i < A.n;
    if (!active) i = 0;

    const float4 q4 = A.poses[2 * i];
    const float4 t4 = A.poses[2 * i + 1];
    const mpdet::mat3 Rm = mpdet::qmat(mpdet::quat{q4.x, q4.y, q4.z, q4.w});
    const float3 t = make_float3(t4.x, t4.y, t4.z);
    const float a = A.map.gicp_a;

    Acc S;
    acc_zero(S);

    const int k0 = chunk * A.chunk_len;
    const int k1 = min(A.ns, k0 + A.chunk_len);
    for (int kt = k0; kt < k1; kt += kTile) {
        const int cnt = min(kTile, k1 - kt);
        __syncthreads();
        for (int j = threadIdx.x; j < cnt; j += kLanes) {
            float4 r0 = A.scan[(size_t)(kt + j) * 3], r1 = A.scan[(size_t)(kt + j) * 3 + 1];
            float4 r2 = A.scan[(size_t)(kt + j) * 3 + 2];
            if (SC != MP_SCORER_SCOREFIELD) stage_inverse(r0, r1, r2);
            tile[3 * j] = r0;
            tile[3 * j + 1] = r1;
            tile[3 * j + 2] = r2;
        }
        __syncthreads();
        if (!active) continue;
        for (int kb = 0; kb < cnt; kb += BATCH) {
            const int nbat = min(BATCH, cnt - kb);
            int32_t g[BATCH];
            float3 pk[BATCH];   // transformed points, kept for the second pass
#pragma unroll
            for (int b = 0; b < BATCH; ++b) {
                g[b] = lik_none<BACKEND>(A.map);
                pk[b] = make_float3(0.0f, 0.0f, 0.0f);
                if (b < nbat) {
                    const float4 r0 = tile[3 * (kb + b)];
                    pk[b] = mpdet::xform(Rm.m, t, make_float3(r0.x, r0.y, r0.z));
                    g[b] = lik_cell<BACKEND>(A.map, pk[b]);
                }
            }
            float4 gm[BATCH], gn[BATCH];
#pragma unroll
            for (int b = 0; b < 2 && b < BATCH; ++b) lik_record<BACKEND>(A.map, g[b], gm[b], gn[b]);
#pragma unroll
            for (int b = 0; b < BATCH; ++b) {
                if (b + 2 < BATCH) lik_record<BACKEND>(A.map, g[b + 2], gm[b + 2], gn[b + 2]);
                if (b < nbat) {
                    const float4 r0 = tile[3 * (kb + b)], r1 = tile[3 * (kb + b) + 1], r2 = tile[3 * (kb + b) + 2];
                    if (SC == MP_SCORER_SCOREFIELD)
                        accumulate_sf<true>(S, Rm, a, A.dmax2, A.cmax, A.sig2, A.ib, A.r_floor, A.r_out, r0, pk[b],
                                            lik_hit<BACKEND>(g[b]), gm[b], gn[b], true);
                    else
                        accumulate<true>(S, Rm, a, A.dmax2, A.cmax, r0, r1, r2, pk[b], lik_hit<BACKEND>(g[b]), gm[b],
                                         gn[b]);
                }
            }
        }
    }
    if (!active) return;
    float* out = A.partial + (size_t)chunk * kNumPartial * A.n + i;
    const size_t st = (size_t)A.n;
#pragma unroll
    for (int m = 0; m < 21; ++m) out[m * st] = S.h[m];
    out[21 * st] = S.bw0;
    out[22 * st] = S.bw1;
    out[23 * st] = S.bw2;
    out[24 * st] = -S.oe0;
    out[25 * st] = -S.oe1;
    out[26 * st] = -S.oe2;
    out[27 * st] = S.cost - S.comp;
    out[28 * st] = (float)(k1 - k0 - S.nin);   // outliers of this chunk
}

// Grouped layout: 16 lanes per particle.  A workgroup (8 waves) keeps a
// chunk of 1024 scan records in LDS and takes 256 LSH-sorted particles, 32 at
// a time; the 16 lanes of a particle walk its points with stride 16, so one
// gather instruction of a wave touches the records of 4 particles x 16
// consecutive (Morton-ordered) scan points: a few compact clusters of cells
// instead of 64 scattered ones.  The 29 sums of a particle are reduced across
// its 16 lanes by shuffles and written per (chunk, sorted position).
constexpr int kGLanes = 16;
constexpr int kGChunk = 1024;
constexpr int kGThreads = 512;
constexpr int kGParticles = 256;

// One tile of the grouped layout: scan chunk `chunk` (kGChunk points) against
// the kGParticles particles of sorted block `pblk`; the whole workgroup takes
// part (it stages the chunk in `tile`).
template <int BACKEND, int BATCH, int SC>
__device__ __forceinline__ void grp_tile(const LikArgs& A, const int chunk, const int pblk, float4* tile) {
    const int k0 = chunk * kGChunk;
    const int cnt = min(kGChunk, A.ns - k0);
    // the whole chunk is staged; records past the scan's end are zero (a
    // finite point at the origin that the walk below marks invalid)
    for (int j = threadIdx.x; j < kGChunk; j += kGThreads) {
        float4 r0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), r1 = r0, r2 = r0;
        if (j < cnt) {
            r0 = A.scan[(size_t)(k0 + j) * 3];
            r1 = A.scan[(size_t)(k0 + j) * 3 + 1];
            r2 = A.scan[(size_t)(k0 + j) * 3 + 2];
            if (SC != MP_SCORER_SCOREFIELD) stage_inverse(r0, r1, r2);
        }
        tile[3 * j] = r0;
        tile[3 * j + 1] = r1;
        tile[3 * j + 2] = r2;
    }
    __syncthreads();
    const int grp = threadIdx.x / kGLanes;   // particle slot in the workgroup (0..31)
    const int gl = threadIdx.x % kGLanes;    // lane within the particle's group
    const float a = A.map.gicp_a;
    constexpr int kSlots = kGThreads / kGLanes;
    static_assert(kGChunk % (kGLanes * BATCH) == 0, "a batch never runs past the staged chunk");
    for (int round = 0; round < kGParticles / kSlots; ++round) {
        const int sp = pblk * kGParticles + round * kSlots + grp;   // sorted position
        int i = sp < A.n ? (A.order ? A.order[sp] : sp) : 0;
        const bool active = sp < A.n && i >= 0 && i < A.n;
        if (!active) i = 0;   // evaluated like particle 0, never written
        const float4 q4 = A.poses[2 * i];
        const float4 t4 = A.poses[2 * i + 1];
        const mpdet::mat3 Rm = mpdet::qmat(mpdet::quat{q4.x, q4.y, q4.z, q4.w});
        const float3 t = make_float3(t4.x, t4.y, t4.z);
        Acc S;
        acc_zero(S);
        // every lane walks whole batches; a point past the chunk's end gets
        // no Gaussian (g = -1) and is excluded from the sums and counts
        for (int kb = 0; kb < cnt; kb += kGLanes * BATCH) {
            int32_t g[BATCH];
            float3 pk[BATCH];
#pragma unroll
            for (int b = 0; b < BATCH; ++b) {
                const int k = kb + gl + kGLanes * b;
                const float4 r0 = tile[3 * k];
                pk[b] = mpdet::xform(Rm.m, t, make_float3(r0.x, r0.y, r0.z));
                const int32_t c = lik_cell<BACKEND>(A.map, pk[b]);
                g[b] = k < cnt ? c : lik_none<BACKEND>(A.map);
            }
            float4 gm[BATCH], gn[BATCH];
#pragma unroll
            for (int b = 0; b < 2 && b < BATCH; ++b) lik_record<BACKEND>(A.map, g[b], gm[b], gn[b]);
#pragma unroll
            for (int b = 0; b < BATCH; ++b) {
                if (b + 2 < BATCH) lik_record<BACKEND>(A.map, g[b + 2], gm[b + 2], gn[b + 2]);
                const int k = kb + gl + kGLanes * b;
                const float4 r0 = tile[3 * k], r1 = tile[3 * k + 1], r2 = tile[3 * k + 2];
                if (SC == MP_SCORER_SCOREFIELD)
                    accumulate_sf<false>(S, Rm, a, A.dmax2, A.cmax, A.sig2, A.ib, A.r_floor, A.r_out, r0, pk[b],
                                         lik_hit<BACKEND>(g[b]), gm[b], gn[b], k < cnt);
                else
                    accumulate<false>(S, Rm, a, A.dmax2, A.cmax, r0, r1, r2, pk[b], lik_hit<BACKEND>(g[b]), gm[b],
                                      gn[b]);
            }
        }
        // the group's 16 partial sums, combined by a butterfly within the group
        // (per-lane runs are at most 64 points: plain FP32 sums)
        float v[kNumPartial];
#pragma unroll
        for (int m = 0; m < 21; ++m) v[m] = S.h[m];
        v[21] = S.bw0;
        v[22] = S.bw1;
        v[23] = S.bw2;
        v[24] = -S.oe0;
        v[25] = -S.oe1;
        v[26] = -S.oe2;
        v[27] = S.cost;
        v[28] = (float)S.nin;   // exact: at most kGChunk
#pragma unroll
        for (int m = 0; m < kNumPartial; ++m)
#pragma unroll
            for (int off = kGLanes / 2; off >= 1; off >>= 1) v[m] += __shfl_xor(v[m], off, 64);
        if (gl == 0 && active) {
            float* out = A.partial + (size_t)chunk * kNumPartial * A.n + sp;
            v[28] = (float)cnt - v[28];   // outliers of this chunk
#pragma unroll
            for (int m = 0; m < kNumPartial; ++m) out[(size_t)m * A.n] = v[m];
        }
    }
}

template <int BACKEND, int BATCH, int SC>
__global__ __launch_bounds__(kGThreads) void k_lik_grp(LikArgs A) {
    __shared__ float4 tile[kGChunk * 3];
    const int nb = A.nbx * A.nchunks;
    const int logical = remap_xcd(blockIdx.x, nb);
    const int chunk = logical / A.nbx;
    grp_tile<BACKEND, BATCH, SC>(A, chunk, logical - chunk * A.nbx, tile);
}

// Persistent likelihood over the tiles of several filters (one pass each,
// dense field maps): a fixed grid of workgroups takes tiles from a queue (an
// atomic counter, zero at launch) until none is left.  Tile t belongs to the last instance whose
// first tile is <= t; within an instance, tiles run chunk-major as in
// k_lik_grp.  Results equal k_lik_grp's on each instance bit for bit (same
// tile arithmetic, same partial layout).
struct LikQueueArgs {
    const LikArgs* __restrict__ tab;    // per instance
    const int32_t* __restrict__ first;  // first tile of each instance (ascending)
    int32_t* __restrict__ counter;      // next tile to take
    int32_t n_inst, tiles;
};

template <int BATCH>
__global__ __launch_bounds__(kGThreads) void k_lik_queue(LikQueueArgs Q) {
    __shared__ float4 tile[kGChunk * 3];
    __shared__ int32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(Q.counter, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();   // `next` is read by every wave before thread 0 overwrites it
        if (t >= Q.tiles) break;
        int lo = 0, hi = Q.n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (Q.first[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        // the table is read-only while the kernel runs: its words are read
        // through the constant address space, so that the uniform arguments
        // land in scalar registers
        typedef const __attribute__((address_space(4))) uint32_t ConstWord;
        static_assert(sizeof(LikArgs) % 4 == 0, "word copy");
        LikArgs A;
        ConstWord* src = (ConstWord*)(Q.tab + lo);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&A);
#pragma unroll
        for (int wd = 0; wd < (int)(sizeof(LikArgs) / 4); ++wd) dst[wd] = src[wd];
        const int local = t - Q.first[lo];
        const int chunk = local / A.nbx;
        grp_tile<MP_NNF_DENSE, BATCH, MP_SCORER_PLAIN>(A, chunk, local - chunk * A.nbx, tile);
    }
}

template <int BACKEND>
void launch_lik_batch(int batch, unsigned grid, hipStream_t s, const LikArgs& A) {
    switch (batch) {
        case 1: k_lik<BACKEND, 1><<<grid, kLanes, 0, s>>>(A); break;
        case 2: k_lik<BACKEND, 2><<<grid, kLanes, 0, s>>>(A); break;
        case 4: k_lik<BACKEND, 4><<<grid, kLanes, 0, s>>>(A); break;
        case 8: k_lik<BACKEND, 8><<<grid, kLanes, 0, s>>>(A); break;
        case 32: k_lik<BACKEND, 32><<<grid, kLanes, 0, s>>>(A); break;
        case 16: k_lik<BACKEND, 16><<<grid, kLanes, 0, s>>>(A); break;
        default: k_lik<BACKEND, 4><<<grid, kLanes, 0, s>>>(A); break;
    }
}

struct SolveArgs {
    const float* __restrict__ partial;
    const int32_t* __restrict__ order;   // partials indexed by sorted position (or null: by particle)
    float4* __restrict__ psi;   // N x 2 float4: (psi0..3), (psi4, psi5, loglik, inliers)
    float* __restrict__ hb;     // N x 28 or null
    int32_t* __restrict__ flags; // [0]: FP64 re-solves
    int32_t* __restrict__ how;   // N or null: 0 FP32 Cholesky, 1 FP64 re-solve, 2 both failed
    int32_t n, nchunks, ns;
    float cmax, lam_rel, lam_abs;
};

__global__ __launch_bounds__(256) void k_solve(SolveArgs A) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;   // partial column
    if (col >= A.n) return;
    const int i = A.order ? A.order[col] : col;
    if (i < 0 || i >= A.n) return;
    // compensated sum of the chunk partials
    float v[kNumPartial], c[kNumPartial];
#pragma unroll
    for (int m = 0; m < kNumPartial; ++m) {
        v[m] = 0.0f;
        c[m] = 0.0f;
    }
    for (int ch = 0; ch < A.nchunks; ++ch) {
        const float* src = A.partial + (size_t)ch * kNumPartial * A.n + col;
#pragma unroll
        for (int m = 0; m < kNumPartial; ++m) {
            const float y = src[(size_t)m * A.n] - c[m];
            const float t = v[m] + y;
            c[m] = (t - v[m]) - y;
            v[m] = t;
        }
    }
    const float nout = v[28];
    const float loglik = -(v[27] + nout * A.cmax);
    float psi[6];
    float kappa = 0.0f;
    bool ok = chol_solve6<float>(v, v + 21, A.lam_rel, A.lam_abs, psi, kappa);
    for (int m = 0; m < 6; ++m) ok = ok && isfinite(psi[m]);
    int how = 0;
    if (!ok || kappa > 1.0e6f) {
        double H64[21], b64[6], p64[6], k64 = 0.0;
        for (int m = 0; m < 21; ++m) H64[m] = v[m];
        for (int m = 0; m < 6; ++m) b64[m] = v[21 + m];
        const bool ok64 = chol_solve6<double>(H64, b64, (double)A.lam_rel, (double)A.lam_abs, p64, k64);
        for (int m = 0; m < 6; ++m) psi[m] = ok64 ? (float)p64[m] : 0.0f;
        atomicAdd(&A.flags[0], 1);
        how = ok64 ? 1 : 2;
    }
    if (A.how) A.how[i] = how;
    A.psi[2 * i] = make_float4(psi[0], psi[1], psi[2], psi[3]);
    A.psi[2 * i + 1] = make_float4(psi[4], psi[5], loglik, (float)A.ns - nout);
    if (A.hb) {
        float* o = A.hb + (size_t)i * 28;
        for (int m = 0; m < 27; ++m) o[m] = v[m];
        o[27] = v[27] + nout * A.cmax;
    }
}


// Morton key (8 bits per axis over the map box, z y x interleaved from the
// top bit) of each particle's translation, and the particle's index
__global__ void k_walk_keys(const float4* __restrict__ poses, int n, float lo0, float lo1, float lo2, float s0,
                            float s1, float s2, uint32_t* __restrict__ keys, int32_t* __restrict__ idx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 t = poses[2 * i + 1];
    const float c0 = fminf(fmaxf((t.x - lo0) * s0, 0.0f), 255.0f);
    const float c1 = fminf(fmaxf((t.y - lo1) * s1, 0.0f), 255.0f);
    const float c2 = fminf(fmaxf((t.z - lo2) * s2, 0.0f), 255.0f);
    const uint32_t x = (uint32_t)c0, y = (uint32_t)c1, z = (uint32_t)c2;   // NaN -> 0
    uint32_t key = 0;
#pragma unroll
    for (int b = 7; b >= 0; --b) key = (key << 3) | (((z >> b) & 1u) << 2) | (((y >> b) & 1u) << 1) | ((x >> b) & 1u);
    keys[i] = key;
    idx[i] = i;
}
}  // namespace

// layout of the likelihood launch: lane per particle, or 16 lanes per particle
static bool lik_grouped(mp_filter f) {
    if (f->p.lik_layout == MP_LIK_LAYOUT_PARTICLE) return false;
    if (f->p.lik_layout == MP_LIK_LAYOUT_GROUPED) return true;
    return f->n >= 2048 && f->scan_n >= 512;
}

// Walk order of the particles in a likelihood pass.  With enough work per
// pass the particles are visited in Morton order of their translations, so
// that the workgroups running at once (and each XCD's contiguous share of
// them) gather records of one part of the map: 26.6 -> 24.6 ms per launch at
// 1M x 8192 against the LSH order, whose adjacent codes are not neighbours in
// space while the particles are spread.  The order changes no particle's sums.
static bool lik_spatial(mp_filter f, int scorer) {
    return scorer != MP_SCORER_SURROGATE && lik_grouped(f) && (int64_t)f->n * (int64_t)f->scan_n >= (1LL << 27);
}

static const int32_t* lik_order(mp_filter f, int scorer) {
    return lik_spatial(f, scorer) ? f->lorder.as<int32_t>() : f->sorted.as<int32_t>();
}

// the spatial walk order of the current poses into lorder (a stable sort of
// the 24-bit keys: ties keep ascending particle index); the LSH sort's
// ping-pong buffers and scratch are free while the likelihood runs
static void lik_prepare_order(mp_filter f, int scorer, hipStream_t s) {
    if (!lik_spatial(f, scorer)) return;
    const int n = f->n;
    float lo[3], sc[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = f->lsh_lo[a];
        sc[a] = 256.0f / std::max(1e-3f, f->lsh_hi[a] - f->lsh_lo[a]);
    }
    constexpr int kBits = 24;
    // start on the side that makes the last pass land in (lkeys, lorder)
    const bool odd = mp_radix_passes(n, kBits) % 2 == 1;
    uint32_t* k0 = odd ? f->tmp_keys.as<uint32_t>() : f->lkeys.as<uint32_t>();
    int32_t* v0 = odd ? f->tmp_vals.as<int32_t>() : f->lorder.as<int32_t>();
    uint32_t* k1 = odd ? f->lkeys.as<uint32_t>() : f->tmp_keys.as<uint32_t>();
    int32_t* v1 = odd ? f->lorder.as<int32_t>() : f->tmp_vals.as<int32_t>();
    k_walk_keys<<<(n + 255) / 256, 256, 0, s>>>(f->poses[f->cur].as<float4>(), n, lo[0], lo[1], lo[2], sc[0], sc[1],
                                                 sc[2], k0, v0);
    MP_CHECK_LAUNCH();
    mp_radix_sort_u32_inplace_parity(k0, v0, k1, v1, n, kBits, f->hist, s);
}

// scan-point chunks per particle tile and the chunk length
static int lik_chunks(mp_filter f, int& clen) {
    const int n = f->n;
    const int ns = std::max(0, f->scan_n);
    if (lik_grouped(f)) {
        clen = kGChunk;
        return std::max(1, (ns + kGChunk - 1) / kGChunk);
    }
    const int nbx = (n + kLanes - 1) / kLanes;
    int nch = f->p.lik_chunks;
    if (nch <= 0) {
        // enough workgroups to fill 256 CUs several times, chunks of >= 256 points
        nch = std::max(1, std::min((2048 + nbx - 1) / nbx, (ns + kTile - 1) / kTile));
    }
    nch = std::max(1, std::min(nch, std::max(1, ns)));
    clen = (ns + nch - 1) / nch;
    return std::max(1, (ns + clen - 1) / std::max(1, clen));
}

size_t mp_lik_partial_bytes(mp_filter f) {
    int clen = 0;
    const int nch = lik_chunks(f, clen);
    return sizeof(float) * (size_t)kNumPartial * (size_t)nch * (size_t)f->n;
}

namespace {
// arguments of one likelihood pass on the filter's current state
struct LikPlan {
    LikArgs A;
    int scorer;    // of this pass: SURROGATE runs as PLAIN while its check has it fall back
    int nch;       // scan chunks (partials per particle)
    bool grouped;  // GROUPED layout: partials indexed by sorted position
};

LikPlan lik_plan(mp_filter f) {
    LikPlan P;
    P.scorer = (f->p.scorer == MP_SCORER_SURROGATE && f->sur_fallback) ? (int)MP_SCORER_PLAIN : f->p.scorer;
    if (P.scorer == MP_SCORER_SURROGATE && !f->sur)
        mp_throw(MP_E_STATE, "SURROGATE scorer without a network (mp_filter_set_surrogate)");
    const int n = f->n;
    const int ns = f->scan_n;
    P.grouped = lik_grouped(f) && P.scorer != MP_SCORER_SURROGATE;
    const int nbx = P.grouped ? (n + kGParticles - 1) / kGParticles : (n + kLanes - 1) / kLanes;
    int clen = 0;
    P.nch = lik_chunks(f, clen);
    f->lik_chunks = P.nch;
    f->lik_chunk_len = clen;
    f->partial.ensure(mp_lik_partial_bytes(f));
    LikArgs& A = P.A;
    A.map = f->map->view;
    A.poses = f->poses[f->cur].as<float4>();
    A.order = lik_order(f, P.scorer);
    A.scan = f->scan.as<float4>();
    A.partial = f->partial.as<float>();
    A.n = n;
    A.ns = ns;
    A.chunk_len = std::max(1, clen);
    A.nchunks = P.nch;
    A.nbx = nbx;
    A.dmax2 = f->p.d_max * f->p.d_max;
    A.cmax = f->p.c_max;
    A.sig2 = f->p.sigma_s * f->p.sigma_s;
    A.ib = 1.0f / (1.0f + A.sig2);
    A.r_floor = 1e-2f;
    A.r_out = mp_residual_r_out(f->p.d_max, f->p.sigma_s, f->map->params.cov_eps);
    return P;
}

// psi, log-likelihood and inliers from the pass's chunk partials (GROUPED:
// indexed by position in the pass's walk order)
void lik_solve(mp_filter f, bool grouped, int nch, const int32_t* order, hipStream_t s) {
    const int n = f->n;
    const int ns = f->scan_n;
    SolveArgs S;
    S.partial = f->partial.as<float>();
    S.order = (grouped && ns > 0) ? order : nullptr;
    S.psi = f->psi.as<float4>();
    S.hb = f->capture_hb ? f->hb.as<float>() : nullptr;
    S.how = f->capture_hb ? f->solve_how.as<int32_t>() : nullptr;
    S.flags = f->flags.as<int32_t>();
    S.n = n;
    S.nchunks = nch;
    S.ns = ns;
    S.cmax = f->p.c_max;
    S.lam_rel = f->p.lambda_rel;
    S.lam_abs = f->p.lambda_abs;
    k_solve<<<(n + 255) / 256, 256, 0, s>>>(S);
    MP_CHECK_LAUNCH();
}
}  // namespace

void mp_launch_likelihood(mp_filter f, hipStream_t s) {
    LikPlan P = lik_plan(f);
    lik_prepare_order(f, P.scorer, s);
    const LikArgs& A = P.A;
    const int scorer = P.scorer;
    const int n = f->n;
    const int ns = f->scan_n;
    const bool grouped = P.grouped;
    const int nbx = A.nbx;
    int nch = P.nch;
    if (ns > 0 && scorer == MP_SCORER_SURROGATE) {
        nch = 1;
        f->lik_chunks = 1;
        f->lik_chunk_len = ns;
        mp_tick(f, MP_STAGE_LIK_CORE, true, s);
        mp_sur_likelihood(f, A.partial, s);
        mp_tick(f, MP_STAGE_LIK_CORE, false, s);
    } else if (ns > 0 && grouped) {
        mp_tick(f, MP_STAGE_LIK_CORE, true, s);
        const unsigned grid = (unsigned)(A.nbx * nch);
        const bool dense = A.map.backend == MP_NNF_DENSE;
        if (scorer == MP_SCORER_SCOREFIELD) {
            if (dense) k_lik_grp<MP_NNF_DENSE, 4, MP_SCORER_SCOREFIELD><<<grid, kGThreads, 0, s>>>(A);
            else k_lik_grp<MP_NNF_HASH, 4, MP_SCORER_SCOREFIELD><<<grid, kGThreads, 0, s>>>(A);
        } else if (f->p.lik_batch == 8) {
            if (dense) k_lik_grp<MP_NNF_DENSE, 8, MP_SCORER_PLAIN><<<grid, kGThreads, 0, s>>>(A);
            else k_lik_grp<MP_NNF_HASH, 8, MP_SCORER_PLAIN><<<grid, kGThreads, 0, s>>>(A);
        } else if (f->p.lik_batch == 4) {
            if (dense) k_lik_grp<MP_NNF_DENSE, 4, MP_SCORER_PLAIN><<<grid, kGThreads, 0, s>>>(A);
            else k_lik_grp<MP_NNF_HASH, 4, MP_SCORER_PLAIN><<<grid, kGThreads, 0, s>>>(A);
        } else {   // 2, and the default: two records in flight keep the kernel at 94 VGPRs
            if (dense) k_lik_grp<MP_NNF_DENSE, 2, MP_SCORER_PLAIN><<<grid, kGThreads, 0, s>>>(A);
            else k_lik_grp<MP_NNF_HASH, 2, MP_SCORER_PLAIN><<<grid, kGThreads, 0, s>>>(A);
        }
        MP_CHECK_LAUNCH();
        mp_tick(f, MP_STAGE_LIK_CORE, false, s);
    } else if (ns > 0 && scorer == MP_SCORER_SCOREFIELD) {
        mp_tick(f, MP_STAGE_LIK_CORE, true, s);
        if (A.map.backend == MP_NNF_DENSE)
            k_lik<MP_NNF_DENSE, 4, MP_SCORER_SCOREFIELD><<<nbx * nch, kLanes, 0, s>>>(A);
        else
            k_lik<MP_NNF_HASH, 4, MP_SCORER_SCOREFIELD><<<nbx * nch, kLanes, 0, s>>>(A);
        MP_CHECK_LAUNCH();
        mp_tick(f, MP_STAGE_LIK_CORE, false, s);
    } else if (ns > 0) {
        mp_tick(f, MP_STAGE_LIK_CORE, true, s);
        if (A.map.backend == MP_NNF_DENSE) launch_lik_batch<MP_NNF_DENSE>(f->p.lik_batch, nbx * nch, s, A);
        else launch_lik_batch<MP_NNF_HASH>(f->p.lik_batch, nbx * nch, s, A);
        MP_CHECK_LAUNCH();
        mp_tick(f, MP_STAGE_LIK_CORE, false, s);
    } else {
        mp_fill_u32(A.partial, 0u, (size_t)kNumPartial * n, s);
        nch = 1;
    }
    lik_solve(f, grouped, nch, A.order, s);
}

// ------------------------------------------------------------ tile queue
size_t mp_lik_args_bytes() { return sizeof(LikArgs); }

bool mp_lik_queue_plan(mp_filter f, void* args_out, int32_t* tiles, hipStream_t s) {
    if (f->scan_n <= 0) return false;
    const LikPlan P = lik_plan(f);
    if (!P.grouped || P.scorer != MP_SCORER_PLAIN || P.A.map.backend != MP_NNF_DENSE) return false;
    lik_prepare_order(f, P.scorer, s);
    std::memcpy(args_out, &P.A, sizeof(LikArgs));
    *tiles = P.A.nbx * P.nch;
    return true;
}

void mp_lik_queue_solve(mp_filter f, hipStream_t s) {
    const LikPlan P = lik_plan(f);
    lik_solve(f, P.grouped, P.nch, P.A.order, s);
}

static int queue_batch(int batch) { return batch == 8 ? 8 : (batch == 4 ? 4 : 2); }

int mp_lik_queue_grid(int batch) {
    int dev = 0, cus = 0, per_cu = 0;
    MP_HIP(hipGetDevice(&dev));
    MP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    switch (queue_batch(batch)) {
        case 8: MP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_lik_queue<8>, kGThreads, 0)); break;
        case 4: MP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_lik_queue<4>, kGThreads, 0)); break;
        default: MP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_lik_queue<2>, kGThreads, 0)); break;
    }
    return std::max(1, cus) * std::max(1, per_cu);
}

void mp_launch_lik_queue(const void* tab_dev, const int32_t* first_dev, int32_t* counter_dev, int n_inst, int tiles,
                         int batch, int grid, hipStream_t s) {
    LikQueueArgs Q;
    Q.tab = static_cast<const LikArgs*>(tab_dev);
    Q.first = first_dev;
    Q.counter = counter_dev;
    Q.n_inst = n_inst;
    Q.tiles = tiles;
    const unsigned g = (unsigned)std::max(1, std::min(grid, tiles));
    switch (queue_batch(batch)) {
        case 8: k_lik_queue<8><<<g, kGThreads, 0, s>>>(Q); break;
        case 4: k_lik_queue<4><<<g, kGThreads, 0, s>>>(Q); break;
        default: k_lik_queue<2><<<g, kGThreads, 0, s>>>(Q); break;
    }
    MP_CHECK_LAUNCH();
}
