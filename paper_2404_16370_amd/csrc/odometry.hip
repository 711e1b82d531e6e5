// odometry.hip -- GICP scan-to-scan odometry (Sec. III-B): the sensor motion
// dT between the previous and the current scan, and its covariance from the
// Hessian of the match, the inputs of the prediction step (Eq. 1); GICP after
// Segal et al. (2009).
//
// Source = the current scan (points mu_k, covariances S_k), target = the
// previous scan (points q_j, covariances T_j); dT maps current-frame points
// into the previous frame (T_t = T_{t-1} dT).  At pose (R, t):
//   p_k = R mu_k + t (FP32, the filter's transform program),
//   j(k) = argmin_j |q_j - p_k|^2 (FP32, the residual gate's fma order,
//          ties to the lower index), an inlier iff that is <= d_max^2;
//   e = q_j - p_k; in the body frame e_b = R^T e,
//   C_b = R^T T_j R + S_k, Omega_b = C_b^-1, J_b = [[mu]x, -I]:
//   H += J_b^T Omega_b J_b, b += J_b^T Omega_b e_b, cost += e_b^T Omega_b e_b
//   (FP32 per point, FP64 sums in a fixed order).
// Each iteration: psi = -(H + diag(lam_rel H_ii + lam_abs))^-1 b (FP64),
// dT <- dT exp(psi) (FP64 pose, FP32 copy for the next evaluation).  After
// the last update the terms are evaluated once more: Sigma^dT = scale H^-1.
//
// Launch shape per iteration: the neighbour search over a grid of (source
// block, target block) pairs, each target block staged in LDS and read as
// broadcasts, one source point per lane; a block's minimum goes into the
// point's 64-bit key (distance bits, index) by an atomic minimum, which for
// non-negative distances is the lowest distance and, among equal ones, the
// lowest index, whatever the order of the blocks.  Then one lane per source
// point forms its terms and each workgroup sums its points' terms in FP64 in
// a fixed order; one workgroup adds the workgroups' sums in order and takes
// the step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "megapf.h"
#include "mp_det.hpp"
#include "mp_internal.hpp"
#include "mp_solve.hpp"

namespace {

constexpr int kNnThreads = 256;   // source points per search workgroup
constexpr int kNnTargets = 256;   // target points per search workgroup (LDS)
constexpr int kTB = 256;          // source points per terms workgroup
constexpr int kOTerms = 29;       // H (21), b (6), cost, inlier count per source point
constexpr int kSumGroups = 8;     // terms of a workgroup summed in 8 runs of kTB / 8 points
constexpr uint64_t kNoMatch = ~0ull;

__device__ __forceinline__ float3 odo_point(const float* pose, const mpdet::mat3& Rm, const float4 r) {
    return mpdet::xform(Rm.m, make_float3(pose[4], pose[5], pose[6]), make_float3(r.x, r.y, r.z));
}

struct OdoNnArgs {
    const float4* __restrict__ trec;   // previous scan records (3 float4 per point)
    const float4* __restrict__ srec;   // current scan records
    const float* __restrict__ pose;    // FP32 pose (qw, qx, qy, qz, tx, ty, tz, 0)
    unsigned long long* __restrict__ key;   // ns: (distance bits << 32) | index, kNoMatch before the search
    int32_t nt, ns;
};

__global__ __launch_bounds__(kNnThreads) void k_odo_nn(OdoNnArgs A) {
    __shared__ float3 tile[kNnTargets];
    const int j0 = blockIdx.y * kNnTargets;
    const int cnt = min(kNnTargets, A.nt - j0);
    for (int u = threadIdx.x; u < cnt; u += kNnThreads) {
        const float4 r = A.trec[3 * (j0 + u)];
        tile[u] = make_float3(r.x, r.y, r.z);
    }
    __syncthreads();
    const int k = blockIdx.x * kNnThreads + threadIdx.x;
    if (k >= A.ns) return;
    const mpdet::mat3 Rm = mpdet::qmat(mpdet::quat{A.pose[0], A.pose[1], A.pose[2], A.pose[3]});
    const float3 p = odo_point(A.pose, Rm, A.srec[3 * k]);
    float bd = __builtin_inff();
    int bj = j0;
    for (int u = 0; u < cnt; ++u) {   // ascending j, strict <: the lower index wins ties
        const float3 q = tile[u];
        const float dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
        const float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
        if (d2 < bd) {
            bd = d2;
            bj = j0 + u;
        }
    }
    // d2 >= +0 (a sum of squares, never -0): its bits order as the values do
    atomicMin(A.key + k, ((unsigned long long)__float_as_uint(bd) << 32) | (uint32_t)bj);
}

struct OdoTermArgs {
    const float4* __restrict__ trec;
    const float4* __restrict__ srec;
    const float* __restrict__ pose;
    unsigned long long* __restrict__ key;   // read, then reset to kNoMatch for the next search
    int32_t* __restrict__ nn;          // ns: target index or -1
    double* __restrict__ part;         // per workgroup: kOTerms FP64 sums
    int32_t ns;
    float dmax2;
};

// The GICP terms of one source point given its nearest target (zero for an
// outlier); t[28] is the inlier count.
__device__ __forceinline__ void odo_point_terms(const OdoTermArgs& A, const mpdet::mat3& Rm, const int k,
                                                const int bj, float t[kOTerms]) {
    const float4 s0 = A.srec[3 * k];
    const float3 mu = make_float3(s0.x, s0.y, s0.z);
    const float3 p = odo_point(A.pose, Rm, s0);
    const float4 t0 = A.trec[3 * bj], t1 = A.trec[3 * bj + 1], t2 = A.trec[3 * bj + 2];
    const float4 s1 = A.srec[3 * k + 1], s2 = A.srec[3 * k + 2];
    const float3 eb = mpdet::rot_t(Rm, make_float3(t0.x - p.x, t0.y - p.y, t0.z - p.z));
    // R^T T R: columns of T R, then R^T times them
    const float T[3][3] = {{t0.w, t1.x, t1.y}, {t1.x, t1.z, t1.w}, {t1.y, t1.w, t2.x}};
    float TR[3][3], C[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            TR[r][c] = T[r][0] * Rm.m[c] + T[r][1] * Rm.m[3 + c] + T[r][2] * Rm.m[6 + c];
    const float S[3][3] = {{s0.w, s1.x, s1.y}, {s1.x, s1.z, s1.w}, {s1.y, s1.w, s2.x}};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            C[r][c] = Rm.m[r] * TR[0][c] + Rm.m[3 + r] * TR[1][c] + Rm.m[6 + r] * TR[2][c] + S[r][c];
    // Omega_b = C_b^-1 (adjugate of the symmetrised matrix)
    const float c00 = C[0][0], c01 = 0.5f * (C[0][1] + C[1][0]), c02 = 0.5f * (C[0][2] + C[2][0]);
    const float c11 = C[1][1], c12 = 0.5f * (C[1][2] + C[2][1]), c22 = C[2][2];
    const float i00 = c11 * c22 - c12 * c12, i01 = c02 * c12 - c01 * c22, i02 = c01 * c12 - c02 * c11;
    const float i11 = c00 * c22 - c02 * c02, i12 = c01 * c02 - c00 * c12, i22 = c00 * c11 - c01 * c01;
    const float rd = 1.0f / (c00 * i00 + c01 * i01 + c02 * i02);
    const float O[3][3] = {{i00 * rd, i01 * rd, i02 * rd}, {i01 * rd, i11 * rd, i12 * rd}, {i02 * rd, i12 * rd, i22 * rd}};
    const float e[3] = {eb.x, eb.y, eb.z};
    float w[3];
    for (int r = 0; r < 3; ++r) w[r] = O[r][0] * e[0] + O[r][1] * e[1] + O[r][2] * e[2];
    // J_b = [[mu]x, -I]
    const float J[3][6] = {{0.0f, -mu.z, mu.y, -1.0f, 0.0f, 0.0f},
                           {mu.z, 0.0f, -mu.x, 0.0f, -1.0f, 0.0f},
                           {-mu.y, mu.x, 0.0f, 0.0f, 0.0f, -1.0f}};
    float OJ[3][6];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 6; ++c) OJ[r][c] = O[r][0] * J[0][c] + O[r][1] * J[1][c] + O[r][2] * J[2][c];
    int q = 0;
    for (int r = 0; r < 6; ++r)
        for (int c = r; c < 6; ++c) t[q++] = J[0][r] * OJ[0][c] + J[1][r] * OJ[1][c] + J[2][r] * OJ[2][c];
    for (int r = 0; r < 6; ++r) t[21 + r] = J[0][r] * w[0] + J[1][r] * w[1] + J[2][r] * w[2];
    t[27] = e[0] * w[0] + e[1] * w[1] + e[2] * w[2];
    t[28] = 1.0f;
}

// One lane per source point: its match, its terms into LDS, then the
// workgroup's FP64 sums in a fixed order (kSumGroups runs of consecutive
// points per term, then the runs in order).
__global__ __launch_bounds__(kTB) void k_odo_terms(OdoTermArgs A) {
    __shared__ float tt[kOTerms][kTB];
    __shared__ double run[kOTerms][kSumGroups];
    const int k = blockIdx.x * kTB + threadIdx.x;
    float t[kOTerms];
    for (int m = 0; m < kOTerms; ++m) t[m] = 0.0f;
    if (k < A.ns) {
        const unsigned long long key = A.key[k];
        A.key[k] = kNoMatch;
        const float bd = __uint_as_float((uint32_t)(key >> 32));
        const int bj = (int)(uint32_t)key;
        const bool inl = key != kNoMatch && bd <= A.dmax2;
        A.nn[k] = inl ? bj : -1;
        if (inl) {
            const mpdet::mat3 Rm = mpdet::qmat(mpdet::quat{A.pose[0], A.pose[1], A.pose[2], A.pose[3]});
            odo_point_terms(A, Rm, k, bj, t);
        }
    }
    for (int m = 0; m < kOTerms; ++m) tt[m][threadIdx.x] = t[m];
    __syncthreads();
    constexpr int kRun = kTB / kSumGroups;
    for (int q = threadIdx.x; q < kOTerms * kSumGroups; q += kTB) {
        const int m = q / kSumGroups, g = q % kSumGroups;
        double acc = 0.0;
        for (int i = 0; i < kRun; ++i) acc += (double)tt[m][g * kRun + i];
        run[m][g] = acc;
    }
    __syncthreads();
    if (threadIdx.x < kOTerms) {
        double acc = 0.0;
        for (int g = 0; g < kSumGroups; ++g) acc += run[threadIdx.x][g];
        A.part[(size_t)blockIdx.x * kOTerms + threadIdx.x] = acc;
    }
}

// SE(3) exponential of [omega; v] (FP64): unit quaternion + translation V v
__device__ void se3_exp_d(const double xi[6], double T[7]) {
    const double* w = xi;
    const double* v = xi + 3;
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = sqrt(th2);
    double A, B, hs, hc;
    if (th < 1e-5) {   // series of (1 - cos)/th^2, (th - sin)/th^3, sin(th/2)/th, cos(th/2)
        A = 0.5 - th2 / 24.0;
        B = 1.0 / 6.0 - th2 / 120.0;
        hs = 0.5 - th2 / 48.0;
        hc = 1.0 - th2 / 8.0;
    } else {
        A = (1.0 - cos(th)) / th2;
        B = (th - sin(th)) / (th2 * th);
        hs = sin(0.5 * th) / th;
        hc = cos(0.5 * th);
    }
    T[0] = hc;
    T[1] = hs * w[0];
    T[2] = hs * w[1];
    T[3] = hs * w[2];
    const double c1[3] = {w[1] * v[2] - w[2] * v[1], w[2] * v[0] - w[0] * v[2], w[0] * v[1] - w[1] * v[0]};
    const double c2[3] = {w[1] * c1[2] - w[2] * c1[1], w[2] * c1[0] - w[0] * c1[2], w[0] * c1[1] - w[1] * c1[0]};
    for (int k = 0; k < 3; ++k) T[4 + k] = v[k] + A * c1[k] + B * c2[k];
}

struct OdoStepArgs {
    const double* __restrict__ part;   // nparts x kOTerms workgroup sums
    double* __restrict__ pose64;   // 7
    float* __restrict__ pose32;    // 8
    double* __restrict__ out;      // final: H 21, b 6, cost, inliers, cov 36, ok
    int32_t nparts, final_eval;
    double lam_rel, lam_abs, cov_scale;
};

// One workgroup: the workgroup sums added in order, then the step or the
// covariance.
__global__ __launch_bounds__(64) void k_odo_step(OdoStepArgs A) {
    __shared__ double tot[kOTerms];
    if (threadIdx.x < kOTerms) {
        double acc = 0.0;
        for (int g = 0; g < A.nparts; ++g) acc += A.part[(size_t)g * kOTerms + threadIdx.x];
        tot[threadIdx.x] = acc;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double* H = tot;
    const double* b = tot + 21;
    if (!A.final_eval) {
        double psi[6], kappa = 0.0;
        if (!chol_solve6<double>(H, b, A.lam_rel, A.lam_abs, psi, kappa))
            for (int m = 0; m < 6; ++m) psi[m] = 0.0;
        double D[7];
        se3_exp_d(psi, D);
        const double* P = A.pose64;
        // P exp(psi): Hamilton product and P's rotation applied to D's translation
        double q[4] = {P[0] * D[0] - P[1] * D[1] - P[2] * D[2] - P[3] * D[3],
                       P[0] * D[1] + P[1] * D[0] + P[2] * D[3] - P[3] * D[2],
                       P[0] * D[2] - P[1] * D[3] + P[2] * D[0] + P[3] * D[1],
                       P[0] * D[3] + P[1] * D[2] - P[2] * D[1] + P[3] * D[0]};
        const double w = P[0], x = P[1], y = P[2], z = P[3];
        const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                             2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                             2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
        double tn[3];
        for (int a = 0; a < 3; ++a) tn[a] = P[4 + a] + R[3 * a] * D[4] + R[3 * a + 1] * D[5] + R[3 * a + 2] * D[6];
        const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        for (int a = 0; a < 4; ++a) q[a] /= nq;
        for (int a = 0; a < 4; ++a) A.pose64[a] = q[a];
        for (int a = 0; a < 3; ++a) A.pose64[4 + a] = tn[a];
        for (int a = 0; a < 7; ++a) A.pose32[a] = (float)A.pose64[a];
        A.pose32[7] = 0.0f;
        return;
    }
    for (int m = 0; m < 27; ++m) A.out[m] = tot[m];
    A.out[27] = tot[27];
    A.out[28] = tot[28];
    // Sigma = scale H^-1: column j solves H x = e_j (the undamped solve with b = -e_j)
    bool ok = true;
    for (int jc = 0; jc < 6; ++jc) {
        double e[6], x[6], kappa = 0.0;
        for (int m = 0; m < 6; ++m) e[m] = m == jc ? -1.0 : 0.0;
        if (!chol_solve6<double>(H, e, 0.0, 0.0, x, kappa)) {
            ok = false;
            for (int m = 0; m < 6; ++m) x[m] = 0.0;
        }
        for (int m = 0; m < 6; ++m) A.out[29 + 6 * m + jc] = A.cov_scale * x[m];
    }
    A.out[65] = ok ? 1.0 : 0.0;
}

}  // namespace

extern "C" void mp_odometry_default_params(mp_odometry_params* p) {
    if (!p) return;
    p->iterations = 20;
    p->d_max = 1.0f;
    p->lambda_rel = 1e-3f;
    p->lambda_abs = 1e-6f;
    p->cov_scale = 1.0f;
}

mp_status mp_guarded_call(const char* where, void (*fn)(void*), void* ctx);

namespace {
struct OdoCall {
    mp_filter f;
    const mp_odometry_params* p;
    const float* init;
    float* dT_out;
    float* cov_out;
    mp_odometry_result* res;
    hipStream_t s;
    char* scratch;   // device address of the fixed work area, or null: the filter's buffers
};

// Layout of the work area: match keys, matches, workgroup sums, then the
// pose state.
constexpr size_t kNoAllocScan = 16384;   // largest current scan of mp_odometry_noalloc
constexpr size_t kStateBytes = sizeof(double) * (8 + 66) + sizeof(float) * 8;
constexpr size_t kScrNn = sizeof(unsigned long long) * kNoAllocScan;
constexpr size_t kScrPart = kScrNn + sizeof(int32_t) * kNoAllocScan;
constexpr size_t kScrState = kScrPart + sizeof(double) * kOTerms * (kNoAllocScan / kTB);
constexpr size_t kScratchBytes = kScrState + kStateBytes;
static_assert(kNoAllocScan % kTB == 0, "whole workgroups");
static_assert(kScrNn % 256 == 0 && kScrPart % 256 == 0 && kScrState % 256 == 0, "aligned sections");

void odometry_impl(void* ctx) {
    OdoCall& c = *static_cast<OdoCall*>(ctx);
    mp_filter f = c.f;
    if (!f || !c.p || !c.dT_out) mp_throw(MP_E_ARG, "null filter, parameters or output");
    const mp_odometry_params& P = *c.p;
    if (P.iterations < 0 || P.iterations > 1000 || !(P.d_max > 0.0f) || !std::isfinite(P.d_max) ||
        !(P.lambda_rel >= 0.0f) || !(P.lambda_abs >= 0.0f) || !(P.cov_scale > 0.0f) || !std::isfinite(P.cov_scale))
        mp_throw(MP_E_ARG, "iterations 0..1000, d_max > 0, damping >= 0 and cov_scale > 0 expected");
    if (f->scan_n <= 0 || f->prev_n <= 0)
        mp_throw(MP_E_STATE, "odometry needs two non-empty scans (mp_scan_upload twice)");
    double init[7] = {1, 0, 0, 0, 0, 0, 0};
    if (c.init) {
        for (int k = 0; k < 7; ++k) init[k] = c.init[k];
        double nq = 0.0;
        for (int k = 0; k < 4; ++k) nq += init[k] * init[k];
        for (int k = 0; k < 7; ++k)
            if (!std::isfinite(init[k])) mp_throw(MP_E_ARG, "non-finite initial dT");
        if (!(nq > 1e-12)) mp_throw(MP_E_ARG, "zero quaternion in the initial dT");
        for (int k = 0; k < 4; ++k) init[k] /= std::sqrt(nq);
    }
    hipStream_t s = c.s;
    const int ns = f->scan_n, nt = f->prev_n;
    const int nparts = (ns + kTB - 1) / kTB;
    unsigned long long* key = nullptr;
    int32_t* nn = nullptr;
    double* part = nullptr;
    double* pose64 = nullptr;
    if (c.scratch) {
        // the caller's fixed work area: no allocation
        if ((size_t)ns > kNoAllocScan)
            mp_throw(MP_E_ARG, "mp_odometry_noalloc: current scan of %d points exceeds its limit of %d", ns,
                     (int)kNoAllocScan);
        key = reinterpret_cast<unsigned long long*>(c.scratch);
        nn = reinterpret_cast<int32_t*>(c.scratch + kScrNn);
        part = reinterpret_cast<double*>(c.scratch + kScrPart);
        pose64 = reinterpret_cast<double*>(c.scratch + kScrState);
    } else {
        f->odo_key.ensure(sizeof(unsigned long long) * (size_t)ns);
        f->odo_nn.ensure(sizeof(int32_t) * (size_t)ns);
        f->odo_part.ensure(sizeof(double) * kOTerms * (size_t)nparts);
        // state: pose64 (8 doubles), out (66 doubles), pose32 (8 floats)
        f->odo_state.ensure(kStateBytes);
        key = f->odo_key.as<unsigned long long>();
        nn = f->odo_nn.as<int32_t>();
        part = f->odo_part.as<double>();
        pose64 = f->odo_state.as<double>();
    }
    double* out = pose64 + 8;
    float* pose32 = reinterpret_cast<float*>(out + 66);
    double h_state[8 + 66];
    std::memset(h_state, 0, sizeof(h_state));
    for (int k = 0; k < 7; ++k) h_state[k] = init[k];
    float h_pose32[8];
    for (int k = 0; k < 7; ++k) h_pose32[k] = (float)init[k];
    h_pose32[7] = 0.0f;
    MP_HIP(hipMemcpyAsync(pose64, h_state, sizeof(h_state), hipMemcpyHostToDevice, s));
    MP_HIP(hipMemcpyAsync(pose32, h_pose32, sizeof(h_pose32), hipMemcpyHostToDevice, s));
    // every key starts unmatched; each terms pass leaves them so again
    mp_fill_u32(key, 0xFFFFFFFFu, 2 * (size_t)ns, s);
    OdoNnArgs Q;
    Q.trec = f->prev_orig.as<float4>();
    Q.srec = f->scan_orig.as<float4>();
    Q.pose = pose32;
    Q.key = key;
    Q.nt = nt;
    Q.ns = ns;
    OdoTermArgs T;
    T.trec = Q.trec;
    T.srec = Q.srec;
    T.pose = pose32;
    T.key = key;
    T.nn = nn;
    T.part = part;
    T.ns = ns;
    T.dmax2 = P.d_max * P.d_max;
    OdoStepArgs U;
    U.part = part;
    U.pose64 = pose64;
    U.pose32 = pose32;
    U.out = out;
    U.nparts = nparts;
    U.lam_rel = P.lambda_rel;
    U.lam_abs = P.lambda_abs;
    U.cov_scale = P.cov_scale;
    const dim3 nn_grid((unsigned)((ns + kNnThreads - 1) / kNnThreads), (unsigned)((nt + kNnTargets - 1) / kNnTargets));
    for (int it = 0; it <= P.iterations; ++it) {
        k_odo_nn<<<nn_grid, kNnThreads, 0, s>>>(Q);
        MP_CHECK_LAUNCH();
        k_odo_terms<<<(unsigned)nparts, kTB, 0, s>>>(T);
        MP_CHECK_LAUNCH();
        U.final_eval = it == P.iterations ? 1 : 0;
        k_odo_step<<<1, 64, 0, s>>>(U);
        MP_CHECK_LAUNCH();
    }
    MP_HIP(hipMemcpyAsync(h_state, pose64, sizeof(h_state), hipMemcpyDeviceToHost, s));
    MP_HIP(hipStreamSynchronize(s));
    const double* ho = h_state + 8;
    for (int k = 0; k < 7; ++k) c.dT_out[k] = (float)h_state[k];
    if (c.cov_out)
        for (int k = 0; k < 36; ++k) c.cov_out[k] = (float)ho[29 + k];
    if (c.res) {
        std::memset(c.res, 0, sizeof(*c.res));
        for (int k = 0; k < 21; ++k) c.res->H[k] = ho[k];
        for (int k = 0; k < 6; ++k) c.res->b[k] = ho[21 + k];
        c.res->cost = ho[27];
        c.res->inliers = (int32_t)ho[28];
        c.res->iterations = P.iterations;
        c.res->cov_ok = ho[65] != 0.0 ? 1 : 0;
        for (int k = 0; k < 7; ++k) c.res->dT64[k] = h_state[k];
    }
    f->last_stream = s;
}
}  // namespace

extern "C" mp_status mp_odometry(mp_filter f, const mp_odometry_params* params, const float init_dT[7], float dT_out[7],
                                 float cov_out[36], mp_odometry_result* result, void* stream) {
    OdoCall c{f, params, init_dT, dT_out, cov_out, result, static_cast<hipStream_t>(stream), nullptr};
    return mp_guarded_call("mp_odometry", odometry_impl, &c);
}

// Work area of mp_odometry_noalloc (0.21 MB): one copy per device, held until
// the process ends.  Host code never uses this name as an address: the device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device (looked up on the
// first call there)
char* scratch_on_current_device() {
    int dev = -1;
    MP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) mp_throw(MP_E_UNSUPPORTED, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        MP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) mp_throw(MP_E_HIP, "hipGetSymbolAddress returned a null work area");
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    return g_scratch_ptr[dev];
}

void odometry_noalloc_impl(void* ctx) {
    OdoCall& c = *static_cast<OdoCall*>(ctx);
    c.scratch = scratch_on_current_device();
    odometry_impl(ctx);
}
}  // namespace

extern "C" mp_status mp_odometry_noalloc(mp_filter f, const mp_odometry_params* params, const float init_dT[7],
                                         float dT_out[7], float cov_out[36], mp_odometry_result* result,
                                         void* stream) {
    OdoCall c{f, params, init_dT, dT_out, cov_out, result, static_cast<hipStream_t>(stream), nullptr};
    return mp_guarded_call("mp_odometry_noalloc", odometry_noalloc_impl, &c);
}
