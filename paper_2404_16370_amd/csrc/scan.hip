// scan.hip -- scan point Gaussians (Sec. III-C: every scan point is modelled
// as N(mu, Sigma), GICP after Segal et al. 2009).
//
// mu is the point itself.  Without caller covariances, Sigma is the
// GICP-normalised covariance I - (1-eps) n n^T of the point and its k nearest
// other scan points: k-NN by FP32 squared distance (fixed fma order, ties to
// the lower index; scan tiles staged in LDS), FP64 mean and 1/(k+1)
// covariance summed self-first in neighbour order, FP64 cyclic Jacobi with a
// fixed operation order.  Fewer than 5 points give Sigma = I.
//
// Record layout consumed by the likelihood kernel (3 float4 per point):
//   (mu_x, mu_y, mu_z, S_xx), (S_xy, S_xz, S_yy, S_yz), (S_zz, 0, 0, 0)
#include <hip/hip_runtime.h>

#include "mp_internal.hpp"

namespace {

constexpr int kB = 128;
constexpr int kKMax = 32;
constexpr int kPtsTile = 2048;

__device__ void jacobi_min_vec(double A[9], double nrm[3]) {
    double V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int sweep = 0; sweep < 60; ++sweep) {
        const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        const double dg = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-300 || off <= 1e-34 * dg) break;
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0;
            const int q = pq == 0 ? 1 : 2;
            const double apq = A[3 * p + q];
            if (apq == 0.0) continue;
            const double app = A[3 * p + p], aqq = A[3 * q + q];
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0);
            const double s = t * c;
            for (int k = 0; k < 3; ++k) {
                const double x = A[3 * k + p], y = A[3 * k + q];
                A[3 * k + p] = c * x - s * y;
                A[3 * k + q] = s * x + c * y;
            }
            for (int k = 0; k < 3; ++k) {
                const double x = A[3 * p + k], y = A[3 * q + k];
                A[3 * p + k] = c * x - s * y;
                A[3 * q + k] = s * x + c * y;
            }
            for (int k = 0; k < 3; ++k) {
                const double x = V[3 * k + p], y = V[3 * k + q];
                V[3 * k + p] = c * x - s * y;
                V[3 * k + q] = s * x + c * y;
            }
        }
    }
    const double ev[3] = {A[0], A[4], A[8]};
    int o[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (ev[o[j]] < ev[o[i]]) {
                const int tmp = o[i];
                o[i] = o[j];
                o[j] = tmp;
            }
    nrm[0] = V[o[0]];
    nrm[1] = V[3 + o[0]];
    nrm[2] = V[6 + o[0]];
}

__global__ __launch_bounds__(kB) void k_scan_knn_cov(const float* __restrict__ xyz, int n, int k, float eps,
                                                     float4* __restrict__ rec) {
    __shared__ float3 tile[kPtsTile];
    const int i = blockIdx.x * kB + threadIdx.x;
    const bool active = i < n;
    const float3 pi = active ? make_float3(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]) : make_float3(0, 0, 0);
    const int kk = min(k, n - 1);
    float bd[kKMax];
    int bj[kKMax];
#pragma unroll
    for (int m = 0; m < kKMax; ++m) {
        bd[m] = __builtin_inff();
        bj[m] = 0x7FFFFFFF;
    }
    for (int base = 0; base < n; base += kPtsTile) {
        const int cnt = min(kPtsTile, n - base);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += kB)
            tile[t] = make_float3(xyz[3 * (base + t)], xyz[3 * (base + t) + 1], xyz[3 * (base + t) + 2]);
        __syncthreads();
        if (!active) continue;
        for (int t = 0; t < cnt; ++t) {
            const int j = base + t;
            if (j == i) continue;
            const float3 pj = tile[t];
            const float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
            const float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
            // candidates arrive in ascending j, so a strict comparison keeps (d2, j) order
            if (d2 < bd[kKMax - 1]) {
#pragma unroll
                for (int m = kKMax - 1; m >= 1; --m) {
                    const bool sh = d2 < bd[m - 1];
                    const bool here = d2 < bd[m];
                    bd[m] = sh ? bd[m - 1] : (here ? d2 : bd[m]);
                    bj[m] = sh ? bj[m - 1] : (here ? j : bj[m]);
                }
                if (d2 < bd[0]) {
                    bd[0] = d2;
                    bj[0] = j;
                }
            }
        }
    }
    if (!active) return;
    double c6[6];
    if (kk + 1 < 5) {
        c6[0] = 1; c6[1] = 0; c6[2] = 0; c6[3] = 1; c6[4] = 0; c6[5] = 1;
    } else {
        double sm[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
        for (int a = 0; a < kKMax; ++a) {
            if (a >= kk) break;
            const int j = bj[a];
            sm[0] = sm[0] + (double)xyz[3 * j];
            sm[1] = sm[1] + (double)xyz[3 * j + 1];
            sm[2] = sm[2] + (double)xyz[3 * j + 2];
        }
        const double dn = (double)(kk + 1);
        const double mu[3] = {sm[0] / dn, sm[1] / dn, sm[2] / dn};
        double S[6] = {0, 0, 0, 0, 0, 0};
        for (int a = -1; a < kk; ++a) {
            const int j = a < 0 ? i : bj[a];
            const double d0 = (double)xyz[3 * j] - mu[0];
            const double d1 = (double)xyz[3 * j + 1] - mu[1];
            const double d2 = (double)xyz[3 * j + 2] - mu[2];
            S[0] += d0 * d0; S[1] += d0 * d1; S[2] += d0 * d2;
            S[3] += d1 * d1; S[4] += d1 * d2; S[5] += d2 * d2;
        }
        for (int a = 0; a < 6; ++a) S[a] /= dn;
        double A[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
        double nv[3];
        jacobi_min_vec(A, nv);
        const double a = 1.0 - (double)eps;
        c6[0] = 1.0 - a * nv[0] * nv[0];
        c6[1] = -a * nv[0] * nv[1];
        c6[2] = -a * nv[0] * nv[2];
        c6[3] = 1.0 - a * nv[1] * nv[1];
        c6[4] = -a * nv[1] * nv[2];
        c6[5] = 1.0 - a * nv[2] * nv[2];
    }
    rec[3 * i] = make_float4(pi.x, pi.y, pi.z, (float)c6[0]);
    rec[3 * i + 1] = make_float4((float)c6[1], (float)c6[2], (float)c6[3], (float)c6[4]);
    rec[3 * i + 2] = make_float4((float)c6[5], 0.0f, 0.0f, 0.0f);
}

__global__ void k_scan_given_cov(const float* __restrict__ xyz, const float* __restrict__ cov, int n,
                                 float4* __restrict__ rec) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* c = cov + 6 * (size_t)i;
    rec[3 * i] = make_float4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], c[0]);
    rec[3 * i + 1] = make_float4(c[1], c[2], c[3], c[4]);
    rec[3 * i + 2] = make_float4(c[5], 0.0f, 0.0f, 0.0f);
}

__global__ void k_scan_permute(const float4* __restrict__ in, const int32_t* __restrict__ perm, int n,
                               float4* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int j = perm[k];
    out[3 * k] = in[3 * j];
    out[3 * k + 1] = in[3 * j + 1];
    out[3 * k + 2] = in[3 * j + 2];
}

}  // namespace

void mp_scan_permute(const float* rec_orig, const int32_t* perm, int32_t n, float* rec_out, hipStream_t s) {
    if (n <= 0) return;
    k_scan_permute<<<(n + 255) / 256, 256, 0, s>>>(reinterpret_cast<const float4*>(rec_orig), perm, n,
                                                    reinterpret_cast<float4*>(rec_out));
    MP_CHECK_LAUNCH();
}

void mp_scan_records(const float* xyz, const float* cov6, int32_t n, int32_t k, float eps, float* rec,
                     hipStream_t s) {
    if (n <= 0) return;
    if (cov6) {
        k_scan_given_cov<<<(n + 255) / 256, 256, 0, s>>>(xyz, cov6, n, reinterpret_cast<float4*>(rec));
    } else {
        if (k > kKMax) mp_throw(MP_E_UNSUPPORTED, "scan_k above %d", kKMax);
        k_scan_knn_cov<<<(n + kB - 1) / kB, kB, 0, s>>>(xyz, n, k, eps, reinterpret_cast<float4*>(rec));
    }
    MP_CHECK_LAUNCH();
}
