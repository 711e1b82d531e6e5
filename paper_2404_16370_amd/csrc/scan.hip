// scan.hip -- scan point Gaussians (Sec. III-C: every scan point is modelled
// as N(mu, Sigma), GICP after Segal et al. 2009).
//
// mu is the point itself.  Without caller covariances, Sigma is the
// GICP-normalised covariance I - (1-eps) n n^T of the point and its k nearest
// other scan points: k-NN by FP32 squared distance (fixed fma order, ties to
// the lower index; scan tiles staged in LDS, 16 lanes per point, 32 points per workgroup), FP64 mean and 1/(k+1)
// covariance summed self-first in neighbour order, FP64 cyclic Jacobi with a
// fixed operation order.  Fewer than 5 points give Sigma = I.
//
// Record layout consumed by the likelihood kernel (3 float4 per point):
//   (mu_x, mu_y, mu_z, S_xx), (S_xy, S_xz, S_yy, S_yz), (S_zz, 0, 0, 0)
#include <hip/hip_runtime.h>

#include "mp_internal.hpp"

namespace {

constexpr int kB = 512;   // 32 points per workgroup share each staged tile
constexpr int kKMax = 32;
constexpr int kPtsTile = 2048;

// Cyclic Jacobi on a symmetric 3x3 (row-major) and the eigenvector of the
// smallest eigenvalue (lowest index on ties).  The rotation loop is unrolled
// so that every index into A and V is a constant and both stay in registers.
__device__ void jacobi_min_vec(double A[9], double nrm[3]) {
    double V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int sweep = 0; sweep < 60; ++sweep) {
        const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        const double dg = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-300 || off <= 1e-34 * dg) break;
#pragma unroll
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
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double x = A[3 * k + p], y = A[3 * k + q];
                A[3 * k + p] = c * x - s * y;
                A[3 * k + q] = s * x + c * y;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double x = A[3 * p + k], y = A[3 * q + k];
                A[3 * p + k] = c * x - s * y;
                A[3 * q + k] = s * x + c * y;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double x = V[3 * k + p], y = V[3 * k + q];
                V[3 * k + p] = c * x - s * y;
                V[3 * k + q] = s * x + c * y;
            }
        }
    }
    int m = 0;
    if (A[4] < A[0]) m = 1;
    if (A[8] < (m == 1 ? A[4] : A[0])) m = 2;
    nrm[0] = m == 0 ? V[0] : (m == 1 ? V[1] : V[2]);
    nrm[1] = m == 0 ? V[3] : (m == 1 ? V[4] : V[5]);
    nrm[2] = m == 0 ? V[6] : (m == 1 ? V[7] : V[8]);
}

// k nearest other scan points of each point, 16 lanes per point: lane l
// keeps the KC best (d2, j) of the candidates j = l, l + 16, ... (ascending j
// with a strict comparison, so equal distances stay in index order) that do
// not exceed a bound on the group's k-th distance; the 16 sorted lists are
// then merged by rounds of a (d2, j) minimum across the group.  Then the
// FP64 Gaussian of the point and its neighbours.
constexpr int kQLanes = 16;
constexpr int kChunk = 32;   // candidates per lane between group-bound updates

template <int KC>
__global__ __launch_bounds__(kB) void k_scan_knn_cov(const float* __restrict__ xyz, int n, int k, float eps,
                                                     float4* __restrict__ rec) {
    __shared__ float3 tile[kPtsTile];
    const int grp = threadIdx.x / kQLanes, gl = threadIdx.x % kQLanes;
    const int i = blockIdx.x * (kB / kQLanes) + grp;
    const bool active = i < n;   // uniform over the point's lanes
    const float3 pi = active ? make_float3(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]) : make_float3(0, 0, 0);
    const int kk = min(k, n - 1);
    float bd[KC];
    int bj[KC];
#pragma unroll
    for (int m = 0; m < KC; ++m) {
        bd[m] = __builtin_inff();
        bj[m] = 0x7FFFFFFF;
    }
    // lists needed per lane to bound the group's kk-th distance (kk <= KC)
    const int mb = kk > kQLanes ? 1 : 0;
    float bound = __builtin_inff();
    // Seed the bound from the 16 (mb + 1) points nearest to i in scan order
    // (sensor order keeps them close in space): each lane measures mb + 1 of
    // them with the same arithmetic as the search below.
    const int nseed = kQLanes * (mb + 1);
    if (active && n - 1 >= nseed) {
        const int start = max(0, min(i - nseed / 2, n - 1 - nseed));
        float own = 0.0f;
        for (int r = 0; r <= mb; ++r) {
            int j = start + kQLanes * r + gl;
            j += j >= i ? 1 : 0;
            const float dx = xyz[3 * j] - pi.x, dy = xyz[3 * j + 1] - pi.y, dz = xyz[3 * j + 2] - pi.z;
            own = fmaxf(own, __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
        }
#pragma unroll
        for (int off = kQLanes / 2; off >= 1; off >>= 1) own = fmaxf(own, __shfl_xor(own, off, 64));
        bound = own;
    }
    for (int base = 0; base < n; base += kPtsTile) {
        const int cnt = min(kPtsTile, n - base);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += kB)
            tile[t] = make_float3(xyz[3 * (base + t)], xyz[3 * (base + t) + 1], xyz[3 * (base + t) + 2]);
        __syncthreads();
        if (!active) continue;
        for (int c0 = 0; c0 < cnt; c0 += kQLanes * kChunk) {
            const int c1 = min(cnt, c0 + kQLanes * kChunk);
            for (int t = c0 + gl; t < c1; t += kQLanes) {
                const int j = base + t;
                if (j == i) continue;
                const float3 pj = tile[t];
                const float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
                const float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
                if (d2 < bd[KC - 1] && d2 <= bound) {
#pragma unroll
                    for (int m = KC - 1; m >= 1; --m) {
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
            // Group bound: every lane holds at least mb + 1 distinct candidates
            // at or below its bd[mb], so 16 (mb + 1) >= kk candidates lie at or
            // below the maximum over the group, and so does every one of the
            // final kk.  Candidates above it are never needed (same lists as
            // without the bound for the entries the merge takes).
            float own = mb >= 1 ? bd[1] : bd[0];
#pragma unroll
            for (int off = kQLanes / 2; off >= 1; off >>= 1) own = fmaxf(own, __shfl_xor(own, off, 64));
            bound = fminf(bound, own);
        }
    }
    if (!active) return;
    // merge: round r takes the smallest head of the group's lists and pops it
    int nb[KC];
#pragma unroll
    for (int r = 0; r < KC; ++r) {
        float d = bd[0];
        int j = bj[0];
#pragma unroll
        for (int off = kQLanes / 2; off >= 1; off >>= 1) {
            const float od = __shfl_xor(d, off, 64);
            const int oj = __shfl_xor(j, off, 64);
            const bool take = od < d || (od == d && oj < j);
            d = take ? od : d;
            j = take ? oj : j;
        }
        nb[r] = j;
        if (bj[0] == j) {   // this lane held the minimum (indices are unique)
#pragma unroll
            for (int m = 0; m + 1 < KC; ++m) {
                bd[m] = bd[m + 1];
                bj[m] = bj[m + 1];
            }
            bd[KC - 1] = __builtin_inff();
            bj[KC - 1] = 0x7FFFFFFF;
        }
    }
    if (gl != 0) return;
    double c6[6];
    if (kk + 1 < 5) {
        c6[0] = 1; c6[1] = 0; c6[2] = 0; c6[3] = 1; c6[4] = 0; c6[5] = 1;
    } else {
        // unrolled over the list capacity so that nb is indexed by constants
        // and stays in registers; sums in list order
        double sm[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
#pragma unroll
        for (int a = 0; a < KC; ++a) {
            if (a < kk) {
                const int j = nb[a];
                sm[0] = sm[0] + (double)xyz[3 * j];
                sm[1] = sm[1] + (double)xyz[3 * j + 1];
                sm[2] = sm[2] + (double)xyz[3 * j + 2];
            }
        }
        const double dn = (double)(kk + 1);
        const double mu[3] = {sm[0] / dn, sm[1] / dn, sm[2] / dn};
        double S[6] = {0, 0, 0, 0, 0, 0};
        {
            const double d0 = (double)pi.x - mu[0];
            const double d1 = (double)pi.y - mu[1];
            const double d2 = (double)pi.z - mu[2];
            S[0] += d0 * d0; S[1] += d0 * d1; S[2] += d0 * d2;
            S[3] += d1 * d1; S[4] += d1 * d2; S[5] += d2 * d2;
        }
#pragma unroll
        for (int a = 0; a < KC; ++a) {
            if (a < kk) {
                const int j = nb[a];
                const double d0 = (double)xyz[3 * j] - mu[0];
                const double d1 = (double)xyz[3 * j + 1] - mu[1];
                const double d2 = (double)xyz[3 * j + 2] - mu[2];
                S[0] += d0 * d0; S[1] += d0 * d1; S[2] += d0 * d2;
                S[3] += d1 * d1; S[4] += d1 * d2; S[5] += d2 * d2;
            }
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

// Finiteness of the points (and covariances) and the minimum corner of the
// points' bounding box: one workgroup (n <= 65536), deterministic (min and or).
constexpr int kChk = 1024;
__global__ __launch_bounds__(kChk) void k_scan_check(const float* __restrict__ xyz, const float* __restrict__ cov,
                                                     int n, float* __restrict__ lo_bad) {
    __shared__ float red[3][kChk];
    __shared__ int rbad[kChk];
    float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    int bad = 0;
    for (int i = threadIdx.x; i < n; i += kChk) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = xyz[3 * i + a];
            bad |= !__builtin_isfinite(v);
            lo[a] = fminf(lo[a], v);
        }
        if (cov)
#pragma unroll
            for (int a = 0; a < 6; ++a) bad |= !__builtin_isfinite(cov[6 * i + a]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) red[a][threadIdx.x] = lo[a];
    rbad[threadIdx.x] = bad;
    __syncthreads();
    for (int h = kChk / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int a = 0; a < 3; ++a) red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + h]);
            rbad[threadIdx.x] |= rbad[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        lo_bad[0] = red[0][0];
        lo_bad[1] = red[1][0];
        lo_bad[2] = red[2][0];
        lo_bad[3] = rbad[0] ? 1.0f : 0.0f;
    }
}

__device__ inline uint32_t spread10(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// 30-bit Morton (Z-order) key of each point's cell (edge `cell`, 1024 cells
// per axis from the box corner, clamped) and the identity permutation
__global__ void k_morton_keys(const float* __restrict__ xyz, int n, const float* __restrict__ lo_bad, float inv_cell,
                              uint32_t* __restrict__ key, int32_t* __restrict__ idx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float q = floorf((xyz[3 * i + a] - lo_bad[a]) * inv_cell);
        c[a] = (uint32_t)fminf(fmaxf(q, 0.0f), 1023.0f);
    }
    key[i] = spread10(c[0]) | (spread10(c[1]) << 1) | (spread10(c[2]) << 2);
    idx[i] = i;
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
        constexpr int per = kB / kQLanes;
        const unsigned grid = (unsigned)((n + per - 1) / per);
        float4* r4 = reinterpret_cast<float4*>(rec);
        if (k <= 8) k_scan_knn_cov<8><<<grid, kB, 0, s>>>(xyz, n, k, eps, r4);
        else if (k <= 16) k_scan_knn_cov<16><<<grid, kB, 0, s>>>(xyz, n, k, eps, r4);
        else k_scan_knn_cov<32><<<grid, kB, 0, s>>>(xyz, n, k, eps, r4);
    }
    MP_CHECK_LAUNCH();
}

void mp_scan_check(const float* xyz_dev, const float* cov6_dev, int32_t n, float* lo_bad_dev, hipStream_t s) {
    k_scan_check<<<1, kChk, 0, s>>>(xyz_dev, cov6_dev, n, lo_bad_dev);
    MP_CHECK_LAUNCH();
}

void mp_scan_walk_order(const float* xyz_dev, int32_t n, float cell, const float* lo_bad_dev, uint32_t* keys,
                        uint32_t* keys_alt, int32_t* perm, int32_t* perm_alt, DevMem& scratch, hipStream_t s) {
    if (n <= 0) return;
    k_morton_keys<<<(n + 255) / 256, 256, 0, s>>>(xyz_dev, n, lo_bad_dev, 1.0f / cell, keys, perm);
    MP_CHECK_LAUNCH();
    mp_radix_sort_u32(keys, perm, keys_alt, perm_alt, n, 30, scratch, s);
}
