// map_build.hip -- per-voxel GICP Gaussians and the nearest-neighbour field.
//
// Sec. III-C ("Likelihood evaluation"): every map element is a Gaussian
// N(mu, Sigma) (GICP, Segal et al. 2009) and a precomputed nearest-neighbour
// field m^nnf maps a voxel of space to the index of the nearest map element.
// Here the elements are per-voxel Gaussians and the field covers the band of
// voxels within Chebyshev radius R of an occupied voxel.
//
// Per-point Gaussians (gauss_mode POINT, the paper's own construction):
// after the same voxel sort, a dense grid of the occupied voxels' runs lets
// each point search the voxel shells around its own for its k nearest other
// points (register-resident sorted list; the search stops after shell s once
// the k-th distance is below s r less a margin, since every point of an outer
// shell is at least s r away); FP64 mean and covariance of the point and its
// list, the same Jacobi normal; kept points compacted in sorted order; each
// kept point proposes (FP32 |p - cell centre|^2 bits << 32 | id) to the cells
// of the block within R around its voxel when that distance is <= R r.
//
// Build pipeline (one-time; synchronises the stream to size its outputs):
//   voxel of each point (FP32 floor(p * 1/r)) and bounds
//   -> linear key in the bounds grid, stable radix sort of (key, point index)
//   -> run starts -> one thread per voxel: FP64 mean and 1/n covariance summed
//      in ascending point index, cyclic Jacobi eigen-solve (fixed operation
//      order), normal = eigenvector of the smallest eigenvalue
//   -> compaction of voxels with >= min_points points; ids in ascending
//      (vz, vy, vx)
//   -> band: every (Gaussian, offset in [-R, R]^3) proposes
//      (squared offset << 32 | id) to its voxel with a 64-bit atomicMin, so a
//      band voxel keeps the nearest Gaussian, ties to the smaller id
//   -> dense grid of ids, or an open-addressing hash map (linear probing,
//      8-byte slots {linear index + 1, id}) sized to twice the band.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "mp_internal.hpp"
#include "mp_lookup.hpp"

namespace {

constexpr int kBlock = 256;

__device__ inline uint32_t grid_hash(int32_t x, int32_t y, int32_t z) { return mp_grid_hash(x, y, z); }

__global__ void k_voxelize(const float* __restrict__ xyz, int64_t n, float inv_r, int3* __restrict__ vox,
                           int32_t* __restrict__ bounds /* minx,miny,minz,maxx,maxy,maxz */,
                           int32_t* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int3 v = make_int3(0, 0, 0);
    bool ok = false;
    if (i < n) {
        const float x = xyz[3 * i] * inv_r, y = xyz[3 * i + 1] * inv_r, z = xyz[3 * i + 2] * inv_r;
        ok = isfinite(x) && isfinite(y) && isfinite(z) && fabsf(x) < 1073741824.0f && fabsf(y) < 1073741824.0f &&
             fabsf(z) < 1073741824.0f;
        if (ok) {
            v = make_int3((int32_t)floorf(x), (int32_t)floorf(y), (int32_t)floorf(z));
        } else {
            atomicOr(bad, 1);
        }
        vox[i] = v;
    }
    // block min/max, then one atomic per block
    __shared__ int32_t smin[3][kBlock], smax[3][kBlock];
    const int t = threadIdx.x;
    smin[0][t] = ok ? v.x : INT32_MAX; smin[1][t] = ok ? v.y : INT32_MAX; smin[2][t] = ok ? v.z : INT32_MAX;
    smax[0][t] = ok ? v.x : INT32_MIN; smax[1][t] = ok ? v.y : INT32_MIN; smax[2][t] = ok ? v.z : INT32_MIN;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
            for (int a = 0; a < 3; ++a) {
                smin[a][t] = min(smin[a][t], smin[a][t + s]);
                smax[a][t] = max(smax[a][t], smax[a][t + s]);
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        for (int a = 0; a < 3; ++a) {
            atomicMin(&bounds[a], smin[a][0]);
            atomicMax(&bounds[3 + a], smax[a][0]);
        }
    }
}

__global__ void k_keys(const int3* __restrict__ vox, int64_t n, int3 lo, int64_t nx, int64_t ny,
                       uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int3 v = vox[i];
    keys[i] = ((uint64_t)(v.z - lo.z) * (uint64_t)ny + (uint64_t)(v.y - lo.y)) * (uint64_t)nx + (uint64_t)(v.x - lo.x);
    vals[i] = (int32_t)i;
}

__global__ void k_run_flags(const uint64_t* __restrict__ keys, int64_t n, uint32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void k_run_starts(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ rid, int64_t n,
                             int32_t* __restrict__ start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (flag[i]) start[rid[i]] = (int32_t)i;
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 in FP64 (Golub & Van
// Loan, sec. 8.5), fixed operation order; returns the unit eigenvector of the
// smallest eigenvalue.
__device__ void jacobi_min_vec(double A[9], double nrm[3]) {
    double V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int sweep = 0; sweep < 60; ++sweep) {
        const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        const double dg = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-300 || off <= 1e-34 * dg) break;
        // unrolled: every index into A and V is a constant (registers, not
        // private memory)
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
    // smallest eigenvalue, the lowest index on ties
    int m = 0;
    if (A[4] < A[0]) m = 1;
    if (A[8] < (m == 1 ? A[4] : A[0])) m = 2;
    nrm[0] = m == 0 ? V[0] : (m == 1 ? V[1] : V[2]);
    nrm[1] = m == 0 ? V[3] : (m == 1 ? V[4] : V[5]);
    nrm[2] = m == 0 ? V[6] : (m == 1 ? V[7] : V[8]);
}

__global__ void k_voxel_stats(const float* __restrict__ xyz, const int32_t* __restrict__ order,
                              const int32_t* __restrict__ start, int64_t nruns, int64_t n, int32_t min_pts,
                              const int3* __restrict__ vox, float gicp_a, float4* __restrict__ st_mu,
                              float4* __restrict__ st_n, int3* __restrict__ st_vox, uint32_t* __restrict__ keep) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nruns) return;
    const int64_t s = start[j];
    const int64_t e = (j + 1 < nruns) ? start[j + 1] : n;
    const int64_t cnt = e - s;
    if (cnt < min_pts) {
        keep[j] = 0;
        return;
    }
    keep[j] = 1;
    double sm[3] = {0.0, 0.0, 0.0};
    for (int64_t k = s; k < e; ++k) {
        const int64_t idx = order[k];
        sm[0] = sm[0] + (double)xyz[3 * idx];
        sm[1] = sm[1] + (double)xyz[3 * idx + 1];
        sm[2] = sm[2] + (double)xyz[3 * idx + 2];
    }
    const double dn = (double)cnt;
    const double mu[3] = {sm[0] / dn, sm[1] / dn, sm[2] / dn};
    double S[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = s; k < e; ++k) {
        const int64_t idx = order[k];
        const double d0 = (double)xyz[3 * idx] - mu[0];
        const double d1 = (double)xyz[3 * idx + 1] - mu[1];
        const double d2 = (double)xyz[3 * idx + 2] - mu[2];
        S[0] += d0 * d0; S[1] += d0 * d1; S[2] += d0 * d2;
        S[3] += d1 * d1; S[4] += d1 * d2; S[5] += d2 * d2;
    }
    for (int a = 0; a < 6; ++a) S[a] /= dn;
    double A[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
    double nv[3];
    jacobi_min_vec(A, nv);
    st_mu[j] = make_float4((float)mu[0], (float)mu[1], (float)mu[2], (float)cnt);
    // the record also carries lam_n = 1 - a |n|^2 of the stored FP32 normal (FP64, then rounded): the
    // eigenvalue of Sigma^M along n, which FP32 arithmetic cannot form without cancellation
    const float n0 = (float)nv[0], n1 = (float)nv[1], n2 = (float)nv[2];
    const double nn = (double)n0 * (double)n0 + (double)n1 * (double)n1 + (double)n2 * (double)n2;
    st_n[j] = make_float4(n0, n1, n2, (float)(1.0 - (double)gicp_a * nn));
    st_vox[j] = vox[order[s]];
}

__global__ void k_compact(const uint32_t* __restrict__ keep, const uint32_t* __restrict__ gid, int64_t nruns,
                          const float4* __restrict__ st_mu, const float4* __restrict__ st_n,
                          const int3* __restrict__ st_vox, float4* __restrict__ gauss, int3* __restrict__ gvox,
                          int32_t* __restrict__ bounds) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nruns || !keep[j]) return;
    const uint32_t g = gid[j];
    gauss[2 * (int64_t)g] = st_mu[j];
    gauss[2 * (int64_t)g + 1] = st_n[j];
    const int3 v = st_vox[j];
    gvox[g] = v;
    atomicMin(&bounds[0], v.x); atomicMin(&bounds[1], v.y); atomicMin(&bounds[2], v.z);
    atomicMax(&bounds[3], v.x); atomicMax(&bounds[4], v.y); atomicMax(&bounds[5], v.z);
}

// ------------------------------------------------------------ per-point Gaussians
__device__ __forceinline__ bool knn_less(float d, int32_t j, float e, int32_t k) {
    return d < e || (d == e && j < k);
}

// One lane per sorted map point: its k nearest other points among the voxels
// within Chebyshev distance S (occupancy grid `occ` over the box lo + [0, dims)
// holds the run of each occupied voxel), then the point's Gaussian.
template <int KC>
__global__ __launch_bounds__(256) void k_point_gauss(const float* __restrict__ xyz, const int32_t* __restrict__ order,
                                                    const int32_t* __restrict__ start, int64_t nruns, int64_t n,
                                                    const int3* __restrict__ vox, const int32_t* __restrict__ occ,
                                                    int3 lo, int3 dims, int k, int S, float r, int32_t min_pts,
                                                    float gicp_a, float4* __restrict__ st_mu, float4* __restrict__ st_n,
                                                    int3* __restrict__ st_vox, uint32_t* __restrict__ keep,
                                                    int32_t* __restrict__ knn_out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t i = order[t];
    const float px = xyz[3 * (int64_t)i], py = xyz[3 * (int64_t)i + 1], pz = xyz[3 * (int64_t)i + 2];
    const int3 v = vox[i];
    float bd[KC];
    int32_t bj[KC];
#pragma unroll
    for (int a = 0; a < KC; ++a) {
        bd[a] = INFINITY;
        bj[a] = INT32_MAX;
    }
    float thd = INFINITY;      // entry k - 1 of the sorted list: the admission bound
    int32_t thj = INT32_MAX;
    int cnt = 0;
    // a point of a voxel outside shell s lies more than s r away; the margin
    // covers the FP32 voxelisation and squared-distance rounding
    const float slop = 1e-3f * r + 5e-7f * (fabsf(px) + fabsf(py) + fabsf(pz));
    for (int sh = 0; sh <= S; ++sh) {
        for (int dz = -sh; dz <= sh; ++dz)
            for (int dy = -sh; dy <= sh; ++dy)
                for (int dx = -sh; dx <= sh; ++dx) {
                    if (max(abs(dx), max(abs(dy), abs(dz))) != sh) continue;
                    const int64_t ux = (int64_t)v.x + dx - lo.x, uy = (int64_t)v.y + dy - lo.y,
                                  uz = (int64_t)v.z + dz - lo.z;
                    if (ux < 0 || uy < 0 || uz < 0 || ux >= dims.x || uy >= dims.y || uz >= dims.z) continue;
                    const int32_t run = occ[(uz * dims.y + uy) * dims.x + ux];
                    if (run < 0) continue;
                    const int64_t q0 = start[run], q1 = run + 1 < nruns ? start[run + 1] : n;
                    for (int64_t q = q0; q < q1; ++q) {
                        const int32_t j = order[q];
                        if (j == i) continue;
                        const float ex = xyz[3 * (int64_t)j] - px, ey = xyz[3 * (int64_t)j + 1] - py,
                                    ez = xyz[3 * (int64_t)j + 2] - pz;
                        float d = __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez));
                        if (!knn_less(d, j, thd, thj)) continue;
                        // insertion into the sorted list by selects: slot a
                        // takes the candidate if it ranks below the old entry
                        // a and not below entry a - 1, else entry a - 1
                        // (slots rewritten from the top, so a - 1 is still old)
                        bool lt[KC];
#pragma unroll
                        for (int a = 0; a < KC; ++a) lt[a] = knn_less(d, j, bd[a], bj[a]);
#pragma unroll
                        for (int a = KC - 1; a >= 0; --a) {
                            const bool up = a > 0 && lt[a > 0 ? a - 1 : 0];
                            const float nd = up ? bd[a > 0 ? a - 1 : 0] : d;
                            const int32_t nj = up ? bj[a > 0 ? a - 1 : 0] : j;
                            bd[a] = lt[a] ? nd : bd[a];
                            bj[a] = lt[a] ? nj : bj[a];
                        }
                        cnt = min(cnt + 1, k);
                        if (cnt == k) {
#pragma unroll
                            for (int a = 0; a < KC; ++a)
                                if (a == k - 1) {
                                    thd = bd[a];
                                    thj = bj[a];
                                }
                        }
                    }
                }
        if (sh >= 1 && cnt == k) {
            const float b = (float)sh * r - slop;
            if (b > 0.0f && thd < b * b) break;   // (b <= 0: cells too small for the bound; search on)
        }
    }
    if (knn_out) {   // test output: the list of point i, -1 pads
#pragma unroll
        for (int a = 0; a < KC; ++a)
            if (a < k) knn_out[(int64_t)i * k + a] = a < cnt ? bj[a] : -1;
    }
    const int m = cnt + 1;
    st_vox[t] = v;
    if (m < min_pts) {
        keep[t] = 0;
        return;
    }
    keep[t] = 1;
    double sm[3] = {(double)px, (double)py, (double)pz};
#pragma unroll
    for (int a = 0; a < KC; ++a)
        if (a < cnt) {
            const int64_t j = bj[a];
            sm[0] = sm[0] + (double)xyz[3 * j];
            sm[1] = sm[1] + (double)xyz[3 * j + 1];
            sm[2] = sm[2] + (double)xyz[3 * j + 2];
        }
    const double dm = (double)m;
    const double mu[3] = {sm[0] / dm, sm[1] / dm, sm[2] / dm};
    double S6[6];
    {
        const double d0 = (double)px - mu[0], d1 = (double)py - mu[1], d2 = (double)pz - mu[2];
        S6[0] = 0.0 + d0 * d0; S6[1] = 0.0 + d0 * d1; S6[2] = 0.0 + d0 * d2;
        S6[3] = 0.0 + d1 * d1; S6[4] = 0.0 + d1 * d2; S6[5] = 0.0 + d2 * d2;
    }
#pragma unroll
    for (int a = 0; a < KC; ++a)
        if (a < cnt) {
            const int64_t j = bj[a];
            const double d0 = (double)xyz[3 * j] - mu[0], d1 = (double)xyz[3 * j + 1] - mu[1],
                         d2 = (double)xyz[3 * j + 2] - mu[2];
            S6[0] += d0 * d0; S6[1] += d0 * d1; S6[2] += d0 * d2;
            S6[3] += d1 * d1; S6[4] += d1 * d2; S6[5] += d2 * d2;
        }
    for (int a = 0; a < 6; ++a) S6[a] /= dm;
    double A[9] = {S6[0], S6[1], S6[2], S6[1], S6[3], S6[4], S6[2], S6[4], S6[5]};
    double nv[3];
    jacobi_min_vec(A, nv);
    st_mu[t] = make_float4(px, py, pz, (float)m);
    const float n0 = (float)nv[0], n1 = (float)nv[1], n2 = (float)nv[2];
    const double nn = (double)n0 * (double)n0 + (double)n1 * (double)n1 + (double)n2 * (double)n2;
    st_n[t] = make_float4(n0, n1, n2, (float)(1.0 - (double)gicp_a * nn));
}

// occupancy grid: the run index of every occupied voxel (keys are the linear
// index of the voxel in the box of all map voxels)
__global__ void k_occ_fill(const uint64_t* __restrict__ keys, const int32_t* __restrict__ start, int64_t nruns,
                           int32_t* __restrict__ occ) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nruns) return;
    occ[keys[start[j]]] = (int32_t)j;
}

struct BandGrid {
    int32_t org[3];
    int32_t dim[3];
};

// every (Gaussian, offset) proposes (d2 << 32 | gid) to its band voxel
// (grid-stride: G (2R+1)^3 proposals can exceed the 2^32 work-items of one dispatch)
__global__ void k_band_dense(const int3* __restrict__ gvox, int64_t G, int R, BandGrid bg,
                             unsigned long long* __restrict__ cells) {
    const int side = 2 * R + 1;
    const int64_t vol = (int64_t)side * side * side;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < G * vol; t += stride) {
        const int64_t g = t / vol;
        const int o = (int)(t - g * vol);
        const int dx = o % side - R, dy = (o / side) % side - R, dz = o / (side * side) - R;
        const int3 u = gvox[g];
        const int64_t x = (int64_t)u.x + dx - bg.org[0], y = (int64_t)u.y + dy - bg.org[1],
                      z = (int64_t)u.z + dz - bg.org[2];
        const int64_t L = (z * bg.dim[1] + y) * bg.dim[0] + x;
        const unsigned long long val =
            ((unsigned long long)(dx * dx + dy * dy + dz * dz) << 32) | (unsigned long long)g;
        atomicMin(&cells[L], val);
    }
}

// per-point field: every (kept point, offset) proposes (bits of the FP32
// squared distance to the cell's centre << 32 | id) when within R r
__global__ void k_band_points_dense(const int3* __restrict__ gvox, const float4* __restrict__ gauss, int64_t G,
                                    int R, float r, float lim2, BandGrid bg, unsigned long long* __restrict__ cells) {
    const int side = 2 * R + 1;
    const int64_t vol = (int64_t)side * side * side;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < G * vol; t += stride) {
        const int64_t g = t / vol;
        const int o = (int)(t - g * vol);
        const int dx = o % side - R, dy = (o / side) % side - R, dz = o / (side * side) - R;
        const int3 u = gvox[g];
        const float4 p = gauss[2 * g];
        const int32_t cx = u.x + dx, cy = u.y + dy, cz = u.z + dz;
        const float ex = p.x - ((float)cx + 0.5f) * r;
        const float ey = p.y - ((float)cy + 0.5f) * r;
        const float ez = p.z - ((float)cz + 0.5f) * r;
        const float d2 = (ex * ex + ey * ey) + ez * ez;
        if (!(d2 <= lim2)) continue;
        const int64_t x = (int64_t)cx - bg.org[0], y = (int64_t)cy - bg.org[1], z = (int64_t)cz - bg.org[2];
        const int64_t L = (z * bg.dim[1] + y) * bg.dim[0] + x;
        const unsigned long long val = ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned long long)g;
        atomicMin(&cells[L], val);
    }
}

__global__ void k_dense_finalize(const unsigned long long* __restrict__ cells, int64_t ncell,
                                 int32_t* __restrict__ dense, unsigned long long* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int hit = 0;
    if (i < ncell) {
        const unsigned long long c = cells[i];
        hit = c != ~0ull;
        dense[i] = hit ? (int32_t)(uint32_t)(c & 0xFFFFFFFFull) : -1;
    }
    const uint64_t b = __ballot(hit);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
}

constexpr float kFarMean = 1.0e15f;

// per-cell copy of the nearest Gaussian's record (the likelihood's one-fetch
// path), followed by one record for points outside the grid
__global__ void k_dense_records(const int32_t* __restrict__ dense, int64_t ncell, const float4* __restrict__ gauss,
                                float4* __restrict__ drec) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncell) return;
    const int32_t g = c < ncell ? dense[c] : -1;   // record ncell: the miss record
    if (g >= 0) {
        drec[2 * c] = gauss[2 * (int64_t)g];
        drec[2 * c + 1] = gauss[2 * (int64_t)g + 1];
    } else {
        // no Gaussian: a mean 1e15 m away fails every residual gate, while
        // squares and products of the residual stay finite in FP32; no normal
        // (lam_n = 1 - a |0|^2 = 1 keeps the masked Omega finite)
        drec[2 * c] = make_float4(kFarMean, kFarMean, kFarMean, 0.0f);
        drec[2 * c + 1] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
    }
}

// wide build table: slot = {key (linear index + 1, 0 empty), value}
__global__ void k_band_hash(const int3* __restrict__ gvox, int64_t G, int R, BandGrid bg,
                            unsigned long long* __restrict__ tkey, unsigned long long* __restrict__ tval,
                            uint64_t mask) {
    const int side = 2 * R + 1;
    const int64_t vol = (int64_t)side * side * side;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < G * vol; t += stride) {
        const int64_t g = t / vol;
        const int o = (int)(t - g * vol);
        const int dx = o % side - R, dy = (o / side) % side - R, dz = o / (side * side) - R;
        const int3 u = gvox[g];
        const int32_t x = u.x + dx - bg.org[0], y = u.y + dy - bg.org[1], z = u.z + dz - bg.org[2];
        const unsigned long long key = (((unsigned long long)z * bg.dim[1] + y) * bg.dim[0] + x) + 1ull;
        const unsigned long long val =
            ((unsigned long long)(dx * dx + dy * dy + dz * dz) << 32) | (unsigned long long)g;
        uint64_t h = grid_hash(x, y, z) & mask;
        for (;;) {
            const unsigned long long prev = atomicCAS(&tkey[h], 0ull, key);
            if (prev == 0ull || prev == key) {
                atomicMin(&tval[h], val);
                break;
            }
            h = (h + 1) & mask;
        }
    }
}

// grid-stride over the slots; lane 0 holds the wave's smallest index, so it is
// active in every iteration any lane of its wave takes
__global__ void k_count_slots(const unsigned long long* __restrict__ tkey, int64_t cap,
                              unsigned long long* __restrict__ count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < cap; i0 += stride) {
        const int64_t i = i0 + threadIdx.x;
        const int hit = (i < cap) && tkey[i] != 0ull;
        const uint64_t b = __ballot(hit);
        if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
    }
}

__global__ void k_rehash(const unsigned long long* __restrict__ tkey, const unsigned long long* __restrict__ tval,
                         int64_t cap, BandGrid bg, uint2* __restrict__ table, uint32_t mask) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += stride) {
        const unsigned long long k = tkey[i];
        if (k == 0ull) continue;
        const uint64_t L = k - 1ull;
        const int32_t x = (int32_t)(L % (uint64_t)bg.dim[0]);
        const int32_t y = (int32_t)((L / (uint64_t)bg.dim[0]) % (uint64_t)bg.dim[1]);
        const int32_t z = (int32_t)(L / ((uint64_t)bg.dim[0] * (uint64_t)bg.dim[1]));
        uint32_t h = grid_hash(x, y, z) & mask;
        const uint32_t key32 = (uint32_t)k;
        const uint32_t gid = (uint32_t)(tval[i] & 0xFFFFFFFFull);
        for (;;) {
            const uint32_t prev = atomicCAS(&table[h].x, 0u, key32);
            if (prev == 0u) {
                table[h].y = gid;
                break;
            }
            h = (h + 1) & mask;
        }
    }
}

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// grid of a grid-stride launch over n items: at most 2^20 workgroups
// (2^28 work-items, well inside the 2^32 of one dispatch)
inline unsigned nblk_capped(int64_t n, int b = kBlock) {
    return (unsigned)std::min<int64_t>((n + b - 1) / b, (int64_t)1 << 20);
}

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

// ------------------------------------------------------------ lookup (the likelihood kernel takes the same path)

namespace {
__global__ void k_lookup(MapView v, const float* __restrict__ xyz, int64_t n, int32_t* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = mp_nnf_lookup(v, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
}
}  // namespace

void mp_map_lookup_launch(const MapView& v, const float* xyz_dev, int64_t n, int32_t* gid_dev, hipStream_t s) {
    if (n <= 0) return;
    k_lookup<<<nblk_capped(n), kBlock, 0, s>>>(v, xyz_dev, n, gid_dev);
    MP_CHECK_LAUNCH();
}

void mp_build_map(mp_map m, const float* xyz, int64_t n, hipStream_t s) {
    const mp_map_params& P = m->params;
    const float r = P.voxel;
    const float inv_r = 1.0f / r;
    const int R = P.nnf_radius;
    MapView& view = m->view;
    std::memset(&view, 0, sizeof(view));
    view.inv_r = inv_r;
    view.gicp_a = 1.0f - P.cov_eps;
    mp_map_info& info = m->info;
    std::memset(&info, 0, sizeof(info));

    auto finish_empty = [&]() {
        view.backend = MP_NNF_DENSE;
        view.dim[0] = view.dim[1] = view.dim[2] = 0;
        info.backend = MP_NNF_DENSE;
        for (int a = 0; a < 3; ++a) { m->box_lo[a] = 0; m->box_hi[a] = 0; }
    };
    if (n == 0) {
        finish_empty();
        return;
    }

    DevMem d_vox, d_bounds, d_bad, d_keys, d_keys2, d_vals, d_vals2, d_flag, d_rid, d_start, scratch;
    d_vox.alloc(sizeof(int3) * (size_t)n);
    d_bounds.alloc(sizeof(int32_t) * 8);
    d_bad.alloc(sizeof(int32_t));
    int32_t hb[8] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN, 0, 0};
    MP_HIP(hipMemcpyAsync(d_bounds.p, hb, sizeof(hb), hipMemcpyHostToDevice, s));
    MP_HIP(hipMemsetAsync(d_bad.p, 0, 4, s));
    k_voxelize<<<nblk(n), kBlock, 0, s>>>(xyz, n, inv_r, d_vox.as<int3>(), d_bounds.as<int32_t>(), d_bad.as<int32_t>());
    MP_CHECK_LAUNCH();
    int32_t bad = 0;
    MP_HIP(hipMemcpyAsync(hb, d_bounds.p, sizeof(hb), hipMemcpyDeviceToHost, s));
    MP_HIP(hipMemcpyAsync(&bad, d_bad.p, 4, hipMemcpyDeviceToHost, s));
    MP_HIP(hipStreamSynchronize(s));
    if (bad) mp_throw(MP_E_ARG, "mp_map_build: non-finite or out-of-range map coordinate (|p/r| >= 2^30)");

    const int3 lo = make_int3(hb[0], hb[1], hb[2]);
    const int64_t nx = (int64_t)hb[3] - hb[0] + 1, ny = (int64_t)hb[4] - hb[1] + 1, nz = (int64_t)hb[5] - hb[2] + 1;
    const double cells = (double)nx * (double)ny * (double)nz;
    if (cells >= 9.0e18) mp_throw(MP_E_UNSUPPORTED, "mp_map_build: map extent too large for 64-bit voxel keys");
    int bits = 1;
    while (bits < 64 && std::ldexp(1.0, bits) < cells) ++bits;

    d_keys.alloc(sizeof(uint64_t) * (size_t)n);
    d_keys2.alloc(sizeof(uint64_t) * (size_t)n);
    d_vals.alloc(sizeof(int32_t) * (size_t)n);
    d_vals2.alloc(sizeof(int32_t) * (size_t)n);
    k_keys<<<nblk(n), kBlock, 0, s>>>(d_vox.as<int3>(), n, lo, nx, ny, d_keys.as<uint64_t>(), d_vals.as<int32_t>());
    MP_CHECK_LAUNCH();
    mp_radix_sort_u64(d_keys.as<uint64_t>(), d_vals.as<int32_t>(), d_keys2.as<uint64_t>(), d_vals2.as<int32_t>(), n,
                      bits, scratch, s);
    d_keys2.release();
    d_vals2.release();

    d_flag.alloc(sizeof(uint32_t) * (size_t)n);
    d_rid.alloc(sizeof(uint32_t) * (size_t)n);
    DevMem d_total;
    d_total.alloc(16);
    k_run_flags<<<nblk(n), kBlock, 0, s>>>(d_keys.as<uint64_t>(), n, d_flag.as<uint32_t>());
    MP_CHECK_LAUNCH();
    mp_scan_exclusive_u32(d_flag.as<uint32_t>(), d_rid.as<uint32_t>(), n, d_total.as<uint32_t>(), scratch, s);
    uint32_t nruns = 0;
    MP_HIP(hipMemcpyAsync(&nruns, d_total.p, 4, hipMemcpyDeviceToHost, s));
    MP_HIP(hipStreamSynchronize(s));
    d_start.alloc(sizeof(int32_t) * (size_t)nruns);
    k_run_starts<<<nblk(n), kBlock, 0, s>>>(d_flag.as<uint32_t>(), d_rid.as<uint32_t>(), n, d_start.as<int32_t>());
    MP_CHECK_LAUNCH();

    // per-point Gaussians: one candidate per point (sorted order), found
    // through an occupancy grid of the voxel runs; per-voxel: one per run
    const bool per_point = P.gauss_mode == MP_GAUSS_POINT;
    DevMem occ;
    if (per_point) {
        if (cells > 268435456.0)
            mp_throw(MP_E_UNSUPPORTED, "mp_map_build: per-point Gaussians need the box of map voxels <= 2^28 cells");
        occ.alloc(sizeof(int32_t) * (size_t)cells);
        MP_HIP(hipMemsetAsync(occ.p, 0xFF, sizeof(int32_t) * (size_t)cells, s));
        k_occ_fill<<<nblk(nruns), kBlock, 0, s>>>(d_keys.as<uint64_t>(), d_start.as<int32_t>(), nruns,
                                                   occ.as<int32_t>());
        MP_CHECK_LAUNCH();
    }
    d_keys.release();
    const int64_t nst = per_point ? n : (int64_t)nruns;

    DevMem st_mu, st_n, st_vox, keep, gid;
    st_mu.alloc(sizeof(float4) * nst);
    st_n.alloc(sizeof(float4) * nst);
    st_vox.alloc(sizeof(int3) * nst);
    keep.alloc(sizeof(uint32_t) * nst);
    gid.alloc(sizeof(uint32_t) * nst);
    if (per_point) {
        const int3 dims = make_int3((int)nx, (int)ny, (int)nz);
        auto launch = [&](auto kern) {
            kern<<<nblk(n), kBlock, 0, s>>>(xyz, d_vals.as<int32_t>(), d_start.as<int32_t>(), (int64_t)nruns, n,
                                            d_vox.as<int3>(), occ.as<int32_t>(), lo, dims, P.point_k, P.point_search,
                                            r, P.min_points, 1.0f - P.cov_eps, st_mu.as<float4>(), st_n.as<float4>(),
                                            st_vox.as<int3>(), keep.as<uint32_t>(), m->knn_dbg);
        };
        if (P.point_k <= 8) launch(k_point_gauss<8>);
        else if (P.point_k <= 16) launch(k_point_gauss<16>);
        else launch(k_point_gauss<32>);
        MP_CHECK_LAUNCH();
    } else {
        k_voxel_stats<<<nblk(nruns, 64), 64, 0, s>>>(xyz, d_vals.as<int32_t>(), d_start.as<int32_t>(), nruns, n,
                                                      P.min_points, d_vox.as<int3>(), 1.0f - P.cov_eps,
                                                      st_mu.as<float4>(), st_n.as<float4>(), st_vox.as<int3>(),
                                                      keep.as<uint32_t>());
        MP_CHECK_LAUNCH();
    }
    mp_scan_exclusive_u32(keep.as<uint32_t>(), gid.as<uint32_t>(), nst, d_total.as<uint32_t>(), scratch, s);
    uint32_t G = 0;
    MP_HIP(hipMemcpyAsync(&G, d_total.p, 4, hipMemcpyDeviceToHost, s));
    MP_HIP(hipStreamSynchronize(s));
    if (G == 0) {
        finish_empty();
        return;
    }
    m->gauss.alloc(sizeof(float4) * 2 * (size_t)G);
    DevMem& gvox = m->vox;
    gvox.alloc(sizeof(int3) * G);
    int32_t hb2[8] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN, 0, 0};
    MP_HIP(hipMemcpyAsync(d_bounds.p, hb2, sizeof(hb2), hipMemcpyHostToDevice, s));
    k_compact<<<nblk(nst), kBlock, 0, s>>>(keep.as<uint32_t>(), gid.as<uint32_t>(), nst, st_mu.as<float4>(),
                                              st_n.as<float4>(), st_vox.as<int3>(), m->gauss.as<float4>(),
                                              gvox.as<int3>(), d_bounds.as<int32_t>());
    MP_CHECK_LAUNCH();
    MP_HIP(hipMemcpyAsync(hb2, d_bounds.p, sizeof(hb2), hipMemcpyDeviceToHost, s));
    MP_HIP(hipStreamSynchronize(s));
    d_vox.release(); d_vals.release(); d_flag.release(); d_rid.release(); d_start.release(); occ.release();
    st_mu.release(); st_n.release(); st_vox.release(); keep.release(); gid.release();

    BandGrid bg;
    for (int a = 0; a < 3; ++a) {
        bg.org[a] = hb2[a] - R;
        const int64_t d = (int64_t)hb2[3 + a] - hb2[a] + 1 + 2 * R;
        if (d > INT32_MAX) mp_throw(MP_E_UNSUPPORTED, "mp_map_build: band grid extent exceeds 2^31 voxels");
        bg.dim[a] = (int32_t)d;
        m->box_lo[a] = (float)hb2[a] * r;
        m->box_hi[a] = (float)(hb2[3 + a] + 1) * r;
    }
    const double bcells = (double)bg.dim[0] * (double)bg.dim[1] * (double)bg.dim[2];
    int backend = P.backend;
    // dense: 4 B id + 32 B record per cell of the band grid's box
    // (cell indices are formed with 24-bit multiplies and records addressed by
    // 32-bit byte offsets: dim_x dim_y < 2^24 and cells + 1 < 2^27)
    const double bplane = (double)bg.dim[0] * (double)bg.dim[1];
    if (backend == MP_NNF_AUTO)
        backend = (per_point || (bcells <= 67108864.0 && bplane < 16777216.0)) ? MP_NNF_DENSE : MP_NNF_HASH;
    if (backend == MP_NNF_DENSE && (bcells > 134217726.0 || bplane >= 16777216.0))
        mp_throw(MP_E_UNSUPPORTED, "mp_map_build: dense band grid exceeds 2^27 - 2 cells or 2^24 cells per plane");
    if (backend == MP_NNF_HASH && bcells > 4294967294.0)
        mp_throw(MP_E_UNSUPPORTED, "mp_map_build: hashed band grid exceeds 2^32 - 2 cells");

    const int side = 2 * R + 1;
    const int64_t emits = (int64_t)G * side * side * side;
    DevMem d_count;
    d_count.alloc(8);
    MP_HIP(hipMemsetAsync(d_count.p, 0, 8, s));
    unsigned long long band = 0;
    if (backend == MP_NNF_DENSE) {
        const int64_t nc = (int64_t)bcells;
        DevMem wide;
        wide.alloc(sizeof(unsigned long long) * (size_t)nc);
        MP_HIP(hipMemsetAsync(wide.p, 0xFF, sizeof(unsigned long long) * (size_t)nc, s));
        if (per_point) {
            const float lim = (float)R * r;
            k_band_points_dense<<<nblk_capped(emits), kBlock, 0, s>>>(gvox.as<int3>(), m->gauss.as<float4>(), G, R, r,
                                                               lim * lim, bg, wide.as<unsigned long long>());
        } else {
            k_band_dense<<<nblk_capped(emits), kBlock, 0, s>>>(gvox.as<int3>(), G, R, bg, wide.as<unsigned long long>());
        }
        MP_CHECK_LAUNCH();
        m->dense.alloc(sizeof(int32_t) * (size_t)nc);
        k_dense_finalize<<<nblk(nc), kBlock, 0, s>>>(wide.as<unsigned long long>(), nc, m->dense.as<int32_t>(),
                                                     d_count.as<unsigned long long>());
        MP_CHECK_LAUNCH();
        MP_HIP(hipMemcpyAsync(&band, d_count.p, 8, hipMemcpyDeviceToHost, s));
        MP_HIP(hipStreamSynchronize(s));
        m->drec.alloc(sizeof(float4) * 2 * (size_t)(nc + 1));   // + the miss record
        k_dense_records<<<nblk(nc + 1), kBlock, 0, s>>>(m->dense.as<int32_t>(), nc, m->gauss.as<float4>(),
                                                        m->drec.as<float4>());
        MP_CHECK_LAUNCH();
        MP_HIP(hipStreamSynchronize(s));
        view.dense = m->dense.as<int32_t>();
        view.drec = m->drec.as<float4>();
        view.dxy = (uint32_t)bg.dim[0] * (uint32_t)bg.dim[1];
        view.dmiss = (uint32_t)nc;
        info.table_slots = nc;
    } else {
        const uint64_t wcap = next_pow2((uint64_t)std::max<int64_t>(2 * emits, 64));
        DevMem tk, tv;
        tk.alloc(sizeof(unsigned long long) * wcap);
        tv.alloc(sizeof(unsigned long long) * wcap);
        MP_HIP(hipMemsetAsync(tk.p, 0, sizeof(unsigned long long) * wcap, s));
        MP_HIP(hipMemsetAsync(tv.p, 0xFF, sizeof(unsigned long long) * wcap, s));
        k_band_hash<<<nblk_capped(emits), kBlock, 0, s>>>(gvox.as<int3>(), G, R, bg, tk.as<unsigned long long>(),
                                                   tv.as<unsigned long long>(), wcap - 1);
        MP_CHECK_LAUNCH();
        k_count_slots<<<nblk_capped((int64_t)wcap), kBlock, 0, s>>>(tk.as<unsigned long long>(), (int64_t)wcap,
                                                              d_count.as<unsigned long long>());
        MP_CHECK_LAUNCH();
        MP_HIP(hipMemcpyAsync(&band, d_count.p, 8, hipMemcpyDeviceToHost, s));
        MP_HIP(hipStreamSynchronize(s));
        const uint64_t cap = next_pow2(std::max<uint64_t>(2 * band, 64));
        if (cap > (1ull << 32)) mp_throw(MP_E_UNSUPPORTED, "mp_map_build: hash table would exceed 2^32 slots");
        m->table.alloc(sizeof(uint2) * cap);
        MP_HIP(hipMemsetAsync(m->table.p, 0, sizeof(uint2) * cap, s));
        k_rehash<<<nblk_capped((int64_t)wcap), kBlock, 0, s>>>(tk.as<unsigned long long>(), tv.as<unsigned long long>(),
                                                         (int64_t)wcap, bg, m->table.as<uint2>(),
                                                         (uint32_t)(cap - 1));
        MP_CHECK_LAUNCH();
        MP_HIP(hipStreamSynchronize(s));
        view.table = m->table.as<uint2>();
        view.mask = (uint32_t)(cap - 1);
        info.table_slots = (int64_t)cap;
    }
    view.backend = backend;
    view.gauss = m->gauss.as<float4>();
    for (int a = 0; a < 3; ++a) {
        view.org[a] = bg.org[a];
        view.dim[a] = bg.dim[a];
        info.grid_origin[a] = bg.org[a];
        info.grid_dim[a] = bg.dim[a];
        info.box_min[a] = m->box_lo[a];
        info.box_max[a] = m->box_hi[a];
    }
    info.num_gauss = G;
    info.num_band = (int64_t)band;
    info.backend = backend;
    info.device_bytes = (int64_t)(m->gauss.bytes + m->dense.bytes + m->drec.bytes + m->table.bytes + m->vox.bytes);
}
