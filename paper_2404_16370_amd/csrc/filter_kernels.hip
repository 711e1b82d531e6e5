// filter_kernels.hip -- prediction (Eq. 1), SVGD update (Eq. 5-8),
// posterior propagation on the neighbour graph (Eq. 11) and initialisation.
#include <hip/hip_runtime.h>

#include <cmath>

#include "mp_det.hpp"
#include "mp_internal.hpp"

namespace {

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// SE(3) exponential of [omega; v] as (unit quaternion, translation), FP32.
//   q = (cos(th/2), sin(th/2)/th omega),  t = V v,
//   V = I + A [w]x + B [w]x^2, A = (1 - cos th)/th^2 = (sin(th/2)/(th/2))^2 / 2,
//   B = (th - sin th)/th^3 (series below th = 0.5).
__device__ inline void se3_exp(const float xi[6], mpdet::quat& q, float3& t) {
    const float wx = xi[0], wy = xi[1], wz = xi[2];
    const float th2 = wx * wx + wy * wy + wz * wz;
    const float th = sqrtf(th2);
    float hs, hc, A, B;
    if (th < 1e-4f) {
        hs = 0.5f - th2 * (1.0f / 48.0f);
        hc = 1.0f - th2 * 0.125f;
        A = 0.5f - th2 * (1.0f / 24.0f);
        B = 1.0f / 6.0f - th2 * (1.0f / 120.0f);
    } else {
        float sh, ch;
        sincosf(0.5f * th, &sh, &ch);
        hs = sh / th;
        hc = ch;
        const float sinc_half = sh / (0.5f * th);
        A = 0.5f * sinc_half * sinc_half;
        if (th < 0.5f) {
            B = 1.0f / 6.0f + th2 * (-1.0f / 120.0f + th2 * (1.0f / 5040.0f - th2 * (1.0f / 362880.0f)));
        } else {
            B = (th - sinf(th)) / (th2 * th);
        }
    }
    q = mpdet::quat{hc, hs * wx, hs * wy, hs * wz};
    const float vx = xi[3], vy = xi[4], vz = xi[5];
    const float c1x = wy * vz - wz * vy, c1y = wz * vx - wx * vz, c1z = wx * vy - wy * vx;
    const float c2x = wy * c1z - wz * c1y, c2y = wz * c1x - wx * c1z, c2z = wx * c1y - wy * c1x;
    t = make_float3(vx + A * c1x + B * c2x, vy + A * c1y + B * c2y, vz + A * c1z + B * c2z);
}

// (q, t) (x) (dq, dt) = (q dq, t + R(q) dt), quaternion renormalised
__device__ inline void compose(mpdet::quat& q, float3& t, const mpdet::quat dq, const float3 dt) {
    const mpdet::mat3 R = mpdet::qmat(q);
    t.x += R.m[0] * dt.x + R.m[1] * dt.y + R.m[2] * dt.z;
    t.y += R.m[3] * dt.x + R.m[4] * dt.y + R.m[5] * dt.z;
    t.z += R.m[6] * dt.x + R.m[7] * dt.y + R.m[8] * dt.z;
    mpdet::quat r = mpdet::qmul(q, dq);
    const float inv = rsqrtf(r.w * r.w + r.x * r.x + r.y * r.y + r.z * r.z);
    q = mpdet::quat{r.w * inv, r.x * inv, r.y * inv, r.z * inv};
}

__device__ inline void load_pose(const float4* P, int i, mpdet::quat& q, float3& t) {
    const float4 a = P[2 * i], b = P[2 * i + 1];
    q = mpdet::quat{a.x, a.y, a.z, a.w};
    t = make_float3(b.x, b.y, b.z);
}

__device__ inline void store_pose(float4* P, int i, const mpdet::quat q, const float3 t) {
    P[2 * i] = make_float4(q.w, q.x, q.y, q.z);
    P[2 * i + 1] = make_float4(t.x, t.y, t.z, 0.0f);
}

// ------------------------------------------------------------ SVGD
struct SvgdArgs {
    const float4* __restrict__ pin;
    float4* __restrict__ pout;
    const float4* __restrict__ psi;
    const int32_t* __restrict__ nbr;
    const float* __restrict__ kval;
    int32_t n, K;
    float sr, st;
};

__device__ inline float3 cross3(const float3 a, const float3 b) {
    return float3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline float3 axpy3(float s, const float3 x, const float3 y) {
    return float3{s * x.x + y.x, s * x.y + y.y, s * x.z + y.z};
}

// J_r^-1(d)^T a for d = [om; rho], a = [aw; ar] (tangent order rotation
// first).  With M = I + 1/2 om^ + beta om^2 (the SO(3) inverse right
// Jacobian; beta as in the SE(3) logarithm) and Q(rho, om) the off-diagonal
// block of the SE(3) left Jacobian (Barfoot and Furgale, IEEE T-RO 2014):
//   J_r^-1(d) = [[M, 0], [-M Q(-rho, -om) M, M]],  Q(-rho, -om)^T = Q(rho, om),
// so that  v_r = M^T ar,  v_w = M^T (aw - Q(rho, om) v_r),
// M^T x = x - 1/2 om x x + beta om x (om x x).
__device__ inline void jr_inv_t(const float3 om, const float3 rho, float beta, const float3 aw, const float3 ar,
                                float3& vw, float3& vr) {
    auto mt = [&](const float3 x) {
        const float3 c1 = cross3(om, x);
        const float3 c2 = cross3(om, c1);
        return float3{(x.x - 0.5f * c1.x) + beta * c2.x, (x.y - 0.5f * c1.y) + beta * c2.y,
                      (x.z - 0.5f * c1.z) + beta * c2.z};
    };
    vr = mt(ar);
    const float th2 = (om.x * om.x + om.y * om.y) + om.z * om.z;
    float c1, c2, c3;   // (th - sin th)/th^3, (th^2 + 2 cos th - 2)/(2 th^4), (2 th - 3 sin th + th cos th)/(2 th^5)
    if (th2 < 1.0f) {   // Taylor series (cancellation in the closed forms below th = 1)
        c1 = fmaf(fmaf(fmaf(-1.0f / 362880.0f, th2, 1.0f / 5040.0f), th2, -1.0f / 120.0f), th2, 1.0f / 6.0f);
        c2 = fmaf(fmaf(fmaf(-1.0f / 3628800.0f, th2, 1.0f / 40320.0f), th2, -1.0f / 720.0f), th2, 1.0f / 24.0f);
        c3 = fmaf(fmaf(fmaf(-1.0f / 9979200.0f, th2, 1.0f / 120960.0f), th2, -1.0f / 2520.0f), th2, 1.0f / 120.0f);
    } else {
        const float th = sqrtf(th2);
        float sn, cs;
        sincosf(th, &sn, &cs);
        const float th4 = th2 * th2;
        c1 = (th - sn) / (th2 * th);
        c2 = (th2 + 2.0f * cs - 2.0f) / (2.0f * th4);
        c3 = (2.0f * th - 3.0f * sn + th * cs) / (2.0f * th4 * th);
    }
    // Q(rho, om) x = 1/2 rho^x + c1 (om^rho^ + rho^om^ + om^rho^om^) x
    //   + c2 (om^om^rho^ + rho^om^om^ - 3 om^rho^om^) x + c3 (om^rho^om^om^ + om^om^rho^om^) x
    const float3 b0 = cross3(rho, vr);
    const float3 a1 = cross3(om, vr);
    const float3 a2 = cross3(om, a1);
    const float3 b1 = cross3(rho, a1);
    const float3 b2 = cross3(rho, a2);
    const float3 wb0 = cross3(om, b0);
    const float3 wb1 = cross3(om, b1);
    const float3 wwb0 = cross3(om, wb0);
    const float3 wb2 = cross3(om, b2);
    const float3 wwb1 = cross3(om, wb1);
    float3 y;
    y.x = 0.5f * b0.x + c1 * (wb0.x + b1.x + wb1.x) + c2 * (wwb0.x + b2.x - 3.0f * wb1.x) + c3 * (wb2.x + wwb1.x);
    y.y = 0.5f * b0.y + c1 * (wb0.y + b1.y + wb1.y) + c2 * (wwb0.y + b2.y - 3.0f * wb1.y) + c3 * (wb2.y + wwb1.y);
    y.z = 0.5f * b0.z + c1 * (wb0.z + b1.z + wb1.z) + c2 * (wwb0.z + b2.z - 3.0f * wb1.z) + c3 * (wb2.z + wwb1.z);
    vw = mt(float3{aw.x - y.x, aw.y - y.y, aw.z - y.z});
}

// phi_i = sum_j v_ij / sum_j k_ij over the list of i, d_ij = log(T_i^-1 T_j),
// v_ij = k_ij psi_j + g_ij with the kernel gradient
//   EXACT = false   g = -2 k W d
//   EXACT = true    g = -2 k J_r^-1(d)^T W d
// and, with TRANSPORT, v_ij carried to T_i's tangent by Ad_{T_i^-1 T_j}:
//   [R v_w; t x (R v_w) + R v_r] with (R, t) = T_i^-1 T_j.
// T_i <- T_i exp(phi_i) (Jacobi: all j at pre-update poses).
template <bool EXACT, bool TRANSPORT>
__global__ __launch_bounds__(256) void k_svgd(SvgdArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    mpdet::quat qi;
    float3 ti;
    load_pose(A.pin, i, qi, ti);
    float num[6] = {0, 0, 0, 0, 0, 0};
    float den = 0.0f;
    for (int a = 0; a < A.K; ++a) {
        const int j = A.nbr[(size_t)a * A.n + i];
        if (j < 0 || j >= A.n) continue;
        const float k = A.kval[(size_t)a * A.n + i];
        mpdet::quat qj;
        float3 tj;
        load_pose(A.pin, j, qj, tj);
        float3 om, rho, tr;
        mpdet::quat qr;
        float beta;
        mpdet::se3_between_ex(qi, ti, qj, tj, om, rho, qr, tr, beta);
        const float4 p0 = A.psi[2 * j], p1 = A.psi[2 * j + 1];
        if (!EXACT && !TRANSPORT) {
            const float k2r = 2.0f * k * A.sr, k2t = 2.0f * k * A.st;
            num[0] += k * p0.x - k2r * om.x;
            num[1] += k * p0.y - k2r * om.y;
            num[2] += k * p0.z - k2r * om.z;
            num[3] += k * p0.w - k2t * rho.x;
            num[4] += k * p1.x - k2t * rho.y;
            num[5] += k * p1.y - k2t * rho.z;
        } else {
            float3 gw = float3{A.sr * om.x, A.sr * om.y, A.sr * om.z};
            float3 gr = float3{A.st * rho.x, A.st * rho.y, A.st * rho.z};
            if (EXACT) jr_inv_t(om, rho, beta, gw, gr, gw, gr);
            const float m2k = -2.0f * k;
            float3 vw = axpy3(m2k, gw, float3{k * p0.x, k * p0.y, k * p0.z});
            float3 vr = axpy3(m2k, gr, float3{k * p0.w, k * p1.x, k * p1.y});
            if (TRANSPORT) {
                const mpdet::mat3 R = mpdet::qmat(qr);
                const float3 rw = float3{R.m[0] * vw.x + R.m[1] * vw.y + R.m[2] * vw.z,
                                         R.m[3] * vw.x + R.m[4] * vw.y + R.m[5] * vw.z,
                                         R.m[6] * vw.x + R.m[7] * vw.y + R.m[8] * vw.z};
                const float3 rr = float3{R.m[0] * vr.x + R.m[1] * vr.y + R.m[2] * vr.z,
                                         R.m[3] * vr.x + R.m[4] * vr.y + R.m[5] * vr.z,
                                         R.m[6] * vr.x + R.m[7] * vr.y + R.m[8] * vr.z};
                const float3 tx = cross3(tr, rw);
                vw = rw;
                vr = float3{tx.x + rr.x, tx.y + rr.y, tx.z + rr.z};
            }
            num[0] += vw.x;
            num[1] += vw.y;
            num[2] += vw.z;
            num[3] += vr.x;
            num[4] += vr.y;
            num[5] += vr.z;
        }
        den += k;
    }
    float phi[6];
    const float inv = den > 0.0f ? 1.0f / den : 0.0f;
    for (int m = 0; m < 6; ++m) phi[m] = num[m] * inv;
    mpdet::quat dq;
    float3 dt;
    se3_exp(phi, dq, dt);
    compose(qi, ti, dq, dt);
    store_pose(A.pout, i, qi, ti);
}

// ------------------------------------------------------------ prediction
struct PredArgs {
    float4* __restrict__ poses;
    int32_t n;
    uint32_t frame;
    uint64_t seed;
    float dq[4], dt[3];
    float L[21];  // lower-triangular Cholesky factor of the noise covariance, row-major packed
    int32_t noise;
    uint32_t purpose;                 // generator purpose of z (prediction, or Gaussian initialisation)
    const StepDyn* __restrict__ dyn;  // captured step: frame, increment and noise from here
};

__global__ __launch_bounds__(256) void k_predict(PredArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    if (A.dyn) {
        if (!A.dyn->do_pred) return;
        A.frame = A.dyn->frame;
        A.noise = A.dyn->noise;
        for (int k = 0; k < 4; ++k) A.dq[k] = A.dyn->dq[k];
        for (int k = 0; k < 3; ++k) A.dt[k] = A.dyn->dt[k];
        for (int k = 0; k < 21; ++k) A.L[k] = A.dyn->L[k];
    }
    mpdet::quat q;
    float3 t;
    load_pose(A.poses, i, q, t);
    compose(q, t, mpdet::quat{A.dq[0], A.dq[1], A.dq[2], A.dq[3]}, make_float3(A.dt[0], A.dt[1], A.dt[2]));
    if (A.noise) {
        float z[6];
        mpdet::gauss6(A.seed, (uint32_t)i, A.frame, 0u, A.purpose, z);
        float d[6];
        int p = 0;
        for (int r = 0; r < 6; ++r) {
            float s = 0.0f;
            for (int c = 0; c <= r; ++c) s += A.L[p++] * z[c];
            d[r] = s;
        }
        mpdet::quat eq;
        float3 et;
        se3_exp(d, eq, et);
        compose(q, t, eq, et);
    }
    store_pose(A.poses, i, q, t);
}

// ------------------------------------------------------------ initialisation
struct InitArgs {
    float4* __restrict__ poses;
    int32_t n;
    uint64_t seed;
    float lo[3], hi[3];
};

__global__ __launch_bounds__(256) void k_init_uniform(InitArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    mpdet::quat q;
    float3 t;
    mpdet::random_pose(A.seed, (uint32_t)i, 0u, 0u, mpdet::PURPOSE_INIT, A.lo, A.hi, q, t);
    store_pose(A.poses, i, q, t);
}

// ------------------------------------------------------------ posterior
// Deterministic two-level reductions: per-block partials, then one block.
constexpr int kRB = 256;

__device__ inline double block_max(double v) {
    __shared__ double sh[kRB];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ inline double block_sum(double v) {
    __shared__ double sh[kRB];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// (value, index) max, ties to the smaller index
__device__ inline void block_argmax(double& v, int& idx) {
    __shared__ double sv[kRB];
    __shared__ int si[kRB];
    sv[threadIdx.x] = v;
    si[threadIdx.x] = idx;
    __syncthreads();
    for (int s = kRB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double a = sv[threadIdx.x], b = sv[threadIdx.x + s];
            const int ia = si[threadIdx.x], ib = si[threadIdx.x + s];
            if (b > a || (b == a && ib < ia)) {
                sv[threadIdx.x] = b;
                si[threadIdx.x] = ib;
            }
        }
        __syncthreads();
    }
    v = sv[0];
    idx = si[0];
    __syncthreads();
}

// stepinfo layout (doubles): 0 max l, 1 sum exp, 2 log evidence, 3 z, 4 map weight,
// 5 n_eff, 6 max loglik, 7 map index (as double)
struct PostArgs {
    const float* __restrict__ prior;
    const float4* __restrict__ psi;
    double* __restrict__ l;
    float* __restrict__ p0;
    float* __restrict__ p1;
    const int32_t* __restrict__ nbr;
    const float* __restrict__ kval;
    double* __restrict__ part;      // 4 x nblocks partials
    int* __restrict__ ipart;        // nblocks
    double* __restrict__ info;
    float* __restrict__ prior_out;
    int32_t n, K, nb;
    double inv_tau, floor_p;
};

__global__ __launch_bounds__(kRB) void k_post_logits(PostArgs A) {
    const int i = blockIdx.x * kRB + threadIdx.x;
    double l = -INFINITY, ll = -INFINITY;
    if (i < A.n) {
        const double pr = fmax((double)A.prior[i], A.floor_p);
        ll = (double)A.psi[2 * i + 1].z;
        l = log(pr) + ll * A.inv_tau;
        A.l[i] = l;
    }
    const double m = block_max(l);
    const double mll = block_max(ll);
    if (threadIdx.x == 0) {
        A.part[blockIdx.x] = m;
        A.part[A.nb + blockIdx.x] = mll;
    }
}

__global__ __launch_bounds__(kRB) void k_post_max_final(PostArgs A) {
    double m = -INFINITY, mll = -INFINITY;
    for (int b = threadIdx.x; b < A.nb; b += kRB) {
        m = fmax(m, A.part[b]);
        mll = fmax(mll, A.part[A.nb + b]);
    }
    m = block_max(m);
    mll = block_max(mll);
    if (threadIdx.x == 0) {
        A.info[0] = m;
        A.info[6] = mll;
    }
}

__global__ __launch_bounds__(kRB) void k_post_expsum(PostArgs A) {
    const int i = blockIdx.x * kRB + threadIdx.x;
    const double m = A.info[0];
    const double e = (i < A.n) ? exp(A.l[i] - m) : 0.0;
    const double s = block_sum(e);
    if (threadIdx.x == 0) A.part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRB) void k_post_sum_final(PostArgs A) {
    double s = 0.0;
    for (int b = threadIdx.x; b < A.nb; b += kRB) s += A.part[b];
    s = block_sum(s);
    if (threadIdx.x == 0) {
        A.info[1] = s;
        A.info[2] = A.info[0] + log(s);
    }
}

__global__ __launch_bounds__(kRB) void k_post_normalise(PostArgs A) {
    const int i = blockIdx.x * kRB + threadIdx.x;
    if (i >= A.n) return;
    A.p0[i] = (float)exp(A.l[i] - A.info[2]);
}

// one Jacobi round of Eq. 11: p'_i = sum_j k_ij p_j / sum_j k_ij
__global__ __launch_bounds__(kRB) void k_post_round(const float* __restrict__ pin, float* __restrict__ pout,
                                                    const int32_t* __restrict__ nbr, const float* __restrict__ kval,
                                                    int n, int K) {
    const int i = blockIdx.x * kRB + threadIdx.x;
    if (i >= n) return;
    float num = 0.0f, den = 0.0f;
    for (int a = 0; a < K; ++a) {
        const int j = nbr[(size_t)a * n + i];
        if (j < 0 || j >= n) continue;
        const float k = kval[(size_t)a * n + i];
        num += k * pin[j];
        den += k;
    }
    pout[i] = den > 0.0f ? num / den : pin[i];
}

__global__ __launch_bounds__(kRB) void k_post_z(PostArgs A, const float* __restrict__ p) {
    const int i = blockIdx.x * kRB + threadIdx.x;
    double v = -INFINITY;
    int idx = 0x7FFFFFFF;
    double s = 0.0;
    if (i < A.n) {
        v = (double)p[i];
        idx = i;
        s = v;
    }
    s = block_sum(s);
    block_argmax(v, idx);
    if (threadIdx.x == 0) {
        A.part[blockIdx.x] = s;
        A.part[A.nb + blockIdx.x] = v;
        A.ipart[blockIdx.x] = idx;
    }
}

__global__ __launch_bounds__(kRB) void k_post_z_final(PostArgs A) {
    double s = 0.0, v = -INFINITY;
    int idx = 0x7FFFFFFF;
    for (int b = threadIdx.x; b < A.nb; b += kRB) {
        s += A.part[b];
        const double vb = A.part[A.nb + b];
        const int ib = A.ipart[b];
        if (vb > v || (vb == v && ib < idx)) {
            v = vb;
            idx = ib;
        }
    }
    s = block_sum(s);
    block_argmax(v, idx);
    if (threadIdx.x == 0) {
        A.info[3] = s;
        A.info[4] = v / s;
        A.info[7] = (double)idx;
    }
}

__global__ __launch_bounds__(kRB) void k_post_store(PostArgs A, const float* __restrict__ p) {
    const int i = blockIdx.x * kRB + threadIdx.x;
    double q = 0.0;
    if (i < A.n) {
        q = (double)p[i] / A.info[3];
        A.prior_out[i] = (float)q;
    }
    const double s = block_sum(q * q);
    if (threadIdx.x == 0) A.part[2 * A.nb + blockIdx.x] = s;
}

__global__ __launch_bounds__(kRB) void k_post_neff_final(PostArgs A) {
    double s = 0.0;
    for (int b = threadIdx.x; b < A.nb; b += kRB) s += A.part[2 * A.nb + b];
    s = block_sum(s);
    if (threadIdx.x == 0) A.info[5] = 1.0 / s;
}

}  // namespace

void mp_launch_svgd(mp_filter f, hipStream_t s) {
    SvgdArgs A;
    A.pin = f->poses[f->cur].as<float4>();
    A.pout = f->poses[1 - f->cur].as<float4>();
    A.psi = f->psi.as<float4>();
    A.nbr = f->nbr.as<int32_t>();
    A.kval = f->kval.as<float>();
    A.n = f->n;
    A.K = f->K;
    A.sr = f->p.sigma_r;
    A.st = f->p.sigma_t;
    const bool exact = f->p.svgd_grad == MP_SVGD_GRAD_EXACT;
    const bool transport = f->p.svgd_transport == MP_SVGD_TRANSPORT_ADJOINT;
    if (exact && transport) k_svgd<true, true><<<nblk(f->n), 256, 0, s>>>(A);
    else if (exact) k_svgd<true, false><<<nblk(f->n), 256, 0, s>>>(A);
    else if (transport) k_svgd<false, true><<<nblk(f->n), 256, 0, s>>>(A);
    else k_svgd<false, false><<<nblk(f->n), 256, 0, s>>>(A);
    MP_CHECK_LAUNCH();
    f->cur = 1 - f->cur;
}

void mp_launch_predict(mp_filter f, const float dT[7], const float L[36], bool noise, hipStream_t s,
                       bool gauss_init) {
    PredArgs A;
    A.purpose = gauss_init ? mpdet::PURPOSE_INIT_GAUSS : mpdet::PURPOSE_PRED;
    A.poses = f->poses[f->cur].as<float4>();
    A.n = f->n;
    A.frame = (uint32_t)f->frame;
    A.seed = f->p.seed;
    for (int k = 0; k < 4; ++k) A.dq[k] = dT[k];
    for (int k = 0; k < 3; ++k) A.dt[k] = dT[4 + k];
    int p = 0;
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c <= r; ++c) A.L[p++] = noise ? L[6 * r + c] : 0.0f;
    A.noise = noise ? 1 : 0;
    A.dyn = f->dyn;
    k_predict<<<nblk(f->n), 256, 0, s>>>(A);
    MP_CHECK_LAUNCH();
}

void mp_launch_init_uniform(mp_filter f, const float lo[3], const float hi[3], hipStream_t s) {
    InitArgs A;
    A.poses = f->poses[f->cur].as<float4>();
    A.n = f->n;
    A.seed = f->p.seed;
    for (int a = 0; a < 3; ++a) {
        A.lo[a] = lo[a];
        A.hi[a] = hi[a];
    }
    k_init_uniform<<<nblk(f->n), 256, 0, s>>>(A);
    MP_CHECK_LAUNCH();
}

size_t mp_post_scratch_bytes(mp_filter f) {
    // l (n doubles), partials (3 nb doubles), index partials (nb ints)
    const int nb = (int)nblk(f->n, kRB);
    return sizeof(double) * ((size_t)f->n + 3 * (size_t)nb) + sizeof(int) * (size_t)nb + 64;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void mp_fill_u32(void* p, uint32_t v, size_t n, hipStream_t s) {
    if (n == 0) return;
    k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(static_cast<uint32_t*>(p), v, n);
    MP_CHECK_LAUNCH();
}

__global__ void k_copy_f4(const float4* __restrict__ src, float4* __restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

void mp_copy_poses(mp_filter f, int from, int to, hipStream_t s) {
    const size_t n = 2 * (size_t)f->n;
    k_copy_f4<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(f->poses[from].as<float4>(), f->poses[to].as<float4>(), n);
    MP_CHECK_LAUNCH();
}

void mp_launch_posterior(mp_filter f, hipStream_t s) {
    const int n = f->n;
    const int nb = (int)nblk(n, kRB);
    f->red.ensure(mp_post_scratch_bytes(f));
    PostArgs A;
    A.prior = f->prior.as<float>();
    A.psi = f->psi.as<float4>();
    A.l = f->red.as<double>();
    A.part = A.l + n;
    A.ipart = reinterpret_cast<int*>(A.part + 3 * (size_t)nb);
    A.p0 = f->post0.as<float>();
    A.p1 = f->post1.as<float>();
    A.nbr = f->nbr.as<int32_t>();
    A.kval = f->kval.as<float>();
    A.info = f->stepinfo.as<double>();
    A.prior_out = f->prior.as<float>();
    A.n = n;
    A.K = f->K;
    A.nb = nb;
    A.inv_tau = 1.0 / (double)f->p.temperature;
    A.floor_p = (double)f->p.prior_floor;
    k_post_logits<<<nb, kRB, 0, s>>>(A);
    k_post_max_final<<<1, kRB, 0, s>>>(A);
    k_post_expsum<<<nb, kRB, 0, s>>>(A);
    k_post_sum_final<<<1, kRB, 0, s>>>(A);
    k_post_normalise<<<nb, kRB, 0, s>>>(A);
    MP_CHECK_LAUNCH();
    float* a = A.p0;
    float* b = A.p1;
    for (int r = 0; r < f->p.post_iters; ++r) {
        k_post_round<<<nb, kRB, 0, s>>>(a, b, A.nbr, A.kval, n, f->K);
        float* t = a;
        a = b;
        b = t;
    }
    MP_CHECK_LAUNCH();
    k_post_z<<<nb, kRB, 0, s>>>(A, a);
    k_post_z_final<<<1, kRB, 0, s>>>(A);
    k_post_store<<<nb, kRB, 0, s>>>(A, a);
    k_post_neff_final<<<1, kRB, 0, s>>>(A);
    MP_CHECK_LAUNCH();
}
