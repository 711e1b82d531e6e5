// neighbors.hip -- LSH bucketing and the iterative neighbour-list refresh
// (Eq. 9-10 and Alg. 1, IterativeNeighborParticleSearch).
//
//   k_lsh        per particle: zeta = alpha W^K x_i + delta_i with the tangent
//                x_i = [log(R_L^T R_i); R_L^T (t_i - t_L)] (decoupled) or
//                log(T_LSH^-1 T_i) (coupled SE(3) logarithm),
//                cell = floor(zeta) (deterministic FP32), code =
//                hash6(cell) & (2^bits - 1).  T^LSH is drawn from Philox for
//                (frame, iteration); every lane derives it, lane 0 records it.
//   sort         stable radix sort of (code, index)  -> buckets as runs
//   k_bucket_bounds  bucket head/end per sorted position (search of the runs)
//   k_refresh    one lane per particle (its sorted position from a rank
//                array): candidates = previous list U
//                window of up to C bucket-mates after the particle (cyclic in
//                its bucket); each ranked by q_ij = d^T W^K d (deterministic
//                FP32), the K-1 smallest (q, j) kept behind the particle itself
//                in a register-resident insertion network; k_ij = exp(-q_ij)
//                cached for the SVGD update and the posterior propagation.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mp_det.hpp"
#include "mp_internal.hpp"

namespace {

struct LshArgs {
    const float4* __restrict__ poses;
    uint32_t* __restrict__ codes;     // particle order
    uint32_t* __restrict__ keys;      // the bucket sort's input keys (a copy of codes)
    int32_t* __restrict__ idx;        // the bucket sort's input values (0..n-1)
    float* __restrict__ tlsh;
    int32_t n;
    uint32_t mask, frame, it;
    float ar, at, sl;
    int32_t coupled;                  // tangent: 0 decoupled, 1 coupled SE(3) log
    float lo[3], hi[3];
    uint64_t seed;
    const StepDyn* __restrict__ dyn;   // captured step: frame from here
};

__global__ __launch_bounds__(256) void k_lsh(LshArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (A.dyn) A.frame = A.dyn->frame;
    // T^LSH is the same for every particle: one lane of the workgroup draws it
    __shared__ float sL[8];
    if (threadIdx.x == 0) {
        mpdet::quat q0;
        float3 t0;
        mpdet::random_pose(A.seed, 0u, A.frame, A.it, mpdet::PURPOSE_TLSH, A.lo, A.hi, q0, t0);
        sL[0] = q0.w; sL[1] = q0.x; sL[2] = q0.y; sL[3] = q0.z;
        sL[4] = t0.x; sL[5] = t0.y; sL[6] = t0.z; sL[7] = 0.0f;
        if (blockIdx.x == 0)
            for (int k = 0; k < 8; ++k) A.tlsh[k] = sL[k];
    }
    __syncthreads();
    const mpdet::quat qL{sL[0], sL[1], sL[2], sL[3]};
    const float3 tL = make_float3(sL[4], sL[5], sL[6]);
    if (i >= A.n) return;
    const float4 q4 = A.poses[2 * i], t4 = A.poses[2 * i + 1];
    const mpdet::quat qi{q4.x, q4.y, q4.z, q4.w};
    float3 om, u;
    if (A.coupled) {
        mpdet::se3_between(qL, tL, qi, make_float3(t4.x, t4.y, t4.z), om, u);
    } else {
        const mpdet::quat qr = mpdet::qmul(mpdet::qconj(qL), qi);
        float w, sc;
        om = mpdet::qlog(qr, w, sc);
        const mpdet::mat3 RL = mpdet::qmat(qL);
        u = mpdet::rot_t(RL, make_float3(t4.x - tL.x, t4.y - tL.y, t4.z - tL.z));
    }
    float z[6];
    mpdet::gauss6(A.seed, (uint32_t)i, A.frame, A.it, mpdet::PURPOSE_LSH, z);
    int32_t c[6];
    c[0] = mpdet::floor_i32(A.ar * om.x + A.sl * z[0]);
    c[1] = mpdet::floor_i32(A.ar * om.y + A.sl * z[1]);
    c[2] = mpdet::floor_i32(A.ar * om.z + A.sl * z[2]);
    c[3] = mpdet::floor_i32(A.at * u.x + A.sl * z[3]);
    c[4] = mpdet::floor_i32(A.at * u.y + A.sl * z[4]);
    c[5] = mpdet::floor_i32(A.at * u.z + A.sl * z[5]);
    const uint32_t code = mpdet::hash6(c) & A.mask;
    A.codes[i] = code;
    A.keys[i] = code;
    A.idx[i] = i;
}

// Bucket head and end of every sorted position: the run of equal codes around
// s, found by an exponential then binary search on each side (a bucket of m
// particles costs about 2 log2(m) reads per position).
__global__ void k_bucket_bounds(const uint32_t* __restrict__ sc, int n, int32_t* __restrict__ head,
                                int32_t* __restrict__ end) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t c = sc[s];
    // left: lo is known to hold c, the first position holding c is in (lo - step, lo]
    int lo = s, step = 1;
    while (lo - step >= 0 && sc[lo - step] == c) {
        lo -= step;
        step <<= 1;
    }
    int a = max(lo - step, -1), b = lo;   // sc[a] != c (or a = -1), sc[b] == c
    while (b - a > 1) {
        const int mid = a + (b - a) / 2;
        if (sc[mid] == c) b = mid;
        else a = mid;
    }
    head[s] = b;
    // right: the last position holding c is in [hi, hi + step)
    int hi = s;
    step = 1;
    while (hi + step < n && sc[hi + step] == c) {
        hi += step;
        step <<= 1;
    }
    a = hi;
    b = min(hi + step, n);   // sc[a] == c, sc[b] != c (or b = n)
    while (b - a > 1) {
        const int mid = a + (b - a) / 2;
        if (sc[mid] == c) a = mid;
        else b = mid;
    }
    end[s] = b;
}

struct RefreshArgs {
    const float4* __restrict__ poses;
    const int32_t* __restrict__ sorted;
    const int32_t* __restrict__ rank;   // sorted position of each particle
    const int32_t* __restrict__ head;
    const int32_t* __restrict__ end;
    int32_t* __restrict__ nbr;    // K x N
    float* __restrict__ kval;     // K x N
    int32_t* __restrict__ cnt;    // N
    int32_t n, K, C;
    float sr, st;
};

template <int KM>
struct TopK {
    float q[KM];
    int32_t j[KM];
    __device__ void init() {
#pragma unroll
        for (int m = 0; m < KM; ++m) {
            q[m] = __builtin_inff();
            j[m] = 0x7FFFFFFF;
        }
    }
    __device__ bool has(int32_t x) const {
        bool h = false;
#pragma unroll
        for (int m = 0; m < KM; ++m) h |= (j[m] == x);
        return h;
    }
    // keep the KM smallest (q, j) in ascending order
    __device__ void insert(float qv, int32_t jv) {
#pragma unroll
        for (int m = KM - 1; m >= 1; --m) {
            const bool lt_prev = (qv < q[m - 1]) || (qv == q[m - 1] && jv < j[m - 1]);
            const bool lt_cur = (qv < q[m]) || (qv == q[m] && jv < j[m]);
            const float nq = lt_prev ? q[m - 1] : (lt_cur ? qv : q[m]);
            const int32_t nj = lt_prev ? j[m - 1] : (lt_cur ? jv : j[m]);
            q[m] = nq;
            j[m] = nj;
        }
        const bool lt0 = (qv < q[0]) || (qv == q[0] && jv < j[0]);
        if (lt0) {
            q[0] = qv;
            j[0] = jv;
        }
    }
};

// rank[sorted[s]] = s
__global__ void k_rank(const int32_t* __restrict__ sorted, int n, int32_t* __restrict__ rank) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = sorted[s];
    if (i >= 0 && i < n) rank[i] = s;
}

// One lane per particle, in particle order, so that the particle's pose, its
// old list and its new list and kernel values are read and written coalesced;
// its sorted position (rank) locates its bucket window.
template <int KM>
__global__ __launch_bounds__(256) void k_refresh(RefreshArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int s = A.rank[i];
    if (s < 0 || s >= A.n || A.sorted[s] != i) return;
    const float4 qi4 = A.poses[2 * i], ti4 = A.poses[2 * i + 1];
    const mpdet::quat qi{qi4.x, qi4.y, qi4.z, qi4.w};
    const float3 ti = make_float3(ti4.x, ti4.y, ti4.z);
    TopK<KM> tk;
    tk.init();
    auto consider = [&](int32_t j) {
        if (j < 0 || j >= A.n || j == i || tk.has(j)) return;
        const float4 qj4 = A.poses[2 * j], tj4 = A.poses[2 * j + 1];
        const float qv = mpdet::qdist(qi, ti, mpdet::quat{qj4.x, qj4.y, qj4.z, qj4.w},
                                      make_float3(tj4.x, tj4.y, tj4.z), A.sr, A.st);
        tk.insert(qv, j);
    };
    // bucket window (Alg. 1 gather loop, capped at C mates)
    int h = A.head[s], e = A.end[s];
    if (!(h >= 0 && h <= s && s < e && e <= A.n)) {
        h = s;
        e = s + 1;
    }
    const int m = e - h;
    const int w = min(m - 1, A.C);
    for (int d = 1; d <= w; ++d) {
        int pos = s + d;
        if (pos >= e) pos -= m;
        consider(A.sorted[pos]);
    }
    // previous list (persists across iterations)
    for (int a = 1; a < A.K; ++a) consider(A.nbr[(size_t)a * A.n + i]);
    // write: the particle itself first, then the K-1 nearest others
    A.nbr[i] = i;
    A.kval[i] = 1.0f;
    int c = 1;
#pragma unroll
    for (int a = 0; a < KM; ++a) {
        if (a + 1 < A.K) {
            const bool ok = tk.j[a] != 0x7FFFFFFF;
            A.nbr[(size_t)(a + 1) * A.n + i] = ok ? tk.j[a] : -1;
            A.kval[(size_t)(a + 1) * A.n + i] = ok ? expf(-tk.q[a]) : 0.0f;
            c += ok ? 1 : 0;
        }
    }
    A.cnt[i] = c;
}

__global__ void k_reset_lists(int32_t* __restrict__ nbr, float* __restrict__ kval, int32_t* __restrict__ cnt,
                              float* __restrict__ prior, int32_t* __restrict__ sorted, int32_t* __restrict__ head,
                              int32_t* __restrict__ end, int n, int K) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // identity order, one particle per bucket, until the first LSH pass
    sorted[i] = i;
    head[i] = i;
    end[i] = i + 1;
    nbr[i] = i;
    kval[i] = 1.0f;
    for (int a = 1; a < K; ++a) {
        nbr[(size_t)a * n + i] = -1;
        kval[(size_t)a * n + i] = 0.0f;
    }
    cnt[i] = 1;
    prior[i] = 1.0f / (float)n;
}

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void mp_launch_lsh(mp_filter f, uint32_t frame, uint32_t it, hipStream_t s) {
    LshArgs A;
    A.poses = f->poses[f->cur].as<float4>();
    A.codes = f->codes.as<uint32_t>();
    // the sort ping-pongs between (tmp_keys, tmp_vals) and (scodes, sorted);
    // start it on the side that makes its last pass land in (scodes, sorted)
    const bool odd = mp_radix_passes(f->n, f->p.lsh_bits) % 2 == 1;
    A.keys = odd ? f->tmp_keys.as<uint32_t>() : f->scodes.as<uint32_t>();
    A.idx = odd ? f->tmp_vals.as<int32_t>() : f->sorted.as<int32_t>();
    A.tlsh = f->tlsh.as<float>();
    A.n = f->n;
    A.mask = f->p.lsh_bits >= 32 ? 0xFFFFFFFFu : ((1u << f->p.lsh_bits) - 1u);
    A.frame = frame;
    A.it = it;
    A.ar = f->p.lsh_alpha * f->p.sigma_r;
    A.at = f->p.lsh_alpha * f->p.sigma_t;
    A.sl = f->p.lsh_sigma;
    A.coupled = f->p.lsh_tangent == MP_LSH_TANGENT_SE3 ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        A.lo[a] = f->lsh_lo[a];
        A.hi[a] = f->lsh_hi[a];
    }
    A.seed = f->p.seed;
    A.dyn = f->dyn;
    k_lsh<<<nblk(f->n), 256, 0, s>>>(A);
    MP_CHECK_LAUNCH();
}

void mp_launch_sort(mp_filter f, hipStream_t s) {
    const int n = f->n;
    // stable sort of (code, index) from the buffers the LSH kernel filled;
    // the result lands in (scodes, sorted) with no copy
    const bool odd = mp_radix_passes(n, f->p.lsh_bits) % 2 == 1;
    if (odd)
        mp_radix_sort_u32_inplace_parity(f->tmp_keys.as<uint32_t>(), f->tmp_vals.as<int32_t>(),
                                         f->scodes.as<uint32_t>(), f->sorted.as<int32_t>(), n, f->p.lsh_bits, f->hist,
                                         s);
    else
        mp_radix_sort_u32_inplace_parity(f->scodes.as<uint32_t>(), f->sorted.as<int32_t>(), f->tmp_keys.as<uint32_t>(),
                                         f->tmp_vals.as<int32_t>(), n, f->p.lsh_bits, f->hist, s);
    k_bucket_bounds<<<nblk(n), 256, 0, s>>>(f->scodes.as<uint32_t>(), n, f->head.as<int32_t>(), f->end.as<int32_t>());
    MP_CHECK_LAUNCH();
}

void mp_launch_refresh(mp_filter f, hipStream_t s, int window) {
    k_rank<<<nblk(f->n), 256, 0, s>>>(f->sorted.as<int32_t>(), f->n, f->rank.as<int32_t>());
    MP_CHECK_LAUNCH();
    RefreshArgs A;
    A.poses = f->poses[f->cur].as<float4>();
    A.sorted = f->sorted.as<int32_t>();
    A.rank = f->rank.as<int32_t>();
    A.head = f->head.as<int32_t>();
    A.end = f->end.as<int32_t>();
    A.nbr = f->nbr.as<int32_t>();
    A.kval = f->kval.as<float>();
    A.cnt = f->cnt.as<int32_t>();
    A.n = f->n;
    A.K = f->K;
    A.C = window < 0 ? f->p.window_c : window;
    A.sr = f->p.sigma_r;
    A.st = f->p.sigma_t;
    if (f->K <= 8) k_refresh<8><<<nblk(f->n), 256, 0, s>>>(A);
    else if (f->K <= 16) k_refresh<16><<<nblk(f->n), 256, 0, s>>>(A);
    else k_refresh<32><<<nblk(f->n), 256, 0, s>>>(A);
    MP_CHECK_LAUNCH();
}

void mp_launch_reset_lists(mp_filter f, hipStream_t s) {
    k_reset_lists<<<nblk(f->n), 256, 0, s>>>(f->nbr.as<int32_t>(), f->kval.as<float>(), f->cnt.as<int32_t>(),
                                               f->prior.as<float>(), f->sorted.as<int32_t>(), f->head.as<int32_t>(),
                                               f->end.as<int32_t>(), f->n, f->K);
    MP_CHECK_LAUNCH();
}
