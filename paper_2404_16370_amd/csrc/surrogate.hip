// surrogate.hip -- learned surrogate of the per-point score, its training
// step, and the scorer that evaluates it inside the likelihood.
//
// Target (residual field): with e = mu_g - p for the NNF Gaussian g of p and
// an inlier (|e| <= d_max), s(p) = e^T (Sigma^M_g + sigma_s^2 I)^-1 e
// untruncated, r = sqrt(s), grad r = -Omega e / max(r, 1e-2); outside the
// gate r = r_out = d_max / sqrt(eps + sigma_s^2) and grad r = 0.
// Sigma^M = I - a n n^T, so with beta = 1 + sigma_s^2 and lam_n = 1 - a|n|^2
// (kept per Gaussian in the normal record):
//   Omega = I / beta + kappa n n^T,  kappa = a / (beta (lam_n + sigma_s^2)).
//
// Network: x = (p - lo) * inv_ext; features sin / cos(2 pi frac(f_l x_a)),
// 32 geometric frequencies per axis, ordered (axis, frequency, sin|cos);
// 192 -> 128 -> 128 -> 4 with SiLU; outputs (r / r_scale, grad r / g_scale).
// Products run on the matrix cores (v_mfma_f32_32x32x16_bf16: bfloat16
// operands, FP32 accumulation); FP32 master weights, Adam in FP32.
//
// Inference keeps all weights of one workgroup in LDS (an image of about
// 82 KB laid out as MFMA operand fragments) and works in the transposed
// form Z^T = W^T X^T: a wave evaluates 64 points at once, hidden units run
// along the MFMA rows, points along its columns, so the accumulators of one
// layer are already the next layer's B operand (after SiLU and conversion)
// with no data exchange between lanes.  The K ordering of layers 2 and 3 is
// permuted to match the accumulator layout; the weight fragments are stored
// in the same permuted order.
//
// Training: one launch evaluates the gradient of the whole batch.  Each
// workgroup (4 waves) takes 32-sample tiles; wave w owns the 32-unit block w
// of both hidden layers, so its weight fragments stay in registers, the
// activations of a tile pass through LDS (sample-major rows for the next
// layer's operands, unit-major rows for the products over samples), and the
// weight gradients accumulate in each wave's accumulation registers over the
// workgroup's tiles.  One partial gradient per workgroup is written; the Adam
// kernel adds the partials in a fixed order, so a step is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "mp_det.hpp"
#include "mp_internal.hpp"
#include "mp_lookup.hpp"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kD0 = 192, kD1 = 128, kD2 = 128;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kD0 * kD1, kOffW2 = kOffB1 + kD1, kOffB2 = kOffW2 + kD1 * kD2,
              kOffW3 = kOffB2 + kD2, kOffB3 = kOffW3 + kD2 * 4, kNParams = kOffB3 + 4;
static_assert(kNParams == MP_SUR_NPARAMS, "parameter count");

// inference image, byte offsets
constexpr int kImgF1 = 0;                          // [4 row tiles][12 k-steps][64 lanes][8] bf16
constexpr int kImgF2 = kImgF1 + 4 * 12 * 64 * 16;  // [4 row tiles][8 k-steps][64 lanes][8] bf16
constexpr int kImgF3 = kImgF2 + 4 * 8 * 64 * 16;   // [8 k-steps][4 outputs][2 lane halves][8] bf16
constexpr int kImgB1 = kImgF3 + 8 * 4 * 2 * 16;    // 128 f32
constexpr int kImgB2 = kImgB1 + 512;               // 128 f32
constexpr int kImgB3 = kImgB2 + 512;               // 4 f32
constexpr int kImgFQ = kImgB3 + 16;                // 32 f32 frequencies
constexpr int kImgBytes = kImgFQ + 128;
static_assert(kImgBytes == MP_SUR_IMAGE_BYTES, "image size");
constexpr int kImg2Bytes = 4 * 8 * 64 * 16;        // [4 row tiles][8 k-steps][64 lanes][8] bf16
static_assert(kImgBytes % 16 == 0, "image in uint4 units");

constexpr int kBatchPad = 512;  // the batch is padded to a multiple of this many rows (zero rows)

__device__ __forceinline__ f32x16 mfma32(const bf16x8 a, const bf16x8 b, const f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float sigmoid_f(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.44269504088896341f * z));
}
__device__ __forceinline__ float silu_f(float z) { return z * sigmoid_f(z); }
__device__ __forceinline__ float silu_grad_f(float z) {
    const float s = sigmoid_f(z);
    return s * __builtin_fmaf(z, 1.0f - s, 1.0f);
}

// sin and cos of 2 pi frac(f x): v_sin / v_cos take revolutions
__device__ __forceinline__ void feature_pair(float f, float x, __bf16& s, __bf16& c) {
    const float u = __builtin_amdgcn_fractf(f * x);
    s = (__bf16)__builtin_amdgcn_sinf(u);
    c = (__bf16)__builtin_amdgcn_cosf(u);
}

// ------------------------------------------------------------ fragment layouts
// Layer-1 A operand (W1^T, rows = hidden o, k = feature f): element (o, f) of
// row tile o/32 and k-step f/16 sits at lane (o%32) + 32 ((f%16)/8), slot f%8.
__host__ __device__ inline int frag1_index(int f, int o) {
    const int r = o >> 5, m = o & 31, s = f >> 4, kk = f & 15;
    return ((r * 12 + s) * 64 + m + 32 * (kk >> 3)) * 8 + (kk & 7);
}
// Hidden unit i of a layer-1/2 accumulator tile: lane half h, register jj of
// row tile r hold unit 32 r + 8 (jj/4) + 4 h + jj%4.  As the next layer's B
// operand, k-step s2 takes registers 8 (s2%2) .. +7 of row tile s2/2, so
// slot j of lane half h at k-step s2 is unit 32 (s2/2) + 16 (s2%2) + 8 (j/4) + 4 h + j%4.
__host__ __device__ inline void hid_slot(int i, int& s2, int& h, int& j) {
    s2 = 2 * (i >> 5) + ((i >> 4) & 1);
    h = (i >> 2) & 1;
    j = 4 * ((i >> 3) & 1) + (i & 3);
}
__host__ __device__ inline int frag2_index(int i, int o) {  // W2[i][o]
    int s2, h, j;
    hid_slot(i, s2, h, j);
    return (((o >> 5) * 8 + s2) * 64 + (o & 31) + 32 * h) * 8 + j;
}
// W2[i][o] as the A operand of the input gradient dH1 = W2 dZ2 (rows = layer-1
// units i, k = layer-2 units o in the accumulator order of layer 2)
__host__ __device__ inline int frag2b_index(int i, int o) {
    int s2, h, j;
    hid_slot(o, s2, h, j);
    return (((i >> 5) * 8 + s2) * 64 + (i & 31) + 32 * h) * 8 + j;
}
// the hidden unit of register jj of accumulator row tile r in lane half h
__host__ __device__ inline int acc_unit(int r, int jj, int h) { return 32 * r + 8 * (jj >> 2) + 4 * h + (jj & 3); }
__host__ __device__ inline int frag3_index(int i, int o) {  // W3[i][o]
    int s2, h, j;
    hid_slot(i, s2, h, j);
    return ((s2 * 4 + o) * 2 + h) * 8 + j;
}

// ------------------------------------------------------------ network on 32 points
// One tile of 32 points per call (accumulators and activations of one tile
// only, so that two waves share each SIMD).  Lane L supplies the normalised
// coordinates x of point L%32 of tile tt; the output layer writes the tile's
// 4 outputs into accumulator rows 4 tt .. 4 tt + 3, which lane half tt holds:
// on return the lanes L with L/32 == tt hold the outputs of point L%32 (the
// other half's y is left as it was).  img points at the inference image (LDS).
__device__ __forceinline__ void mlp32(const char* __restrict__ img, const float x[3], const int tt, float y[4]) {
    const int lane = threadIdx.x & 63, m = lane & 31, h = lane >> 5;
    const bf16x8* f1 = reinterpret_cast<const bf16x8*>(img + kImgF1);
    const bf16x8* f2 = reinterpret_cast<const bf16x8*>(img + kImgF2);
    const bf16x8* f3 = reinterpret_cast<const bf16x8*>(img + kImgF3);
    const float* b1 = reinterpret_cast<const float*>(img + kImgB1);
    const float* b2 = reinterpret_cast<const float*>(img + kImgB2);
    const float* b3 = reinterpret_cast<const float*>(img + kImgB3);
    const float* fq = reinterpret_cast<const float*>(img + kImgFQ);

    f32x16 acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 bb = *reinterpret_cast<const float4*>(b1 + 32 * r + 8 * q + 4 * h);
            acc[r][4 * q] = bb.x;
            acc[r][4 * q + 1] = bb.y;
            acc[r][4 * q + 2] = bb.z;
            acc[r][4 * q + 3] = bb.w;
        }
    // layer 1: k-step s covers axis s/4, frequencies 8 (s%4) + 4 h + 0..3 (sin, cos each)
#pragma unroll
    for (int s = 0; s < 12; ++s) {
        const float4 fr = *reinterpret_cast<const float4*>(fq + 8 * (s & 3) + 4 * h);
        const float xs = x[s >> 2];
        __bf16 v0, v1, v2, v3, v4, v5, v6, v7;
        feature_pair(fr.x, xs, v0, v1);
        feature_pair(fr.y, xs, v2, v3);
        feature_pair(fr.z, xs, v4, v5);
        feature_pair(fr.w, xs, v6, v7);
        const bf16x8 bx = bf16x8{v0, v1, v2, v3, v4, v5, v6, v7};
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = mfma32(f1[(r * 12 + s) * 64 + lane], bx, acc[r]);
    }
    bf16x8 hb[8];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
        for (int j = 0; j < 8; ++j) hb[s2][j] = (__bf16)silu_f(acc[s2 >> 1][8 * (s2 & 1) + j]);
    // layer 2
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 bb = *reinterpret_cast<const float4*>(b2 + 32 * r + 8 * q + 4 * h);
            acc[r][4 * q] = bb.x;
            acc[r][4 * q + 1] = bb.y;
            acc[r][4 * q + 2] = bb.z;
            acc[r][4 * q + 3] = bb.w;
        }
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = mfma32(f2[(r * 8 + s2) * 64 + lane], hb[s2], acc[r]);
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
        for (int j = 0; j < 8; ++j) hb[s2][j] = (__bf16)silu_f(acc[s2 >> 1][8 * (s2 & 1) + j]);
    // layer 3: outputs in rows 4 tt .. 4 tt + 3 (other A rows zero)
    f32x16 o = {};
    const bf16x8 zero = {};
    const int o3 = m - 4 * tt;
    const bool row = o3 >= 0 && o3 < 4;
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) o = mfma32(row ? f3[(s2 * 4 + o3) * 2 + h] : zero, hb[s2], o);
    if (h == tt) {
        y[0] = o[0] + b3[0];
        y[1] = o[1] + b3[1];
        y[2] = o[2] + b3[2];
        y[3] = o[3] + b3[3];
    }
}

__device__ __forceinline__ void load_image(const uint4* __restrict__ src, uint4* dst) {
    for (int q = threadIdx.x; q < kImgBytes / 16; q += blockDim.x) dst[q] = src[q];
    __syncthreads();
}

// ------------------------------------------------------------ residual field
struct LabelArgs {
    MapView map;
    const float* __restrict__ xyz;
    float4* __restrict__ out;
    int64_t n;
    float sig2, ib, dmax2, r_floor, r_out, inv_r, inv_g;
};

__global__ void k_label(LabelArgs A) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const float px = A.xyz[3 * i], py = A.xyz[3 * i + 1], pz = A.xyz[3 * i + 2];
    const int32_t g = mp_nnf_lookup<0>(A.map, px, py, pz);
    float r = A.r_out, gx = 0.0f, gy = 0.0f, gz = 0.0f;
    if (g >= 0) {
        const float4 gm = A.map.gauss[2 * (int64_t)g];
        const float4 gn = A.map.gauss[2 * (int64_t)g + 1];
        const float ex = gm.x - px, ey = gm.y - py, ez = gm.z - pz;
        const float d2 = __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez));
        if (d2 <= A.dmax2) {
            const float kap = A.map.gicp_a / ((1.0f + A.sig2) * (gn.w + A.sig2));
            const float ne = __builtin_fmaf(gn.x, ex, __builtin_fmaf(gn.y, ey, gn.z * ez));
            const float ee = __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez));
            const float c = __builtin_fmaf(kap * ne, ne, ee * A.ib);
            r = __builtin_sqrtf(c);
            const float id = 1.0f / fmaxf(r, A.r_floor);
            const float kn = kap * ne;
            gx = -id * __builtin_fmaf(kn, gn.x, ex * A.ib);
            gy = -id * __builtin_fmaf(kn, gn.y, ey * A.ib);
            gz = -id * __builtin_fmaf(kn, gn.z, ez * A.ib);
        }
    }
    A.out[i] = make_float4(r * A.inv_r, gx * A.inv_g, gy * A.inv_g, gz * A.inv_g);
}

// ------------------------------------------------------------ weights
__global__ void k_init_weights(float* __restrict__ P, uint64_t seed) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kNParams) return;
    float bound = 0.0f;
    if (q < kOffB1) bound = 0.07216878364870322f;        // 1 / sqrt(192)
    else if (q >= kOffW2 && q < kOffB2) bound = 0.08838834764831845f;  // 1 / sqrt(128)
    else if (q >= kOffW3 && q < kOffB3) bound = 0.08838834764831845f;
    const mpdet::u32x4 r = mpdet::rng(seed, (uint32_t)q, 0u, 0u, mpdet::PURPOSE_WINIT, 0u);
    P[q] = bound * (2.0f * mpdet::unit_co(r.v[0]) - 1.0f);
}

struct PublishArgs {
    __bf16* w3b;  // [128][4]
    char* img;
    __bf16* img2;
};

__device__ __forceinline__ void publish(const PublishArgs& W, int q, float w) {
    const __bf16 wb = (__bf16)w;
    __bf16* f1 = reinterpret_cast<__bf16*>(W.img + kImgF1);
    __bf16* f2 = reinterpret_cast<__bf16*>(W.img + kImgF2);
    __bf16* f3 = reinterpret_cast<__bf16*>(W.img + kImgF3);
    if (q < kOffB1) {
        const int f = q / kD1, o = q % kD1;
        f1[frag1_index(f, o)] = wb;
    } else if (q < kOffW2) {
        reinterpret_cast<float*>(W.img + kImgB1)[q - kOffB1] = w;
    } else if (q < kOffB2) {
        const int i = (q - kOffW2) / kD2, o = (q - kOffW2) % kD2;
        f2[frag2_index(i, o)] = wb;
        W.img2[frag2b_index(i, o)] = wb;
    } else if (q < kOffW3) {
        reinterpret_cast<float*>(W.img + kImgB2)[q - kOffB2] = w;
    } else if (q < kOffB3) {
        const int i = (q - kOffW3) / 4, o = (q - kOffW3) % 4;
        W.w3b[i * 4 + o] = wb;
        f3[frag3_index(i, o)] = wb;
    } else {
        reinterpret_cast<float*>(W.img + kImgB3)[q - kOffB3] = w;
    }
}

__global__ void k_publish(const float* __restrict__ P, PublishArgs W) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kNParams) return;
    publish(W, q, P[q]);
}

// ------------------------------------------------------------ fused training step
// One gradient evaluation of the batch in one launch.  A workgroup of four
// waves takes 32-sample tiles; wave w owns the 32-unit block w of both hidden
// layers, and its fragments of W1^T (rows: layer-1 units of the block), W2^T
// (rows: layer-2 units) and W2 (rows: layer-1 units, for the input gradient)
// stay in registers for the whole launch.  Per tile the activations pass
// through LDS as sample-major rows: features, H1 and dZ2 shared by the four
// waves, H2 and dZ1 of each wave's own block.  The weight gradients are
// products over samples: their operands are read from those rows eight
// samples at a time (slot i of lane half h at k-step kq is sample
// 16 kq + 8 h + i on both sides), and each wave accumulates its share (the
// dW1 columns, dW2 rows and dW3 rows of its block) in accumulation registers
// over the workgroup's tiles.  The workgroup writes one partial gradient and
// its squared error; the Adam kernel adds the partials in a fixed order.
// Rounding points: features, H1, H2, dZ2 and dZ1 in bf16;
// pre-activations, outputs, dY and dH2 in FP32; dY enters the dW3 product as
// a bf16 pair (hi + lo).
constexpr int kFThreads = 256;
constexpr int kXS = kD0 + 8;   // feature row stride (bf16): 400 B
constexpr int kHS = kD1 + 8;   // hidden row stride (bf16): 272 B
constexpr int kTS = 32 + 8;    // transposed row stride (bf16, one unit's 32 samples): 80 B
constexpr int kFPart = kNParams + 1;   // partial gradient + squared error of a workgroup
constexpr int kFPartPad = (kFPart + 3) / 4 * 4;   // partial row stride: 16-byte aligned rows

struct FusedArgs {
    const uint4* __restrict__ img;     // inference image: W1^T, W2^T fragments; b1, b2, b3; frequencies
    const uint4* __restrict__ img2;    // W2 fragments of the input gradient
    const __bf16* __restrict__ w3b;    // [128][4]
    const float* __restrict__ xyz;     // staged batch [bp][3] (draw == 0; zero rows past n_real)
    const float4* __restrict__ tgt;    // staged scaled targets [bp]
    const float* __restrict__ dxyz;    // training set (draw == 1): points
    const float4* __restrict__ dlab;   // scaled labels
    float* __restrict__ part;          // [gridDim.x][kFPartPad]
    int64_t n_data;
    int32_t tiles, n_real, draw, full;
    uint32_t step;
    uint64_t seed;
    float two_over_n;
    float lo[3], inv[3];
};

// Sample b of the batch: the staged row, or drawn from the training set (the
// whole set in order when it fits the batch, else index floor(x n / 2^64) of
// a Philox draw x keyed by the step counter); zero past n_real.
__device__ __forceinline__ void fused_sample(const FusedArgs& A, int b, float4& p, float4& tg) {
    p = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    tg = p;
    if (!A.draw) {
        p = make_float4(A.xyz[3 * b], A.xyz[3 * b + 1], A.xyz[3 * b + 2], 0.0f);
        tg = A.tgt[b];
        return;
    }
    if (b >= A.n_real) return;
    int64_t idx = b;
    if (!A.full) {
        const mpdet::u32x4 r = mpdet::rng(A.seed, (uint32_t)b, A.step, 0u, mpdet::PURPOSE_BATCH, 0u);
        const uint64_t x = ((uint64_t)r.v[1] << 32) | r.v[0];
        idx = (int64_t)__umul64hi(x, (uint64_t)A.n_data);
    }
    p = make_float4(A.dxyz[3 * idx], A.dxyz[3 * idx + 1], A.dxyz[3 * idx + 2], 0.0f);
    tg = A.dlab[idx];
}

__device__ __forceinline__ void store4(__bf16* p, float a, float b, float c, float d) {
    typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
    *reinterpret_cast<bf16x4*>(p) = bf16x4{(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
}

__global__ __launch_bounds__(kFThreads) void k_train_fused(FusedArgs A) {
    __shared__ __attribute__((aligned(16))) __bf16 xs[32 * kXS];    // [sample][feature]
    __shared__ __attribute__((aligned(16))) __bf16 h1s[32 * kHS];   // [sample][unit]
    __shared__ __attribute__((aligned(16))) __bf16 dz2s[32 * kHS];
    __shared__ __attribute__((aligned(16))) __bf16 xT[kD0 * kTS];   // the same, [feature][sample]
    __shared__ __attribute__((aligned(16))) __bf16 h1T[kD1 * kTS];  // [unit][sample]
    __shared__ __attribute__((aligned(16))) __bf16 dz2T[kD2 * kTS];
    __shared__ __attribute__((aligned(16))) __bf16 h2T[kD2 * kTS];
    __shared__ __attribute__((aligned(16))) __bf16 dz1T[kD1 * kTS];
    __shared__ float ys[4][32][4];
    __shared__ float dys[32][4];
    __shared__ float w3s[kD2 * 4];
    __shared__ float bias[kD1 + kD2 + 4];
    __shared__ __attribute__((aligned(16))) float fqs[32];
    __shared__ float4 sxyz[2][32], stgt[2][32];   // the samples of the tile and of the next one
    const char* img = reinterpret_cast<const char*>(A.img);
    for (int q = threadIdx.x; q < kD2 * 4; q += kFThreads) w3s[q] = (float)A.w3b[q];
    for (int q = threadIdx.x; q < kD1; q += kFThreads) {
        bias[q] = reinterpret_cast<const float*>(img + kImgB1)[q];
        bias[kD1 + q] = reinterpret_cast<const float*>(img + kImgB2)[q];
    }
    if (threadIdx.x < 4) bias[kD1 + kD2 + threadIdx.x] = reinterpret_cast<const float*>(img + kImgB3)[threadIdx.x];
    if (threadIdx.x < 32) fqs[threadIdx.x] = reinterpret_cast<const float*>(img + kImgFQ)[threadIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, m = lane & 31, h = lane >> 5;
    // this wave's weight fragments
    const bf16x8* f1 = reinterpret_cast<const bf16x8*>(img + kImgF1);
    const bf16x8* f2 = reinterpret_cast<const bf16x8*>(img + kImgF2);
    const bf16x8* f2b = reinterpret_cast<const bf16x8*>(A.img2);
    bf16x8 a1[12], a2[8], a2b[8];
#pragma unroll
    for (int sk = 0; sk < 12; ++sk) a1[sk] = f1[(w * 12 + sk) * 64 + lane];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
        a2[s2] = f2[(w * 8 + s2) * 64 + lane];
        a2b[s2] = f2b[(w * 8 + s2) * 64 + lane];
    }
    f32x16 g1[6], g2[4], g3;
#pragma unroll
    for (int r = 0; r < 6; ++r) g1[r] = f32x16{};
#pragma unroll
    for (int r = 0; r < 4; ++r) g2[r] = f32x16{};
    g3 = f32x16{};
    float db1 = 0.0f, db2 = 0.0f, sse = 0.0f;
    float db3[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (w == 0 && h == 0 && (int)blockIdx.x < A.tiles) {
        float4 p, tg;
        fused_sample(A, 32 * blockIdx.x + m, p, tg);
        sxyz[0][m] = p;
        stgt[0][m] = tg;
    }
    __syncthreads();
    int it = 0;
    for (int t = blockIdx.x; t < A.tiles; t += gridDim.x, ++it) {
        const int cur = it & 1;
        // the next tile's samples, requested by one half-wave now and stored
        // at the end of this tile (the other buffer's readers finished before
        // the last barrier; the stores are read after this tile's last one)
        const bool fetch = w == 0 && h == 0 && t + (int)gridDim.x < A.tiles;
        float4 nxt_p, nxt_t;
        if (fetch) fused_sample(A, 32 * (t + gridDim.x) + m, nxt_p, nxt_t);
        const int b = 32 * t + m;   // this lane's sample
        const float4 pm = sxyz[cur][m];
        float x[3];
        x[0] = (pm.x - A.lo[0]) * A.inv[0];
        x[1] = (pm.y - A.lo[1]) * A.inv[1];
        x[2] = (pm.z - A.lo[2]) * A.inv[2];
        // features of k-steps 3w .. 3w + 2 (axis sk / 4, frequencies 8 (sk % 4) + 4 h + 0..3)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int sk = 3 * w + q;
            const float4 fr = *reinterpret_cast<const float4*>(fqs + 8 * (sk & 3) + 4 * h);
            const int ax = sk >> 2;
            const float xv = ax == 0 ? x[0] : (ax == 1 ? x[1] : x[2]);
            __bf16 v0, v1, v2, v3, v4, v5, v6, v7;
            feature_pair(fr.x, xv, v0, v1);
            feature_pair(fr.y, xv, v2, v3);
            feature_pair(fr.z, xv, v4, v5);
            feature_pair(fr.w, xv, v6, v7);
            *reinterpret_cast<bf16x8*>(xs + m * kXS + 16 * sk + 8 * h) = bf16x8{v0, v1, v2, v3, v4, v5, v6, v7};
            __bf16* xt = xT + (16 * sk + 8 * h) * kTS + m;
            xt[0] = v0;
            xt[kTS] = v1;
            xt[2 * kTS] = v2;
            xt[3 * kTS] = v3;
            xt[4 * kTS] = v4;
            xt[5 * kTS] = v5;
            xt[6 * kTS] = v6;
            xt[7 * kTS] = v7;
        }
        __syncthreads();
        // layer 1 of the block: Z1 = W1^T x + b1 (kept), H1 to the shared rows
        f32x16 z1;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) z1[jj] = bias[acc_unit(w, jj, h)];
#pragma unroll
        for (int sk = 0; sk < 12; ++sk)
            z1 = mfma32(a1[sk], *reinterpret_cast<const bf16x8*>(xs + m * kXS + 16 * sk + 8 * h), z1);
        float s1[16];   // sigmoid(Z1), kept for silu'
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) s1[jj] = sigmoid_f(z1[jj]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float hv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int jj = 4 * q + i;
                hv[i] = z1[jj] * s1[jj];
                h1T[acc_unit(w, jj, h) * kTS + m] = (__bf16)hv[i];
            }
            store4(h1s + m * kHS + 32 * w + 8 * q + 4 * h, hv[0], hv[1], hv[2], hv[3]);
        }
        __syncthreads();
        // layer 2 of the block: Z2 = W2^T H1 + b2 (kept); H2 of the block; the
        // block's share of the output layer
        f32x16 z2;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) z2[jj] = bias[kD1 + acc_unit(w, jj, h)];
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) {
            const __bf16* r = h1s + m * kHS + 32 * (s2 >> 1) + 16 * (s2 & 1) + 4 * h;
            typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
            const bf16x4 lo4 = *reinterpret_cast<const bf16x4*>(r);
            const bf16x4 hi4 = *reinterpret_cast<const bf16x4*>(r + 8);
            z2 = mfma32(a2[s2], bf16x8{lo4[0], lo4[1], lo4[2], lo4[3], hi4[0], hi4[1], hi4[2], hi4[3]}, z2);
        }
        float s2v[16];   // sigmoid(Z2), kept for silu'
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) s2v[jj] = sigmoid_f(z2[jj]);
        float y0 = 0.0f, y1 = 0.0f, y2 = 0.0f, y3 = 0.0f;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int u = acc_unit(w, jj, h);
            const __bf16 hb = (__bf16)(z2[jj] * s2v[jj]);
            h2T[u * kTS + m] = hb;
            const float hv = (float)hb;
            const float* wv = w3s + 4 * u;
            y0 = __builtin_fmaf(wv[0], hv, y0);
            y1 = __builtin_fmaf(wv[1], hv, y1);
            y2 = __builtin_fmaf(wv[2], hv, y2);
            y3 = __builtin_fmaf(wv[3], hv, y3);
        }
        y0 += __shfl_xor(y0, 32, 64);
        y1 += __shfl_xor(y1, 32, 64);
        y2 += __shfl_xor(y2, 32, 64);
        y3 += __shfl_xor(y3, 32, 64);
        if (h == 0) {
            ys[w][m][0] = y0;
            ys[w][m][1] = y1;
            ys[w][m][2] = y2;
            ys[w][m][3] = y3;
        }
        __syncthreads();
        // loss and dY of the tile's samples (the four blocks' shares added in order)
        float yv[4];
#pragma unroll
        for (int c = 0; c < 4; ++c)
            yv[c] = bias[kD1 + kD2 + c] + (((ys[0][m][c] + ys[1][m][c]) + ys[2][m][c]) + ys[3][m][c]);
        const float4 tg = stgt[cur][m];
        const bool valid = b < A.n_real;
        const float r0 = yv[0] - tg.x, r1 = yv[1] - tg.y, r2 = yv[2] - tg.z, r3 = yv[3] - tg.w;
        const float e = valid ? __builtin_fmaf(r0, r0, __builtin_fmaf(r1, r1, __builtin_fmaf(r2, r2, r3 * r3))) : 0.0f;
        const float kk = valid ? A.two_over_n : 0.0f;
        const float d0 = r0 * kk, d1 = r1 * kk, d2 = r2 * kk, d3 = r3 * kk;
        if (w == 0 && h == 0) {
            sse += e;
            db3[0] += d0;
            db3[1] += d1;
            db3[2] += d2;
            db3[3] += d3;
            dys[m][0] = d0;
            dys[m][1] = d1;
            dys[m][2] = d2;
            dys[m][3] = d3;
        }
        // dZ2 = (W3 dY) silu'(Z2) of the block, to the shared rows
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float dv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int jj = 4 * q + i;
                const int u = acc_unit(w, jj, h);
                const float* wv = w3s + 4 * u;
                const float dh = __builtin_fmaf(wv[0], d0, __builtin_fmaf(wv[1], d1, __builtin_fmaf(wv[2], d2, wv[3] * d3)));
                dv[i] = dh * (s2v[jj] * __builtin_fmaf(z2[jj], 1.0f - s2v[jj], 1.0f));
                dz2T[u * kTS + m] = (__bf16)dv[i];
            }
            store4(dz2s + m * kHS + 32 * w + 8 * q + 4 * h, dv[0], dv[1], dv[2], dv[3]);
        }
        __syncthreads();
        // dH1 = W2 dZ2 of the block, dZ1 = dH1 silu'(Z1) to the block's rows
        f32x16 g = {};
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) {
            const __bf16* r = dz2s + m * kHS + 32 * (s2 >> 1) + 16 * (s2 & 1) + 4 * h;
            typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
            const bf16x4 lo4 = *reinterpret_cast<const bf16x4*>(r);
            const bf16x4 hi4 = *reinterpret_cast<const bf16x4*>(r + 8);
            g = mfma32(a2b[s2], bf16x8{lo4[0], lo4[1], lo4[2], lo4[3], hi4[0], hi4[1], hi4[2], hi4[3]}, g);
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
            dz1T[acc_unit(w, jj, h) * kTS + m] = (__bf16)(g[jj] * (s1[jj] * __builtin_fmaf(z1[jj], 1.0f - s1[jj], 1.0f)));
        // the block's dZ1 rows are read back by this wave only
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // weight gradients: products over the tile's samples
#pragma unroll
        for (int kq = 0; kq < 2; ++kq) {
            const int s0 = 16 * kq + 8 * h;
            const bf16x8 bz1 = *reinterpret_cast<const bf16x8*>(dz1T + (32 * w + m) * kTS + s0);
            const bf16x8 ah = *reinterpret_cast<const bf16x8*>(h1T + (32 * w + m) * kTS + s0);
            const bf16x8 a3 = *reinterpret_cast<const bf16x8*>(h2T + (32 * w + m) * kTS + s0);
            bf16x8 bhi, blo;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float d = m < 4 ? dys[s0 + i][m & 3] : 0.0f;
                bhi[i] = (__bf16)d;
                blo[i] = (__bf16)(d - (float)bhi[i]);
                db1 += (float)bz1[i];
            }
#pragma unroll
            for (int rb = 0; rb < 6; ++rb)
                g1[rb] = mfma32(*reinterpret_cast<const bf16x8*>(xT + (32 * rb + m) * kTS + s0), bz1, g1[rb]);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const bf16x8 bz = *reinterpret_cast<const bf16x8*>(dz2T + (32 * cb + m) * kTS + s0);
                if (cb == w) {
#pragma unroll
                    for (int i = 0; i < 8; ++i) db2 += (float)bz[i];
                }
                g2[cb] = mfma32(ah, bz, g2[cb]);
            }
            g3 = mfma32(a3, bhi, g3);
            g3 = mfma32(a3, blo, g3);
        }
        if (fetch) {
            sxyz[cur ^ 1][m] = nxt_p;
            stgt[cur ^ 1][m] = nxt_t;
        }
        __syncthreads();   // the tile's rows are read; the next tile overwrites them
    }
    // this workgroup's partial gradient, in parameter order
    float* out = A.part + (size_t)blockIdx.x * kFPartPad;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int row = 8 * (j >> 2) + 4 * h + (j & 3);   // accumulator row of register j
#pragma unroll
        for (int rb = 0; rb < 6; ++rb) out[kOffW1 + (32 * rb + row) * kD1 + 32 * w + m] = g1[rb][j];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) out[kOffW2 + (32 * w + row) * kD2 + 32 * cb + m] = g2[cb][j];
        if (m < 4) out[kOffW3 + (32 * w + row) * 4 + m] = g3[j];
    }
    db1 += __shfl_xor(db1, 32, 64);
    db2 += __shfl_xor(db2, 32, 64);
    if (h == 0) {
        out[kOffB1 + 32 * w + m] = db1;
        out[kOffB2 + 32 * w + m] = db2;
    }
    if (w == 0) {
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) {
            sse += __shfl_xor(sse, off, 64);
#pragma unroll
            for (int c = 0; c < 4; ++c) db3[c] += __shfl_xor(db3[c], off, 64);
        }
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) out[kOffB3 + c] = db3[c];
            out[kNParams] = sse;
        }
    }
}

// Gradient of every parameter from the workgroups' partials (added in a fixed
// order), the loss, then the Adam update.
struct AdamSumArgs {
    float* __restrict__ P;
    float* __restrict__ Mo;
    float* __restrict__ Vo;
    float* __restrict__ G;
    const float* __restrict__ part;   // [nparts][kFPartPad]
    float* __restrict__ loss_out;     // one float
    int32_t nparts, update;
    float inv_n, lr, beta1, beta2, eps, c1, c2;
    PublishArgs W;
};

// A workgroup takes 4 x kSumQ consecutive parameters (the squared error is
// the last "parameter"); thread (quad, row) reads four consecutive partials
// of every kSumRows-th workgroup at once; the rows' sums are added in order.
constexpr int kSumQ = 32, kSumRows = 8;
__global__ __launch_bounds__(kSumQ * kSumRows) void k_adam_sum(AdamSumArgs A) {
    __shared__ float4 part[kSumRows][kSumQ];
    const int qi = threadIdx.x % kSumQ, row = threadIdx.x / kSumQ;
    const int q0 = 4 * (blockIdx.x * kSumQ + qi);   // first of this thread's four parameters
    float4 g = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (q0 < kFPart) {
        float4 acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        int z = row;
        for (; z + 3 * kSumRows < A.nparts; z += 4 * kSumRows) {
            float4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                v[u] = *reinterpret_cast<const float4*>(A.part + (size_t)(z + u * kSumRows) * kFPartPad + q0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc[u].x += v[u].x;
                acc[u].y += v[u].y;
                acc[u].z += v[u].z;
                acc[u].w += v[u].w;
            }
        }
        for (; z < A.nparts; z += kSumRows) {
            const float4 v = *reinterpret_cast<const float4*>(A.part + (size_t)z * kFPartPad + q0);
            acc[0].x += v.x;
            acc[0].y += v.y;
            acc[0].z += v.z;
            acc[0].w += v.w;
        }
        g.x = (acc[0].x + acc[1].x) + (acc[2].x + acc[3].x);
        g.y = (acc[0].y + acc[1].y) + (acc[2].y + acc[3].y);
        g.z = (acc[0].z + acc[1].z) + (acc[2].z + acc[3].z);
        g.w = (acc[0].w + acc[1].w) + (acc[2].w + acc[3].w);
    }
    part[row][qi] = g;
    __syncthreads();
    // thread (quad, row) finishes parameter q0 + row of quad qi (rows 0..3)
    if (row >= 4) return;
    const int q = q0 + row;
    if (q >= kFPart) return;
    float gq = 0.0f;
#pragma unroll
    for (int r = 0; r < kSumRows; ++r) {
        const float4 v = part[r][qi];
        gq += row == 0 ? v.x : (row == 1 ? v.y : (row == 2 ? v.z : v.w));
    }
    if (q == kNParams) {
        if (A.loss_out) *A.loss_out = gq * A.inv_n;
        return;
    }
    A.G[q] = gq;
    if (!A.update) return;
    const float m = __builtin_fmaf(A.beta1, A.Mo[q], (1.0f - A.beta1) * gq);
    const float v = __builtin_fmaf(A.beta2, A.Vo[q], (1.0f - A.beta2) * gq * gq);
    A.Mo[q] = m;
    A.Vo[q] = v;
    const float mh = m / A.c1, vh = v / A.c2;
    const float w = A.P[q] - A.lr * mh / (sqrtf(vh) + A.eps);
    A.P[q] = w;
    publish(A.W, q, w);
}

// ------------------------------------------------------------ inference kernels
constexpr int kInferThreads = 512;   // 8 waves: two per SIMD share one LDS copy of the weights

struct EvalArgs {
    const uint4* __restrict__ img;
    const float* __restrict__ xyz;
    float4* __restrict__ out;
    int64_t n;
    float lo[3], inv[3];
    float r_scale, g_scale;
};

__global__ __launch_bounds__(kInferThreads) void k_sur_eval(EvalArgs A) {
    __shared__ uint4 simg[kImgBytes / 16];
    load_image(A.img, simg);
    const char* img = reinterpret_cast<const char*>(simg);
    const int lane = threadIdx.x & 63, m = lane & 31, h = lane >> 5;
    const int64_t nw = (int64_t)gridDim.x * (kInferThreads / 64);
    for (int64_t g = (int64_t)blockIdx.x * (kInferThreads / 64) + (threadIdx.x >> 6); g * 64 < A.n; g += nw) {
        // keeps the weight-fragment reads inside the loop (hoisting them would
        // need some 320 registers per lane)
        asm volatile("" ::: "memory");
        float xa[2][3];
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int64_t k = g * 64 + 32 * tt + m;
            const bool v = k < A.n;
#pragma unroll
            for (int a = 0; a < 3; ++a) xa[tt][a] = ((v ? A.xyz[3 * k + a] : A.lo[a]) - A.lo[a]) * A.inv[a];
        }
        float y[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        mlp32(img, xa[0], 0, y);
        asm volatile("" ::: "memory");
        mlp32(img, xa[1], 1, y);
        const int64_t k = g * 64 + 32 * h + m;
        if (k < A.n) A.out[k] = make_float4(y[0] * A.r_scale, y[1] * A.g_scale, y[2] * A.g_scale, y[3] * A.g_scale);
    }
}

struct SurLikArgs {
    const uint4* __restrict__ img;
    const float4* __restrict__ poses;   // N x 2 float4 (q; t, 0)
    const int32_t* __restrict__ order;  // sorted position -> particle (or null)
    const float4* __restrict__ scan;    // ns x 3 float4 records (mu in the first)
    float* __restrict__ partial;        // [29][N]
    int32_t n, ns;
    float cmax, r_scale, g_scale;
    float lo[3], inv[3];
};

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wave per particle at a time (persistent over particles); 64 scan points
// per network evaluation.  Per-lane sums of H (21), b (6), cost and outliers
// are reduced across the wave once per particle.
__global__ __launch_bounds__(kInferThreads) void k_lik_sur(SurLikArgs A) {
    __shared__ uint4 simg[kImgBytes / 16];
    load_image(A.img, simg);
    const char* img = reinterpret_cast<const char*>(simg);
    const int lane = threadIdx.x & 63, m = lane & 31, h = lane >> 5;
    const int nw = gridDim.x * (kInferThreads / 64);
    for (int sidx = blockIdx.x * (kInferThreads / 64) + (threadIdx.x >> 6); sidx < A.n; sidx += nw) {
        const int i = A.order ? A.order[sidx] : sidx;
        if (i < 0 || i >= A.n) continue;
        const float4 q4 = A.poses[2 * i];
        const float4 t4 = A.poses[2 * i + 1];
        const mpdet::mat3 Rm = mpdet::qmat(mpdet::quat{q4.x, q4.y, q4.z, q4.w});
        const float3 t = make_float3(t4.x, t4.y, t4.z);
        float hs[21], bs[6];
#pragma unroll
        for (int k = 0; k < 21; ++k) hs[k] = 0.0f;
#pragma unroll
        for (int k = 0; k < 6; ++k) bs[k] = 0.0f;
        float cost = 0.0f, comp = 0.0f, nout = 0.0f;
        for (int k0 = 0; k0 < A.ns; k0 += 64) {
            asm volatile("" ::: "memory");   // as in k_sur_eval: no hoisting of fragment reads
            float xa[2][3];
            float3 mu_mine = make_float3(0.0f, 0.0f, 0.0f);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const int k = k0 + 32 * tt + m;
                const float4 r0 = k < A.ns ? A.scan[3 * k] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                const float3 mu = make_float3(r0.x, r0.y, r0.z);
                const float3 p = mpdet::xform(Rm.m, t, mu);
                xa[tt][0] = (p.x - A.lo[0]) * A.inv[0];
                xa[tt][1] = (p.y - A.lo[1]) * A.inv[1];
                xa[tt][2] = (p.z - A.lo[2]) * A.inv[2];
                if (tt == h) mu_mine = mu;
            }
            float y[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            mlp32(img, xa[0], 0, y);
            asm volatile("" ::: "memory");
            mlp32(img, xa[1], 1, y);
            // rank-1 terms of the predicted residual: g = [mu x w; w], w = R^T grad r,
            // H += g g^T, b += r g, cost min(r^2, c_max) (r^2 >= c_max: outlier)
            const bool valid = k0 + 32 * h + m < A.ns;
            const float r = valid ? fmaxf(y[0] * A.r_scale, 0.0f) : 0.0f;
            const float gs = valid ? A.g_scale : 0.0f;
            const float3 w = mpdet::rot_t(Rm, make_float3(y[1] * gs, y[2] * gs, y[3] * gs));
            const float3 mu = mu_mine;
            const float g6[6] = {mu.y * w.z - mu.z * w.y, mu.z * w.x - mu.x * w.z, mu.x * w.y - mu.y * w.x,
                                 w.x, w.y, w.z};
            int q = 0;
#pragma unroll
            for (int rr = 0; rr < 6; ++rr)
#pragma unroll
                for (int c = rr; c < 6; ++c) {
                    hs[q] = __builtin_fmaf(g6[rr], g6[c], hs[q]);
                    ++q;
                }
#pragma unroll
            for (int k = 0; k < 6; ++k) bs[k] = __builtin_fmaf(r, g6[k], bs[k]);
            const float sq = r * r;
            const bool below = valid && sq < A.cmax;
            nout += (valid && !below) ? 1.0f : 0.0f;
            const float yv = (below ? sq : 0.0f) - comp;
            const float tv = cost + yv;
            comp = (tv - cost) - yv;
            cost = tv;
        }
        float* out = A.partial + i;
        const size_t st = (size_t)A.n;
#pragma unroll
        for (int k = 0; k < 21; ++k) {
            const float v = wave_sum(hs[k]);
            if (lane == 0) out[k * st] = v;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const float v = wave_sum(bs[k]);
            if (lane == 0) out[(21 + k) * st] = v;
        }
        const float cs = wave_sum(cost - comp);
        const float no = wave_sum(nout);
        if (lane == 0) {
            out[27 * st] = cs;
            out[28 * st] = no;
        }
    }
}

int num_cus() {
    int dev = 0, cus = 0;
    MP_HIP(hipGetDevice(&dev));
    MP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return std::max(1, cus);
}

PublishArgs publish_args(mp_surrogate S) {
    PublishArgs W;
    W.w3b = S->w3b.as<__bf16>();
    W.img = S->img.as<char>();
    W.img2 = S->img2.as<__bf16>();
    return W;
}

// ------------------------------------------------------------ scorer check
// Scan points (every kstride-th record of the walk order) transformed by
// every pstride-th particle: the sample on which the network is compared with
// the exact residual field.
struct CheckPtsArgs {
    const float4* __restrict__ poses;
    const float4* __restrict__ scan;
    float* __restrict__ xyz;
    int32_t n, pstride, ns, kstride, nk;
    int64_t m;
};

__global__ void k_check_points(CheckPtsArgs A) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= A.m) return;
    const int i = (int)(q / A.nk) * A.pstride;
    const int k = (int)(q % A.nk) * A.kstride;
    const float4 q4 = A.poses[2 * i], t4 = A.poses[2 * i + 1];
    const mpdet::mat3 Rm = mpdet::qmat(mpdet::quat{q4.x, q4.y, q4.z, q4.w});
    const float4 r0 = A.scan[3 * k];
    const float3 p = mpdet::xform(Rm.m, make_float3(t4.x, t4.y, t4.z), make_float3(r0.x, r0.y, r0.z));
    A.xyz[3 * q] = p.x;
    A.xyz[3 * q + 1] = p.y;
    A.xyz[3 * q + 2] = p.z;
}

constexpr int kChkBlocks = 256;

// per-block sums of |min(r_net^2, c) - min(r^2, c)| (fixed grid: deterministic)
__global__ __launch_bounds__(256) void k_check_sum(const float4* __restrict__ net, const float4* __restrict__ ref,
                                                   int64_t m, float cmax, double* __restrict__ part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < m; q += (int64_t)kChkBlocks * 256) {
        const float a = net[q].x, b = ref[q].x;
        acc += (double)fabsf(fminf(a * a, cmax) - fminf(b * b, cmax));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_check_final(const double* __restrict__ part, int64_t m, float* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (int b = 0; b < kChkBlocks; ++b) t += part[b];
    out[0] = (float)(t / (double)m);
}

}  // namespace

// ------------------------------------------------------------ host launchers
void mp_sur_alloc(mp_surrogate S, hipStream_t s) {
    S->cus = num_cus();
    S->P.alloc(sizeof(float) * kNParams);
    S->Mo.alloc(sizeof(float) * kNParams);
    S->Vo.alloc(sizeof(float) * kNParams);
    S->G.alloc(sizeof(float) * kNParams);
    S->img.alloc(kImgBytes);
    S->img2.alloc(kImg2Bytes);
    S->w3b.alloc(2 * kD2 * 4);
    MP_HIP(hipMemsetAsync(S->img.p, 0, kImgBytes, s));
    MP_HIP(hipMemcpyAsync(S->img.as<char>() + kImgFQ, S->info.freqs, sizeof(float) * 32, hipMemcpyHostToDevice, s));
    MP_HIP(hipStreamSynchronize(s));
}

void mp_sur_reset_adam(mp_surrogate S, hipStream_t s) {
    MP_HIP(hipMemsetAsync(S->Mo.p, 0, sizeof(float) * kNParams, s));
    MP_HIP(hipMemsetAsync(S->Vo.p, 0, sizeof(float) * kNParams, s));
    S->info.steps = 0;
}

void mp_sur_publish(mp_surrogate S, hipStream_t s) {
    k_publish<<<(kNParams + 255) / 256, 256, 0, s>>>(S->P.as<float>(), publish_args(S));
    MP_CHECK_LAUNCH();
}

void mp_sur_init_weights(mp_surrogate S, hipStream_t s) {
    k_init_weights<<<(kNParams + 255) / 256, 256, 0, s>>>(S->P.as<float>(), S->p.seed);
    MP_CHECK_LAUNCH();
    mp_sur_reset_adam(S, s);
    mp_sur_publish(S, s);
}

void mp_sur_label(mp_surrogate S, const float* xyz_dev, int64_t n, float* out4_dev, bool scaled, hipStream_t s) {
    if (n <= 0) return;
    LabelArgs A;
    A.map = S->map->view;
    A.xyz = xyz_dev;
    A.out = reinterpret_cast<float4*>(out4_dev);
    A.n = n;
    A.sig2 = S->p.sigma_s * S->p.sigma_s;
    A.ib = 1.0f / (1.0f + A.sig2);
    A.dmax2 = S->p.d_max * S->p.d_max;
    A.r_floor = 1e-2f;
    A.r_out = S->info.r_scale;
    A.inv_r = scaled ? 1.0f / S->info.r_scale : 1.0f;
    A.inv_g = scaled ? 1.0f / S->info.g_scale : 1.0f;
    k_label<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(A);
    MP_CHECK_LAUNCH();
}

void mp_sur_eval(mp_surrogate S, const float* xyz_dev, int64_t n, float* out4_dev, hipStream_t s) {
    if (n <= 0) return;
    EvalArgs A;
    A.img = S->img.as<uint4>();
    A.xyz = xyz_dev;
    A.out = reinterpret_cast<float4*>(out4_dev);
    A.n = n;
    for (int a = 0; a < 3; ++a) {
        A.lo[a] = S->info.lo[a];
        A.inv[a] = S->info.inv_ext[a];
    }
    A.r_scale = S->info.r_scale;
    A.g_scale = S->info.g_scale;
    const int64_t groups = (n + 63) / 64;
    const int64_t blocks = std::min<int64_t>((int64_t)S->cus, (groups + kInferThreads / 64 - 1) / (kInferThreads / 64));
    k_sur_eval<<<(unsigned)std::max<int64_t>(1, blocks), kInferThreads, 0, s>>>(A);
    MP_CHECK_LAUNCH();
}

// padded batch rows: a multiple of the reduction chunk
static int32_t padded_rows(int64_t n) { return (int32_t)((n + kBatchPad - 1) / kBatchPad * kBatchPad); }

void mp_sur_ensure_batch(mp_surrogate S, int64_t cap) {
    const int32_t bp = padded_rows(cap);
    if (bp <= S->cap) return;
    const size_t b = (size_t)bp;
    S->bxyz.alloc(sizeof(float) * 3 * b);
    S->btgt.alloc(sizeof(float) * 4 * b);
    S->pf.ensure(sizeof(float) * (size_t)std::max(1, S->cus) * kFPartPad);
    S->cap = bp;
}

// One gradient evaluation over n_real samples, staged (bxyz, btgt) or drawn
// from the training set with step counter `step`, optionally followed by an
// Adam step with learning rate lr.
static void fused_step(mp_surrogate S, int32_t n_real, bool draw, bool full, uint32_t step, bool update, float lr,
                       float* loss_dev, hipStream_t s) {
    const int32_t bp = padded_rows(n_real);
    if (bp > S->cap) mp_throw(MP_E_STATE, "surrogate batch buffers too small");
    FusedArgs F;
    F.img = S->img.as<uint4>();
    F.img2 = S->img2.as<uint4>();
    F.w3b = S->w3b.as<__bf16>();
    F.xyz = S->bxyz.as<float>();
    F.tgt = S->btgt.as<float4>();
    F.dxyz = S->dxyz.as<float>();
    F.dlab = S->dlab.as<float4>();
    F.part = S->pf.as<float>();
    F.n_data = S->info.n_data;
    F.draw = draw ? 1 : 0;
    F.full = full ? 1 : 0;
    F.step = step;
    F.seed = S->p.seed;
    F.tiles = bp / 32;
    F.n_real = n_real;
    F.two_over_n = (float)(2.0 / (double)n_real);
    for (int a = 0; a < 3; ++a) {
        F.lo[a] = S->info.lo[a];
        F.inv[a] = S->info.inv_ext[a];
    }
    const int groups = std::max(1, std::min(S->cus, F.tiles));
    k_train_fused<<<groups, kFThreads, 0, s>>>(F);
    MP_CHECK_LAUNCH();
    AdamSumArgs A;
    A.P = S->P.as<float>();
    A.Mo = S->Mo.as<float>();
    A.Vo = S->Vo.as<float>();
    A.G = S->G.as<float>();
    A.part = S->pf.as<float>();
    A.loss_out = loss_dev;
    A.nparts = groups;
    A.update = update ? 1 : 0;
    A.inv_n = (float)(1.0 / (double)n_real);
    A.lr = lr;
    A.beta1 = S->p.beta1;
    A.beta2 = S->p.beta2;
    A.eps = S->p.adam_eps;
    const double t = (double)(S->info.steps + 1);
    A.c1 = (float)(1.0 - std::pow((double)S->p.beta1, t));
    A.c2 = (float)(1.0 - std::pow((double)S->p.beta2, t));
    A.W = publish_args(S);
    k_adam_sum<<<(kFPart + 4 * kSumQ - 1) / (4 * kSumQ), kSumQ * kSumRows, 0, s>>>(A);
    MP_CHECK_LAUNCH();
    if (update) S->info.steps += 1;
}

void mp_sur_grad_step(mp_surrogate S, int32_t n_real, bool update, float lr, float* loss_dev, hipStream_t s) {
    fused_step(S, n_real, false, false, 0u, update, lr, loss_dev, s);
}

void mp_sur_train_step(mp_surrogate S, int32_t n_real, bool full, uint32_t step, float lr, float* loss_dev,
                       hipStream_t s) {
    fused_step(S, n_real, true, full, step, true, lr, loss_dev, s);
}

void mp_sur_likelihood(mp_filter f, float* partial, hipStream_t s) {
    mp_surrogate S = f->sur;
    SurLikArgs A;
    A.img = S->img.as<uint4>();
    A.poses = f->poses[f->cur].as<float4>();
    A.order = f->sorted.as<int32_t>();
    A.scan = f->scan.as<float4>();
    A.partial = partial;
    A.n = f->n;
    A.ns = f->scan_n;
    A.cmax = f->p.c_max;
    A.r_scale = S->info.r_scale;
    A.g_scale = S->info.g_scale;
    for (int a = 0; a < 3; ++a) {
        A.lo[a] = S->info.lo[a];
        A.inv[a] = S->info.inv_ext[a];
    }
    // one workgroup per CU (the weights fill its LDS); no device query: this may run under graph capture
    const int blocks = std::min(S->cus, (f->n + kInferThreads / 64 - 1) / (kInferThreads / 64));
    k_lik_sur<<<std::max(1, blocks), kInferThreads, 0, s>>>(A);
    MP_CHECK_LAUNCH();
}

float mp_sur_check(mp_filter f, int32_t pstride, hipStream_t s) {
    const int n = f->n, ns = f->scan_n;
    if (!f->sur || n <= 0 || ns <= 0) return 0.0f;
    const int np = (n + pstride - 1) / pstride;
    int kstride = 1;   // keep the sample at most 2^22 pairs
    while ((int64_t)np * ((ns + kstride - 1) / kstride) > ((int64_t)1 << 22)) ++kstride;
    const int nk = (ns + kstride - 1) / kstride;
    const int64_t m = (int64_t)np * nk;
    // layout: net and ref outputs (float4), block sums (double), result, points
    f->chk_buf.ensure(32 * (size_t)m + sizeof(double) * kChkBlocks + 16 + 12 * (size_t)m);
    char* base = f->chk_buf.as<char>();
    float* net = reinterpret_cast<float*>(base);
    float* ref = reinterpret_cast<float*>(base + 16 * (size_t)m);
    double* part = reinterpret_cast<double*>(base + 32 * (size_t)m);
    float* res = reinterpret_cast<float*>(part + kChkBlocks);
    float* xyz = res + 4;
    CheckPtsArgs A;
    A.poses = f->poses[f->cur].as<float4>();
    A.scan = f->scan.as<float4>();
    A.xyz = xyz;
    A.n = n;
    A.pstride = pstride;
    A.ns = ns;
    A.kstride = kstride;
    A.nk = nk;
    A.m = m;
    k_check_points<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(A);
    MP_CHECK_LAUNCH();
    mp_sur_eval(f->sur, xyz, m, net, s);
    mp_sur_label(f->sur, xyz, m, ref, false, s);
    k_check_sum<<<kChkBlocks, 256, 0, s>>>(reinterpret_cast<const float4*>(net), reinterpret_cast<const float4*>(ref),
                                           m, f->p.c_max, part);
    MP_CHECK_LAUNCH();
    k_check_final<<<1, 64, 0, s>>>(part, m, res);
    MP_CHECK_LAUNCH();
    float out = 0.0f;
    MP_HIP(hipMemcpyAsync(&out, res, sizeof(float), hipMemcpyDeviceToHost, s));
    MP_HIP(hipStreamSynchronize(s));
    return out;
}
