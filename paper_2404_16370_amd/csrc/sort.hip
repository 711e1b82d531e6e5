// sort.hip -- device-wide exclusive scan and stable LSD radix sort.
//
// The radix sort distributes particles into LSH buckets (Alg. 1, distribute
// loop) and groups map points by voxel.  Each pass handles one 8-bit digit:
//   1. per-tile digit histograms (tile = 1024 items, LDS atomics),
//   2. exclusive scan of the digit-major histogram matrix -> global offsets,
//   3. stable scatter: tiles are walked in 4 rounds of 256 items; within a
//      wavefront the rank among lanes with the same digit comes from eight
//      64-lane ballots (one per digit bit); per-wavefront counts are
//      prefix-summed across the four wavefronts in LDS.
// Stability of every pass makes the LSD sort stable, so equal keys keep
// ascending value order when the values start as 0..n-1.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mp_internal.hpp"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 4;
constexpr int kTile = kThreads * kItems;

__device__ inline uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// block-wide exclusive scan of one value per thread; returns the block total
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t& excl) {
    __shared__ uint32_t wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v, lane);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t base = 0, total = 0;
#pragma unroll
    for (int k = 0; k < kThreads / 64; ++k) {
        if (k < w) base += wsum[k];
        total += wsum[k];
    }
    excl = base + inc - v;
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                          uint32_t* __restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + r * kThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t ex;
    const uint32_t tot = block_excl_scan(s, ex);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// exclusive scan of each tile plus the tile's offset; in == out allowed
__global__ __launch_bounds__(kThreads) void k_scan_apply(const uint32_t* in, uint32_t* out, int64_t n,
                                                         const uint32_t* __restrict__ offsets,
                                                         uint32_t* __restrict__ total) {
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t i = base + j;
        v[j] = i < n ? in[i] : 0u;
        s += v[j];
    }
    uint32_t ex;
    const uint32_t tot = block_excl_scan(s, ex);
    const uint32_t off = offsets ? offsets[blockIdx.x] : 0u;
    uint32_t run = off + ex;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t i = base + j;
        if (i < n) out[i] = run;
        run += v[j];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
}

size_t scan_scratch_words(int64_t n) {
    size_t w = 0;
    while (n > kTile) {
        n = (n + kTile - 1) / kTile;
        w += (size_t)n;
    }
    return w;
}

void scan_rec(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* scratch, hipStream_t s) {
    if (n <= 0) {
        if (total) mp_fill_u32(total, 0u, 1, s);
        return;
    }
    if (n <= kTile) {
        k_scan_apply<<<1, kThreads, 0, s>>>(in, out, n, nullptr, total);
        MP_CHECK_LAUNCH();
        return;
    }
    const int64_t nb = (n + kTile - 1) / kTile;
    uint32_t* sums = scratch;
    k_scan_reduce<<<(unsigned)nb, kThreads, 0, s>>>(in, n, sums);
    MP_CHECK_LAUNCH();
    scan_rec(sums, sums, nb, nullptr, scratch + nb, s);
    k_scan_apply<<<(unsigned)nb, kThreads, 0, s>>>(in, out, n, sums, total);
    MP_CHECK_LAUNCH();
}

template <class K>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const K* __restrict__ keys, int64_t n, int shift,
                                                         uint32_t* __restrict__ counts, int64_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + r * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

template <class K>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const K* __restrict__ kin, const int32_t* __restrict__ vin,
                                                            K* __restrict__ kout, int32_t* __restrict__ vout,
                                                            int64_t n, int shift, const uint32_t* __restrict__ offs,
                                                            int64_t nblocks) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kThreads / 64][256];
    __shared__ uint32_t wpre[kThreads / 64][256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    run[t] = offs[(int64_t)t * nblocks + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kItems; ++r) {
#pragma unroll
        for (int j = 0; j < kThreads / 64; ++j) wcnt[j][t] = 0;
        __syncthreads();
        const int64_t i = base + r * kThreads + t;
        const bool valid = i < n;
        const K key = valid ? kin[i] : (K)0;
        const int32_t val = valid ? vin[i] : 0;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint64_t lower = peers & below;
        const uint32_t rank = (uint32_t)__popcll(lower);
        if (valid && lower == 0ull) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        uint32_t s = run[t];
#pragma unroll
        for (int j = 0; j < kThreads / 64; ++j) {
            wpre[j][t] = s;
            s += wcnt[j][t];
        }
        run[t] = s;
        __syncthreads();
        if (valid) {
            const uint32_t pos = wpre[w][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

// Sorts (keys, vals) in 8-bit passes, ping-ponging with the alt arrays.  With
// copy_back the result is always left in (keys, vals); without it the result
// stays where the last pass wrote it, (keys_alt, vals_alt) after an odd
// number of passes.
template <class K>
void radix_sort(K* keys, int32_t* vals, K* keys_alt, int32_t* vals_alt, int64_t n, int bits, DevMem& scratch,
                hipStream_t s, bool copy_back = true) {
    if (n <= 1 || bits <= 0) return;
    const int passes = (bits + 7) / 8;
    const int64_t nb = (n + kTile - 1) / kTile;
    const int64_t m = 256 * nb;
    scratch.ensure(sizeof(uint32_t) * (size_t)(2 * m + scan_scratch_words(m) + 16));
    uint32_t* counts = scratch.as<uint32_t>();
    uint32_t* offs = counts + m;
    uint32_t* sscr = offs + m;
    K* ka = keys;
    int32_t* va = vals;
    K* kb = keys_alt;
    int32_t* vb = vals_alt;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        k_radix_hist<K><<<(unsigned)nb, kThreads, 0, s>>>(ka, n, shift, counts, nb);
        MP_CHECK_LAUNCH();
        scan_rec(counts, offs, m, nullptr, sscr, s);
        k_radix_scatter<K><<<(unsigned)nb, kThreads, 0, s>>>(ka, va, kb, vb, n, shift, offs, nb);
        MP_CHECK_LAUNCH();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (copy_back && ka != keys) {
        MP_HIP(hipMemcpyAsync(keys, ka, sizeof(K) * (size_t)n, hipMemcpyDeviceToDevice, s));
        MP_HIP(hipMemcpyAsync(vals, va, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    }
}

}  // namespace

void mp_scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev, DevMem& scratch,
                           hipStream_t s) {
    scratch.ensure(sizeof(uint32_t) * (scan_scratch_words(n) + 16));
    scan_rec(in, out, n, total_dev, scratch.as<uint32_t>(), s);
}

size_t mp_radix_scratch_bytes(int64_t n) {
    const int64_t nb = (n + kTile - 1) / kTile;
    const int64_t m = 256 * nb;
    return sizeof(uint32_t) * (size_t)(2 * m + scan_scratch_words(m) + 16);
}

void mp_radix_sort_u32(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                       DevMem& scratch, hipStream_t s) {
    radix_sort<uint32_t>(keys, vals, keys_alt, vals_alt, n, bits, scratch, s);
}

int mp_radix_passes(int64_t n, int bits) {
    return (n <= 1 || bits <= 0) ? 0 : (bits + 7) / 8;
}

void mp_radix_sort_u32_inplace_parity(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n,
                                      int bits, DevMem& scratch, hipStream_t s) {
    radix_sort<uint32_t>(keys, vals, keys_alt, vals_alt, n, bits, scratch, s, false);
}

void mp_radix_sort_u64(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                       DevMem& scratch, hipStream_t s) {
    radix_sort<uint64_t>(keys, vals, keys_alt, vals_alt, n, bits, scratch, s);
}
