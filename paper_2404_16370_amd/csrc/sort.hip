// sort.hip -- device-wide exclusive scan and stable radix sorts.
//
// The radix sorts distribute particles into LSH buckets (Alg. 1, distribute
// loop), order the scan points for the likelihood's walk and group map points
// by voxel.  Every pass handles one 8-bit digit and is stable, so the sort is
// stable: equal keys keep ascending value order when the values start as
// 0..n-1.
//
// 32-bit keys (the per-iteration sorts) take a one-sweep form: one launch
// counts the digits of every pass at once, then each pass is one launch in
// which a workgroup ranks its 4096-key tile locally, publishes its digit
// counts, reads the counts of the tiles before it (a decoupled look-back:
// each tile publishes first its own count, then its inclusive prefix, and a
// tile adds its predecessors' counts until it reaches an inclusive prefix)
// and writes its keys to their sorted places through LDS.  Tiles take their
// index from a counter in the order they start, so every tile a workgroup
// waits for belongs to a workgroup that is already running and publishes
// without waiting on later tiles; the wait is bounded all the same.
//
// 64-bit keys (the one-time voxel grouping of a map build) take three
// launches per pass: per-tile digit histograms (LDS atomics), an exclusive
// scan of the digit-major histogram matrix, and a stable scatter in which the
// rank among lanes with the same digit comes from eight 64-lane ballots.
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

// ------------------------------------------------------------ one-sweep sort of 32-bit keys
constexpr int kOsThreads = 512;
constexpr int kOsWaves = kOsThreads / 64;
constexpr int kOsItems = 8;                      // keys per thread: a wave ranks 8 rounds of 64
constexpr int kOsTile = kOsThreads * kOsItems;   // 4096 keys per tile
static_assert(kOsThreads == 512, "two threads per digit sum the histogram blocks");
constexpr int kOsWaveKeys = kOsTile / kOsWaves;  // 512 consecutive keys per wave
constexpr int kOsMaxPasses = 4;
constexpr int kOsHistThreads = 1024;
constexpr int kOsHistKeys = 16;                  // consecutive keys per histogram thread and round
constexpr int kOsMaxHistBlocks = 64;
constexpr int kOsWindow = 16;                    // predecessor tiles read per look-back step
constexpr uint32_t kOsSpinLimit = 1u << 20;      // look-back steps without progress before giving up
// a tile's published word for one digit: flag in the top two bits, count below
constexpr uint32_t kStAgg = 1u << 30;            // the tile's own count
constexpr uint32_t kStInc = 2u << 30;            // the count of all keys up to and including the tile
constexpr uint32_t kStVal = (1u << 30) - 1u;
// scratch words: [0, 4) tile counters of the passes, [4] wait flag, then the
// published words [pass][tile][digit], then the histogram blocks' counts
// [block][pass][digit]
constexpr int kOsHead = 16;

__device__ inline uint32_t os_load(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void os_store(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct OsHistArgs {
    const uint32_t* __restrict__ keys;
    int64_t n;
    int32_t passes;
    int32_t vec;                     // keys 16-byte aligned: read four at a time
    uint32_t* __restrict__ part;     // [gridDim.x][kOsMaxPasses][256]
    uint32_t* __restrict__ clear;    // counters, flag and published words: zeroed
    int64_t clear_words;
};

// Digit counts of every pass over all keys.  A thread takes 16 consecutive
// keys and adds runs of equal digits with one LDS atomic per run (keys of a
// converged filter share codes over long runs).
__global__ __launch_bounds__(kOsHistThreads) void k_os_hist(OsHistArgs A) {
    __shared__ uint32_t h[kOsMaxPasses * 256];
    const int64_t gt = (int64_t)blockIdx.x * kOsHistThreads + threadIdx.x;
    const int64_t gstride = (int64_t)gridDim.x * kOsHistThreads;
    for (int j = threadIdx.x; j < kOsMaxPasses * 256; j += kOsHistThreads) h[j] = 0;
    for (int64_t j = gt; j < A.clear_words; j += gstride) A.clear[j] = 0;
    __syncthreads();
    for (int64_t i0 = gt * kOsHistKeys; i0 < A.n; i0 += gstride * kOsHistKeys) {
        uint32_t k[kOsHistKeys];
        if (A.vec && i0 + kOsHistKeys <= A.n) {
            const uint4* q = reinterpret_cast<const uint4*>(A.keys + i0);
#pragma unroll
            for (int c = 0; c < kOsHistKeys / 4; ++c) {
                const uint4 v = q[c];
                k[4 * c] = v.x;
                k[4 * c + 1] = v.y;
                k[4 * c + 2] = v.z;
                k[4 * c + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int c = 0; c < kOsHistKeys; ++c) k[c] = i0 + c < A.n ? A.keys[i0 + c] : 0u;
        }
        const int cnt = (int)min<int64_t>(kOsHistKeys, A.n - i0);
        for (int p = 0; p < A.passes; ++p) {
            uint32_t cur = (k[0] >> (8 * p)) & 255u, run = 1;
#pragma unroll
            for (int c = 1; c < kOsHistKeys; ++c) {
                const uint32_t d = (k[c] >> (8 * p)) & 255u;
                if (c < cnt && d == cur) {
                    ++run;
                } else if (c < cnt) {
                    atomicAdd(&h[p * 256 + cur], run);
                    cur = d;
                    run = 1;
                }
            }
            atomicAdd(&h[p * 256 + cur], run);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kOsMaxPasses * 256; j += kOsHistThreads)
        A.part[(size_t)blockIdx.x * kOsMaxPasses * 256 + j] = h[j];
}

struct OsScatterArgs {
    const uint32_t* __restrict__ kin;
    const int32_t* __restrict__ vin;
    uint32_t* __restrict__ kout;
    int32_t* __restrict__ vout;
    int64_t n;
    int32_t shift, pass, nhist;
    const uint32_t* __restrict__ part;   // [nhist][kOsMaxPasses][256]
    uint32_t* status;                    // this pass: [tiles][256], zero at launch
    uint32_t* ticket;                    // this pass's tile counter, zero at launch
    uint32_t* wait_flag;                 // 1: a look-back gave up; 2: a key fell outside the output
};

// One pass: the grid has exactly one workgroup per tile.
__global__ __launch_bounds__(kOsThreads) void k_os_scatter(OsScatterArgs A) {
    __shared__ uint32_t wc[kOsWaves][256];   // per-wave digit counts, then the waves' exclusive offsets
    __shared__ uint32_t sk[kOsTile];
    __shared__ int32_t sv[kOsTile];
    __shared__ uint32_t tstart[256];         // first local position of each digit in the tile
    __shared__ uint32_t gbase[256];          // global position of a digit's keys minus tstart
    __shared__ uint32_t htot[2][256];        // digit totals summed by the two halves of the workgroup
    __shared__ uint32_t wsc[4], wsg[4];
    __shared__ uint32_t s_tile;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) s_tile = atomicAdd(A.ticket, 1u);
    for (int j = t; j < kOsWaves * 256; j += kOsThreads) (&wc[0][0])[j] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t tbase = (int64_t)tile * kOsTile;
    const int64_t wbase = tbase + w * kOsWaveKeys;
    uint32_t key[kOsItems], lr[kOsItems];
    int32_t val[kOsItems];
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        const int64_t i = wbase + r * 64 + lane;
        key[r] = i < A.n ? A.kin[i] : 0u;
        val[r] = i < A.n ? A.vin[i] : 0;
    }
    // digit totals of this pass over all keys, from the histogram blocks:
    // each half of the workgroup sums every other block (loads in flight together)
    {
        const int d = t & 255, hb = t >> 8;
        uint32_t pv[kOsMaxHistBlocks / 2];
#pragma unroll
        for (int b = 0; b < kOsMaxHistBlocks / 2; ++b) {
            const int blk = 2 * b + hb;
            pv[b] = blk < A.nhist ? A.part[((size_t)blk * kOsMaxPasses + A.pass) * 256 + d] : 0u;
        }
        uint32_t sum = 0;
#pragma unroll
        for (int b = 0; b < kOsMaxHistBlocks / 2; ++b) sum += pv[b];
        htot[hb][d] = sum;
    }
    // rank of each key among the keys of its wave with the same digit, in
    // key order: the lanes of a round sharing the digit (eight ballots), plus
    // the wave's running count of that digit from earlier rounds
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        const bool valid = wbase + r * 64 + lane < A.n;
        const uint32_t d = (key[r] >> A.shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t rk = (uint32_t)__popcll(peers & below);
        const uint32_t b0 = wc[w][d];
        if (valid && rk == 0) wc[w][d] = b0 + (uint32_t)__popcll(peers);
        lr[r] = b0 + rk;
    }
    __syncthreads();
    uint32_t cnt = 0, incc = 0, incg = 0, tot = 0;
    if (t < 256) {
        tot = htot[0][t] + htot[1][t];
        for (int v = 0; v < kOsWaves; ++v) {
            const uint32_t c = wc[v][t];
            wc[v][t] = cnt;
            cnt += c;
        }
        os_store(A.status + (size_t)tile * 256 + t, (tile == 0 ? kStInc : kStAgg) | cnt);
        incc = wave_incl_scan(cnt, lane);
        incg = wave_incl_scan(tot, lane);
        if (lane == 63) {
            wsc[w] = incc;
            wsg[w] = incg;
        }
    }
    __syncthreads();
    if (t < 256) {
        uint32_t bc = 0, bg = 0;
        for (int v = 0; v < w; ++v) {
            bc += wsc[v];
            bg += wsg[v];
        }
        const uint32_t ts = bc + incc - cnt;   // tile-local start of digit t
        const uint32_t gs = bg + incg - tot;   // global start of digit t
        // keys of digit t in the tiles before this one
        uint32_t excl = 0;
        int64_t tp = (int64_t)tile - 1;
        uint32_t idle = 0;
        while (tp >= 0) {
            uint32_t st[kOsWindow];
#pragma unroll
            for (int k = 0; k < kOsWindow; ++k)
                st[k] = tp - k >= 0 ? os_load(A.status + (size_t)(tp - k) * 256 + t) : kStInc;
            int used = 0;
            bool done = false;
#pragma unroll
            for (int k = 0; k < kOsWindow; ++k) {
                if (done || used < k) continue;              // stopped earlier in the window
                const uint32_t sw = st[k];
                if ((sw & ~kStVal) == 0u) continue;          // not published yet: read again from here
                excl += sw & kStVal;
                used = k + 1;
                done = (sw & kStInc) != 0u;
            }
            if (done) break;
            tp -= used;
            if (used == 0) {
                if (++idle > kOsSpinLimit) {
                    os_store(A.wait_flag, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (tile > 0) os_store(A.status + (size_t)tile * 256 + t, kStInc | (excl + cnt));
        tstart[t] = ts;
        gbase[t] = gs + excl - ts;
    }
    __syncthreads();
    // keys to their sorted places in the tile
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        if (wbase + r * 64 + lane < A.n) {
            const uint32_t d = (key[r] >> A.shift) & 255u;
            const uint32_t lp = tstart[d] + wc[w][d] + lr[r];
            sk[lp] = key[r];
            sv[lp] = val[r];
        }
    }
    __syncthreads();
    const int64_t tn = min<int64_t>(kOsTile, A.n - tbase);
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        const int j = r * kOsThreads + t;
        if (j < tn) {
            const uint32_t kk = sk[j];
            const uint32_t pos = gbase[(kk >> A.shift) & 255u] + (uint32_t)j;
            // a pass whose input is not a permutation of the counted keys (the
            // keys changed under the sort) could place a key past the end:
            // such keys are dropped and the sort flagged
            if ((int64_t)pos < A.n) {
                A.kout[pos] = kk;
                A.vout[pos] = sv[j];
            } else {
                os_store(A.wait_flag, 2u);
            }
        }
    }
}

int64_t os_tiles(int64_t n) { return (n + kOsTile - 1) / kOsTile; }

int os_hist_blocks(int64_t n) {
    const int64_t per = (int64_t)kOsHistThreads * kOsHistKeys;
    return (int)std::max<int64_t>(1, std::min<int64_t>(kOsMaxHistBlocks, (n + per - 1) / per));
}

size_t os_scratch_words(int64_t n) {
    return (size_t)kOsHead + (size_t)kOsMaxPasses * (size_t)os_tiles(n) * 256 +
           (size_t)kOsMaxHistBlocks * kOsMaxPasses * 256;
}

// Stable sort of 32-bit keys by their low `bits` bits (one launch for the
// digit counts, one per 8-bit pass), ping-ponging with the alt arrays; the
// result lands as in radix_sort.
void onesweep_sort(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                   DevMem& scratch, hipStream_t s, bool copy_back) {
    if (n <= 1 || bits <= 0) return;
    if (n > (int64_t)kStVal) mp_throw(MP_E_UNSUPPORTED, "radix sort of more than 2^30 - 1 keys");
    const int passes = std::min(kOsMaxPasses, (bits + 7) / 8);
    const int64_t tiles = os_tiles(n);
    const int nhist = os_hist_blocks(n);
    scratch.ensure(sizeof(uint32_t) * os_scratch_words(n));
    uint32_t* base = scratch.as<uint32_t>();
    uint32_t* status = base + kOsHead;
    uint32_t* part = status + (size_t)kOsMaxPasses * (size_t)tiles * 256;
    OsHistArgs H;
    H.keys = keys;
    H.n = n;
    H.passes = passes;
    H.vec = ((uintptr_t)keys & 15u) == 0 ? 1 : 0;
    H.part = part;
    H.clear = base;
    H.clear_words = kOsHead + (int64_t)passes * tiles * 256;
    k_os_hist<<<nhist, kOsHistThreads, 0, s>>>(H);
    MP_CHECK_LAUNCH();
    uint32_t* ka = keys;
    int32_t* va = vals;
    uint32_t* kb = keys_alt;
    int32_t* vb = vals_alt;
    for (int p = 0; p < passes; ++p) {
        OsScatterArgs A;
        A.kin = ka;
        A.vin = va;
        A.kout = kb;
        A.vout = vb;
        A.n = n;
        A.shift = 8 * p;
        A.pass = p;
        A.nhist = nhist;
        A.part = part;
        A.status = status + (size_t)p * (size_t)tiles * 256;
        A.ticket = base + p;
        A.wait_flag = base + 4;
        k_os_scatter<<<(unsigned)tiles, kOsThreads, 0, s>>>(A);
        MP_CHECK_LAUNCH();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (copy_back && ka != keys) {
        MP_HIP(hipMemcpyAsync(keys, ka, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
        MP_HIP(hipMemcpyAsync(vals, va, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    }
}

}  // namespace

void mp_scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev, DevMem& scratch,
                           hipStream_t s) {
    scratch.ensure(sizeof(uint32_t) * (scan_scratch_words(n) + 16));
    scan_rec(in, out, n, total_dev, scratch.as<uint32_t>(), s);
}

size_t mp_radix_scratch_bytes(int64_t n) { return sizeof(uint32_t) * os_scratch_words(n); }

void mp_radix_sort_u32(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                       DevMem& scratch, hipStream_t s) {
    onesweep_sort(keys, vals, keys_alt, vals_alt, n, bits, scratch, s, true);
}

int mp_radix_passes(int64_t n, int bits) {
    return (n <= 1 || bits <= 0) ? 0 : std::min(kOsMaxPasses, (bits + 7) / 8);
}

void mp_radix_sort_u32_inplace_parity(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n,
                                      int bits, DevMem& scratch, hipStream_t s) {
    onesweep_sort(keys, vals, keys_alt, vals_alt, n, bits, scratch, s, false);
}

uint32_t* mp_radix_wait_flag(DevMem& scratch) { return scratch.as<uint32_t>() + 4; }

void mp_radix_sort_u64(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                       DevMem& scratch, hipStream_t s) {
    radix_sort<uint64_t>(keys, vals, keys_alt, vals_alt, n, bits, scratch, s);
}
