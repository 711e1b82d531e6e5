// mp_lookup.hpp -- nearest-neighbour-field lookup of a transformed scan point.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mp_det.hpp"
#include "mp_internal.hpp"

// spatial hash of band-grid coordinates (Teschner et al. 2003 primes)
__host__ __device__ inline uint32_t mp_grid_hash(int32_t x, int32_t y, int32_t z) {
    return ((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349663u) ^ ((uint32_t)z * 83492791u);
}

// Gaussian id of the voxel floor(p * 1/r), or -1 outside the band.
// BACKEND: MP_NNF_DENSE, MP_NNF_HASH, or 0 to branch on v.backend.
template <int BACKEND = 0>
__device__ __forceinline__ int32_t mp_nnf_lookup(const MapView& v, float px, float py, float pz) {
    const uint32_t x = (uint32_t)mpdet::floor_i32(px * v.inv_r) - (uint32_t)v.org[0];
    const uint32_t y = (uint32_t)mpdet::floor_i32(py * v.inv_r) - (uint32_t)v.org[1];
    const uint32_t z = (uint32_t)mpdet::floor_i32(pz * v.inv_r) - (uint32_t)v.org[2];
    if (x >= (uint32_t)v.dim[0] || y >= (uint32_t)v.dim[1] || z >= (uint32_t)v.dim[2]) return -1;
    const bool dense = BACKEND == 0 ? v.backend == MP_NNF_DENSE : BACKEND == MP_NNF_DENSE;
    if (dense) return v.dense[((uint32_t)z * (uint32_t)v.dim[1] + y) * (uint32_t)v.dim[0] + x];
    const uint64_t L = ((uint64_t)z * (uint32_t)v.dim[1] + y) * (uint32_t)v.dim[0] + x;
    const uint32_t key = (uint32_t)L + 1u;
    uint32_t h = mp_grid_hash((int32_t)x, (int32_t)y, (int32_t)z) & v.mask;
    for (;;) {
        const uint2 s = v.table[h];
        if (s.x == key) return (int32_t)s.y;
        if (s.x == 0u) return -1;
        h = (h + 1u) & v.mask;
    }
}

// floor to int32 in one instruction (saturating outside the int32 range);
// for |z| >= 2^30 both this and the clamped floor put the point outside any
// band grid (|origin| < 2^30, extent < 2^30), so the lookup decisions agree
__device__ __forceinline__ int32_t floor_cell(float z) {
    int32_t r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(z));
    return r;
}

// dense band-grid cell of floor(p * 1/r) (x fastest), or `miss` outside the
// grid's box.  The map build keeps dim_x dim_y < 2^24, so for in-box cells the
// 24-bit products are exact; outside the box the index is discarded.
__device__ __forceinline__ uint32_t mp_nnf_cell_or(const MapView& v, float px, float py, float pz, uint32_t miss) {
    const uint32_t x = (uint32_t)floor_cell(px * v.inv_r) - (uint32_t)v.org[0];
    const uint32_t y = (uint32_t)floor_cell(py * v.inv_r) - (uint32_t)v.org[1];
    const uint32_t z = (uint32_t)floor_cell(pz * v.inv_r) - (uint32_t)v.org[2];
    const bool in = (x < (uint32_t)v.dim[0]) & (y < (uint32_t)v.dim[1]) & (z < (uint32_t)v.dim[2]);
    const uint32_t c = __umul24(z, v.dxy) + __umul24(y, (uint32_t)v.dim[0]) + x;
    return in ? c : miss;
}

// dense band-grid cell of floor(p * 1/r), or -1 outside the grid's box
__device__ __forceinline__ int32_t mp_nnf_cell(const MapView& v, float px, float py, float pz) {
    return (int32_t)mp_nnf_cell_or(v, px, py, pz, 0xFFFFFFFFu);
}

// the two float4 of dense record c (a cell, or the miss record), addressed by
// a 32-bit byte offset from the array's base
__device__ __forceinline__ void mp_dense_record(const MapView& v, uint32_t c, float4& m, float4& n) {
    const char* b = reinterpret_cast<const char*>(v.drec) + (c << 5);
    m = *reinterpret_cast<const float4*>(b);
    n = *reinterpret_cast<const float4*>(b + 16);
}
