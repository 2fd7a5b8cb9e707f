// Device helpers shared by the docking, scoring and refinement kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gd_internal.h"

namespace gd {

// --------------------------------------------------------------------------
// wavefront helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t lo = __shfl_xor((uint32_t)v, o);
        uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o);
        uint64_t w = ((uint64_t)hi << 32) | lo;
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// --------------------------------------------------------------------------
// exact distance field lookups

// D by brute force over the occupied cells (cells outside the tabulated box).
static __device__ int D_brute(const PocketDev& P, int cx, int cy, int cz) {
    int best = 0x7fffffff;
    for (int i = 0; i < P.n_occ; i++) {
        int dx = cx - P.occ[3 * i], dy = cy - P.occ[3 * i + 1], dz = cz - P.occ[3 * i + 2];
        int d = dx * dx + dy * dy + dz * dz;
        best = d < best ? d : best;
    }
    return best;
}

// D of a box-relative cell; outside the box falls back to brute force.
__device__ __forceinline__ int D_box(const PocketDev& P, int ix, int iy, int iz, int& oob) {
    if ((unsigned)ix < (unsigned)P.dim[0] && (unsigned)iy < (unsigned)P.dim[1] && (unsigned)iz < (unsigned)P.dim[2])
        return P.edt[((size_t)iz * P.dim[1] + iy) * P.dim[0] + ix];
    oob++;
    return D_brute(P, ix + P.lo[0], iy + P.lo[1], iz + P.lo[2]);
}

// D of the cell containing an FP64 point (global frame): floor(x / h) is
// floor(x * (1/h)) exactly because h is a power of two.
__device__ __forceinline__ int D_exact(const PocketDev& P, double x, double y, double z, int& oob) {
    int cx = (int)floor(x * P.inv_h), cy = (int)floor(y * P.inv_h), cz = (int)floor(z * P.inv_h);
    return D_box(P, cx - P.lo[0], cy - P.lo[1], cz - P.lo[2], oob);
}

__device__ __forceinline__ double dist2(double ax, double ay, double az, double bx, double by, double bz) {
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    return dx * dx + dy * dy + dz * dz;
}

}  // namespace gd
