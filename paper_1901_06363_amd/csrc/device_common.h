// Device helpers shared by the docking, scoring and refinement kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gd_internal.h"

namespace gd {

// --------------------------------------------------------------------------
// wavefront helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }
// The lane index computed where it is used: code that runs once per sweep or
// pose takes it from here, so that the compiler does not keep lane-derived
// addresses from the start of the kernel in registers (or scratch memory)
// across the inner loops.
__device__ __forceinline__ int lane_id_here() {
    int r;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(r));
    return r;
}
// 0.0f in a vector register, formed where it is used (for the same reason).
__device__ __forceinline__ float zero_here() {
    float r;
    asm volatile("v_mov_b32 %0, 0" : "=v"(r));
    return r;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane reductions with DPP row shifts (inclusive prefix within each row
// of 16 lanes) and readlane of the four row results: no LDS round trips.
// DPP controls: row_shr:n = 0x110 + n; row_mask/bank_mask 0xf; invalid source
// lanes read the identity passed as `old`.
template <class Op>
__device__ __forceinline__ int dpp_row_scan(int v, int ident, Op op) {
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x111, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x112, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x114, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x118, 0xf, 0xf, false));
    return v;
}

__device__ __forceinline__ int wave_sum(int v) {
    v = dpp_row_scan(v, 0, [](int a, int b) { return a + b; });
    return __builtin_amdgcn_readlane(v, 15) + __builtin_amdgcn_readlane(v, 31) + __builtin_amdgcn_readlane(v, 47) +
           __builtin_amdgcn_readlane(v, 63);
}

// 64-bit wave sum (for exact scores of atoms far outside the grid box), in
// three limbs of 24, 24 and 16 bits summed as 32-bit integers (64 lanes add at
// most 6 bits), so it needs no lane-index registers; exact modulo 2^64.
__device__ __forceinline__ long long wave_sum64(long long v) {
    const unsigned long long u = (unsigned long long)v;
    const int l0 = wave_sum((int)(u & 0xffffffu));
    const int l1 = wave_sum((int)((u >> 24) & 0xffffffu));
    const int l2 = wave_sum((int)(short)(u >> 48));
    return (long long)((unsigned long long)(long long)l0 + ((unsigned long long)(long long)l1 << 24) +
                       ((unsigned long long)(long long)l2 << 48));
}

// Scores are reported in 31 bits: a pose whose S reaches 2^31 - 1 (an atom
// some kilometres from the pocket) saturates there.
constexpr long long kSMax = 0x7fffffffLL;
__device__ __forceinline__ int sat_S(long long s) { return s < kSMax ? (int)s : (int)kSMax; }

__device__ __forceinline__ float wave_maxf(float v) {
    // non-negative inputs: the integer order of the bit patterns is the float order
    int b = dpp_row_scan(__float_as_int(v), 0, [](int a, int c) { return a > c ? a : c; });
    int m = max(max(__builtin_amdgcn_readlane(b, 15), __builtin_amdgcn_readlane(b, 31)),
                max(__builtin_amdgcn_readlane(b, 47), __builtin_amdgcn_readlane(b, 63)));
    return __int_as_float(m);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    int b = dpp_row_scan((int)v, -1, [](int a, int c) { return (uint32_t)a < (uint32_t)c ? a : c; });
    uint32_t m0 = (uint32_t)__builtin_amdgcn_readlane(b, 15), m1 = (uint32_t)__builtin_amdgcn_readlane(b, 31);
    uint32_t m2 = (uint32_t)__builtin_amdgcn_readlane(b, 47), m3 = (uint32_t)__builtin_amdgcn_readlane(b, 63);
    m0 = m0 < m1 ? m0 : m1;
    m2 = m2 < m3 ? m2 : m3;
    return m0 < m2 ? m0 : m2;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    const uint32_t hi = wave_min_u32((uint32_t)(v >> 32));
    const uint32_t lo = wave_min_u32((uint32_t)(v >> 32) == hi ? (uint32_t)v : 0xffffffffu);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The double held by one lane (a wave-uniform lane index), in scalar registers.
__device__ __forceinline__ double readlane_d(double v, int l) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// A wave-uniform double moved to scalar registers.
__device__ __forceinline__ double uniform_d(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Load through a global-address-space pointer.  Pointers read out of the
// device descriptors are generic to the compiler, and generic (flat) loads
// also hold the LDS wait counter, so every LDS access after a gather would
// wait for the gather; the cast gives plain global loads.
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}

// The same for a plain record, word by word (records have no copy from the
// global address space).
template <class T>
__device__ __forceinline__ T ldg_record(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "whole words");
    T v;
    uint32_t* d = reinterpret_cast<uint32_t*>(&v);
    const uint32_t* s = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); i++) d[i] = ldg(s + i);
    return v;
}

// Loads of wave-uniform data that no kernel writes (the batch and pocket
// tables) through the constant address space: with a uniform address the
// compiler issues scalar loads and keeps the value in scalar registers rather
// than a copy in every lane.
template <class T>
__device__ __forceinline__ T ldc(const T* p) {
    return *(const __attribute__((address_space(4))) T*)p;
}

template <class T>
__device__ __forceinline__ T ldc_record(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "whole words");
    T v;
    uint32_t* d = reinterpret_cast<uint32_t*>(&v);
    const uint32_t* s = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); i++) d[i] = ldc(s + i);
    return v;
}

// --------------------------------------------------------------------------
// exact distance field lookups

// D by brute force over the occupied cells (cells outside the tabulated box),
// in 64 bits; a cell more than about 46,000 cells from every occupied cell
// (23 km at h = 0.5 A) saturates at 2^31 - 1, so a sum over at most 128
// atoms stays below 2^38.
constexpr long long kDMax = 0x7fffffffLL;
static __device__ long long D_brute(const PocketDev& P, int cx, int cy, int cz) {
    long long best = kDMax;
    for (int i = 0; i < P.n_occ; i++) {
        long long dx = (long long)cx - ldg(P.occ + 3 * i), dy = (long long)cy - ldg(P.occ + 3 * i + 1),
                  dz = (long long)cz - ldg(P.occ + 3 * i + 2);
        long long d = dx * dx + dy * dy + dz * dz;
        best = d < best ? d : best;
    }
    return best;
}

// D of a box-relative cell; outside the box falls back to brute force.
__device__ __forceinline__ long long D_box(const PocketDev& P, int ix, int iy, int iz, int& oob) {
    if ((unsigned)ix < (unsigned)P.dim[0] && (unsigned)iy < (unsigned)P.dim[1] && (unsigned)iz < (unsigned)P.dim[2])
        return ldg(P.edt + ((size_t)iz * P.dim[1] + iy) * P.dim[0] + ix);
    oob++;
    return D_brute(P, ix + P.lo[0], iy + P.lo[1], iz + P.lo[2]);
}

// D of the cell containing an FP64 point (global frame): floor(x / h) is
// floor(x * (1/h)) exactly because h is a power of two.
__device__ __forceinline__ long long D_exact(const PocketDev& P, double x, double y, double z, int& oob) {
    int cx = (int)floor(x * P.inv_h), cy = (int)floor(y * P.inv_h), cz = (int)floor(z * P.inv_h);
    return D_box(P, cx - P.lo[0], cy - P.lo[1], cz - P.lo[2], oob);
}

__device__ __forceinline__ double dist2(double ax, double ay, double az, double bx, double by, double bz) {
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    return dx * dx + dy * dy + dz * dz;
}

}  // namespace gd
