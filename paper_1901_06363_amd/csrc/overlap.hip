// Eq. 1 without the lattice (Section III-A): every atom's smallest squared
// distance to the pocket's points, then per pose the sum over its atoms in
// index order and the overlap o = l / sum.  The brute-force O(l p) form of the
// paper's overlap measure, in FP64.
//
// Layout: the points live on the device as three FP64 planes (x, y, z) of
// `pitch` doubles each, padded to a multiple of kOvUnroll with far points
// (1e150 per axis: their squared distance to any finite atom exceeds that of
// every real point).  Lanes own atoms (kOvAtoms per lane, consecutive blocks of
// the flattened pose rows, coalesced FP32 loads); every wave walks the same
// point sequence, so the point reads are wave-uniform scalar loads and each
// point feeds 64 x kOvAtoms distance evaluations from registers.  The bound is
// FP64 VALU issue: per pair 3 subtractions, a multiply, two fused
// multiply-adds and a minimum.
#include <hip/hip_runtime.h>

#include <math.h>

#include "gd_internal.h"

namespace gd {

constexpr int kOvBlock = 256;  // threads per block
constexpr int kOvAtoms = 2;    // atoms per lane

__global__ void __launch_bounds__(kOvBlock) overlap_min_kernel(const double* __restrict__ pts, int n_pad, int pitch,
                                                              const float* __restrict__ px,
                                                              const float* __restrict__ py,
                                                              const float* __restrict__ pz, int64_t n_atoms,
                                                              double* __restrict__ min_out) {
    const int64_t base = (int64_t)blockIdx.x * (kOvBlock * kOvAtoms) + threadIdx.x;
    double ax[kOvAtoms], ay[kOvAtoms], az[kOvAtoms], best[kOvAtoms];
#pragma unroll
    for (int k = 0; k < kOvAtoms; k++) {
        const int64_t i = base + (int64_t)k * kOvBlock;
        const bool ok = i < n_atoms;
        ax[k] = ok ? (double)px[i] : 0.0;
        ay[k] = ok ? (double)py[i] : 0.0;
        az[k] = ok ? (double)pz[i] : 0.0;
        best[k] = HUGE_VAL;
    }
    const double* qx = pts;
    const double* qy = pts + pitch;
    const double* qz = pts + 2 * (size_t)pitch;
    for (int j = 0; j < n_pad; j += kOvUnroll) {
#pragma unroll
        for (int u = 0; u < kOvUnroll; u++) {
            const double x = qx[j + u], y = qy[j + u], z = qz[j + u];
#pragma unroll
            for (int k = 0; k < kOvAtoms; k++) {
                const double dx = ax[k] - x, dy = ay[k] - y, dz = az[k] - z;
                best[k] = fmin(best[k], fma(dz, dz, fma(dy, dy, dx * dx)));
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kOvAtoms; k++) {
        const int64_t i = base + (int64_t)k * kOvBlock;
        if (i < n_atoms) min_out[i] = best[k];
    }
}

// One thread per pose: the in-order sum of its atoms' minima and l / sum.
// Offsets are clamped to [0, n_atoms] so that a malformed offset array never
// reads outside the minima.
__global__ void __launch_bounds__(kOvBlock) overlap_sum_kernel(const int32_t* __restrict__ pose_off, int n_poses,
                                                              int64_t n_atoms, const double* __restrict__ min_d2,
                                                              double* __restrict__ sum_out,
                                                              double* __restrict__ o_out) {
    const int p = blockIdx.x * kOvBlock + threadIdx.x;
    if (p >= n_poses) return;
    const int64_t a = min((int64_t)max(pose_off[p], 0), n_atoms);
    const int64_t b = max(a, min((int64_t)pose_off[p + 1], n_atoms));
    double s = 0.0;
    for (int64_t i = a; i < b; i++) s += min_d2[i];
    sum_out[p] = s;
    if (o_out) o_out[p] = (double)(b - a) / s;
}

hipError_t launch_overlap(const double* pts, int n_pad, int pitch, const int32_t* pose_off, int n_poses,
                          const float* px, const float* py, const float* pz, int64_t n_atoms, double* min_out,
                          double* sum_out, double* o_out, hipStream_t s) {
    if (n_atoms > 0) {
        const int64_t per_block = (int64_t)kOvBlock * kOvAtoms;
        const int64_t blocks = (n_atoms + per_block - 1) / per_block;
        overlap_min_kernel<<<dim3((unsigned)blocks), dim3(kOvBlock), 0, s>>>(pts, n_pad, pitch, px, py, pz, n_atoms,
                                                                            min_out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_poses > 0) {
        overlap_sum_kernel<<<dim3((n_poses + kOvBlock - 1) / kOvBlock), dim3(kOvBlock), 0, s>>>(
            pose_off, n_poses, n_atoms, min_out, sum_out, o_out);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace gd
