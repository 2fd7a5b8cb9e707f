// Exact scoring of given FP32 poses: the overlap count S of Eq. 1 on the
// lattice and the whole-ligand bump flag (Section III-B).  For FP32 inputs
// the cell floor(x/h) is exact in FP32 (h a power of two), and the pair
// distances are formed in FP64 from the widened coordinates.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_common.h"
#include "gd_internal.h"

namespace gd {

// one wave per pose; lanes over atoms, then over the ligand's far pairs
__global__ void __launch_bounds__(256) score_kernel(PocketDev P, ScoreDev Sd, int n_poses, double cd2, int32_t* S_out,
                                                    uint8_t* clash_out) {
    const int lane = lane_id();
    const int pose = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (pose >= n_poses) return;
    const int lig = Sd.pose_lig[pose];
    const int off = Sd.pose_off[pose];
    const int l = Sd.n_atoms[lig];
    const float inv_h = (float)P.inv_h;
    int oob = 0;
    long long s = 0;
    for (int i = lane; i < l; i += kWave) {
        int cx = (int)floorf(Sd.px[off + i] * inv_h) - P.lo[0];
        int cy = (int)floorf(Sd.py[off + i] * inv_h) - P.lo[1];
        int cz = (int)floorf(Sd.pz[off + i] * inv_h) - P.lo[2];
        s += D_box(P, cx, cy, cz, oob);
    }
    s = wave_sum64(s);
    bool c = false;
    const uint16_t* fp = Sd.efar + Sd.far_off[lig];
    const int nf = Sd.n_far[lig];
    for (int q = lane; q < nf; q += kWave) {
        uint16_t pr = fp[q];
        int i = off + (pr & 0xff), j = off + (pr >> 8);
        c |= dist2((double)Sd.px[i], (double)Sd.py[i], (double)Sd.pz[i], (double)Sd.px[j], (double)Sd.py[j],
                   (double)Sd.pz[j]) < cd2;
    }
    c = __ballot(c) != 0;
    if (lane == 0) {
        S_out[pose] = sat_S(s);
        clash_out[pose] = (uint8_t)c;
    }
}

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free scoring call: one static array per
// device the library runs on (each holds it until the process ends).  Host
// code must not use the array's name as a device address; the per-device
// address comes from hipGetSymbolAddress, taken once per device with that
// device current.

static __device__ __align__(256) uint8_t scratch[kNoAllocScratch];

hipError_t noalloc_scratch(void** out) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_score(const PocketDev& P, const ScoreDev& S, int n_poses, double cd2, int32_t* S_out,
                        uint8_t* clash_out, hipStream_t s) {
    if (n_poses <= 0) return hipSuccess;
    const int waves = 4;
    hipLaunchKernelGGL(score_kernel, dim3((n_poses + waves - 1) / waves), dim3(waves * kWave), 0, s, P, S, n_poses,
                       cd2, S_out, clash_out);
    return hipGetLastError();
}

}  // namespace gd
