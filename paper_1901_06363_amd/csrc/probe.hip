// Measurement only (not part of the docking library): the achievable rate of
// random gathers from a small table that stays resident in the L2 caches, the
// reference peak for the kernels whose work is lookups in the distance grid
// (2-byte cells) and the density grid (4-byte nodes).  Every lane walks its
// own pseudo-random index sequences (a 32-bit linear congruential step per
// gather, 8 independent sequences for memory-level parallelism), adds the
// values it reads and writes one sum, so the only memory traffic besides the
// gathers is one 4-byte store per lane.  Built as its own library, loaded by
// bench.py.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;

template <class T>
__global__ void __launch_bounds__(256) gather_probe(const T* __restrict__ table, uint32_t mask, int iters,
                                                    uint32_t* __restrict__ out) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t x[kChains];
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; c++) x[c] = (tid * kChains + c) * 2654435761u + 12345u;
    const __attribute__((address_space(1))) T* tb = (const __attribute__((address_space(1))) T*)table;
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int c = 0; c < kChains; c++) {
            x[c] = x[c] * 1664525u + 1013904223u;
            acc += (uint32_t)tb[(x[c] >> 7) & mask];
        }
    }
    out[tid] = acc;
}

}  // namespace

extern "C" {

// Time `reps` launches of random gathers of 2-byte (elem_bytes 2) or 4-byte
// (4) elements from a table of 2^log2_elems elements: `blocks` blocks of 256
// lanes, iters * 8 gathers per lane.  Writes the mean kernel time (ms, HIP
// events on `stream`) and returns 0, or a HIP error code.
int gd_probe_gather(int elem_bytes, int log2_elems, int blocks, int iters, int reps, void* stream, float* ms_out) {
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)1 << log2_elems;
    void* table = nullptr;
    uint32_t* out = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&table, n * elem_bytes)) != hipSuccess) return (int)e;
    if ((e = hipMalloc(&out, (size_t)blocks * 256 * 4)) != hipSuccess) {
        (void)hipFree(table);
        return (int)e;
    }
    (void)hipMemsetAsync(table, 1, n * elem_bytes, s);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const uint32_t mask = (uint32_t)(n - 1);
    auto launch = [&]() {
        if (elem_bytes == 2)
            hipLaunchKernelGGL(gather_probe<uint16_t>, dim3(blocks), dim3(256), 0, s, (const uint16_t*)table, mask,
                               iters, out);
        else
            hipLaunchKernelGGL(gather_probe<uint32_t>, dim3(blocks), dim3(256), 0, s, (const uint32_t*)table, mask,
                               iters, out);
    };
    launch();  // warm-up: brings the table into the caches
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; r++) launch();
    (void)hipEventRecord(e1, s);
    e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) e = hipGetLastError();
    *ms_out = ms / (reps > 0 ? reps : 1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    (void)hipFree(table);
    return (int)e;
}

}  // extern "C"
