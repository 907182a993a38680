// Plain-copy probe of the achievable HBM rate (a measurement helper beside
// the stage kernels, not a step of the method).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "imexlb.h"

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte element per thread: the widest access per lane and the most
// requests in flight, the form that reached the highest copy rate on gfx950
// among grid-stride and unrolled variants.
__global__ void __launch_bounds__(256) copy16_kernel(const u32x4* __restrict__ a, u32x4* __restrict__ b,
                                                     unsigned long long n) {
    const unsigned long long i = (unsigned long long)blockIdx.x * 256u + threadIdx.x;
    if (i < n) b[i] = a[i];
}

}  // namespace

extern "C" imexlb_status imexlb_copy_probe(const void* d_src, void* d_dst, size_t bytes, int reps,
                                           void* hip_stream, double* gbs) {
    if (!d_src || !d_dst || !gbs || reps < 1) return IMEXLB_EINVAL;
    if (bytes == 0 || bytes % 16 != 0 || bytes > (size_t(1) << 40)) return IMEXLB_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_src) % 16 != 0 || reinterpret_cast<uintptr_t>(d_dst) % 16 != 0)
        return IMEXLB_EINVAL;
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(d_src), d0 = reinterpret_cast<uintptr_t>(d_dst);
    if (s0 < d0 + bytes && d0 < s0 + bytes) return IMEXLB_EINVAL;  // overlapping ranges
    const unsigned long long n = bytes / 16;
    const unsigned blocks = (unsigned)((n + 255) / 256);  // at most 2^28
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return IMEXLB_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return IMEXLB_EHIP;
    }
    imexlb_status st = IMEXLB_OK;
    float best = 0.0f;
    for (int r = 0; r <= reps && st == IMEXLB_OK; ++r) {  // r = 0: untimed warm-up
        float ms = 0.0f;
        if (hipEventRecord(e0, s) != hipSuccess) st = IMEXLB_EHIP;
        if (st == IMEXLB_OK) {
            copy16_kernel<<<blocks, 256, 0, s>>>(static_cast<const u32x4*>(d_src), static_cast<u32x4*>(d_dst), n);
            if (hipGetLastError() != hipSuccess) st = IMEXLB_EHIP;
        }
        if (st == IMEXLB_OK && hipEventRecord(e1, s) != hipSuccess) st = IMEXLB_EHIP;
        if (st == IMEXLB_OK && hipEventSynchronize(e1) != hipSuccess) st = IMEXLB_EHIP;
        if (st == IMEXLB_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = IMEXLB_EHIP;
        if (st == IMEXLB_OK && r > 0 && (best == 0.0f || ms < best)) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != IMEXLB_OK) return st;
    *gbs = best > 0.0f ? 2.0 * (double)bytes / ((double)best * 1e-3) / 1e9 : 0.0;
    return IMEXLB_OK;
}
