// Allocation-free domain sums (imexlb library, gfx950) for callers that
// cannot allocate device memory: code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc.  Same kernels and results as
// imexlb_domain_sums.
#include <cstdio>
#include <mutex>

#include "common.hpp"
#include "imexlb.h"

// ---------------------------------------------------------------------------
// Domain sums that allocate nothing (imexlb_domain_sums_noalloc): the
// per-work-group partials live in this file-scope device array instead of
// library-allocated memory.  Each GPU holds its own copy until the process
// ends; host code reaches it only through the device address returned by
// hipGetSymbolAddress, looked up once per device.
// ---------------------------------------------------------------------------
namespace imexlb {

// Partials of the kSumBlocks work-groups of the sums: 32 KiB per GPU.
static __device__ __align__(256) double scratch[kSumBlocks * 4];

namespace {

constexpr long long kNoAllocMaxCells = (1LL << 31) - 1;  // the library's cell limit
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (nullptr and the error on failure).
hipError_t scratch_on_current_device(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace imexlb

extern "C" imexlb_status imexlb_domain_sums_noalloc(int d, int K, const double* d_M, long long cells,
                                                    double* d_out, void* hip_stream) {
    using namespace imexlb;
    if (d != 1 && d != 2) {
        std::fprintf(stderr, "imexlb_domain_sums_noalloc: d must be 1 or 2 (got %d)\n", d);
        return IMEXLB_EINVAL;
    }
    if (K < 0 || !d_M || !d_out) {
        std::fprintf(stderr, "imexlb_domain_sums_noalloc: K < 0 or a NULL buffer\n");
        return IMEXLB_EINVAL;
    }
    if (cells < 1 || cells > kNoAllocMaxCells) {
        std::fprintf(stderr, "imexlb_domain_sums_noalloc: cells = %lld outside [1, %lld]\n", cells,
                     kNoAllocMaxCells);
        return IMEXLB_EINVAL;
    }
    double* part = nullptr;
    hipError_t e = scratch_on_current_device(&part);
    if (e == hipSuccess)
        e = launch_domain_sums(d, d_M, cells, cells, (double)(kDTotal + K), part, kSumBlocks, d_out,
                               (hipStream_t)hip_stream);
    if (e != hipSuccess) {
        std::fprintf(stderr, "imexlb_domain_sums_noalloc: %s\n", hipGetErrorString(e));
        return IMEXLB_EHIP;
    }
    return IMEXLB_OK;
}
