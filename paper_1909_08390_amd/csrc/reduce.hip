// Reductions over the cells of a grid (imexlb library, gfx950): the domain
// sums of mass, momentum and energy, the density loss 1/2 sum (n - n*)^2
// and the physical-state check.
//
// The step conserves the three sums on periodic grids: the MP-9 fluxes
// telescope (Sec. IV) and the BGK terms carry no mass, momentum or energy
// (Sec. III).  The sums are deterministic: each work-group owns a fixed
// contiguous range of cells and each lane a fixed strided subset of it; the
// 64 lanes of a wavefront combine by an xor butterfly of cross-lane
// shuffles, the four wavefronts of the work-group in index order through
// LDS, and the per-work-group partials in a second, single-work-group pass
// that reduces them the same way.
#include <climits>

#include "common.hpp"

namespace imexlb {
namespace {

constexpr int kRedThreads = 256;  // four wavefronts of 64 lanes
constexpr int kRedWaves = kRedThreads / 64;

// Sum over the 64 lanes of a wavefront.  Lanes i and i^m add the same two
// values at every level, so every lane ends with the same total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Work-group sums of NV per-lane values: thread t < NV writes total t to
// dst[t].
template <int NV>
__device__ __forceinline__ void group_sum(double (&s)[NV], double* dst) {
    __shared__ double red[NV][kRedWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = wave_sum(s[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[k][wave] = s[k];
    }
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        double t = red[threadIdx.x][0];
        for (int w = 1; w < kRedWaves; ++w) t += red[threadIdx.x][w];
        dst[threadIdx.x] = t;
    }
}

// Cells [beg, end) owned by this work-group.
__device__ __forceinline__ void block_range(long long cells, long long& beg, long long& end) {
    const long long per = (cells + gridDim.x - 1) / gridDim.x;
    beg = (long long)blockIdx.x * per;
    end = beg + per < cells ? beg + per : cells;
}

// Partial sums of mass n, momentum n u and total energy
// (D+K)/2 n T + n |u|^2 / 2 (Sec. II, Eq. Moments) from the moment fields
// M = (n, ux, [uy], T), field stride ms.
template <int D>
__global__ void __launch_bounds__(kRedThreads) sums_kernel(const double* __restrict__ M, long long ms,
                                                           long long cells, double dk, double* partial) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    long long beg, end;
    block_range(cells, beg, end);
    for (long long c = beg + threadIdx.x; c < end; c += kRedThreads) {
        const double n = M[c], ux = M[ms + c];
        const double uy = D == 2 ? M[2 * ms + c] : 0.0;
        const double T = M[(D + 1) * ms + c];
        s[0] += n;
        s[1] += n * ux;
        s[2] += n * uy;
        s[3] += 0.5 * dk * n * T + 0.5 * n * (ux * ux + uy * uy);
    }
    group_sum<4>(s, partial + (size_t)blockIdx.x * 4);
}

// Partial sums of 1/2 (n - n*)^2; the gradient n - n* per cell when grad is
// not NULL.
__global__ void __launch_bounds__(kRedThreads) loss_kernel(const double* __restrict__ n,
                                                           const double* __restrict__ target,
                                                           long long cells, double* grad, double* partial) {
    double s[1] = {0.0};
    long long beg, end;
    block_range(cells, beg, end);
    for (long long c = beg + threadIdx.x; c < end; c += kRedThreads) {
        const double r = n[c] - target[c];
        s[0] += 0.5 * r * r;
        if (grad) grad[c] = r;
    }
    group_sum<1>(s, partial + blockIdx.x);
}

// Sum of the nblocks partials (NV values each) into out[0 .. NV-1].
template <int NV>
__global__ void __launch_bounds__(kRedThreads) final_sum_kernel(const double* __restrict__ partial, int nblocks,
                                                                double* out) {
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kRedThreads) {
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += partial[(size_t)b * NV + k];
    }
    group_sum<NV>(s, out);
}

// flag = min(flag, code) if some cell has n <= 0, T <= 0 or a non-finite
// moment; one atomic per wavefront that found one.
template <int D>
__global__ void __launch_bounds__(256) check_kernel(const double* __restrict__ M, long long ms, long long cells,
                                                    int code, int* flag) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (c < cells) {
        for (int f = 0; f < D + 2; ++f) bad |= !isfinite(M[f * ms + c]);
        bad |= !(M[c] > 0.0) || !(M[(D + 1) * ms + c] > 0.0);
    }
    const unsigned long long m = __ballot(bad);
    if (m != 0ull && (int)(threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicMin(flag, code);
}

__global__ void set_flag_kernel(int* flag, int v) { *flag = v; }

}  // namespace

hipError_t launch_domain_sums(int d, const double* M, long long ms, long long cells, double dk, double* partial,
                              int nblocks, double* out4, hipStream_t s) {
    if (d == 2) hipLaunchKernelGGL((sums_kernel<2>), dim3(nblocks), dim3(kRedThreads), 0, s, M, ms, cells, dk, partial);
    else hipLaunchKernelGGL((sums_kernel<1>), dim3(nblocks), dim3(kRedThreads), 0, s, M, ms, cells, dk, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((final_sum_kernel<4>), dim3(1), dim3(kRedThreads), 0, s, partial, nblocks, out4);
    return hipGetLastError();
}

hipError_t launch_density_loss(const double* n, const double* target, long long cells, double* grad,
                               double* partial, int nblocks, double* out1, hipStream_t s) {
    hipLaunchKernelGGL(loss_kernel, dim3(nblocks), dim3(kRedThreads), 0, s, n, target, cells, grad, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((final_sum_kernel<1>), dim3(1), dim3(kRedThreads), 0, s, partial, nblocks, out1);
    return hipGetLastError();
}

hipError_t launch_check_reset(int* flag, hipStream_t s) {
    hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(1), 0, s, flag, INT_MAX);
    return hipGetLastError();
}

hipError_t launch_check(int d, const double* M, long long ms, long long cells, int code, int* flag, hipStream_t s) {
    const long long grid = (cells + 255) / 256;
    if (d == 2) hipLaunchKernelGGL((check_kernel<2>), dim3((unsigned)grid), dim3(256), 0, s, M, ms, cells, code, flag);
    else hipLaunchKernelGGL((check_kernel<1>), dim3((unsigned)grid), dim3(256), 0, s, M, ms, cells, code, flag);
    return hipGetLastError();
}

}  // namespace imexlb
