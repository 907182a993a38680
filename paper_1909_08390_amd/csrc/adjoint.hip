// Adjoint (reverse-mode) kernels of the IMEX-SSP3(4,3,3) step for gfx950.
//
// The reverse sweep through the stages of Table I (orchestrated by
// imexlb_adjoint_step in imexlb.cpp) needs four operations, each the
// transpose of a forward building block:
//   * materialise a stage value  F_i = a S_i + b E(M_i)   (relax on read, Sec. III);
//   * MP-9 advection transposed: dF = V^T dA, with V the flux difference of
//     Sec. IV.  A face value is linear in its nine upwind-biased nodes with
//     the weights of F^L unless the monotonicity test clips it; a clipped
//     face takes the derivative of the candidate the clip selected (F^min or
//     F^max, through the minmod selections).  Gather form: each cell sums
//     the contributions of the faces whose stencils read it (ghost nodes
//     route to the cell they copy);
//   * the equilibrium Jacobian transposed: dM = (dE/dM)^T dE per cell, with
//     dg/du = sum_l h_l l a_{l-1} and dg/dT = sum_l h_l l (l-1)/2 a_{l-2}
//     (Eq. gExpanded; the a_l are Appell polynomials in u with variance T-1);
//   * the moment Jacobian transposed: dF_v = dM . dM/dF_v (Sec. II,
//     Eq. Moments_discrete).
// All adjoint arrays are FP64 plane-sets F[v][cell] and FP64 moment sets
// M[field][cell] (d + 2 fields: n, u_x, [u_y], T).
#include "common.hpp"
#include "device.hpp"

namespace imexlb {
namespace {

constexpr int kAdjBlock = 256;

// Up to four FP64 plane-sets combined as sum_j c_j Y_j.
struct Lin4 {
    const double* y[4];
    double c[4];
    int n;
};

__device__ __forceinline__ double lin_at(const Lin4& L, size_t i) {
    double r = 0.0;
    for (int j = 0; j < L.n; ++j) r = fma(L.c[j], L.y[j][i], r);
    return r;
}

// g, dg/du, dg/dT of one axis factor (runtime order Q <= kQMax).
__device__ __forceinline__ void herm_factor_d(CDp h, int Q, double u, double th, double& g, double& gu,
                                              double& gT) {
    double am2 = 0.0, am1 = 0.0, a = 1.0;  // a_{l-2}, a_{l-1}, a_l
    g = 0.0;
    gu = 0.0;
    gT = 0.0;
    for (int l = 0; l < Q; ++l) {
        if (l == 1) {
            am2 = am1;
            am1 = a;
            a = u;
        } else if (l > 1) {
            const double an = fma(u, a, (double)(l - 1) * th * am1);
            am2 = am1;
            am1 = a;
            a = an;
        }
        g = fma(h[l], a, g);
        if (l >= 1) gu = fma(h[l] * (double)l, am1, gu);
        if (l >= 2) gT = fma(h[l] * (0.5 * l * (l - 1)), am2, gT);
    }
}

// ---------------------------------------------------- clipped-face derivative
// Index of the smallest / largest of four values, the first on ties (the
// order the forward's nested min / max resolves them).
__device__ __forceinline__ int argmin4(const double (&x)[4]) {
    int i = 0;
    if (x[1] < x[i]) i = 1;
    if (x[2] < x[i]) i = 2;
    if (x[3] < x[i]) i = 3;
    return i;
}
__device__ __forceinline__ int argmax4(const double (&x)[4]) {
    int i = 0;
    if (x[1] > x[i]) i = 1;
    if (x[2] > x[i]) i = 2;
    if (x[3] > x[i]) i = 3;
    return i;
}

// Four-argument minmod: the selected argument (0..3), or -1 for 0.
__device__ __forceinline__ int minmod4_sel(const double (&x)[4], double& val) {
    const int lo = argmin4(x), hi = argmax4(x);
    if (x[lo] > 0.0) {
        val = x[lo];
        return lo;
    }
    if (x[hi] < 0.0) {
        val = x[hi];
        return hi;
    }
    val = 0.0;
    return -1;
}

// d/d(w_k) of the curvatures C_{s-1}, C_s, C_{s+1} (w_4 = F_s).
__device__ __forceinline__ double dcurv(int j, int k) {  // C at node j: w_{j-1} - 2 w_j + w_{j+1}
    return (k == j - 1 ? 1.0 : 0.0) + (k == j ? -2.0 : 0.0) + (k == j + 1 ? 1.0 : 0.0);
}

// Component k of the gradient of the selected argument of
// minmod4(4 Ca - Cb, 4 Cb - Ca, Ca, Cb), curvatures at nodes ja, jb.
__device__ __forceinline__ double dminmod_arg(int sel, int ja, int jb, int k) {
    const double ga = dcurv(ja, k), gb = dcurv(jb, k);
    switch (sel) {
        case 0: return 4.0 * ga - gb;
        case 1: return 4.0 * gb - ga;
        case 2: return ga;
        case 3: return gb;
        default: return 0.0;
    }
}

// Weights of F^L on the nine nodes F_{s-4} .. F_{s+4} (Sec. IV), times 2520.
__device__ __forceinline__ double linear_weight(int k) {
    constexpr double c[9] = {4.0, -41.0, 199.0, -641.0, 1879.0, 1375.0, -305.0, 55.0, -5.0};
    return c[k] * (1.0 / 2520.0);
}

// d(face)/d(w[k]) for the upwind-first window w[0..8] (w[4] = F_s): the same
// decision as the forward (mp9_face_linear), the linear weights when the
// face is not clipped, else the derivative of the clip's selected branch
// (candidates F_s, F_{s+1}, MD, UL, LC; F^min / F^max by three-way min /
// max as in the forward).
__device__ double face_jacobian(const double (&w)[9], int k) {
    double dd[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) dd[j] = w[j + 1] - w[j];
    double t, q;
    const double fl = mp9_face_linear<double>(dd, w[4], t, q);
    if (!(q > 0.0)) return linear_weight(k);
    const double f = w[4], g = w[5], ul = f + t;
    const double cm = dd[3] - dd[2], c0 = dd[4] - dd[3], cp = dd[5] - dd[4];
    double vm, v0;
    const double am[4] = {fma(4.0, cm, -c0), fma(4.0, c0, -cm), cm, c0};
    const double a0[4] = {fma(4.0, c0, -cp), fma(4.0, cp, -c0), c0, cp};
    const int sm = minmod4_sel(am, vm);   // d^M4 at s - 1/2
    const int s0 = minmod4_sel(a0, v0);   // d^M4 at s + 1/2
    const double lc = fma(4.0 / 3.0, vm, fma(0.5, dd[3], f));
    const double md = fma(0.5, dd[4] - v0, f);
    // candidates: 0 f, 1 g, 2 md, 3 ul, 4 lc
    const double cv[5] = {f, g, md, ul, lc};
    auto pick_min3 = [&](int i, int j, int l) {  // fmin(fmin(x_i, x_j), x_l)
        int r = cv[j] < cv[i] ? j : i;
        return cv[l] < cv[r] ? l : r;
    };
    auto pick_max3 = [&](int i, int j, int l) {
        int r = cv[j] > cv[i] ? j : i;
        return cv[l] > cv[r] ? l : r;
    };
    const int a = pick_min3(0, 1, 2), b = pick_min3(0, 3, 4);
    const int lo = cv[b] > cv[a] ? b : a;
    const int c = pick_max3(0, 1, 2), e = pick_max3(0, 3, 4);
    const int hi = cv[e] < cv[c] ? e : c;
    int sel;
    if (fl < cv[lo]) sel = lo;
    else if (fl > cv[hi]) sel = hi;
    else return linear_weight(k);
    const double ek3 = k == 3 ? 1.0 : 0.0, ek4 = k == 4 ? 1.0 : 0.0, ek5 = k == 5 ? 1.0 : 0.0;
    switch (sel) {
        case 0: return ek4;                                               // F_s
        case 1: return ek5;                                               // F_{s+1}
        case 2: return 0.5 * ek4 + 0.5 * ek5 - 0.5 * dminmod_arg(s0, 4, 5, k);  // MD
        case 3: return 5.0 * ek4 - 4.0 * ek3;                             // UL
        default: return 1.5 * ek4 - 0.5 * ek3 + (4.0 / 3.0) * dminmod_arg(sm, 3, 4, k);  // LC
    }
}

// The whole row d(face)/d(w[0..8]) of one face: the limiter's decisions
// are taken once (as in face_jacobian), then all nine entries follow.
__device__ __forceinline__ void face_jacobian_row(const double (&w)[9], double (&J)[9]) {
    double dd[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) dd[j] = w[j + 1] - w[j];
    double t, q;
    const double fl = mp9_face_linear<double>(dd, w[4], t, q);
#pragma unroll
    for (int k = 0; k < 9; ++k) J[k] = linear_weight(k);
    if (!(q > 0.0)) return;
    const double f = w[4], g = w[5], ul = f + t;
    const double cm = dd[3] - dd[2], c0 = dd[4] - dd[3], cp = dd[5] - dd[4];
    double vm, v0;
    const double am[4] = {fma(4.0, cm, -c0), fma(4.0, c0, -cm), cm, c0};
    const double a0[4] = {fma(4.0, c0, -cp), fma(4.0, cp, -c0), c0, cp};
    const int sm = minmod4_sel(am, vm);
    const int s0 = minmod4_sel(a0, v0);
    const double lc = fma(4.0 / 3.0, vm, fma(0.5, dd[3], f));
    const double md = fma(0.5, dd[4] - v0, f);
    const double cv[5] = {f, g, md, ul, lc};
    auto pick_min3 = [&](int i, int j, int l) {
        int r = cv[j] < cv[i] ? j : i;
        return cv[l] < cv[r] ? l : r;
    };
    auto pick_max3 = [&](int i, int j, int l) {
        int r = cv[j] > cv[i] ? j : i;
        return cv[l] > cv[r] ? l : r;
    };
    const int a = pick_min3(0, 1, 2), b = pick_min3(0, 3, 4);
    const int lo = cv[b] > cv[a] ? b : a;
    const int c = pick_max3(0, 1, 2), e = pick_max3(0, 3, 4);
    const int hi = cv[e] < cv[c] ? e : c;
    int sel;
    if (fl < cv[lo]) sel = lo;
    else if (fl > cv[hi]) sel = hi;
    else return;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double ek3 = k == 3 ? 1.0 : 0.0, ek4 = k == 4 ? 1.0 : 0.0, ek5 = k == 5 ? 1.0 : 0.0;
        double r;
        switch (sel) {
            case 0: r = ek4; break;
            case 1: r = ek5; break;
            case 2: r = 0.5 * ek4 + 0.5 * ek5 - 0.5 * dminmod_arg(s0, 4, 5, k); break;
            case 3: r = 5.0 * ek4 - 4.0 * ek3; break;
            default: r = 1.5 * ek4 - 0.5 * ek3 + (4.0 / 3.0) * dminmod_arg(sm, 3, 4, k); break;
        }
        J[k] = r;
    }
}

// Adjoint contribution along one axis to node t of a line of n nodes
// (stride st): sum over the faces whose stencils read t (or a ghost node
// that copies t) of d(face)/d(node) * d(face), where d(face s) =
// p/ds (dA_s - dA_{s+1}) for the face between s and s+1 and dA is zero
// outside the line (outflow) or wraps (periodic).  FWD: p > 0 (window
// F_{s-4} .. F_{s+4}), else the mirrored window F_{s+5} .. F_{s-3}.
template <bool FWD>
__device__ double adj_axis_dir(const double* F, const Lin4& dA, size_t base, long long st, int n, int bc, int t,
                               double pinv) {
    int vlo = t, vhi = t;
    if (bc == 0) {
        if (t == 0) vlo = -5;
        if (t == n - 1) vhi = n + 4;
    }
    double acc = 0.0;
    for (int tv = vlo; tv <= vhi; ++tv) {
        double w17[17];  // nodes tv-8 .. tv+8
#pragma unroll
        for (int i = 0; i < 17; ++i) w17[i] = F[base + (size_t)bc_map(tv - 8 + i, n, bc) * st];
        double a10[10];  // dA at faces' nodes: FWD s = tv-4 .. tv+5, else s = tv-5 .. tv+4
#pragma unroll
        for (int i = 0; i < 10; ++i) {
            int j = (FWD ? tv - 4 : tv - 5) + i;
            double v = 0.0;
            if (bc == 0) {
                if (j >= 0 && j < n) v = lin_at(dA, base + (size_t)j * st);
            } else {
                v = lin_at(dA, base + (size_t)bc_map(j, n, 1) * st);
            }
            a10[i] = v;
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int s = FWD ? tv + 4 - k : tv - 5 + k;  // face between s and s+1
            if (bc == 0 && (s < -1 || s > n - 1)) continue;
            double fw[9];
#pragma unroll
            for (int kk = 0; kk < 9; ++kk) fw[kk] = w17[FWD ? 8 - k + kk : 8 + k - kk];
            const int ia = FWD ? 8 - k : k;  // a10 index of s
            const double dface = pinv * (a10[ia] - a10[ia + 1]);
            acc = fma(face_jacobian(fw, k), dface, acc);
        }
    }
    return acc;
}

__device__ __forceinline__ double adj_axis(const double* F, const Lin4& dA, size_t base, long long st, int n,
                                           int bc, int t, double p, double inv_ds) {
    if (p == 0.0) return 0.0;
    return p > 0.0 ? adj_axis_dir<true>(F, dA, base, st, n, bc, t, p * inv_ds)
                   : adj_axis_dir<false>(F, dA, base, st, n, bc, t, p * inv_ds);
}

// Face-major form along a line (used for y columns): the thread owns the
// kAdjSeg nodes t0 .. t0+kAdjSeg-1 and streams over the kAdjSeg + 8 faces whose
// stencils read them, each evaluated once with its whole Jacobian row (a
// face is evaluated (kAdjSeg + 8) / kAdjSeg times per node instead of nine).
// Positions p = 0 .. kAdjSeg+15 stand for node t0 - 8 + p; a rolling window
// holds F at the nine positions of the current face and a rolling
// accumulator their contributions, so the position leaving the window is
// complete.  Positions left / right of the segment are the ghost nodes of an
// outflow line (folded into its end nodes) or, on a periodic line, nodes of
// other segments (dropped here, counted there).
constexpr int kAdjSeg = 32;

template <bool FWD>
__device__ __forceinline__ void adj_stream(const double* F, const Lin4& dA, size_t base, long long st, int n,
                                           int bc, int t0, double pinv, double* out, int accumulate) {
    constexpr int L = kAdjSeg;
    auto fat = [&](int p) { return F[base + (size_t)bc_map(t0 - 8 + p, n, bc) * st]; };
    const int sa = t0 - (FWD ? 4 : 5);  // node s of face 0
    auto dat = [&](int q) {             // dA at node sa + q, zero outside an outflow line
        const int j = sa + q;
        if (bc == 1) return lin_at(dA, base + (size_t)bc_map(j, n, 1) * st);
        return (j >= 0 && j < n) ? lin_at(dA, base + (size_t)j * st) : 0.0;
    };
    auto emit = [&](int t, double val) {
        const size_t o = base + (size_t)t * st;
        __builtin_nontemporal_store(accumulate ? out[o] + val : val, out + o);
    };
    double w[9], r[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        w[k] = fat(k);
        r[k] = 0.0;
    }
    double a0 = dat(0), a1 = dat(1);
    double gl = 0.0, gend = 0.0;  // left ghosts; the last node of an outflow line and its ghosts
    const bool outflow = bc == 0;
#pragma unroll 1
    for (int f = 0; f < L + 8; ++f) {
        const double dface = pinv * (a0 - a1);
        double fw[9];
#pragma unroll
        for (int kk = 0; kk < 9; ++kk) fw[kk] = w[FWD ? kk : 8 - kk];
        double J[9];
        face_jacobian_row(fw, J);
#pragma unroll
        for (int kk = 0; kk < 9; ++kk) r[FWD ? kk : 8 - kk] = fma(J[kk], dface, r[FWD ? kk : 8 - kk]);
        // position f is complete
        const double val = r[0];
        if (f < 8) {
            gl += val;
        } else {
            const int t = t0 + f - 8;
            if (outflow && t >= n - 1) {
                gend += val;
            } else if (t < n) {
                emit(t, (outflow && t == 0) ? val + gl : val);
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            r[k] = r[k + 1];
            w[k] = w[k + 1];
        }
        r[8] = 0.0;
        if (f + 1 < L + 8) {
            w[8] = fat(f + 9);
            a0 = a1;
            a1 = dat(f + 2);
        }
    }
    if (outflow && n - 1 >= t0 && n - 1 < t0 + L) {  // this segment holds the last node
        double g = gend;
#pragma unroll
        for (int k = 1; k < 9; ++k) g += r[k - 1];  // positions L+8 .. L+15, shifted once
        emit(n - 1, (n - 1 == 0) ? g + gl : g);
    }
}

// x lines, wave-cooperative: one wavefront per chunk of kChunk nodes of a
// row, kChunkWaves chunks per work-group.  Lane l evaluates face
// s = c0 - 4 + l (flow to +x; else c0 - 5 + l), the 64 faces whose stencils
// read the chunk's nodes, with coalesced window loads, and writes its nine
// weighted Jacobian entries to LDS; node c0 + i then gathers the nine
// entries addressed to it (from lanes i + 8 - k, or i + k for flow to -x).
// The end nodes of an outflow row also collect the entries at ghost
// positions.
constexpr int kChunk = 56;

__device__ __forceinline__ int chunk_pos(bool fwd, int c0, int lane, int kk) {  // node index written by (lane, kk)
    return fwd ? c0 - 8 + lane + kk : c0 + lane - kk;
}

// Chunks per work-group of the x-row kernel: one per wavefront.
constexpr int kChunkWaves = 4;

__global__ void __launch_bounds__(64 * kChunkWaves) advect_adjoint_xchunk_kernel(const DevTables* __restrict__ tabp,
                                                                                 const double* __restrict__ F,
                                                                                 Lin4 dA, double* out, int nx, int ny,
                                                                                 int bc, double inv_dx,
                                                                                 int accumulate) {
    // per wavefront: F at nodes c0-8 .. c0+63, dA at c0-5 .. c0+66, and the
    // 9 x 64 weighted Jacobian entries of its faces
    __shared__ double contrib_all[kChunkWaves][9 * 64];
    __shared__ double sF_all[kChunkWaves][72], sA_all[kChunkWaves][72];
    CTab* tab = (CTab*)tabp;
    const long long cells = (long long)nx * ny;
    const int v = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, n = nx;
    double* contrib = contrib_all[wave];
    double* sF = sF_all[wave];
    double* sA = sA_all[wave];
    const int nch = (nx + kChunk - 1) / kChunk;
    const long long chunk = (long long)blockIdx.x * kChunkWaves + wave;
    // a wavefront past the last chunk still takes part in the barriers
    const bool live = chunk < (long long)nch * ny;
    const int y = live ? (int)(chunk / nch) : 0, c0 = live ? (int)(chunk % nch) * kChunk : 0;
    const size_t base = (size_t)v * cells + (size_t)y * nx;
    const double p = tab->plane[v].px;  // one plane per work-group
    const int t = c0 + lane;
    if (p == 0.0) {
        if (live && !accumulate && lane < kChunk && t < n) out[base + t] = 0.0;
        return;
    }
    const bool fwd = p > 0.0;
    // the chunk's windows, read once into LDS (coalesced)
    auto dat = [&](int j) {
        if (bc == 1) return lin_at(dA, base + (size_t)bc_map(j, n, 1));
        return (j >= 0 && j < n) ? lin_at(dA, base + (size_t)j) : 0.0;
    };
    if (live) {
        for (int i = lane; i < 72; i += 64) {
            sF[i] = F[base + bc_map(c0 - 8 + i, n, bc)];
            sA[i] = dat(c0 - 5 + i);
        }
    }
    __syncthreads();
    // face s = c0 - 4 + lane (flow to +x) or c0 - 5 + lane: window nodes
    // s - 4 + kk = c0 - 8 + lane + kk, or s + 5 - kk = c0 + lane - kk
    if (live) {
        double w[9];
#pragma unroll
        for (int kk = 0; kk < 9; ++kk) w[kk] = sF[fwd ? lane + kk : lane + 8 - kk];
        const int ia = lane + (fwd ? 1 : 0);  // sA index of node s
        const double dface = p * inv_dx * (sA[ia] - sA[ia + 1]);
        double J[9];
        face_jacobian_row(w, J);
#pragma unroll
        for (int kk = 0; kk < 9; ++kk) contrib[kk * 64 + lane] = J[kk] * dface;
    }
    __syncthreads();
    if (live && lane < kChunk && t < n) {
        double val = 0.0;
#pragma unroll
        for (int kk = 0; kk < 9; ++kk) val += contrib[kk * 64 + (fwd ? lane + 8 - kk : lane + kk)];
        if (bc == 0 && (t == 0 || t == n - 1)) {  // ghost positions copy the end nodes
            for (int l = 0; l < 64; ++l)
                for (int kk = 0; kk < 9; ++kk) {
                    const int j = chunk_pos(fwd, c0, l, kk);
                    if ((t == 0 && j < 0) || (t == n - 1 && j > n - 1)) val += contrib[kk * 64 + l];
                }
        }
        const size_t o = base + (size_t)t;
        __builtin_nontemporal_store(accumulate ? out[o] + val : val, out + o);
    }
}

// y lines: thread per segment of a column, adjacent lanes on adjacent
// columns (coalesced), out[v][c] += the y contribution.
__global__ void __launch_bounds__(kAdjBlock) advect_adjoint_ycol_kernel(const DevTables* __restrict__ tabp,
                                                                        const double* __restrict__ F, Lin4 dA,
                                                                        double* out, int nx, int ny, int bc,
                                                                        double inv_dy) {
    constexpr int L = kAdjSeg;
    CTab* tab = (CTab*)tabp;
    const long long cells = (long long)nx * ny;
    const int v = blockIdx.y;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nseg = (ny + L - 1) / L;
    if (i >= (long long)nseg * nx) return;
    const int t0 = (int)(i / nx) * L;
    const size_t base = (size_t)v * cells + (size_t)(i % nx);
    const double p = tab->plane[v].py;
    if (p > 0.0) adj_stream<true>(F, dA, base, nx, ny, bc, t0, p * inv_dy, out, 1);
    else if (p < 0.0) adj_stream<false>(F, dA, base, nx, ny, bc, t0, p * inv_dy, out, 1);
}

// out[v][c] (=|+=) V^T dA at every node, both axes in 2D.
template <int D>
__global__ void __launch_bounds__(kAdjBlock) advect_adjoint_kernel(const DevTables* __restrict__ tabp,
                                                                   const double* __restrict__ F, Lin4 dA,
                                                                   double* out, int nx, int ny, int bcx,
                                                                   int bcy, double inv_dx, double inv_dy,
                                                                   int accumulate) {
    CTab* tab = (CTab*)tabp;
    const long long cells = (long long)nx * ny;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (c >= cells) return;
    const double px = tab->plane[v].px, py = tab->plane[v].py;
    const int x = (int)(c % nx), y = (int)(c / nx);
    const size_t pl = (size_t)v * cells;
    double r = adj_axis(F, dA, pl + (size_t)y * nx, 1, nx, bcx, x, px, inv_dx);
    if (D == 2) r += adj_axis(F, dA, pl + (size_t)x, nx, ny, bcy, y, py, inv_dy);
    out[pl + c] = accumulate ? out[pl + c] + r : r;
}

// out = a src + b E(M) as FP64 (stage value rebuilt from its moments).
template <typename S, int D>
__global__ void __launch_bounds__(kAdjBlock) materialise_kernel(const DevTables* __restrict__ tabp,
                                                                const S* __restrict__ src,
                                                                const double* __restrict__ M, double a,
                                                                double b, double* out, long long cells,
                                                                double chi_fac) {
    CTab* tab = (CTab*)tabp;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const double nn = M[c], u = M[cells + c], w = D == 2 ? M[2 * cells + c] : 0.0;
    const double th = M[(D + 1) * cells + c] - 1.0;
    int v = 0;
    for (int set = 0; set < 2; ++set) {
        const int Q = tab->q[set];
        const double pre = set ? chi_fac * nn * (th + 1.0) : nn;
        for (int ky = 0; ky < (D == 2 ? Q : 1); ++ky) {
            const double gy = D == 2 ? pre * herm_factor(tab->h[set][ky], Q, w, th) : pre;
            for (int kx = 0; kx < Q; ++kx, ++v) {
                const size_t i = (size_t)v * cells + c;
                out[i] = fma(a, (double)src[i], b * gy * herm_factor(tab->h[set][kx], Q, u, th));
            }
        }
    }
}

// dM = (dE/dM)^T dE per cell, dE = sum_j c_j Y_j.  Moments (n, u, T) of M.
// The x factors (and their u and T derivatives) of the QM or fewer nodes of
// a set are evaluated once per cell and set, then reused by every y group.
template <int D, int QM>
__global__ void __launch_bounds__(kAdjBlock) eq_adjoint_kernel(const DevTables* __restrict__ tabp,
                                                               const double* __restrict__ M, Lin4 dE,
                                                               double* dM, long long cells, double chi_fac) {
    CTab* tab = (CTab*)tabp;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const double nn = M[c], u = M[cells + c], w = D == 2 ? M[2 * cells + c] : 0.0;
    const double T = M[(D + 1) * cells + c], th = T - 1.0;
    double dn = 0.0, dux = 0.0, duy = 0.0, dT = 0.0;
    int v = 0;
    for (int set = 0; set < 2; ++set) {
        const int Q = tab->q[set];
        const double pre = set ? chi_fac * nn * T : nn;       // P_phi = n, P_chi = (K+D-d) n T
        const double pre_n = set ? chi_fac * T : 1.0;
        const double pre_T = set ? chi_fac * nn : 0.0;
        double gx[QM], gxu[QM], gxT[QM];
#pragma unroll
        for (int kx = 0; kx < QM; ++kx) {
            gx[kx] = 0.0;
            gxu[kx] = 0.0;
            gxT[kx] = 0.0;
            if (kx < Q) herm_factor_d(tab->h[set][kx], Q, u, th, gx[kx], gxu[kx], gxT[kx]);
        }
        for (int ky = 0; ky < (D == 2 ? Q : 1); ++ky) {
            double gy = 1.0, gyu = 0.0, gyT = 0.0;
            if (D == 2) herm_factor_d(tab->h[set][ky], Q, w, th, gy, gyu, gyT);
#pragma unroll
            for (int kx = 0; kx < QM; ++kx) {
                if (kx < Q) {
                    const double e = lin_at(dE, (size_t)(v + kx) * cells + c);
                    dn = fma(e, pre_n * gx[kx] * gy, dn);
                    dux = fma(e, pre * gxu[kx] * gy, dux);
                    if (D == 2) duy = fma(e, pre * gx[kx] * gyu, duy);
                    dT = fma(e, pre_T * gx[kx] * gy + pre * (gxT[kx] * gy + gx[kx] * gyT), dT);
                }
            }
            v += Q;
        }
    }
    dM[c] = dn;
    dM[cells + c] = dux;
    if (D == 2) dM[2 * cells + c] = duy;
    dM[(D + 1) * cells + c] = dT;
}

// out (=|+=) sum_j c_j Y_j + (dM/dF)^T dM per plane (dM may be NULL).
// n = sum_phi F, n u = sum_phi p F, (D+K) n T = sum_phi |p|^2 F + sum_chi F - n |u|^2:
//   dn/dF = [phi], du/dF = [phi] (p - u)/n,
//   dT/dF = ([phi] |p - u|^2 + [chi]) / ((D+K) n) - [phi] T / n.
template <int D>
__global__ void __launch_bounds__(kAdjBlock) mom_adjoint_kernel(const DevTables* __restrict__ tabp,
                                                                const double* __restrict__ M,
                                                                const double* __restrict__ dM, Lin4 Y,
                                                                double* out, long long cells, double dk,
                                                                int accumulate) {
    CTab* tab = (CTab*)tabp;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    double nn = 1.0, u = 0.0, w = 0.0, T = 0.0, gn = 0.0, gu = 0.0, gw = 0.0, gT = 0.0;
    if (dM) {
        nn = M[c];
        u = M[cells + c];
        w = D == 2 ? M[2 * cells + c] : 0.0;
        T = M[(D + 1) * cells + c];
        gn = dM[c];
        gu = dM[cells + c];
        gw = D == 2 ? dM[2 * cells + c] : 0.0;
        gT = dM[(D + 1) * cells + c];
    }
    const double inv_n = 1.0 / nn, inv_dkn = 1.0 / (dk * nn);
    const int np = tab->nplanes;
    for (int v = 0; v < np; ++v) {
        const size_t i = (size_t)v * cells + c;
        double r = lin_at(Y, i);
        if (dM) {
            const double px = tab->plane[v].px, py = tab->plane[v].py;
            if (tab->plane[v].set == 0) {
                const double ex = px - u, ey = py - w;
                r += gn + (gu * ex + gw * ey) * inv_n + gT * ((ex * ex + ey * ey) * inv_dkn - T * inv_n);
            } else {
                r += gT * inv_dkn;
            }
        }
        out[i] = accumulate ? out[i] + r : r;
    }
}

Lin4 make_lin(int n, const double* const* y, const double* cf) {
    Lin4 L;
    L.n = n;
    for (int j = 0; j < 4; ++j) {
        L.y[j] = j < n ? y[j] : nullptr;
        L.c[j] = j < n ? cf[j] : 0.0;
    }
    return L;
}

}  // namespace

hipError_t launch_materialise(int d, bool f32, const DevTables* tab, const void* src, const double* M,
                              double a, double b, double* out, long long cells, double chi_fac,
                              hipStream_t s) {
    const int grid = (int)((cells + kAdjBlock - 1) / kAdjBlock);
    if (d == 2) {
        if (f32) hipLaunchKernelGGL((materialise_kernel<float, 2>), dim3(grid), dim3(kAdjBlock), 0, s, tab, (const float*)src, M, a, b, out, cells, chi_fac);
        else hipLaunchKernelGGL((materialise_kernel<double, 2>), dim3(grid), dim3(kAdjBlock), 0, s, tab, (const double*)src, M, a, b, out, cells, chi_fac);
    } else {
        if (f32) hipLaunchKernelGGL((materialise_kernel<float, 1>), dim3(grid), dim3(kAdjBlock), 0, s, tab, (const float*)src, M, a, b, out, cells, chi_fac);
        else hipLaunchKernelGGL((materialise_kernel<double, 1>), dim3(grid), dim3(kAdjBlock), 0, s, tab, (const double*)src, M, a, b, out, cells, chi_fac);
    }
    return hipGetLastError();
}

hipError_t launch_advect_adjoint(int d, const DevTables* tab, int nplanes, const double* F, int ny_in,
                                 const double* const* y, const double* cf, double* out, int nx, int ny,
                                 int bcx, int bcy, double inv_dx, double inv_dy, bool accumulate,
                                 hipStream_t s) {
    const Lin4 L = make_lin(ny_in, y, cf);
    const long long cells = (long long)nx * ny;
    // Face-major forms: x rows in 64-face chunks, y columns in streamed
    // segments.  They need periodic lines of at least kAdjSeg + 8 nodes (on a
    // shorter ring a segment's face range, or a face's window, would hold one
    // node twice); shorter periodic lines take the gather form.
    const bool short_ring = (bcx == 1 && nx < kAdjSeg + 8) || (d == 2 && bcy == 1 && ny < kAdjSeg + 8);
    if (short_ring) {
        const dim3 grid((unsigned)((cells + kAdjBlock - 1) / kAdjBlock), (unsigned)nplanes);
        if (d == 2)
            hipLaunchKernelGGL((advect_adjoint_kernel<2>), grid, dim3(kAdjBlock), 0, s, tab, F, L, out, nx, ny, bcx, bcy, inv_dx, inv_dy, (int)accumulate);
        else
            hipLaunchKernelGGL((advect_adjoint_kernel<1>), grid, dim3(kAdjBlock), 0, s, tab, F, L, out, nx, 1, bcx, 0, inv_dx, 0.0, (int)accumulate);
        return hipGetLastError();
    }
    const int nyl = d == 2 ? ny : 1;
    const long long chx = (long long)((nx + kChunk - 1) / kChunk) * nyl;
    const long long gx = (chx + kChunkWaves - 1) / kChunkWaves;
    hipLaunchKernelGGL(advect_adjoint_xchunk_kernel, dim3((unsigned)gx, (unsigned)nplanes), dim3(64 * kChunkWaves), 0, s,
                       tab, F, L, out, nx, nyl, bcx, inv_dx, (int)accumulate);
    if (d == 2) {
        const long long segy = (long long)((ny + kAdjSeg - 1) / kAdjSeg) * nx;
        const dim3 gy((unsigned)((segy + kAdjBlock - 1) / kAdjBlock), (unsigned)nplanes);
        hipLaunchKernelGGL(advect_adjoint_ycol_kernel, gy, dim3(kAdjBlock), 0, s, tab, F, L, out, nx, ny, bcy, inv_dy);
    }
    return hipGetLastError();
}

hipError_t launch_eq_adjoint(int d, int qm, const DevTables* tab, const double* M, int ny_in,
                             const double* const* y, const double* cf, double* dM, long long cells,
                             double chi_fac, hipStream_t s) {
    const Lin4 L = make_lin(ny_in, y, cf);
    const int grid = (int)((cells + kAdjBlock - 1) / kAdjBlock);
    if (d == 2) {
        if (qm == 8) hipLaunchKernelGGL((eq_adjoint_kernel<2, 8>), dim3(grid), dim3(kAdjBlock), 0, s, tab, M, L, dM, cells, chi_fac);
        else hipLaunchKernelGGL((eq_adjoint_kernel<2, 16>), dim3(grid), dim3(kAdjBlock), 0, s, tab, M, L, dM, cells, chi_fac);
    } else {
        if (qm == 8) hipLaunchKernelGGL((eq_adjoint_kernel<1, 8>), dim3(grid), dim3(kAdjBlock), 0, s, tab, M, L, dM, cells, chi_fac);
        else hipLaunchKernelGGL((eq_adjoint_kernel<1, 16>), dim3(grid), dim3(kAdjBlock), 0, s, tab, M, L, dM, cells, chi_fac);
    }
    return hipGetLastError();
}

hipError_t launch_mom_adjoint(int d, const DevTables* tab, const double* M, const double* dM, int ny_in,
                              const double* const* y, const double* cf, double* out, long long cells,
                              double dk, bool accumulate, hipStream_t s) {
    const Lin4 L = make_lin(ny_in, y, cf);
    const int grid = (int)((cells + kAdjBlock - 1) / kAdjBlock);
    if (d == 2) hipLaunchKernelGGL((mom_adjoint_kernel<2>), dim3(grid), dim3(kAdjBlock), 0, s, tab, M, dM, L, out, cells, dk, (int)accumulate);
    else hipLaunchKernelGGL((mom_adjoint_kernel<1>), dim3(grid), dim3(kAdjBlock), 0, s, tab, M, dM, L, out, cells, dk, (int)accumulate);
    return hipGetLastError();
}

}  // namespace imexlb
