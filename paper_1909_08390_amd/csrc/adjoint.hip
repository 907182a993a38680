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
//     F^max, through the minmod selections).  A node sums the contributions
//     of the faces whose stencils read it (ghost nodes route to the node
//     they copy): in 2D one tiled kernel for both axes, in 1D a row kernel
//     with one face per lane;
//   * the equilibrium Jacobian transposed: dM = (dE/dM)^T dE per cell, with
//     dg/du = sum_l h_l l a_{l-1} and dg/dT = sum_l h_l l (l-1)/2 a_{l-2}
//     (Eq. gExpanded; the a_l are Appell polynomials in u with variance T-1);
//   * the moment Jacobian transposed: dF_v = dM . dM/dF_v (Sec. II,
//     Eq. Moments_discrete).
// Adjoint plane-sets F[v][cell] between the kernels are held in the storage
// type (the adjoint of the following step, lam^{n+1}, in FP64), moment sets
// M[field][cell] (d + 2 fields: n, u_x, [u_y], T) in FP64; all arithmetic is
// FP64.
#include "common.hpp"
#include "device.hpp"

namespace imexlb {
namespace {

constexpr int kAdjBlock = 256;

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
// Selected argument of the four-argument minmod, as the weights (al, be) of
// the two curvatures a, b in it: 4a - b -> (4, -1), 4b - a -> (-1, 4),
// a -> (1, 0), b -> (0, 1), 0 -> (0, 0).  The smallest / largest argument is
// the first one on ties, the order the forward's nested min / max resolves
// them.  The comparisons run in the precision R of the forward's sweep.
template <typename R>
__device__ __forceinline__ void minmod4_weights(R a, R b, double& al, double& be) {
    const R x0 = fma(R(4), a, -b), x1 = fma(R(4), b, -a);
    // argmin and argmax over (x0, x1, a, b), first on ties
    R vmin = x0, vmax = x0;
    double amin = 4.0, bmin = -1.0, amax = 4.0, bmax = -1.0;
    if (x1 < vmin) { vmin = x1; amin = -1.0; bmin = 4.0; }
    if (a < vmin) { vmin = a; amin = 1.0; bmin = 0.0; }
    if (b < vmin) { vmin = b; amin = 0.0; bmin = 1.0; }
    if (x1 > vmax) { vmax = x1; amax = -1.0; bmax = 4.0; }
    if (a > vmax) { vmax = a; amax = 1.0; bmax = 0.0; }
    if (b > vmax) { vmax = b; amax = 0.0; bmax = 1.0; }
    const bool pos = vmin > R(0), neg = vmax < R(0);
    al = pos ? amin : (neg ? amax : 0.0);
    be = pos ? bmin : (neg ? bmax : 0.0);
}

// The Jacobian row d(face)/d(w[0..8]) of one face, upwind-first window w
// (w[4] = F_s, w[5] = F_{s+1}), with the forward's decisions: the linear
// weights of F^L (Sec. IV) unless the monotonicity test fails and F^L lies
// outside [F^min, F^max]; then the derivative of the bound it is clipped
// to, i.e. of the candidate that bound selected (F_s, F_{s+1}, F^MD, F^UL
// or F^LC; three-way min / max first on ties).  The candidates are linear
// in w apart from the M4 limits, whose selected arguments are linear in the
// curvatures C_{s-1}, C_s, C_{s+1} (stencils (1, -2, 1) at nodes s-1, s,
// s+1, i.e. slots 2-4, 3-5, 4-6), so a clipped row has entries in slots 2
// to 6 only:
//   F_s: e4;  F_{s+1}: e5;  F^UL = 5 F_s - 4 F_{s-1}: 5 e4 - 4 e3;
//   F^MD = (F_s + F_{s+1})/2 - d^M4_{s+1/2}/2;
//   F^LC = 3/2 F_s - 1/2 F_{s-1} + 4/3 d^M4_{s-1/2}.
// The decisions are taken in the precision R of the forward's sweep (the
// storage type), with the forward's operations, so that they are the
// forward's own; the row's weights are exact in FP64.  Returns true when
// the row is a clipped one.
template <typename R>
__device__ __forceinline__ bool face_jacobian_row(const R (&w)[9], double (&J)[9]) {
    constexpr double W[9] = {4.0 / 2520.0,    -41.0 / 2520.0, 199.0 / 2520.0, -641.0 / 2520.0, 1879.0 / 2520.0,
                             1375.0 / 2520.0, -305.0 / 2520.0, 55.0 / 2520.0, -5.0 / 2520.0};
    R dd[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) dd[j] = w[j + 1] - w[j];
    R t, q;
    const R fl = mp9_face_linear<R>(dd, w[4], t, q);
#pragma unroll
    for (int k = 0; k < 9; ++k) J[k] = W[k];
    if (!(q > R(0))) return false;
    const R f = w[4], g = w[5], ul = f + t;
    const R cm = dd[3] - dd[2], c0 = dd[4] - dd[3], cp = dd[5] - dd[4];
    double am, bm, a0, b0;
    minmod4_weights(cm, c0, am, bm);  // d^M4 at s - 1/2 = am C_{s-1} + bm C_s
    minmod4_weights(c0, cp, a0, b0);  // d^M4 at s + 1/2 = a0 C_s + b0 C_{s+1}
    // the selected M4 arguments (exact: the weights are 0, +-1 or 4)
    const R vm = fma(R(am), cm, R(bm) * c0), v0 = fma(R(a0), c0, R(b0) * cp);
    const R lc = fma(R(4.0 / 3.0), vm, fma(R(0.5), dd[3], f));
    const R md = fma(R(0.5), dd[4] - v0, f);
    // candidates 0 F_s, 1 F_{s+1}, 2 MD, 3 UL, 4 LC: F^min = max(min(0, 1, 2),
    // min(0, 3, 4)), F^max = min(max(0, 1, 2), max(0, 3, 4))
    R va = f, vb = f, vc = f, ve = f;
    int ia = 0, ib = 0, ic = 0, ie = 0;
    if (g < va) { va = g; ia = 1; }
    if (md < va) { va = md; ia = 2; }
    if (ul < vb) { vb = ul; ib = 3; }
    if (lc < vb) { vb = lc; ib = 4; }
    if (g > vc) { vc = g; ic = 1; }
    if (md > vc) { vc = md; ic = 2; }
    if (ul > ve) { ve = ul; ie = 3; }
    if (lc > ve) { ve = lc; ie = 4; }
    const R lo = vb > va ? vb : va, hi = ve < vc ? ve : vc;
    const int ilo = vb > va ? ib : ia, ihi = ve < vc ? ie : ic;
    int sel;
    if (fl < lo) sel = ilo;
    else if (fl > hi) sel = ihi;
    else return false;
    // coefficients of the selected candidate on e3, e4, e5 and on the
    // curvature stencils at s-1, s, s+1
    const double A3 = sel == 3 ? -4.0 : (sel == 4 ? -0.5 : 0.0);
    const double A4 = sel == 0 ? 1.0 : (sel == 2 ? 0.5 : (sel == 3 ? 5.0 : (sel == 4 ? 1.5 : 0.0)));
    const double A5 = sel == 1 ? 1.0 : (sel == 2 ? 0.5 : 0.0);
    const double gm = sel == 4 ? 4.0 / 3.0 : 0.0, g0 = sel == 2 ? -0.5 : 0.0;
    const double Cm = gm * am, C0 = fma(gm, bm, g0 * a0), Cp = g0 * b0;
#pragma unroll
    for (int k = 0; k < 9; ++k) J[k] = 0.0;
    J[2] = Cm;
    J[3] = fma(-2.0, Cm, A3 + C0);
    J[4] = fma(-2.0, C0, A4 + Cm + Cp);
    J[5] = fma(-2.0, Cp, A5 + C0);
    J[6] = Cp;
    return true;
}

// One entry d(face)/d(w[k]) of the row above.
template <typename R>
__device__ __forceinline__ double face_jacobian(const R (&w)[9], int k) {
    double J[9];
    face_jacobian_row(w, J);
    double r = 0.0;
#pragma unroll
    for (int j = 0; j < 9; ++j) r = j == k ? J[j] : r;
    return r;
}

// ------------------------------------------------ transposed advection V^T
// The adjoint of the fluxes is dA = sum_j c_j z_j; every form below
// evaluates V = V^T dA at a node and hands it to adj_store, which writes
// y1 = e0 V + sum_j e_j z_j and (when y2 is set) y2 = f0 V + sum_j f_j z_j.
// The face between nodes s and s + 1 of a line carries
// d(face) = p/ds (dA_s - dA_{s+1}) (dA zero outside an outflow line,
// wrapped on a periodic one); a node receives, from every face whose
// window reads it, the face's Jacobian entry times d(face).
// NZ = o.n, a compile-time constant so that the loads of all z_j issue
// together.
// Element i of adjoint input j: z[0] is FP64, the others are in the storage
// type S (j is a compile-time constant at every use).
template <typename S>
__device__ __forceinline__ double adj_z(const AdvAdjIO& o, int j, size_t i) {
    return j == 0 ? static_cast<const double*>(o.z[0])[i] : (double)static_cast<const S*>(o.z[j])[i];
}

template <int NZ, typename S>
__device__ __forceinline__ double adj_dA(const AdvAdjIO& o, size_t i) {
    double r = 0.0;
#pragma unroll
    for (int j = 0; j < NZ; ++j) r = fma(o.c[j], adj_z<S>(o, j, i), r);
    return r;
}

// dA at element i, and the combinations sum_j e[j] z[j], sum_j f[j] z[j]
// of the same loads.
template <int NZ, typename S>
__device__ __forceinline__ double adj_dA_ef(const AdvAdjIO& o, size_t i, double& ze, double& zf) {
    double r = 0.0;
    ze = 0.0;
    zf = 0.0;
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        const double z = adj_z<S>(o, j, i);
        r = fma(o.c[j], z, r);
        ze = fma(o.e[j], z, ze);
        zf = fma(o.f[j], z, zf);
    }
    return r;
}

// y1 = e0 V + ze, y2 = f0 V + zf from the combinations formed at load time.
template <typename S>
__device__ __forceinline__ void adj_store_ef(const AdvAdjIO& o, size_t i, double V, double ze, double zf) {
    __builtin_nontemporal_store((S)fma(o.e0, V, ze), static_cast<S*>(o.y1) + i);
    if (o.y2) {
        const double y2 = fma(o.f0, V, zf);
        if (o.y2_f64) __builtin_nontemporal_store(y2, static_cast<double*>(o.y2) + i);
        else __builtin_nontemporal_store((S)y2, static_cast<S*>(o.y2) + i);
    }
}

template <int NZ, typename S>
__device__ __forceinline__ void adj_store(const AdvAdjIO& o, size_t i, double V) {
    double y1 = o.e0 * V, y2 = o.f0 * V;
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        const double z = adj_z<S>(o, j, i);
        y1 = fma(o.e[j], z, y1);
        y2 = fma(o.f[j], z, y2);
    }
    __builtin_nontemporal_store((S)y1, static_cast<S*>(o.y1) + i);
    if (o.y2) {
        if (o.y2_f64) __builtin_nontemporal_store(y2, static_cast<double*>(o.y2) + i);
        else __builtin_nontemporal_store((S)y2, static_cast<S*>(o.y2) + i);
    }
}

// Gather form along one line (used for 1D periodic lines shorter than 40
// nodes): node t of a line of n nodes (stride st) sums the faces whose
// windows read t or a ghost node that copies t; each face is evaluated once
// per node it feeds.  FWD: p > 0 (window F_{s-4} .. F_{s+4}), else the
// mirrored window F_{s+5} .. F_{s-3}.
template <bool FWD, int NZ, typename S>
__device__ double adj_axis_dir(const S* F, const AdvAdjIO& o, size_t base, long long st, int n, int bc,
                               int t, double pinv) {
    int vlo = t, vhi = t;
    if (bc == 0) {
        if (t == 0) vlo = -5;
        if (t == n - 1) vhi = n + 4;
    }
    double acc = 0.0;
    for (int tv = vlo; tv <= vhi; ++tv) {
        S w17[17];  // nodes tv-8 .. tv+8
#pragma unroll
        for (int i = 0; i < 17; ++i) w17[i] = F[base + (size_t)bc_map(tv - 8 + i, n, bc) * st];
        double a10[10];  // dA at faces' nodes: FWD s = tv-4 .. tv+5, else s = tv-5 .. tv+4
#pragma unroll
        for (int i = 0; i < 10; ++i) {
            int j = (FWD ? tv - 4 : tv - 5) + i;
            double v = 0.0;
            if (bc == 0) {
                if (j >= 0 && j < n) v = adj_dA<NZ, S>(o, base + (size_t)j * st);
            } else {
                v = adj_dA<NZ, S>(o, base + (size_t)bc_map(j, n, 1) * st);
            }
            a10[i] = v;
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int s = FWD ? tv + 4 - k : tv - 5 + k;  // face between s and s+1
            if (bc == 0 && (s < -1 || s > n - 1)) continue;
            S fw[9];
#pragma unroll
            for (int kk = 0; kk < 9; ++kk) fw[kk] = w17[FWD ? 8 - k + kk : 8 + k - kk];
            const int ia = FWD ? 8 - k : k;  // a10 index of s
            const double dface = pinv * (a10[ia] - a10[ia + 1]);
            acc = fma(face_jacobian(fw, k), dface, acc);
        }
    }
    return acc;
}

template <int NZ, typename S>
__global__ void __launch_bounds__(kAdjBlock) advect_adjoint_gather1d_kernel(const DevTables* __restrict__ tabp,
                                                                            const S* __restrict__ F,
                                                                            AdvAdjIO o, int nx, int bc,
                                                                            double inv_dx) {
    CTab* tab = (CTab*)tabp;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (x >= nx) return;
    const double p = tab->plane[v].px;
    const size_t pl = (size_t)v * nx;
    double r = 0.0;
    if (p > 0.0) r = adj_axis_dir<true, NZ, S>(F, o, pl, 1, nx, bc, x, p * inv_dx);
    else if (p < 0.0) r = adj_axis_dir<false, NZ, S>(F, o, pl, 1, nx, bc, x, p * inv_dx);
    adj_store<NZ, S>(o, pl + x, r);
}

// x lines, wave-cooperative (1D): one wavefront per chunk of kChunk nodes of
// a row, kChunkWaves chunks per work-group.  Lane l evaluates face
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

template <int NZ, typename S>
__global__ void __launch_bounds__(64 * kChunkWaves) advect_adjoint_xchunk_kernel(const DevTables* __restrict__ tabp,
                                                                                 const S* __restrict__ F,
                                                                                 AdvAdjIO o, int nx, int ny, int bc,
                                                                                 double inv_dx) {
    // per wavefront: F at nodes c0-8 .. c0+63, dA at c0-5 .. c0+66, and the
    // 9 x 64 weighted Jacobian entries of its faces
    __shared__ double contrib_all[kChunkWaves][9 * 64];
    __shared__ S sF_all[kChunkWaves][72];
    __shared__ double sA_all[kChunkWaves][72];
    CTab* tab = (CTab*)tabp;
    const long long cells = (long long)nx * ny;
    const int v = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, n = nx;
    double* contrib = contrib_all[wave];
    S* sF = sF_all[wave];
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
        if (live && lane < kChunk && t < n) adj_store<NZ, S>(o, base + t, 0.0);
        return;
    }
    const bool fwd = p > 0.0;
    // the chunk's windows, read once into LDS (coalesced)
    auto dat = [&](int j) {
        if (bc == 1) return adj_dA<NZ, S>(o, base + (size_t)bc_map(j, n, 1));
        return (j >= 0 && j < n) ? adj_dA<NZ, S>(o, base + (size_t)j) : 0.0;
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
        S w[9];
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
        adj_store<NZ, S>(o, base + (size_t)t, val);
    }
}

// 2D, both axes in one pass over tiles of kTT x kTT nodes, one work-group of
// four wavefronts per tile and kTPB planes.  Per plane the tile's F with an
// 8-node cross halo (the windows of every face that reads a tile node) and
// dA with a 5-node cross halo (the nodes of those faces) are staged in LDS.
// Wavefronts 0-1 take the x lines, 2-3 the y lines: each lane owns kTS
// nodes of a row (column) and evaluates the kTS + 8 faces that read them,
// each with its whole Jacobian row, accumulating by position in registers
// (two face evaluations per node and axis).  Positions left of node 0 and
// right of node n - 1 of an outflow line are its ghost nodes and fold into
// those end nodes; positions outside the lane's own nodes are otherwise
// counted by the lane that owns them.  Both axes' sums meet in LDS and every
// node is written once, coalesced.  Periodic lines of any length wrap through
// bc_map: a node gathers the nine faces t - 4 .. t + 4 (unwrapped), which
// are the faces that read it, so no face is counted twice.
constexpr int kTT = 32;                  // tile edge, nodes
constexpr int kTS = 8;                   // nodes per lane
constexpr int kTF = kTS + 8;             // faces per lane
constexpr int kFE = kTT + 16, kFP = kFE + 1;  // F tile (8-node halo), pitch
constexpr int kAE = kTT + 10, kAP = kAE + 1;  // dA tile (5-node halo), pitch
constexpr int kRP = kTT + 1;                  // pitch of the per-axis results (reusing the F and dA tiles)
constexpr int kZP = kTT;                      // pitch of the own nodes' input combinations (FP32 storage)
constexpr int kTThreads = 256;             // half of them on x lines, half on y lines
constexpr int kCorrStride = kTThreads;     // per-thread LDS column of corrections (entry j at j * kCorrStride)
constexpr int kFLoads = kTT * kFE + 16 * kTT, kALoads = kTT * kAE + 10 * kTT;  // cross sizes
constexpr int kNFL = (kFLoads + kTThreads - 1) / kTThreads;  // F loads per thread
constexpr int kNAL = (kALoads + kTThreads - 1) / kTThreads;  // dA loads per thread
constexpr int kTPB = 8;                                    // planes per work-group
static_assert(kTT % kTS == 0 && (kTT / kTS) * kTT * 2 == kTThreads, "lanes per line");
static_assert(kTT * kRP <= kAE * kAP && kTT * kRP * 2 <= kFE * kFP, "result tiles");
static_assert(kAE * kAP < 4096 && kTT * kZP < (1 << 19), "packed LDS slots");

// The kTF faces of one lane: position q (0 .. kTS + 15) stands for node
// t0 - 8 + q, its F at f[q FS]; face i has node s = t0 - 4 + i (FWD) or
// t0 - 5 + i, with dA_s at a[i AS].  Entries at the lane's own nodes
// (positions 8 .. 8 + kTS - 1) go to own[], those left of them to gl and
// those right of them to gr (ghost nodes of an outflow line, else nodes of
// other lanes).  Every face first carries the linear weights of F^L and
// takes the forward's monotonicity test; then the lane walks its faces that
// failed it (a wavefront takes as many turns as its busiest lane, not one
// per face position) and trades their linear weights for their clipped
// rows, accumulated in face order in corr[] (the lane's LDS column: the
// positions of those entries vary from face to face).
template <bool FWD, int FS, int AS, typename FT>
__device__ __forceinline__ void seg_faces(const FT* f, const double* a, double pinv, double* corr,
                                          double (&own)[kTS], double& gl, double& gr) {
    // 2520 times the weights of F^L: small integers, exact as instruction
    // literals
    constexpr double C[9] = {4.0, -41.0, 199.0, -641.0, 1879.0, 1375.0, -305.0, 55.0, -5.0};
#pragma unroll
    for (int j = 0; j < kTS; ++j) own[j] = 0.0;
    gl = 0.0;
    gr = 0.0;
    unsigned mask = 0u;
#pragma unroll
    for (int i = 0; i < kTF; ++i) {
        // the forward's monotonicity test, in its precision FT
        FT dd[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            dd[k] = FWD ? f[(i + k + 1) * FS] - f[(i + k) * FS] : f[(i + 7 - k) * FS] - f[(i + 8 - k) * FS];
        FT t, q;
        (void)mp9_face_linear<FT>(dd, f[(i + 4) * FS], t, q);
        mask |= (q > FT(0) ? 1u : 0u) << i;
        const double dl = pinv * (a[i * AS] - a[(i + 1) * AS]) * (1.0 / 2520.0);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int p = FWD ? i + k : i + 8 - k;
            if (p < 8) gl = fma(C[k], dl, gl);
            else if (p >= 8 + kTS) gr = fma(C[k], dl, gr);
            else own[p - 8] = fma(C[k], dl, own[p - 8]);
        }
    }
    if (mask) {
#pragma unroll
        for (int j = 0; j < kTS; ++j) corr[j * kCorrStride] = 0.0;
        for (unsigned m = mask; m; m &= m - 1u) {
            const int i = __builtin_ctz(m);
            FT w[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) w[k] = f[(FWD ? i + k : i + 8 - k) * FS];
            double J[9];
            if (face_jacobian_row(w, J)) {
                const double d = pinv * (a[i * AS] - a[(i + 1) * AS]);
                const double dl = d * (1.0 / 2520.0);
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    const int p = FWD ? i + k : i + 8 - k;
                    const double v = fma(J[k], d, -C[k] * dl);
                    if (p < 8) gl += v;
                    else if (p >= 8 + kTS) gr += v;
                    else corr[(p - 8) * kCorrStride] += v;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kTS; ++j) own[j] += corr[j * kCorrStride];
    }
}

// Outflow ghosts of a lane whose nodes start at t0 on a line of n nodes:
// the entries left of node 0 fold into node 0 (t0 = 0), those right of node
// n - 1 into node n - 1 (when the lane owns it; own nodes past n - 1 are
// ghost positions too).
__device__ __forceinline__ void seg_fold(double (&own)[kTS], double gl, double gr, int t0, int n) {
    if (t0 == 0) own[0] += gl;
    const int je = n - 1 - t0;  // own index of node n - 1
    if (je >= 0 && je < kTS) {
        double g = gr;
#pragma unroll
        for (int j = 1; j < kTS; ++j) g += j > je ? own[j] : 0.0;
#pragma unroll
        for (int j = 0; j < kTS; ++j) own[j] += j == je ? g : 0.0;
    }
}

template <int NZ, typename S, bool ZL>
__global__ void __launch_bounds__(kTThreads) advect_adjoint_tile_kernel(const DevTables* __restrict__ tabp,
                                                                        const S* __restrict__ F, AdvAdjIO o,
                                                                        int nx, int ny, int bcx, int bcy,
                                                                        double inv_dx, double inv_dy, int ntx,
                                                                        int nplanes) {
    // ZL (FP32 storage): the combinations sum e_j z_j and sum f_j z_j of the
    // tile's own nodes are formed as the dA halo loads arrive and kept in
    // LDS, so the closing stores need no second round of loads (with FP64
    // storage the LDS would not hold them at three work-groups per compute
    // unit, and the closing stores load the z_j again).  F is staged in its
    // storage type.
    static_assert(!ZL || sizeof(S) == 4, "combinations in LDS with FP32 storage only");
    constexpr bool kZL = ZL;
    __shared__ double sFbuf[(kFE * kFP * sizeof(S) + 7) / 8];  // F, then the x results [row][col] (FP64)
    __shared__ double sA[kAE * kAP];  // then the y results [row][col]
    __shared__ double sCorr[kTS * kCorrStride];  // per thread: clipped-face corrections
    // e.z (FP32, as y1 is stored) and f.z (FP64: y2 may be lam^n) at the own
    // nodes [row][col], then one dummy entry per lane for the loads of other
    // nodes (unconditional stores: a store behind a branch would hold the
    // next loads back)
    constexpr int kZN = kTT * kZP + 64;
    __shared__ float sZe[kZL ? kZN : 1];
    __shared__ double sZf[kZL ? kZN : 1];
    S* const sF = reinterpret_cast<S*>(sFbuf);
    double* const sX = sFbuf;
    CTab* tab = (CTab*)tabp;
    const long long cells = (long long)nx * ny;
    const int tid = threadIdx.x;
    const int x0 = (int)(blockIdx.x % ntx) * kTT, y0 = (int)(blockIdx.x / ntx) * kTT;
    // global offsets and LDS slots of the loads, the same for every plane;
    // the F cross: rows 8 .. 8 + kTT - 1 across the whole width, then the
    // columns 8 .. 8 + kTT - 1 of the 8 rows above and below; dA likewise
    // with a 5-node halo (bit j of amask clear: outside an outflow line,
    // where dA is zero; the load still reads a valid node so that every
    // load issues at once).  al[j] packs the dA slot (bits 0-11) and the
    // slot of the node's combinations in sZ (bits 12 up: its own-node index,
    // or the lane's dummy entry).
    int fo[kNFL], fl[kNFL], ao[kNAL], al[kNAL];
    unsigned amask = 0u;
#pragma unroll
    for (int j = 0; j < kNFL; ++j) {
        // slots past the cross (last round) load node 0 into the unused corner 0
        const int i = min(tid + j * kTThreads, kFLoads);
        int lx, ly;
        if (i == kFLoads) {
            lx = 0;
            ly = 0;
        } else if (i < kTT * kFE) {
            ly = 8 + i / kFE;
            lx = i % kFE;
        } else {
            const int k = i - kTT * kFE, q = k / kTT;
            lx = 8 + k % kTT;
            ly = q < 8 ? q : kTT + q;
        }
        fo[j] = i == kFLoads ? 0 : bc_map(y0 - 8 + ly, ny, bcy) * nx + bc_map(x0 - 8 + lx, nx, bcx);
        fl[j] = ly * kFP + lx;
    }
#pragma unroll
    for (int j = 0; j < kNAL; ++j) {
        const int i = min(tid + j * kTThreads, kALoads);
        int lx, ly;
        if (i == kALoads) {
            lx = 0;
            ly = 0;
        } else if (i < kTT * kAE) {
            ly = 5 + i / kAE;
            lx = i % kAE;
        } else {
            const int k = i - kTT * kAE, q = k / kTT;
            lx = 5 + k % kTT;
            ly = q < 5 ? q : kTT + q;
        }
        const int gx = x0 - 5 + lx, gy = y0 - 5 + ly;
        const bool zero = (bcx == 0 && (gx < 0 || gx >= nx)) || (bcy == 0 && (gy < 0 || gy >= ny));
        ao[j] = i == kALoads ? 0 : bc_map(gy, ny, bcy) * nx + bc_map(gx, nx, bcx);
        amask |= (zero ? 0u : 1u) << j;
        const bool tile_node = i < kTT * kAE && lx >= 5 && lx < 5 + kTT;
        al[j] = ly * kAP + lx + ((tile_node ? (ly - 5) * kZP + lx - 5 : kTT * kZP + (tid & 63)) << 12);
    }
    // the first half of the threads on x lines, the second on y lines: a
    // row (column) `line`, nodes kTS seg .. kTS seg + kTS - 1 of the tile
    const bool xl = tid < kTThreads / 2;
    const int li = xl ? tid : tid - kTThreads / 2;
    const int line = li % kTT, seg = li / kTT;
    const int v1 = min((int)blockIdx.y * kTPB + kTPB, nplanes);
    for (int v = (int)blockIdx.y * kTPB; v < v1; ++v) {
        const size_t pl = (size_t)v * cells;
#pragma unroll
        for (int j = 0; j < kNFL; ++j) sF[fl[j]] = F[pl + fo[j]];
#pragma unroll
        for (int j = 0; j < kNAL; ++j) {
            // (slots from j = kTT kAE / kTThreads on hold halo rows only)
            if (kZL && j * kTThreads < kTT * kAE) {  // constant once unrolled
                double ze, zf;
                const double v = adj_dA_ef<NZ, S>(o, pl + ao[j], ze, zf);
                sA[al[j] & 4095] = (amask >> j) & 1u ? v : 0.0;
                sZe[al[j] >> 12] = (float)ze;
                sZf[al[j] >> 12] = zf;
            } else {
                const double v = adj_dA<NZ, S>(o, pl + ao[j]);
                sA[al[j] & 4095] = (amask >> j) & 1u ? v : 0.0;
            }
        }
        __syncthreads();
        double own[kTS], gl, gr;
        bool live;
        if (xl) {  // x lines: row `line`, nodes t0 .. t0 + kTS - 1
            const double p = tab->plane[v].px;
            const int t0 = x0 + kTS * seg;
            live = p != 0.0 && y0 + line < ny && t0 < nx;
            if (live) {
                const S* f = sF + (8 + line) * kFP + kTS * seg;
                const double* a = sA + (5 + line) * kAP + kTS * seg;
                double* corr = sCorr + tid;
                if (p > 0.0) seg_faces<true, 1, 1>(f, a + 1, p * inv_dx, corr, own, gl, gr);
                else seg_faces<false, 1, 1>(f, a, p * inv_dx, corr, own, gl, gr);
                if (bcx == 0) seg_fold(own, gl, gr, t0, nx);
            }
        } else {  // y lines: column `line`, nodes t0 .. t0 + kTS - 1
            const double p = tab->plane[v].py;
            const int t0 = y0 + kTS * seg;
            live = p != 0.0 && x0 + line < nx && t0 < ny;
            if (live) {
                const S* f = sF + kTS * seg * kFP + 8 + line;
                const double* a = sA + kTS * seg * kAP + 5 + line;
                double* corr = sCorr + tid;
                if (p > 0.0) seg_faces<true, kFP, kAP>(f, a + kAP, p * inv_dy, corr, own, gl, gr);
                else seg_faces<false, kFP, kAP>(f, a, p * inv_dy, corr, own, gl, gr);
                if (bcy == 0) seg_fold(own, gl, gr, t0, ny);
            }
        }
        __syncthreads();  // both tiles are read; they now take the results
        if (xl) {
#pragma unroll
            for (int i = 0; i < kTS; ++i) sX[line * kRP + kTS * seg + i] = live ? own[i] : 0.0;
        } else {
#pragma unroll
            for (int i = 0; i < kTS; ++i) sA[(kTS * seg + i) * kRP + line] = live ? own[i] : 0.0;
        }
        __syncthreads();
        for (int i = tid; i < kTT * kTT; i += kTThreads) {
            const int r = i / kTT, c = i % kTT;
            if (x0 + c < nx && y0 + r < ny) {
                const size_t g = pl + (size_t)(y0 + r) * nx + x0 + c;
                const double V = sX[r * kRP + c] + sA[r * kRP + c];
                if constexpr (kZL) adj_store_ef<S>(o, g, V, (double)sZe[r * kZP + c], sZf[r * kZP + c]);
                else adj_store<NZ, S>(o, g, V);
            }
        }
        __syncthreads();  // before the next plane overwrites the tiles
    }
}

// The pointwise adjoint kernels: a work-group of kParts wavefronts covers 64
// consecutive cells (one per lane), and its wavefronts split the planes
// between them (rows of one y node each, in plane order), so that a grid of
// a few hundred thousand cells still keeps several wavefronts per SIMD, each
// with a row of loads in flight.  (Two parts measured faster than four: each
// part evaluates the x factors of its sets again.)
constexpr int kParts = 2;

// Row r of the plane order: set, y node and first plane; a set holds Q_set
// rows of Q_set planes in 2D and one row of Q_set planes in 1D.
template <int D>
__device__ __forceinline__ void plane_row(CTab* tab, int r, int& set, int& ky, int& v) {
    const int q0 = tab->q[0];
    if (D == 2) {
        set = r >= q0 ? 1 : 0;
        ky = set ? r - q0 : r;
        v = set ? q0 * q0 + ky * tab->q[1] : ky * q0;
    } else {
        set = r;
        ky = 0;
        v = r ? q0 : 0;
    }
}

template <int D>
__device__ __forceinline__ int plane_rows(CTab* tab) {
    return D == 2 ? tab->q[0] + tab->q[1] : 2;
}

// out = a src + b E(M) (stage value rebuilt from its moments), evaluated in
// FP64 and stored in the storage type, as the forward's relax on read
// stores it before the MP-9 sweeps.  The x factors of a set are evaluated
// once per cell and wavefront; a row of planes is read with all its loads in
// flight.
template <typename S, int D, int QM>
__global__ void __launch_bounds__(64 * kParts) materialise_kernel(const DevTables* __restrict__ tabp,
                                                                     const S* __restrict__ src,
                                                                     const double* __restrict__ M, double a,
                                                                     double b, S* __restrict__ out,
                                                                     long long cells, double chi_fac) {
    CTab* tab = (CTab*)tabp;
    const long long c = (long long)blockIdx.x * 64 + (threadIdx.x & 63);
    if (c >= cells) return;
    const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double nn = M[c], u = M[cells + c], w = D == 2 ? M[2 * cells + c] : 0.0;
    const double th = M[(D + 1) * cells + c] - 1.0;
    const int nrow = plane_rows<D>(tab);
    const int r0 = part * nrow / kParts, r1 = (part + 1) * nrow / kParts;
    int cur = -1;
    double pre = 0.0, gx[QM];
#pragma unroll
    for (int kx = 0; kx < QM; ++kx) gx[kx] = 0.0;
    for (int r = r0; r < r1; ++r) {
        int set, ky, v;
        plane_row<D>(tab, r, set, ky, v);
        const int Q = tab->q[set];
        if (set != cur) {
            cur = set;
            pre = set ? chi_fac * nn * (th + 1.0) : nn;
#pragma unroll
            for (int kx = 0; kx < QM; ++kx) gx[kx] = kx < Q ? herm_factor(tab->h[set][kx], Q, u, th) : 0.0;
        }
        double sv[QM];  // every load issued, none behind a branch (past the row's end: its first plane again)
#pragma unroll
        for (int kx = 0; kx < QM; ++kx) sv[kx] = (double)src[(size_t)(v + (kx < Q ? kx : 0)) * cells + c];
        const double gy = b * (D == 2 ? pre * herm_factor(tab->h[set][ky], Q, w, th) : pre);
#pragma unroll
        for (int kx = 0; kx < QM; ++kx)
            if (kx < Q) out[(size_t)(v + kx) * cells + c] = (S)fma(a, sv[kx], gy * gx[kx]);
    }
}

// dM = (dE/dM)^T dE per cell for the plane-set dE (type A).  Moments (n, u, T)
// of M.  With E = P_set g_x g_y per plane, the sums over a set's planes
// factor: the wavefront accumulates, per x node, sum_y e g_y, sum_y e dg_y/du
// and sum_y e dg_y/dT over its rows (three FMAs per plane) and applies the x
// factors and their derivatives once per set.  The wavefronts' partial sums
// meet in LDS and are added in wavefront order (deterministic).
template <int D, int QM, typename A>
__global__ void __launch_bounds__(64 * kParts) eq_adjoint_kernel(const DevTables* __restrict__ tabp,
                                                                    const double* __restrict__ M,
                                                                    const A* __restrict__ dE,
                                                                    double* __restrict__ dM, long long cells,
                                                                    double chi_fac) {
    constexpr int NP = kParts;
    __shared__ double red[NP - 1][4][64];
    CTab* tab = (CTab*)tabp;
    const int lane = threadIdx.x & 63;
    const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long cl = (long long)blockIdx.x * 64 + lane;
    const bool live = cl < cells;
    const long long c = live ? cl : 0;  // lanes past the end work on cell 0 and store nothing
    const double nn = M[c], u = M[cells + c], w = D == 2 ? M[2 * cells + c] : 0.0;
    const double T = M[(D + 1) * cells + c], th = T - 1.0;
    double dn = 0.0, dux = 0.0, duy = 0.0, dT = 0.0;
    const int nrow = plane_rows<D>(tab);
    const int r0 = part * nrow / NP, r1 = (part + 1) * nrow / NP;
    // per x node of the current set: sum_y e g_y, sum_y e g_y,u, sum_y e g_y,T
    double sg[QM], su[QM], sT[QM];
#pragma unroll
    for (int kx = 0; kx < QM; ++kx) {
        sg[kx] = 0.0;
        su[kx] = 0.0;
        sT[kx] = 0.0;
    }
    // folds the sums of set `set` into dn .. dT and clears them
    auto flush = [&](int set) {
        const int Q = tab->q[set];
        const double pre = set ? chi_fac * nn * T : nn;  // P_phi = n, P_chi = (K+D-d) n T
        const double pre_n = set ? chi_fac * T : 1.0;
        const double pre_T = set ? chi_fac * nn : 0.0;
        double xg = 0.0, xu = 0.0, xgy = 0.0, xT = 0.0, xgT = 0.0;
#pragma unroll
        for (int kx = 0; kx < QM; ++kx) {
            if (kx < Q) {
                double gx, gxu, gxT;
                herm_factor_d(tab->h[set][kx], Q, u, th, gx, gxu, gxT);
                xg = fma(gx, sg[kx], xg);     // sum e g_x g_y
                xu = fma(gxu, sg[kx], xu);    // sum e g_x,u g_y
                xgy = fma(gx, su[kx], xgy);   // sum e g_x g_y,u
                xT = fma(gxT, sg[kx], xT);    // sum e g_x,T g_y
                xgT = fma(gx, sT[kx], xgT);   // sum e g_x g_y,T
            }
            sg[kx] = 0.0;
            su[kx] = 0.0;
            sT[kx] = 0.0;
        }
        dn = fma(pre_n, xg, dn);
        dux = fma(pre, xu, dux);
        if (D == 2) duy = fma(pre, xgy, duy);
        dT = fma(pre_T, xg, fma(pre, xT + xgT, dT));
    };
    int cur = -1;
    for (int r = r0; r < r1; ++r) {
        int set, ky, v;
        plane_row<D>(tab, r, set, ky, v);
        const int Q = tab->q[set];
        double ev[QM];  // the row's loads, all in flight (past the row's end: its first plane again)
#pragma unroll
        for (int kx = 0; kx < QM; ++kx) ev[kx] = (double)dE[(size_t)(v + (kx < Q ? kx : 0)) * cells + c];
        if (set != cur) {
            if (cur >= 0) flush(cur);
            cur = set;
        }
        double gy = 1.0, gyu = 0.0, gyT = 0.0;
        if (D == 2) herm_factor_d(tab->h[set][ky], Q, w, th, gy, gyu, gyT);
#pragma unroll
        for (int kx = 0; kx < QM; ++kx) {
            const double e = kx < Q ? ev[kx] : 0.0;
            sg[kx] = fma(e, gy, sg[kx]);
            if (D == 2) su[kx] = fma(e, gyu, su[kx]);
            sT[kx] = fma(e, gyT, sT[kx]);
        }
    }
    if (cur >= 0) flush(cur);
    if (part > 0) {
        red[part - 1][0][lane] = dn;
        red[part - 1][1][lane] = dux;
        red[part - 1][2][lane] = duy;
        red[part - 1][3][lane] = dT;
    }
    __syncthreads();
    if (part == 0 && live) {
#pragma unroll
        for (int p = 0; p < NP - 1; ++p) {
            dn += red[p][0][lane];
            dux += red[p][1][lane];
            duy += red[p][2][lane];
            dT += red[p][3][lane];
        }
        dM[c] = dn;
        dM[cells + c] = dux;
        if (D == 2) dM[2 * cells + c] = duy;
        dM[(D + 1) * cells + c] = dT;
    }
}

// out = y + (dM/dF)^T dM per plane, y and out of type A (y may be NULL:
// zero; it may also be out itself, each element being read before it is
// written).
// n = sum_phi F, n u = sum_phi p F, (D+K) n T = sum_phi |p|^2 F + sum_chi F - n |u|^2:
//   dn/dF = [phi], du/dF = [phi] (p - u)/n,
//   dT/dF = ([phi] |p - u|^2 + [chi]) / ((D+K) n) - [phi] T / n.
// Each wavefront takes a contiguous range of planes, in groups of
// kMomGroup with the group's loads in flight together.
constexpr int kMomGroup = 8;

template <int D, typename A>
__global__ void __launch_bounds__(64 * kParts) mom_adjoint_kernel(const DevTables* __restrict__ tabp,
                                                                     const double* __restrict__ M,
                                                                     const double* __restrict__ dM,
                                                                     const A* y, A* out, long long cells,
                                                                     double dk) {
    CTab* tab = (CTab*)tabp;
    const long long c = (long long)blockIdx.x * 64 + (threadIdx.x & 63);
    if (c >= cells) return;
    const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double nn = M[c], u = M[cells + c], w = D == 2 ? M[2 * cells + c] : 0.0;
    const double T = M[(D + 1) * cells + c];
    const double gn = dM[c], gu = dM[cells + c], gw = D == 2 ? dM[2 * cells + c] : 0.0;
    const double gT = dM[(D + 1) * cells + c];
    const double inv_n = 1.0 / nn, inv_dkn = 1.0 / (dk * nn);
    // the terms of a phi plane: gn + (gu (px - u) + gw (py - w)) / n + gT (|p - u|^2 / ((D+K) n) - T / n);
    // of a chi plane: gT / ((D+K) n)
    const double chi_term = gT * inv_dkn;
    const int np = tab->nplanes;
    const int v0 = part * np / kParts, v1 = (part + 1) * np / kParts;
    for (int vb = v0; vb < v1; vb += kMomGroup) {
        double r[kMomGroup];
#pragma unroll
        for (int k = 0; k < kMomGroup; ++k) r[k] = y ? (double)y[(size_t)(vb + k < v1 ? vb + k : vb) * cells + c] : 0.0;
#pragma unroll
        for (int k = 0; k < kMomGroup; ++k) {
            const int v = vb + k;
            if (v < v1) {
                double t = chi_term;
                if (tab->plane[v].set == 0) {
                    const double ex = tab->plane[v].px - u, ey = tab->plane[v].py - w;
                    t = gn + (gu * ex + gw * ey) * inv_n + gT * ((ex * ex + ey * ey) * inv_dkn - T * inv_n);
                }
                out[(size_t)v * cells + c] = (A)(r[k] + t);
            }
        }
    }
}

}  // namespace

hipError_t launch_materialise(int d, int qm, bool f32, const DevTables* tab, const void* src, const double* M,
                              double a, double b, void* out, long long cells, double chi_fac,
                              hipStream_t s) {
    const int grid = (int)((cells + 63) / 64);
#define IMEXLB_MAT(S, D, QM) \
    hipLaunchKernelGGL((materialise_kernel<S, D, QM>), dim3(grid), dim3(64 * kParts), 0, s, tab, (const S*)src, M, a, b, (S*)out, cells, chi_fac)
    if (d == 2) {
        if (qm == 8) { if (f32) IMEXLB_MAT(float, 2, 8); else IMEXLB_MAT(double, 2, 8); }
        else { if (f32) IMEXLB_MAT(float, 2, 16); else IMEXLB_MAT(double, 2, 16); }
    } else {
        if (qm == 8) { if (f32) IMEXLB_MAT(float, 1, 8); else IMEXLB_MAT(double, 1, 8); }
        else { if (f32) IMEXLB_MAT(float, 1, 16); else IMEXLB_MAT(double, 1, 16); }
    }
#undef IMEXLB_MAT
    return hipGetLastError();
}

namespace {

template <int NZ, typename S>
hipError_t launch_advect_adjoint_n(int d, const DevTables* tab, int nplanes, const S* F, const AdvAdjIO& io,
                                   int nx, int ny, int bcx, int bcy, double inv_dx, double inv_dy, hipStream_t s) {
    if (d == 2) {
        const int ntx = (nx + kTT - 1) / kTT, nty = (ny + kTT - 1) / kTT;
        const dim3 grid((unsigned)(ntx * nty), (unsigned)((nplanes + kTPB - 1) / kTPB));
        hipLaunchKernelGGL((advect_adjoint_tile_kernel<NZ, S, sizeof(S) == 4>), grid, dim3(kTThreads), 0, s, tab, F,
                           io, nx, ny, bcx, bcy, inv_dx, inv_dy, ntx, nplanes);
        return hipGetLastError();
    }
    // 1D: rows in 64-face chunks; periodic lines shorter than a chunk's
    // window range take the gather form
    if (bcx == 1 && nx < 40) {
        const dim3 grid((unsigned)((nx + kAdjBlock - 1) / kAdjBlock), (unsigned)nplanes);
        hipLaunchKernelGGL((advect_adjoint_gather1d_kernel<NZ, S>), grid, dim3(kAdjBlock), 0, s, tab, F, io, nx, bcx,
                           inv_dx);
        return hipGetLastError();
    }
    const long long gx = ((nx + kChunk - 1) / kChunk + kChunkWaves - 1) / kChunkWaves;
    hipLaunchKernelGGL((advect_adjoint_xchunk_kernel<NZ, S>), dim3((unsigned)gx, (unsigned)nplanes),
                       dim3(64 * kChunkWaves), 0, s, tab, F, io, nx, 1, bcx, inv_dx);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_advect_adjoint_s(int d, const DevTables* tab, int nplanes, const S* F, const AdvAdjIO& io,
                                   int nx, int ny, int bcx, int bcy, double inv_dx, double inv_dy, hipStream_t s) {
    switch (io.n) {
        case 1: return launch_advect_adjoint_n<1, S>(d, tab, nplanes, F, io, nx, ny, bcx, bcy, inv_dx, inv_dy, s);
        case 2: return launch_advect_adjoint_n<2, S>(d, tab, nplanes, F, io, nx, ny, bcx, bcy, inv_dx, inv_dy, s);
        case 3: return launch_advect_adjoint_n<3, S>(d, tab, nplanes, F, io, nx, ny, bcx, bcy, inv_dx, inv_dy, s);
        case 4: return launch_advect_adjoint_n<4, S>(d, tab, nplanes, F, io, nx, ny, bcx, bcy, inv_dx, inv_dy, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_advect_adjoint(int d, bool f32, const DevTables* tab, int nplanes, const void* F,
                                 const AdvAdjIO& io, int nx, int ny, int bcx, int bcy, double inv_dx, double inv_dy,
                                 hipStream_t s) {
    return f32 ? launch_advect_adjoint_s<float>(d, tab, nplanes, (const float*)F, io, nx, ny, bcx, bcy, inv_dx, inv_dy, s)
               : launch_advect_adjoint_s<double>(d, tab, nplanes, (const double*)F, io, nx, ny, bcx, bcy, inv_dx,
                                                 inv_dy, s);
}

hipError_t launch_eq_adjoint(int d, int qm, bool f32, const DevTables* tab, const double* M, const void* dE,
                             double* dM, long long cells, double chi_fac, hipStream_t s) {
    const int grid = (int)((cells + 63) / 64);
#define IMEXLB_EQT(D, QM, T) \
    hipLaunchKernelGGL((eq_adjoint_kernel<D, QM, T>), dim3(grid), dim3(64 * kParts), 0, s, tab, M, (const T*)dE, dM, cells, chi_fac)
    if (d == 2) {
        if (qm == 8) { if (f32) IMEXLB_EQT(2, 8, float); else IMEXLB_EQT(2, 8, double); }
        else { if (f32) IMEXLB_EQT(2, 16, float); else IMEXLB_EQT(2, 16, double); }
    } else {
        if (qm == 8) { if (f32) IMEXLB_EQT(1, 8, float); else IMEXLB_EQT(1, 8, double); }
        else { if (f32) IMEXLB_EQT(1, 16, float); else IMEXLB_EQT(1, 16, double); }
    }
#undef IMEXLB_EQT
    return hipGetLastError();
}

hipError_t launch_mom_adjoint(int d, bool f32, const DevTables* tab, const double* M, const double* dM,
                              const void* y, void* out, long long cells, double dk, hipStream_t s) {
    const int grid = (int)((cells + 63) / 64);
#define IMEXLB_MOMT(D, T) \
    hipLaunchKernelGGL((mom_adjoint_kernel<D, T>), dim3(grid), dim3(64 * kParts), 0, s, tab, M, dM, (const T*)y, (T*)out, cells, dk)
    if (d == 2) { if (f32) IMEXLB_MOMT(2, float); else IMEXLB_MOMT(2, double); }
    else { if (f32) IMEXLB_MOMT(1, float); else IMEXLB_MOMT(1, double); }
#undef IMEXLB_MOMT
    return hipGetLastError();
}

}  // namespace imexlb
