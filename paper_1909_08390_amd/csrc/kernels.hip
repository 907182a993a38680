// HIP kernels of the imexlb library for gfx950 (MI355X).
//
// One IMEX-SSP3(4,3,3) step (Sec. III, Table I) runs as three fused stage
// passes over the plane-sets; the BGK stages are closed forms because the
// collision conserves n, u and T (Sec. III):
//
//   c = alpha dt/tau, w = dt/tau, a1 = 1/(1+c), a2 = (1+2c)/(1+c)^2, b2 = 1-a2
//   F1 = a1 F^n + c a1 E^n,  F2 = a2 F^n + b2 E^n          (stages 1-2, pointwise)
//   pass 3: G3 = F^n - dt V F2 - (1-alpha) dF2,  M3 = moments(G3)
//   pass 4: F3 = a1 G3 + c a1 E3 (relax on read),
//           G4 = F^n - (dt/4)(V F2 + V F3) - beta dF1 - eta dF2 - kappa dF3,
//           R  = F^n - (dt/6)(V F2 + V F3) - (dF2 + dF3)/6  (written over F^n),
//           M4 = moments(G4)
//   pass 5: F4 = a1 G4 + c a1 E4 (relax on read),
//           F^{n+1} = R - (2/3)(dt V F4 + dF4),  M^{n+1} = moments(F^{n+1})
//   with dF1 = w a1 (F^n - E^n), dF2 = w a2 (F^n - E^n), dF3 = w a1 (G3 - E3),
//   dF4 = w a1 (G4 - E4), kappa = 1/2 - alpha - beta - eta, and dt V F2
//   recovered pointwise in pass 4 as F^n - (1 - alpha) dF2 - G3.
//
// Every pass streams all planes of a tile of cells through LDS: per plane,
// the tile plus a 5-cell cross-shaped halo is loaded, relaxed on read to
// the stage value F_i = a G + b E_i (the equilibrium E_i rebuilt per cell
// from the stage moments), swept with MP-9 along x and y, combined with the
// pointwise terms, stored, and its moments accumulated in FP64 registers
// across the plane loop.  The advection operator V is the MP-9 flux
// difference of Sec. IV, dimensionally unsplit.
#include "common.hpp"
#include "device.hpp"

namespace imexlb {
namespace {

// MP-9 along a line held in registers, upwind-first window w[0 .. L+8]: the
// face between window positions m and m+1 (m = 4 .. L+4) is reconstructed
// from w[m-4 .. m+4] with w[m] the upwind node.  Returns dif[i] = face(5+i)
// - face(4+i), the flux difference of the node at window position 5+i
// (divide by delta s, multiply by |p|).  The linear parts of all L + 1 faces
// are evaluated first (independent chains the scheduler interleaves), then
// the clipping of each face that needs it.
template <typename R, int L>
__device__ __forceinline__ void mp9_line(const R (&w)[L + 9], R (&dif)[L]) {
    R d[L + 8];
#pragma unroll
    for (int j = 0; j < L + 8; ++j) d[j] = w[j + 1] - w[j];
    R fl[L + 1], t[L + 1], q[L + 1];
#pragma unroll
    for (int i = 0; i <= L; ++i) {
        R dd[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) dd[k] = d[i + k];
        fl[i] = mp9_face_linear<R>(dd, w[i + 4], t[i], q[i]);
    }
    // one branch for the whole line, skipped by every wavefront none of whose
    // lanes needs a clip (the common case in smooth regions); inside it each
    // face takes its clipped value where its test fails.  Neighbouring faces
    // share curvatures and M4 limits (the limit at s + 1/2 of face i is the
    // one at s - 1/2 of face i + 1), so the line evaluates L + 3 curvatures
    // and L + 2 limits instead of three and two per face.
    bool any = false;
#pragma unroll
    for (int i = 0; i <= L; ++i) any |= q[i] > R(0);
    if (any) {
        // opaque copies keep this work inside the branch
        R e[L + 4], f[L + 2];
#pragma unroll
        for (int j = 0; j < L + 4; ++j) {
            e[j] = d[j + 2];
            opaque(e[j]);
        }
#pragma unroll
        for (int j = 0; j < L + 2; ++j) {
            f[j] = w[j + 4];
            opaque(f[j]);
        }
        // e[j] = d[j + 2]: face i reads d[i + 2 .. i + 5] = e[i .. i + 3]
        R c0 = e[2] - e[1];                          // curvature at s of face 0
        R mlo = mp9_m4<R>(e[1] - e[0], c0);          // M4 limit at s - 1/2 of face 0
#pragma unroll
        for (int i = 0; i <= L; ++i) {
            const R cp = e[i + 3] - e[i + 2];        // curvature at s + 1
            const R mhi = mp9_m4<R>(c0, cp);         // M4 limit at s + 1/2
            const R c = mp9_face_bound<R>(f[i], f[i + 1], t[i], e[i + 1], e[i + 2], mlo, mhi, fl[i]);
            fl[i] = q[i] > R(0) ? c : fl[i];
            c0 = cp;
            mlo = mhi;
        }
    }
#pragma unroll
    for (int i = 0; i < L; ++i) dif[i] = fl[i + 1] - fl[i];
}

// mp9_line over a window held in LDS.  lo points at the lowest address of
// the L + 9 window elements, STRIDE apart; FWD: window position m is
// lo[m STRIDE] (flow towards higher addresses), else lo[(L + 8 - m) STRIDE].
// The flux difference of the node at window position 5 + i goes to
// out[i OSTRIDE] (FWD) or out[(L - 1 - i) OSTRIDE], i.e. out addresses the
// node of lowest address either way.  All offsets are compile-time
// constants.
template <typename R, typename S, int L, int STRIDE, int OSTRIDE, bool FWD>
__device__ __forceinline__ void mp9_sweep(const S* lo, R* out) {
    R w[L + 9];
#pragma unroll
    for (int m = 0; m < L + 9; ++m) w[m] = (R)lo[(FWD ? m : L + 8 - m) * STRIDE];
    R dif[L];
    mp9_line<R, L>(w, dif);
#pragma unroll
    for (int i = 0; i < L; ++i) out[(FWD ? i : L - 1 - i) * OSTRIDE] = dif[i];
}

// Raw buffer access to one plane: the plane base sits in SGPRs (a buffer
// resource built per plane with scalar arithmetic) and each lane supplies a
// 32-bit byte offset, so the per-plane address work is scalar.  Offsets
// outside the plane read 0 and drop stores (hardware range check); the host
// keeps every plane below 2^31 bytes.
typedef __amdgpu_buffer_rsrc_t Rsrc;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRawBufferWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format

template <typename S>
__device__ __forceinline__ Rsrc plane_rsrc(const S* p, long long cells) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(p), 0, (int)(cells * (long long)sizeof(S)),
                                             kRawBufferWord3);
}

// Cache policy of a load or store (the buffer intrinsics' last operand): 0
// is the default.  Data that the pass touches once and no neighbouring tile
// reads (the own cells of the state buffer, the output planes) take the
// streaming policies, so that it leaves the L2 early and the halo lines the
// neighbouring tiles still read stay: kStreamLoad = nt, kStreamStore =
// sc1 | nt (gfx950 encodings).
constexpr int kStreamLoad = 2;
constexpr int kStreamStore = 16 | 2;

template <typename S, int POL = 0>
__device__ __forceinline__ double bload1(Rsrc r, int off) {
    if constexpr (sizeof(S) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, POL));
    else
        return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, POL));
}

// Two consecutive elements as one access.
template <typename S, int POL = 0>
__device__ __forceinline__ void bload2(Rsrc r, int off, double* o) {
    if constexpr (sizeof(S) == 8) {
        const double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, POL));
        o[0] = v.x;
        o[1] = v.y;
    } else {
        const float2 v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, POL));
        o[0] = v.x;
        o[1] = v.y;
    }
}

template <typename S, int POL = 0>
__device__ __forceinline__ void bstore1(Rsrc r, int off, S v) {
    if constexpr (sizeof(S) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, POL);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, POL);
}

template <typename S, int POL = 0>
__device__ __forceinline__ void bstore2(Rsrc r, int off, const S* v) {
    if constexpr (sizeof(S) == 8) {
        const double2 x = {v[0], v[1]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x), r, off, 0, POL);
    } else {
        const float2 x = {v[0], v[1]};
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, off, 0, POL);
    }
}

// Moments accumulated per cell in FP64 (Sec. II, Eq. Moments_discrete).
struct Acc {
    double s0, sx, sy, se;
};

template <typename PD>
__device__ __forceinline__ void acc_add(Acc& a, const PD& pd, double f) {
    a.s0 = fma(pd.m0, f, a.s0);
    a.sx = fma(pd.mx, f, a.sx);
    a.sy = fma(pd.my, f, a.sy);
    a.se = fma(pd.me, f, a.se);
}

// ---------------------------------------------------------------------------
// One-axis equilibrium factors of node k and of its mirror -p_k from the
// even/odd Horner table row c (HornerLayout<QM>): g = Ge + u Go, gm = Ge - u Go.
// ---------------------------------------------------------------------------
template <int QM>
__device__ __forceinline__ void g_pair(CDp c, double u, double th,
                                       double& g, double& gm) {
    using H = HornerLayout<QM>;
    const double v = u * u;
    double ge = 0.0, go = 0.0;
#pragma unroll
    for (int s = H::S; s >= 0; --s) {
        CDp ce = c + H::off(s);
        double e = ce[H::ne(s) - 1];
#pragma unroll
        for (int i = H::ne(s) - 2; i >= 0; --i) e = fma(e, v, ce[i]);
        double o = 0.0;
        if (H::no(s) > 0) {
            CDp co = ce + H::ne(s);
            o = co[H::no(s) - 1];
#pragma unroll
            for (int i = H::no(s) - 2; i >= 0; --i) o = fma(o, v, co[i]);
        }
        ge = (s == H::S) ? e : fma(ge, th, e);
        go = (s == H::S) ? o : fma(go, th, o);
    }
    g = fma(u, go, ge);
    gm = fma(-u, go, ge);
}

__device__ __forceinline__ PlaneDesc load_desc(CTab* t, int v) {
    const PlaneDesc IMEXLB_CONST& r = t->plane[v];
    PlaneDesc s;
    s.px = r.px; s.py = r.py; s.m0 = r.m0; s.mx = r.mx; s.my = r.my; s.me = r.me;
    s.set = r.set; s.kx = r.kx; s.ky = r.ky; s.pad = 0;
    return s;
}

// g_pair with the Horner row already in registers (loaded once per plane
// and shared by all cells of the thread).
template <int QM>
__device__ __forceinline__ void g_pair_r(const double (&c)[HornerLayout<QM>::total()], double u,
                                         double th, double& g, double& gm) {
    using H = HornerLayout<QM>;
    const double v = u * u;
    double ge = 0.0, go = 0.0;
#pragma unroll
    for (int s = H::S; s >= 0; --s) {
        constexpr int dummy = 0;
        (void)dummy;
        const int oe = H::off(s), no = H::no(s), ne = H::ne(s);
        double e = c[oe + ne - 1];
#pragma unroll
        for (int i = ne - 2; i >= 0; --i) e = fma(e, v, c[oe + i]);
        double o = 0.0;
        if (no > 0) {
            o = c[oe + ne + no - 1];
#pragma unroll
            for (int i = no - 2; i >= 0; --i) o = fma(o, v, c[oe + ne + i]);
        }
        ge = (s == H::S) ? e : fma(ge, th, e);
        go = (s == H::S) ? o : fma(go, th, o);
    }
    g = fma(u, go, ge);
    gm = fma(-u, go, ge);
}

// One entry of the plane order, unpacked from PackedStep.
struct Step {
    double px, py;
    int v, bits;
    __device__ int set() const { return bits & 1; }
    __device__ bool first() const { return (bits >> 1) & 1; }
    __device__ bool new_group() const { return (bits >> 2) & 1; }
    __device__ bool yfirst() const { return (bits >> 3) & 1; }
    __device__ bool new_tab() const { return (bits >> 4) & 1; }
    __device__ bool last() const { return (bits >> 5) & 1; }
    __device__ int slot() const { return (bits >> 6) & 7; }
    __device__ int tcount() const { return (bits >> 9) & 7; }
    __device__ int hx() const { return (bits >> 12) & 31; }
    __device__ int hy() const { return (bits >> 17) & 31; }
};

__device__ __forceinline__ Step load_pstep(CTab* t, int j) {
    const PackedStep IMEXLB_CONST& r = t->step[j];
    Step s;
    s.px = r.px;
    s.py = r.py;
    s.v = r.v;
    s.bits = r.bits;
    return s;
}

template <int QM>
__device__ __forceinline__ CDp hrow(CTab* t, int set, int k) {
    if constexpr (QM == 8) return t->hc8[set][k];
    else return t->hc16[set][k];
}

// The own cells of a thread (one or two) as one access.
template <typename S, int OWN, int POL = 0>
__device__ __forceinline__ void bload_own(Rsrc r, int off, double* o) {
    if constexpr (OWN == 2) bload2<S, POL>(r, off, o);
    else o[0] = bload1<S, POL>(r, off);
}

template <typename S, int OWN>
__device__ __forceinline__ void bstore_own(Rsrc r, int off, const S* v) {
    if constexpr (OWN == 2) bstore2<S, kStreamStore>(r, off, v);
    else bstore1<S, kStreamStore>(r, off, v[0]);
}

// Tile visiting order: patch rows of kPatchH tile rows (the last one may be
// lower), patches of kPatchW tile columns inside a patch row (the last one
// may be narrower), row-major inside a patch; consecutive logical indices go
// to one XCD (blockIdx % 8 selects the XCD).
__device__ __forceinline__ bool tile_of_block(const StageArgs& a, int& tx, int& ty) {
    const int ntiles = a.ntx * a.nty;
    const int l = (blockIdx.x & 7) * a.tiles_per_xcd + (blockIdx.x >> 3);
    if (l >= ntiles) return false;
    const int ph = min(kPatchH, a.nty);
    const int prow = l / (a.ntx * ph), rem = l - prow * a.ntx * ph;
    const int h = min(ph, a.nty - prow * ph);
    const int pcol = rem / (kPatchW * h), rem2 = rem - pcol * kPatchW * h;
    const int w = min(kPatchW, a.ntx - pcol * kPatchW);
    tx = pcol * kPatchW + rem2 % w;
    ty = prow * ph + rem2 / w;
    return true;
}

// ---------------------------------------------------------------------------
// Two-dimensional stage pass.  Tile of TX x TY cells, TX TY / OWN threads.
//  - own cells: thread t owns the OWN consecutive cells (OWN (t % (TX/OWN))
//    .. +OWN-1) of row t / (TX/OWN) (vector loads/stores on interior tiles,
//    FP64 moment accumulators);
//  - loaded cells: own cells plus the 5-cell cross halo (10 TY + 10 TX
//    cells), spread over the threads; each is relaxed on read into the LDS
//    tile;
//  - sweeps: the first half of the threads slides the MP-9 window along x
//    over L = 2 OWN cells of a row, the second half along y over L cells of
//    a column;
//  - x factors (orders up to 8) from LDS tables of one table group of the
//    plane order (kTabNodes2D nodes: two mirror pairs), built when a group
//    starts; above order 8 from one Horner evaluation per loaded cell for a
//    node and its mirror;
//  - three plane loops (Stage2DShape): the mirror-pair loop (even orders:
//    every FP32 pass; both planes of an x-mirror pair per iteration), the
//    software pipeline (FP64 pass 5, and FP32 passes 3 and 5 of odd orders:
//    sweep plane j and relax plane j + 1 into the other of two LDS tiles,
//    the loads of plane j + 2 in flight, one barrier, pointwise step of
//    plane j) and the plain loop (FP64 passes 3 and 4, FP32 pass 4 of odd
//    orders: relax, barrier, sweeps, barrier, pointwise; FP64 pass 3 at
//    three waves per SIMD);
//  - stage 4 keeps the x factors of E^n at its own cells in a second LDS
//    table, built with the x-factor tables.
// LDS pitches are odd so the row-strided x windows and the column-strided
// results spread over all banks.
// ---------------------------------------------------------------------------
template <typename S, int KIND, int QM, int TY, int OWN, bool PAIR>
struct Stage2DShape {
    static constexpr int TX = kTile2X, NT = TX * TY / OWN, L = 2 * OWN;
    static constexpr int OPR = TX / OWN;          // threads per tile row
    static constexpr int P = TX + 11;             // tile pitch (odd)
    static constexpr int VP = TX + 1;             // VF buffer pitch (odd)
    static constexpr int NH = 10 * TY + 10 * TX;  // cross-shaped halo
    static constexpr int HS = (NH + NT - 1) / NT;
    static constexpr int NS = OWN + HS;
    static constexpr bool RELAX = KIND != kAdvect;
    static constexpr bool TAB = RELAX && (QM == 8);
    static constexpr int NLOAD = TX * TY + NH;
    // x-factor table nodes: the table groups of the plane order built by the
    // host
    static constexpr int TABN = kTabNodes2D;
    // stage 4 with tables also keeps the x factors of E^n at its own cells in
    // LDS (one table group, each thread its own entries)
    static constexpr bool NTAB = TAB && KIND == kStage4;
    // software-pipelined plane loop (double-buffered LDS tile and flux
    // buffers) for FP64 pass 5 and for FP32 passes 3 and 5 without the
    // mirror-pair loop (odd orders); stage 4, whose registers are already
    // full with the E^n factors of its own cells, and FP64 stage 3 (three
    // waves per SIMD, below) keep the two-barrier loop when they do not pair
    static constexpr bool PIPE = KIND != kStage4 && (sizeof(S) == 4 || KIND == kStage5) && !PAIR;
    static constexpr int NBUF = (PIPE || PAIR) ? 2 : 1;
    // waves per SIMD the register budget aims at: two work-groups per
    // compute unit; three for FP64 stage 3 with x-factor tables in the
    // single-buffer loop (49 KB of LDS; the moments of the loaded cells, read
    // only when a factor group starts, spill to scratch and are reloaded
    // there)
    static constexpr int WPE = (sizeof(S) == 8 && KIND == kStage3 && QM == 8 && !PAIR) ? 3 : 2 * NT / 256;
};

template <typename S, int KIND, int QM, int TY, int OWN, bool PAIR, bool VEC, bool REC>
__device__ __forceinline__ void stage2d_body(const StageArgs& a, int txi, int tyi, S* tile, S* vfx,
                                             S* vfy, double* gtab, double* gntab) {
    using Sh = Stage2DShape<S, KIND, QM, TY, OWN, PAIR>;
    constexpr int TX = Sh::TX, NT = Sh::NT, L = Sh::L, OPR = Sh::OPR, P = Sh::P, VP = Sh::VP;
    constexpr int NH = Sh::NH, HS = Sh::HS, NS = Sh::NS;
    constexpr bool RELAX = Sh::RELAX;
    static_assert(TY * (TX / L) == NT / 2 && TX * (TY / L) == NT / 2, "sweep split");
    using R = S;
    const int tid = threadIdx.x;
    const int x0 = txi * TX, y0 = tyi * TY;
    const int nx = a.nx, ny = a.ny;
    const long long ps = a.plane_stride;
    CTab* tab = (CTab*)a.tab;

    const int orow = tid / OPR, ox = (tid % OPR) * OWN;
    const int oy = y0 + orow, ox0 = x0 + ox;
    const bool row_real = oy < ny;

    // gcell: global cell read by each loaded slot (ghost nodes mapped by the
    // boundary rule); slots past the end of the halo list read cell gcell[0]
    // (valid, unused) so that every thread issues the same loads.
    int gcell[NS], lidx[NS];
    bool sval[NS];
    {
        const int gy = bc_map(oy, ny, a.bcy) * nx;
#pragma unroll
        for (int i = 0; i < OWN; ++i) {
            gcell[i] = gy + bc_map(ox0 + i, nx, a.bcx);
            sval[i] = true;
            lidx[i] = (orow + 5) * P + ox + i + 5;
        }
#pragma unroll
        for (int j = 0; j < HS; ++j) {
            const int h = tid + j * NT;
            int lx = 0, ly = 0;
            if (h < 10 * TY) {  // x-halo: 5 left + 5 right nodes of each row
                const int k = h % 10;
                ly = h / 10 + 5;
                lx = k < 5 ? k : TX + k;
            } else {            // y-halo: 5 rows below + 5 above
                const int hh = h - 10 * TY;
                const int k = hh / TX;
                lx = hh % TX + 5;
                ly = k < 5 ? k : TY + k;
            }
            sval[OWN + j] = h < NH;
            if (h < NH) {
                gcell[OWN + j] = bc_map(y0 + ly - 5, ny, a.bcy) * nx + bc_map(x0 + lx - 5, nx, a.bcx);
                lidx[OWN + j] = ly * P + lx;
            } else {
                gcell[OWN + j] = gcell[0];
                lidx[OWN + j] = 0;
            }
        }
    }

    // x-factor tables in LDS (orders up to 8): gtab[t * NLOAD + cid] holds
    // g_x of table slot t (node hx + t / 2 of the group's first pair, or its
    // mirror for odd t) at loaded cell cid; rebuilt when a table group starts.
    constexpr bool TAB = Sh::TAB;
    constexpr int NLOAD = Sh::NLOAD;
    int cid[NS];
#pragma unroll
    for (int i = 0; i < OWN; ++i) cid[i] = i * NT + tid;
#pragma unroll
    for (int jh = 0; jh < HS; ++jh) cid[OWN + jh] = TX * TY + jh * NT + tid;

    // Per loaded cell: u_x and T - 1 of the source moments, the y factor
    // A = P_set g_y (P_phi = n, P_chi = (K + D - d) n T) of the current group
    // and of the mirrored group, and (without tables) the cached x factor of
    // the mirrored node.
    double sux[NS], sth[NS], sA[NS], sAm[NS], sgm[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        sux[s] = 0.0;
        sth[s] = 0.0;
        sA[s] = 0.0;
        sAm[s] = 0.0;
        sgm[s] = 0.0;
        if (RELAX) {
            sux[s] = a.msrc[ps + gcell[s]];
            sth[s] = a.msrc[3 * ps + gcell[s]] - 1.0;
        }
    }
    // n and u_y of the loaded cells (y factors), kept for the whole pass
    double gn[NS], guy[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int c = gcell[s];
        gn[s] = RELAX ? a.msrc[c] : 0.0;
        guy[s] = RELAX ? a.msrc[2 * ps + c] : 0.0;
    }
    // Stage 4 also needs E^n at its own cells (moments of F^n).
    double nux[OWN], nth[OWN], nA[OWN], nAm[OWN], ngm[OWN], gnn[OWN], gnuy[OWN];
#pragma unroll
    for (int i = 0; i < OWN; ++i) {
        nux[i] = 0.0;
        nth[i] = 0.0;
        nA[i] = 0.0;
        nAm[i] = 0.0;
        ngm[i] = 0.0;
        gnn[i] = 0.0;
        gnuy[i] = 0.0;
        if (KIND == kStage4) {
            nux[i] = a.mn[ps + gcell[i]];
            nth[i] = a.mn[3 * ps + gcell[i]] - 1.0;
            gnn[i] = a.mn[gcell[i]];
            gnuy[i] = a.mn[2 * ps + gcell[i]];
        }
    }
    Acc acc[OWN];
#pragma unroll
    for (int i = 0; i < OWN; ++i) acc[i] = Acc{0.0, 0.0, 0.0, 0.0};

    // Global loads of one plane: the source plane at the loaded cells and,
    // for stages 4 and 5, the state buffer at the own cells (byte offsets
    // within the plane; own cells of interior tiles as one vector access).
    static_assert(OWN == 1 || OWN == 2, "own-cell accesses take one or two cells");
    int boff[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) boff[s] = gcell[s] * (int)sizeof(S);
    const int own_off = (oy * nx + ox0) * (int)sizeof(S);
    // element offset of plane v: one 32 x 32 -> 64-bit product (a plane
    // holds fewer than 2^31 elements, checked on the host)
    const unsigned ps32 = (unsigned)ps;
    auto plane_off = [&](int v) -> size_t { return (size_t)((unsigned long long)(unsigned)v * ps32); };
    // Loads of plane v; with live == false (the padding entries past the
    // last plane) the buffer resources have no records, so the loads return
    // zeros without touching memory while every iteration still issues them
    // (a conditional load would make the compiler wait for it right away).
    double pg[NS], pf[OWN];
    auto fetch_to = [&](double (&pg)[NS], double (&pf)[OWN], int v, bool live) IMEXLB_INLINE {
        const long long recs = live ? ps : 0;
        const Rsrc rs = plane_rsrc(static_cast<const S*>(a.src) + plane_off(v), recs);
        if constexpr (VEC) {
            bload_own<S, OWN>(rs, boff[0], pg);
        } else {
#pragma unroll
            for (int i = 0; i < OWN; ++i) pg[i] = bload1<S>(rs, boff[i]);
        }
#pragma unroll
        for (int jh = 0; jh < HS; ++jh) pg[OWN + jh] = bload1<S>(rs, boff[OWN + jh]);
        if constexpr (KIND == kStage4 || KIND == kStage5) {
            const Rsrc rf = plane_rsrc(static_cast<const S*>(a.fbuf) + plane_off(v), recs);
            if constexpr (VEC) {
                bload_own<S, OWN, kStreamLoad>(rf, boff[0], pf);
            } else {
#pragma unroll
                for (int i = 0; i < OWN; ++i) pf[i] = bload1<S, kStreamLoad>(rf, boff[i]);
            }
        }
    };
    auto fetch = [&](int v, bool live) { fetch_to(pg, pf, v, live); };

    constexpr int NC = HornerLayout<QM>::total();
    constexpr int TSZ = (TY + 10) * P, VSZ = TY * VP;
    // relax-time part of the pointwise stage algebra at the own cells: the
    // stage value without its flux term (stage 4: the stage value and R)
    constexpr int NB = KIND == kStage4 ? 2 : 1;

    // Relax on read of plane st (loads in pg / pf) into the LDS tile tl;
    // updates the factor caches when a table group or a y group starts.
    // x factors come from the LDS tables, or (orders above 8, and stage 4's
    // own E^n) from one Horner evaluation per cell on the first plane of a
    // mirror pair, the second plane using the cached mirror factor.
    auto relax_from = [&](const double (&pg)[NS], const double (&pf)[OWN], const Step& st, S* tl,
                          double (&base)[NB][OWN]) IMEXLB_INLINE {
        double g[NS], fb[OWN];
#pragma unroll
        for (int s = 0; s < NS; ++s) g[s] = pg[s];
#pragma unroll
        for (int i = 0; i < OWN; ++i) fb[i] = pf[i];
        if constexpr (RELAX) {
            if constexpr (TAB) {
                if (st.new_tab()) {  // x factors of the mirror pairs of this table group
                    for (int p = 0; p < st.tcount(); ++p) {
                        CDp hx = hrow<QM>(tab, st.set(), st.hx() + p);
                        double cf[NC];
#pragma unroll
                        for (int i = 0; i < NC; ++i) cf[i] = hx[i];
#pragma unroll
                        for (int s = 0; s < NS; ++s) {
                            if (sval[s]) {
                                double gp, gq;
                                g_pair_r<QM>(cf, sux[s], sth[s], gp, gq);
                                gtab[(2 * p) * NLOAD + cid[s]] = gp;
                                gtab[(2 * p + 1) * NLOAD + cid[s]] = gq;
                            }
                        }
                        if constexpr (Sh::NTAB) {
#pragma unroll
                            for (int i = 0; i < OWN; ++i) {
                                double gp, gq;
                                g_pair_r<QM>(cf, nux[i], nth[i], gp, gq);
                                gntab[(2 * p) * (TX * TY) + cid[i]] = gp;
                                gntab[(2 * p + 1) * (TX * TY) + cid[i]] = gq;
                            }
                        }
                    }
                }
            }
            // (both branches of the factor updates assign the same arrays, so
            // that they stay in registers)
            if (st.new_group()) {  // y factors of the group (and of its mirror)
                double tA[NS], tAm[NS], tnA[OWN], tnAm[OWN];
                if (st.yfirst()) {
                    CDp hy = hrow<QM>(tab, st.set(), st.hy());
                    double cf[NC];
#pragma unroll
                    for (int i = 0; i < NC; ++i) cf[i] = hy[i];
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        const double n = gn[s];
                        const double pre = st.set() ? a.chi_fac * n * (sth[s] + 1.0) : n;
                        double gp, gq;
                        g_pair_r<QM>(cf, guy[s], sth[s], gp, gq);
                        tA[s] = pre * gp;
                        tAm[s] = pre * gq;
                    }
#pragma unroll
                    for (int i = 0; i < OWN; ++i) {
                        tnA[i] = 0.0;
                        tnAm[i] = 0.0;
                        if constexpr (KIND == kStage4) {
                            const double n = gnn[i];
                            const double pre = st.set() ? a.chi_fac * n * (nth[i] + 1.0) : n;
                            double gp, gq;
                            g_pair_r<QM>(cf, gnuy[i], nth[i], gp, gq);
                            tnA[i] = pre * gp;
                            tnAm[i] = pre * gq;
                        }
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        tA[s] = sAm[s];
                        tAm[s] = sAm[s];
                    }
#pragma unroll
                    for (int i = 0; i < OWN; ++i) {
                        tnA[i] = nAm[i];
                        tnAm[i] = nAm[i];
                    }
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    sA[s] = tA[s];
                    sAm[s] = tAm[s];
                }
#pragma unroll
                for (int i = 0; i < OWN; ++i) {
                    nA[i] = tnA[i];
                    nAm[i] = tnAm[i];
                }
            }
        }

        double eown[OWN];
        double gxs[NS], gxn[OWN];
        if constexpr (RELAX) {
            if constexpr (TAB) {
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    gxs[s] = gtab[st.slot() * NLOAD + (sval[s] ? cid[s] : cid[0])];
            }
            double tgx[NS], tgm[NS], tgn[OWN], tgnm[OWN];
            if (st.first()) {
                CDp hx = hrow<QM>(tab, st.set(), st.hx());
                double cf[NC];
#pragma unroll
                for (int i = 0; i < NC; ++i) cf[i] = hx[i];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    tgx[s] = 0.0;
                    tgm[s] = 0.0;
                    if constexpr (!TAB) g_pair_r<QM>(cf, sux[s], sth[s], tgx[s], tgm[s]);
                }
#pragma unroll
                for (int i = 0; i < OWN; ++i) {
                    tgn[i] = 0.0;
                    tgnm[i] = 0.0;
                    if constexpr (KIND == kStage4 && !Sh::NTAB) g_pair_r<QM>(cf, nux[i], nth[i], tgn[i], tgnm[i]);
                }
            } else {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    tgx[s] = sgm[s];
                    tgm[s] = sgm[s];
                }
#pragma unroll
                for (int i = 0; i < OWN; ++i) {
                    tgn[i] = ngm[i];
                    tgnm[i] = ngm[i];
                }
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if constexpr (!TAB) gxs[s] = tgx[s];
                sgm[s] = tgm[s];
            }
#pragma unroll
            for (int i = 0; i < OWN; ++i) {
                if constexpr (Sh::NTAB) gxn[i] = gntab[st.slot() * (TX * TY) + cid[i]];
                else gxn[i] = tgn[i];
                ngm[i] = tgnm[i];
            }
        }
        S rec[OWN];  // the stage values at the own cells, as swept
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            double e = 0.0;
            if constexpr (RELAX) e = sA[s] * gxs[s];
            if (s < OWN) eown[s] = e;
            if (sval[s]) {
                const double val = RELAX ? fma(a.a_rel, g[s], a.b_rel * e) : g[s];
                tl[lidx[s]] = (S)val;
                if (s < OWN) rec[s] = (S)val;
            }
        }
        if constexpr (REC && RELAX) {
            const Rsrc rr = plane_rsrc(static_cast<S*>(a.sval_out) + plane_off(st.v), ps);
            if constexpr (VEC) {
                bstore_own<S, OWN>(rr, own_off, rec);
            } else {
#pragma unroll
                for (int i = 0; i < OWN; ++i)
                    if (row_real && ox0 + i < nx) bstore1<S, kStreamStore>(rr, own_off + i * (int)sizeof(S), rec[i]);
            }
        }
        // stage algebra with the host-combined coefficients k[] (see
        // StageArgs), the flux term added in the pointwise step
#pragma unroll
        for (int i = 0; i < OWN; ++i) {
            if constexpr (KIND == kStage3) {
                base[0][i] = fma(-a.k[0], g[i] - eown[i], g[i]);
            } else if constexpr (KIND == kStage4) {
                const double fn = fb[i], g3 = g[i];
                const double dn = fn - nA[i] * gxn[i], d3 = g3 - eown[i];
                base[0][i] = fma(0.75, fn, fma(0.25, g3, fma(a.k[1], dn, -a.k[2] * d3)));
                base[1][i] = fma(5.0 / 6.0, fn, fma(1.0 / 6.0, g3, fma(-a.k[3], dn, -a.k[4] * d3)));
            } else if constexpr (KIND == kStage5) {
                base[0][i] = fma(-a.k[5], g[i] - eown[i], fb[i]);
            } else {
                base[0][i] = 0.0;
            }
        }
        // the bases are computed here, not sunk into the pointwise step: the
        // loaded values then die here and the next loads reuse their
        // registers (no copy, hence no early wait, at the loop latch)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int i = 0; i < OWN; ++i) opaque(base[b][i]);
    };

    auto relax = [&](const Step& st, S* tl, double (&base)[NB][OWN]) { relax_from(pg, pf, st, tl, base); };

    // MP-9 sweeps of one plane from the LDS tile tl into the flux buffers
    // fx, fy: the first half of the threads along x (row tid % TY, cells
    // L (tid / TY) .. +L-1), the second along y (column (tid - NT/2) % TX,
    // cells L seg .. +L-1).
    auto sweep = [&](const Step& st, const S* tl, R* fx, R* fy) IMEXLB_INLINE {
        if (tid < NT / 2) {
            if (st.px != 0.0) {
                const int row = tid % TY, seg = tid / TY;
                const S* lo = tl + (row + 5) * P + seg * L;
                R* o = fx + row * VP + seg * L;
                if (st.px > 0.0) mp9_sweep<R, S, L, 1, 1, true>(lo, o);
                else mp9_sweep<R, S, L, 1, 1, false>(lo + 1, o);
            }
        } else {
            if (st.py != 0.0) {
                const int i2 = tid - NT / 2;
                const int col = i2 % TX, seg = i2 / TX;
                const S* lo = tl + seg * L * P + col + 5;
                R* o = fy + seg * L * VP + col;
                if (st.py > 0.0) mp9_sweep<R, S, L, P, VP, true>(lo, o);
                else mp9_sweep<R, S, L, P, VP, false>(lo + P, o);
            }
        }
    };

    // Flux term, stores and moment accumulation of one plane.
    auto pointwise = [&](const Step& st, const R* fx, const R* fy, const double (&base)[NB][OWN]) IMEXLB_INLINE {
        const double sx = fabs(st.px) * a.inv_dx;
        const double sy = fabs(st.py) * a.inv_dy;
        double vf[OWN];
#pragma unroll
        for (int i = 0; i < OWN; ++i)
            vf[i] = fma((double)fy[orow * VP + ox + i], sy, (double)fx[orow * VP + ox + i] * sx);

        if constexpr (KIND == kAdvect) {
            double* o = static_cast<double*>(a.out) + plane_off(st.v) + (size_t)oy * nx + ox0;
#pragma unroll
            for (int i = 0; i < OWN; ++i)
                if (row_real && ox0 + i < nx) o[i] = vf[i];
        } else {
            S outv[OWN], fbv[OWN];
#pragma unroll
            for (int i = 0; i < OWN; ++i) {
                if constexpr (KIND == kStage3) {
                    outv[i] = (S)fma(-a.dt, vf[i], base[0][i]);
                    fbv[i] = outv[i];
                } else if constexpr (KIND == kStage4) {
                    outv[i] = (S)fma(-0.25 * a.dt, vf[i], base[0][i]);
                    fbv[i] = (S)fma(-(1.0 / 6.0) * a.dt, vf[i], base[1][i]);
                } else {  // kStage5
                    fbv[i] = (S)fma(-(2.0 / 3.0) * a.dt, vf[i], base[0][i]);
                    outv[i] = fbv[i];
                }
            }
            const Rsrc ro = plane_rsrc(static_cast<S*>(KIND == kStage5 ? a.fbuf : a.out) + plane_off(st.v), ps);
            if constexpr (VEC) {
                bstore_own<S, OWN>(ro, own_off, outv);
            } else {
#pragma unroll
                for (int i = 0; i < OWN; ++i)
                    if (row_real && ox0 + i < nx) bstore1<S, kStreamStore>(ro, own_off + i * (int)sizeof(S), outv[i]);
            }
            if constexpr (KIND == kStage4) {
                // R over the state buffer, or (recorded steps, which may be
                // out of place) into rbuf; the plain passes keep one pointer
                const Rsrc rf = plane_rsrc(static_cast<S*>(REC ? a.rbuf : a.fbuf) + plane_off(st.v), ps);
                if constexpr (VEC) {
                    bstore_own<S, OWN>(rf, own_off, fbv);
                } else {
#pragma unroll
                    for (int i = 0; i < OWN; ++i)
                        if (row_real && ox0 + i < nx) bstore1<S, kStreamStore>(rf, own_off + i * (int)sizeof(S), fbv[i]);
                }
            }
            if (st.set() == 0) {
#pragma unroll
                for (int i = 0; i < OWN; ++i) {
                    const double f = (double)outv[i];
                    acc[i].s0 += f;
                    acc[i].sx = fma(st.px, f, acc[i].sx);
                    acc[i].sy = fma(st.py, f, acc[i].sy);
                    acc[i].se = fma(fma(st.px, st.px, st.py * st.py), f, acc[i].se);
                }
            } else {
#pragma unroll
                for (int i = 0; i < OWN; ++i) acc[i].se += (double)outv[i];
            }
        }
    };

    // The flux buffers start at zero: a plane whose velocity component is
    // zero skips that sweep and reads zeros (times a zero speed).  The step
    // table carries two padding entries past the last plane, so the
    // look-ahead loads need no bound test.
    for (int i = tid; i < Sh::NBUF * VSZ; i += NT) {
        vfx[i] = S(0);
        vfy[i] = S(0);
    }
    Step st = load_pstep(tab, 0);  // plane swept in the current iteration
    Step s1 = load_pstep(tab, 1);  // the plane after it
    double bcur[NB][OWN], bnext[NB][OWN];
    fetch(st.v, true);
    if constexpr (PAIR) {
        // Planes in x-mirror pairs (kx, ky), (Q - 1 - kx, ky), consecutive in
        // the plane order (even orders): both planes of a pair per iteration,
        // their global loads issued together one iteration ahead (fixed
        // register sets A and B), x factors of both from the LDS tables (or,
        // above order 8, from one Horner evaluation per loaded cell), relax
        // both into two tiles, barrier, sweep both into two pairs of flux
        // buffers, barrier, pointwise steps of both.
        double pgB[NS], pfB[OWN], bB[NB][OWN];
        fetch_to(pgB, pfB, s1.v, true);
        for (int j = 0;; j += 2) {
            const Step na = load_pstep(tab, j + 2), nb = load_pstep(tab, j + 3);
            const bool more = !s1.last();
            relax_from(pg, pf, st, tile, bcur);
            relax_from(pgB, pfB, s1, tile + TSZ, bB);
            fetch_to(pg, pf, na.v, more);
            fetch_to(pgB, pfB, nb.v, more);
            __syncthreads();
            sweep(st, tile, vfx, vfy);
            sweep(s1, tile + TSZ, vfx + VSZ, vfy + VSZ);
            __syncthreads();
            pointwise(st, vfx, vfy, bcur);
            pointwise(s1, vfx + VSZ, vfy + VSZ, bB);
            if (!more) break;
            st = na;
            s1 = nb;
        }
    } else if constexpr (Sh::PIPE) {
        // Software pipeline over the planes, two LDS tiles and two pairs of
        // flux buffers: iteration j sweeps plane j out of tile j % 2 and
        // relaxes plane j + 1 into the other tile, one barrier, then the
        // pointwise step of plane j.  A tile is rewritten two iterations
        // after it was swept and a flux buffer two iterations after it was
        // read, each time with a barrier in between, so one barrier per
        // plane suffices.
        relax(st, tile, bcur);
        fetch(s1.v, !st.last());
        __syncthreads();
        int buf = 0;
        for (int j = 0;; ++j) {  // ends at the plane flagged last
            const Step sn = s1;
            s1 = load_pstep(tab, j + 2);
            sweep(st, tile + buf * TSZ, vfx + buf * VSZ, vfy + buf * VSZ);
            if (!st.last()) relax(sn, tile + (buf ^ 1) * TSZ, bnext);
            fetch(s1.v, !st.last() && !sn.last());
            __syncthreads();
            pointwise(st, vfx + buf * VSZ, vfy + buf * VSZ, bcur);
            if (st.last()) break;
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int i = 0; i < OWN; ++i) bcur[b][i] = bnext[b][i];
            st = sn;
            buf ^= 1;
        }
    } else {
        // One tile and one pair of flux buffers: relax (the next plane's
        // loads in flight), barrier, sweeps, barrier, pointwise step.
        for (int j = 0;; ++j) {
            const Step sn = s1;
            s1 = load_pstep(tab, j + 2);
            relax(st, tile, bcur);
            fetch(sn.v, !st.last());
            __syncthreads();
            sweep(st, tile, vfx, vfy);
            __syncthreads();
            pointwise(st, vfx, vfy, bcur);
            if (st.last()) break;
            st = sn;
        }
    }

    if constexpr (KIND != kAdvect) {
#pragma unroll
        for (int i = 0; i < OWN; ++i) {
            if (row_real && ox0 + i < nx) {
                const double n = acc[i].s0;
                const double ux = acc[i].sx / n, uy = acc[i].sy / n;
                const double T = (acc[i].se - n * (ux * ux + uy * uy)) / (a.dk * n);
                const size_t c = (size_t)oy * nx + ox0 + i;
                a.mout[c] = n;
                a.mout[ps + c] = ux;
                a.mout[2 * ps + c] = uy;
                a.mout[3 * ps + c] = T;
            }
        }
    }
}

template <typename S, int KIND, int QM, int TY, int OWN, bool PAIR, bool REC>
__global__ void __launch_bounds__(kTile2X * TY / OWN)
__attribute__((amdgpu_waves_per_eu(Stage2DShape<S, KIND, QM, TY, OWN, PAIR>::WPE)))
stage2d_kernel(StageArgs a) {
    using Sh = Stage2DShape<S, KIND, QM, TY, OWN, PAIR>;
    __shared__ S tile[Sh::NBUF * (TY + 10) * Sh::P];
    __shared__ S vfx[Sh::NBUF * TY * Sh::VP];
    __shared__ S vfy[Sh::NBUF * TY * Sh::VP];
    __shared__ double gtab[Sh::TAB ? Sh::TABN * Sh::NLOAD : 1];
    __shared__ double gntab[Sh::NTAB ? Sh::TABN * kTile2X * TY : 1];
    int txi, tyi;
    if (!tile_of_block(a, txi, tyi)) return;
    // interior tiles of a grid whose rows are multiples of OWN take the
    // vector-access path; tiles at a ragged edge the element-wise one
    const bool vec = ((txi + 1) * Sh::TX <= a.nx) && ((tyi + 1) * TY <= a.ny) && (a.nx % OWN == 0);
    if (vec) stage2d_body<S, KIND, QM, TY, OWN, PAIR, true, REC>(a, txi, tyi, tile, vfx, vfy, gtab, gntab);
    else stage2d_body<S, KIND, QM, TY, OWN, PAIR, false, REC>(a, txi, tyi, tile, vfx, vfy, gtab, gntab);
}

// ---------------------------------------------------------------------------
// One-dimensional stage pass over a tile of TX cells, TX / 4 threads, 4
// consecutive cells per thread (one or two vector accesses).
//  - loaded cells: the 4 own cells of every thread plus the 10 halo cells
//    (threads 0..9); cells past the end of the grid map through the
//    boundary rule and act as the ghost nodes of Sec. IV;
//  - planes run set by set with every node followed by its mirror, so one
//    even/odd Horner evaluation per loaded cell gives the x factors of both
//    (the second plane uses the cached mirror factor);
//  - per plane: relax on read into one of two LDS tiles (the next plane's
//    global loads already in flight), one barrier, MP-9 sweep of the
//    thread's own 4 cells (flux differences stay in registers), pointwise
//    stage algebra, stores, FP64 moment accumulation.
// The arguments come by reference so that the batched kernel can read them
// from a per-tube table with scalar loads.
// ---------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ void bload4(Rsrc r, int off, double* o) {
    if constexpr (sizeof(S) == 8) {
        bload2<S>(r, off, o);
        bload2<S>(r, off + 16, o + 2);
    } else {
        const float4 v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
}

template <typename S>
__device__ __forceinline__ void bstore4(Rsrc r, int off, const S* v) {
    if constexpr (sizeof(S) == 8) {
        bstore2<S>(r, off, v);
        bstore2<S>(r, off + 16, v + 2);
    } else {
        const float4 x = {v[0], v[1], v[2], v[3]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x), r, off, 0, 0);
    }
}

template <typename S, int KIND, int QM, int TX, bool VEC, typename A>
__device__ __forceinline__ void stage1d_body(const A& a, int x0, S (*tile)[TX + 10]) {
    constexpr int L = 4, NT = TX / L, NS = L + 1;
    constexpr bool RELAX = KIND != kAdvect;
    static_assert(NT * L == TX && NT >= 10, "tile / thread mismatch");
    using R = S;
    const int tid = threadIdx.x;
    const int nx = a.nx, bcx = a.bcx;
    const long long ps = a.plane_stride, ms = a.mstride;
    const double* msrc = a.msrc;
    CTab* tab = (CTab*)a.tab;
    const int ox0 = x0 + tid * L;

    // loaded slots: own cells 0..3, halo slot 4 (threads 0..9; the others
    // load cell gcell[0] again so that every thread issues the same loads)
    int gcell[NS], lidx[NS];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        gcell[i] = bc_map(ox0 + i, nx, bcx);
        lidx[i] = tid * L + i + 5;
    }
    const bool hval = tid < 10;
    {
        const int lx = tid < 5 ? tid : TX + tid;
        gcell[L] = hval ? bc_map(x0 + lx - 5, nx, bcx) : gcell[0];
        lidx[L] = hval ? lx : 0;
    }
    int boff[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) boff[s] = gcell[s] * (int)sizeof(S);
    const int own_off = ox0 * (int)sizeof(S);

    // source moments at the loaded cells, F^n moments at the own cells (stage 4)
    // sP: the set prefactor P_phi = n, turned into P_chi = (K + D - d) n T
    // at the start of the chi set
    double sux[NS], sth[NS], sP[NS], sgm[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        sux[s] = RELAX ? msrc[ms + gcell[s]] : 0.0;
        sth[s] = RELAX ? msrc[2 * ms + gcell[s]] - 1.0 : 0.0;
        sP[s] = RELAX ? msrc[gcell[s]] : 0.0;
        sgm[s] = 0.0;
    }
    double nux[L], nth[L], nP[L], ngm[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        nux[i] = KIND == kStage4 ? a.mn[ms + gcell[i]] : 0.0;
        nth[i] = KIND == kStage4 ? a.mn[2 * ms + gcell[i]] - 1.0 : 0.0;
        nP[i] = KIND == kStage4 ? a.mn[gcell[i]] : 0.0;
        ngm[i] = 0.0;
    }
    Acc acc[L];
#pragma unroll
    for (int i = 0; i < L; ++i) acc[i] = Acc{0.0, 0.0, 0.0, 0.0};

    // element offset of plane v (a plane holds fewer than 2^31 elements)
    const unsigned ps32 = (unsigned)ps;
    auto plane_off = [&](int v) -> size_t { return (size_t)((unsigned long long)(unsigned)v * ps32); };
    // Loads of plane v; past the last plane (live == false) the resources
    // have no records, so every iteration issues the same loads.
    double pg[NS], pf[L];
    auto fetch = [&](int v, bool live) IMEXLB_INLINE {
        const long long recs = live ? ps : 0;
        const Rsrc rs = plane_rsrc(static_cast<const S*>(a.src) + plane_off(v), recs);
        if constexpr (VEC) {
            bload4<S>(rs, boff[0], pg);
        } else {
#pragma unroll
            for (int i = 0; i < L; ++i) pg[i] = bload1<S>(rs, boff[i]);
        }
        pg[L] = bload1<S>(rs, boff[L]);
        if constexpr (KIND == kStage4 || KIND == kStage5) {
            const Rsrc rf = plane_rsrc(static_cast<const S*>(a.fbuf) + plane_off(v), recs);
            if constexpr (VEC) {
                bload4<S>(rf, boff[0], pf);
            } else {
#pragma unroll
                for (int i = 0; i < L; ++i) pf[i] = bload1<S>(rf, boff[i]);
            }
        }
    };

    constexpr int NC = HornerLayout<QM>::total();
    // relax-time part of the stage algebra at the own cells (the stage value
    // without its flux term; stage 4: the stage value and R)
    constexpr int NB = KIND == kStage4 ? 2 : 1;
    Step st = load_pstep(tab, 0);
    Step s1 = load_pstep(tab, 1);
    fetch(st.v, true);
    for (int j = 0;; ++j) {  // ends at the plane flagged last
        const Step sn = s1;
        s1 = load_pstep(tab, j + 2);
        S* buf = tile[j & 1];

        // relax on read of the loaded planes into the LDS tile
        double e[NS], en[L];
        if constexpr (RELAX) {
            if (st.new_tab() && st.set() == 1) {
#pragma unroll
                for (int s = 0; s < NS; ++s) sP[s] = a.chi_fac * sP[s] * (sth[s] + 1.0);
                if constexpr (KIND == kStage4) {
#pragma unroll
                    for (int i = 0; i < L; ++i) nP[i] = a.chi_fac * nP[i] * (nth[i] + 1.0);
                }
            }
            // (both branches assign the same arrays, so that they stay in registers)
            double gx[NS], tgm[NS], gxn[L], tngm[L];
            if (st.first()) {
                CDp hx = hrow<QM>(tab, st.set(), st.hx());
                double cf[NC];
#pragma unroll
                for (int i = 0; i < NC; ++i) cf[i] = hx[i];
#pragma unroll
                for (int s = 0; s < NS; ++s) g_pair_r<QM>(cf, sux[s], sth[s], gx[s], tgm[s]);
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    gxn[i] = 0.0;
                    tngm[i] = 0.0;
                    if constexpr (KIND == kStage4) g_pair_r<QM>(cf, nux[i], nth[i], gxn[i], tngm[i]);
                }
            } else {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    gx[s] = sgm[s];
                    tgm[s] = sgm[s];
                }
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    gxn[i] = ngm[i];
                    tngm[i] = ngm[i];
                }
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                sgm[s] = tgm[s];
                e[s] = sP[s] * gx[s];
            }
#pragma unroll
            for (int i = 0; i < L; ++i) {
                ngm[i] = tngm[i];
                en[i] = KIND == kStage4 ? nP[i] * gxn[i] : 0.0;
            }
        } else {
#pragma unroll
            for (int s = 0; s < NS; ++s) e[s] = 0.0;
#pragma unroll
            for (int i = 0; i < L; ++i) en[i] = 0.0;
        }
#pragma unroll
        for (int s = 0; s < L; ++s) buf[lidx[s]] = (S)(RELAX ? fma(a.a_rel, pg[s], a.b_rel * e[s]) : pg[s]);
        if (hval) buf[lidx[L]] = (S)(RELAX ? fma(a.a_rel, pg[L], a.b_rel * e[L]) : pg[L]);
        // stage algebra with the host-combined coefficients k[] (see
        // StageArgs), the flux term added after the sweep
        double base[NB][L];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            if constexpr (KIND == kStage3) {
                base[0][i] = fma(-a.k[0], pg[i] - e[i], pg[i]);
            } else if constexpr (KIND == kStage4) {
                const double fn = pf[i], g3 = pg[i];
                const double dn = fn - en[i], d3 = g3 - e[i];
                base[0][i] = fma(0.75, fn, fma(0.25, g3, fma(a.k[1], dn, -a.k[2] * d3)));
                base[1][i] = fma(5.0 / 6.0, fn, fma(1.0 / 6.0, g3, fma(-a.k[3], dn, -a.k[4] * d3)));
            } else if constexpr (KIND == kStage5) {
                base[0][i] = fma(-a.k[5], pg[i] - e[i], pf[i]);
            } else {
                base[0][i] = 0.0;
            }
        }
        // computed here, so that the loaded registers die and the next
        // loads reuse them (no copy, hence no early wait)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int i = 0; i < L; ++i) opaque(base[b][i]);
        fetch(sn.v, !st.last());
        __syncthreads();

        // MP-9 over the own cells: window of L + 9 values around them
        double vf[L];
#pragma unroll
        for (int i = 0; i < L; ++i) vf[i] = 0.0;
        if (st.px != 0.0) {
            R w[L + 9], dif[L];
            const S* lo = buf + tid * L;
            if (st.px > 0.0) {
#pragma unroll
                for (int m = 0; m < L + 9; ++m) w[m] = (R)lo[m];
                mp9_line<R, L>(w, dif);
            } else {
#pragma unroll
                for (int m = 0; m < L + 9; ++m) w[m] = (R)lo[L + 9 - m];
                R dr[L];
                mp9_line<R, L>(w, dr);
#pragma unroll
                for (int i = 0; i < L; ++i) dif[i] = dr[L - 1 - i];
            }
            const double sx = fabs(st.px) * a.inv_dx;
#pragma unroll
            for (int i = 0; i < L; ++i) vf[i] = (double)dif[i] * sx;
        }

        if constexpr (KIND == kAdvect) {
            double* o = static_cast<double*>(a.out) + plane_off(st.v) + ox0;
#pragma unroll
            for (int i = 0; i < L; ++i)
                if (ox0 + i < nx) o[i] = vf[i];
        } else {
            S outv[L], fbv[L];
#pragma unroll
            for (int i = 0; i < L; ++i) {
                if constexpr (KIND == kStage3) {
                    outv[i] = (S)fma(-a.dt, vf[i], base[0][i]);
                    fbv[i] = outv[i];
                } else if constexpr (KIND == kStage4) {
                    outv[i] = (S)fma(-0.25 * a.dt, vf[i], base[0][i]);
                    fbv[i] = (S)fma(-(1.0 / 6.0) * a.dt, vf[i], base[1][i]);
                } else {  // kStage5
                    fbv[i] = (S)fma(-(2.0 / 3.0) * a.dt, vf[i], base[0][i]);
                    outv[i] = fbv[i];
                }
            }
            const Rsrc ro = plane_rsrc(static_cast<S*>(KIND == kStage5 ? a.fbuf : a.out) + plane_off(st.v), ps);
            if constexpr (VEC) {
                bstore4<S>(ro, own_off, outv);
            } else {
#pragma unroll
                for (int i = 0; i < L; ++i)
                    if (ox0 + i < nx) bstore1<S>(ro, own_off + i * (int)sizeof(S), outv[i]);
            }
            if constexpr (KIND == kStage4) {
                const Rsrc rf = plane_rsrc(static_cast<S*>(a.rbuf) + plane_off(st.v), ps);
                if constexpr (VEC) {
                    bstore4<S>(rf, own_off, fbv);
                } else {
#pragma unroll
                    for (int i = 0; i < L; ++i)
                        if (ox0 + i < nx) bstore1<S>(rf, own_off + i * (int)sizeof(S), fbv[i]);
                }
            }
            if (st.set() == 0) {
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    const double f = (double)outv[i];
                    acc[i].s0 += f;
                    acc[i].sx = fma(st.px, f, acc[i].sx);
                    acc[i].se = fma(st.px * st.px, f, acc[i].se);
                }
            } else {
#pragma unroll
                for (int i = 0; i < L; ++i) acc[i].se += (double)outv[i];
            }
        }
        if (st.last()) break;
        st = sn;
    }

    if constexpr (KIND != kAdvect) {
#pragma unroll
        for (int i = 0; i < L; ++i) {
            if (ox0 + i < nx) {
                const double n = acc[i].s0;
                const double ux = acc[i].sx / n;
                const double T = (acc[i].se - n * ux * ux) / (a.dk * n);
                const size_t c = (size_t)ox0 + i;
                a.mout[c] = n;
                a.mout[ms + c] = ux;
                a.mout[2 * ms + c] = T;
            }
        }
    }
}

// interior tiles of a line whose planes start at multiples of 4 elements
// take the vector-access body, tiles at a ragged end the element-wise one
template <typename S, int KIND, int QM, int TX, typename A>
__device__ __forceinline__ void stage1d_tile(const A& a, int x0, S (*tile)[TX + 10]) {
    if ((x0 + TX <= a.nx) && (a.plane_stride % 4 == 0)) stage1d_body<S, KIND, QM, TX, true>(a, x0, tile);
    else stage1d_body<S, KIND, QM, TX, false>(a, x0, tile);
}

template <typename S, int KIND, int QM, int TX>
__global__ void __launch_bounds__(TX / 4) __attribute__((amdgpu_waves_per_eu(2)))
stage1d_kernel(StageArgs a) {
    __shared__ S tile[2][TX + 10];
    const int logical = (blockIdx.x & 7) * a.tiles_per_xcd + (blockIdx.x >> 3);
    if (logical >= a.ntx) return;
    stage1d_tile<S, KIND, QM, TX>(a, logical * TX, tile);
}

// Batched form: block j runs tile tiles[j] = (tube, first cell) with that
// tube's arguments for this pass.
typedef const StageArgs IMEXLB_CONST CArgs;
template <typename S, int KIND, int QM, int TX>
__global__ void __launch_bounds__(TX / 4) __attribute__((amdgpu_waves_per_eu(2)))
stage1d_batch_kernel(const StageArgs* targs, const int2* tiles, int ntiles) {
    __shared__ S tile[2][TX + 10];
    if ((int)blockIdx.x >= ntiles) return;
    const int IMEXLB_CONST* tp = (const int IMEXLB_CONST*)tiles + 2 * blockIdx.x;
    CArgs& a = ((CArgs*)targs)[tp[0]];
    stage1d_tile<S, KIND, QM, TX>(a, tp[1], tile);
}

// Persistent batched form (temporal blocking).  Block b owns a bin of
// items (tubes, or chunks of outflow tubes) for nsteps whole steps.  An
// item's region extends its own cells by 15 cells per step on each side
// (clamped to the tube): a pass's stencil reaches 5 cells, so the values
// that the clamped ghost nodes at an artificial region end make wrong
// spread 5 cells per pass and stay outside the own cells for the whole
// launch; at a true tube end the clamp is the outflow rule.  Each item's
// state and moments are copied into its private area, stepped there (the
// passes of all items of the bin, with a work-group barrier after every
// tile, which also separates the passes), and the own cells copied out to
// buffers distinct from the inputs, so that no block overwrites cells
// another block still reads.  No block waits for another.
template <typename S, int KIND, int QM, int TX>
__device__ __forceinline__ void persist_pass(const StageArgs* iargs, const int* bin_items, int j0, int j1,
                                             int k, S (*tile)[TX + 10]) {
    for (int j = j0; j < j1; ++j) {
        CArgs& a = ((CArgs*)iargs)[3 * bin_items[j] + k];
        const int len = a.nx;
        for (int x0 = 0; x0 < len; x0 += TX) {
            stage1d_tile<S, KIND, QM, TX>(a, x0, tile);
            __syncthreads();
        }
    }
}

template <typename S, int QM, int TX>
__global__ void __launch_bounds__(TX / 4) __attribute__((amdgpu_waves_per_eu(2)))
stage1d_persist_kernel(const StageArgs* iargs, const PersistItem* items, const int* bin_start,
                       const int* bin_items, PersistIO io, int nsteps) {
    __shared__ S tile[2][TX + 10];
    constexpr int NT = TX / 4;
    const int j0 = bin_start[blockIdx.x], j1 = bin_start[blockIdx.x + 1];
    const int P = io.nplanes;
    for (int j = j0; j < j1; ++j) {
        const int it = bin_items[j];
        const PersistItem m = items[it];
        S* Fp = static_cast<S*>(iargs[3 * it + 1].fbuf);
        double* Mp = iargs[3 * it + 2].mout;
        const long long ps = iargs[3 * it].plane_stride, ms = iargs[3 * it].mstride;
        const S* fi = static_cast<const S*>(io.f_in) + m.soff + m.r0;
        for (int v = 0; v < P; ++v)
            for (int x = threadIdx.x; x < m.len; x += NT) Fp[v * ps + x] = fi[(long long)v * m.nx + x];
        const double* mi = io.m_in + m.coff + m.r0;
        for (int f = 0; f < 3; ++f)
            for (int x = threadIdx.x; x < m.len; x += NT) Mp[f * ms + x] = mi[f * io.ctot + x];
    }
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        persist_pass<S, kStage3, QM, TX>(iargs, bin_items, j0, j1, 0, tile);
        persist_pass<S, kStage4, QM, TX>(iargs, bin_items, j0, j1, 1, tile);
        persist_pass<S, kStage5, QM, TX>(iargs, bin_items, j0, j1, 2, tile);
    }
    for (int j = j0; j < j1; ++j) {
        const int it = bin_items[j];
        const PersistItem m = items[it];
        const S* Fp = static_cast<const S*>(iargs[3 * it + 1].fbuf);
        const double* Mp = iargs[3 * it + 2].mout;
        const long long ps = iargs[3 * it].plane_stride, ms = iargs[3 * it].mstride;
        S* fo = static_cast<S*>(io.f_out) + m.soff;
        const int b = m.own0 - m.r0, n = m.own1 - m.own0;
        for (int v = 0; v < P; ++v)
            for (int x = threadIdx.x; x < n; x += NT) fo[(long long)v * m.nx + m.own0 + x] = Fp[v * ps + b + x];
        double* mo = io.m_out + m.coff + m.own0;
        for (int f = 0; f < 3; ++f)
            for (int x = threadIdx.x; x < n; x += NT) mo[f * io.ctot + x] = Mp[f * ms + b + x];
    }
}

// ---------------------------------------------------------------------------
// F = discrete equilibrium of (n, u, T) (Sec. II); one thread per cell.
// ---------------------------------------------------------------------------
template <typename S, int D>
__global__ void __launch_bounds__(256) init_eq_kernel(const DevTables* __restrict__ tabp,
                                                      const double* __restrict__ n,
                                                      const double* __restrict__ ux,
                                                      const double* __restrict__ uy,
                                                      const double* __restrict__ T, S* F,
                                                      long long cells, double chi_fac) {
    CTab* tab = (CTab*)tabp;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const double nn = n[c], u = ux[c], w = D == 2 ? uy[c] : 0.0, th = T[c] - 1.0;
    int v = 0;
    for (int set = 0; set < 2; ++set) {
        const int Q = tab->q[set];
        const double pre = set ? chi_fac * nn * (th + 1.0) : nn;
        for (int ky = 0; ky < (D == 2 ? Q : 1); ++ky) {
            const double gy = D == 2 ? pre * herm_factor(tab->h[set][ky], Q, w, th) : pre;
            for (int kx = 0; kx < Q; ++kx, ++v)
                F[(size_t)v * cells + c] = (S)(gy * herm_factor(tab->h[set][kx], Q, u, th));
        }
    }
}

// Moments of a plane-set (Sec. II, Eq. Moments_discrete): n, n u from the phi
// planes; (D + K) n T = sum_phi |p|^2 phi + sum_chi chi - n |u|^2.
template <typename S, int D>
__global__ void __launch_bounds__(256) moments_kernel(const DevTables* __restrict__ tabp,
                                                      const S* __restrict__ F, double* M,
                                                      long long cells, long long ms, double dk) {
    CTab* tab = (CTab*)tabp;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    Acc a{0.0, 0.0, 0.0, 0.0};
    const int np = tab->nplanes;
    for (int v = 0; v < np; ++v) acc_add(a, load_desc(tab, v), (double)F[(size_t)v * cells + c]);
    const double nn = a.s0, ux = a.sx / nn, uy = a.sy / nn;
    if (D == 2) {
        M[c] = nn;
        M[ms + c] = ux;
        M[2 * ms + c] = uy;
        M[3 * ms + c] = (a.se - nn * (ux * ux + uy * uy)) / (dk * nn);
    } else {
        M[c] = nn;
        M[ms + c] = ux;
        M[2 * ms + c] = (a.se - nn * ux * ux) / (dk * nn);
    }
}

// One launch of a 2D stage pass; REC: the pass also stores the stage values
// at the own cells (sval_out).
template <typename S, int KIND, bool REC>
hipError_t launch_stage_2d(const StageArgs& a, int grid, hipStream_t s) {
    constexpr int TY = kTile2Y, OWN = kOwn2;
    constexpr int NT = kTile2X * TY / OWN;
    // Even orders take the mirror-pair loop for every FP32 pass (FP64 stage
    // 3 runs the single-buffer loop at three waves per SIMD, FP64 stage 5 is
    // as fast in the software pipeline, and FP64 stage 4 has no registers
    // left for a second plane)
    constexpr bool CAN_PAIR = sizeof(S) == 4 && KIND != kAdvect && OWN == 2;
    if constexpr (CAN_PAIR) {
        if (a.paired) {
            if (a.qm == 16)
                hipLaunchKernelGGL((stage2d_kernel<S, KIND, 16, TY, OWN, true, REC>), dim3(grid), dim3(NT), 0, s, a);
            else
                hipLaunchKernelGGL((stage2d_kernel<S, KIND, 8, TY, OWN, true, REC>), dim3(grid), dim3(NT), 0, s, a);
            return hipGetLastError();
        }
    }
    if (a.qm == 16)
        hipLaunchKernelGGL((stage2d_kernel<S, KIND, 16, TY, OWN, false, REC>), dim3(grid), dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((stage2d_kernel<S, KIND, 8, TY, OWN, false, REC>), dim3(grid), dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <typename S, int KIND>
hipError_t launch_stage_t(int d, const StageArgs& a, hipStream_t s) {
    const int ntiles = d == 2 ? a.ntx * a.nty : a.ntx;
    const int grid = 8 * ((ntiles + 7) / 8);
    if (d == 2) {
        if constexpr (KIND != kAdvect) {
            if (a.sval_out) return launch_stage_2d<S, KIND, true>(a, grid, s);
        }
        return launch_stage_2d<S, KIND, false>(a, grid, s);
    }
    constexpr int TX = kTile1X;
    if (a.qm == 16)
        hipLaunchKernelGGL((stage1d_kernel<S, KIND, 16, TX>), dim3(grid), dim3(TX / 4), 0, s, a);
    else
        hipLaunchKernelGGL((stage1d_kernel<S, KIND, 8, TX>), dim3(grid), dim3(TX / 4), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stage(int d, bool f32, int kind, const StageArgs& a, hipStream_t s) {
    switch (kind) {
        case kAdvect: return f32 ? launch_stage_t<float, kAdvect>(d, a, s) : launch_stage_t<double, kAdvect>(d, a, s);
        case kStage3: return f32 ? launch_stage_t<float, kStage3>(d, a, s) : launch_stage_t<double, kStage3>(d, a, s);
        case kStage4: return f32 ? launch_stage_t<float, kStage4>(d, a, s) : launch_stage_t<double, kStage4>(d, a, s);
        case kStage5: return f32 ? launch_stage_t<float, kStage5>(d, a, s) : launch_stage_t<double, kStage5>(d, a, s);
        default: return hipErrorInvalidValue;
    }
}

namespace {

template <typename S, int KIND, int QM>
hipError_t launch_batch_t(int tile, const StageArgs* targs, const int2* tiles, int ntiles, hipStream_t s) {
    switch (tile) {
        case 256: hipLaunchKernelGGL((stage1d_batch_kernel<S, KIND, QM, 256>), dim3(ntiles), dim3(64), 0, s, targs, tiles, ntiles); break;
        case 512: hipLaunchKernelGGL((stage1d_batch_kernel<S, KIND, QM, 512>), dim3(ntiles), dim3(128), 0, s, targs, tiles, ntiles); break;
        case 1024: hipLaunchKernelGGL((stage1d_batch_kernel<S, KIND, QM, 1024>), dim3(ntiles), dim3(256), 0, s, targs, tiles, ntiles); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename S, int KIND>
hipError_t launch_batch_q(int qm, int tile, const StageArgs* targs, const int2* tiles, int ntiles, hipStream_t s) {
    return qm == 16 ? launch_batch_t<S, KIND, 16>(tile, targs, tiles, ntiles, s)
                    : launch_batch_t<S, KIND, 8>(tile, targs, tiles, ntiles, s);
}

}  // namespace

hipError_t launch_stage1d_batch(bool f32, int kind, int qm, int tile, const StageArgs* targs,
                                const int2* tiles, int ntiles, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    switch (kind) {
        case kStage3: return f32 ? launch_batch_q<float, kStage3>(qm, tile, targs, tiles, ntiles, s) : launch_batch_q<double, kStage3>(qm, tile, targs, tiles, ntiles, s);
        case kStage4: return f32 ? launch_batch_q<float, kStage4>(qm, tile, targs, tiles, ntiles, s) : launch_batch_q<double, kStage4>(qm, tile, targs, tiles, ntiles, s);
        case kStage5: return f32 ? launch_batch_q<float, kStage5>(qm, tile, targs, tiles, ntiles, s) : launch_batch_q<double, kStage5>(qm, tile, targs, tiles, ntiles, s);
        default: return hipErrorInvalidValue;
    }
}

namespace {

template <typename S, int QM>
hipError_t launch_persist_t(int tile, const StageArgs* iargs, const PersistItem* items, const int* bin_start,
                            const int* bin_items, int nbins, const PersistIO& io, int nsteps, hipStream_t s) {
    switch (tile) {
        case 256: hipLaunchKernelGGL((stage1d_persist_kernel<S, QM, 256>), dim3(nbins), dim3(64), 0, s, iargs, items, bin_start, bin_items, io, nsteps); break;
        case 512: hipLaunchKernelGGL((stage1d_persist_kernel<S, QM, 512>), dim3(nbins), dim3(128), 0, s, iargs, items, bin_start, bin_items, io, nsteps); break;
        case 1024: hipLaunchKernelGGL((stage1d_persist_kernel<S, QM, 1024>), dim3(nbins), dim3(256), 0, s, iargs, items, bin_start, bin_items, io, nsteps); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stage1d_persist(bool f32, int qm, int tile, const StageArgs* iargs, const PersistItem* items,
                                  const int* bin_start, const int* bin_items, int nbins, const PersistIO& io,
                                  int nsteps, hipStream_t s) {
    if (nbins <= 0 || nsteps <= 0) return hipSuccess;
    if (f32)
        return qm == 16 ? launch_persist_t<float, 16>(tile, iargs, items, bin_start, bin_items, nbins, io, nsteps, s)
                        : launch_persist_t<float, 8>(tile, iargs, items, bin_start, bin_items, nbins, io, nsteps, s);
    return qm == 16 ? launch_persist_t<double, 16>(tile, iargs, items, bin_start, bin_items, nbins, io, nsteps, s)
                    : launch_persist_t<double, 8>(tile, iargs, items, bin_start, bin_items, nbins, io, nsteps, s);
}

hipError_t launch_init_equilibrium(int d, bool f32, const DevTables* tab, const double* n,
                                   const double* ux, const double* uy, const double* T,
                                   void* F, double* M, long long cells, double chi_fac,
                                   hipStream_t s) {
    (void)M;
    const int grid = (int)((cells + 255) / 256);
    if (d == 2) {
        if (f32) hipLaunchKernelGGL((init_eq_kernel<float, 2>), dim3(grid), dim3(256), 0, s, tab, n, ux, uy, T, (float*)F, cells, chi_fac);
        else hipLaunchKernelGGL((init_eq_kernel<double, 2>), dim3(grid), dim3(256), 0, s, tab, n, ux, uy, T, (double*)F, cells, chi_fac);
    } else {
        if (f32) hipLaunchKernelGGL((init_eq_kernel<float, 1>), dim3(grid), dim3(256), 0, s, tab, n, ux, uy, T, (float*)F, cells, chi_fac);
        else hipLaunchKernelGGL((init_eq_kernel<double, 1>), dim3(grid), dim3(256), 0, s, tab, n, ux, uy, T, (double*)F, cells, chi_fac);
    }
    return hipGetLastError();
}

hipError_t launch_moments(int d, bool f32, const DevTables* tab, const void* F, double* M,
                          long long cells, long long ms, double dk, hipStream_t s) {
    const int grid = (int)((cells + 255) / 256);
    if (d == 2) {
        if (f32) hipLaunchKernelGGL((moments_kernel<float, 2>), dim3(grid), dim3(256), 0, s, tab, (const float*)F, M, cells, ms, dk);
        else hipLaunchKernelGGL((moments_kernel<double, 2>), dim3(grid), dim3(256), 0, s, tab, (const double*)F, M, cells, ms, dk);
    } else {
        if (f32) hipLaunchKernelGGL((moments_kernel<float, 1>), dim3(grid), dim3(256), 0, s, tab, (const float*)F, M, cells, ms, dk);
        else hipLaunchKernelGGL((moments_kernel<double, 1>), dim3(grid), dim3(256), 0, s, tab, (const double*)F, M, cells, ms, dk);
    }
    return hipGetLastError();
}

}  // namespace imexlb
