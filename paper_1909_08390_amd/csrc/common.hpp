// Shared host/device definitions of the imexlb library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace imexlb {

constexpr int kQMax = 16;                      // max Gauss-Hermite order per axis
constexpr int kMaxPlanes = 2 * kQMax * kQMax;  // phi + chi planes in 2D
constexpr int kDTotal = 3;                     // D = 3 (Sec. II)

// One discrete velocity (plane).  m0..me are its weights in the moment sums
// of Sec. II (Eq. Moments_discrete): mass, x/y momentum, twice the energy.
struct PlaneDesc {
    double px, py;            // velocity components (py = 0 when d = 1)
    double m0, mx, my, me;    // phi: 1, px, py, px^2+py^2;  chi: 0, 0, 0, 1
    int set;                  // 0 = phi, 1 = chi
    int kx, ky;               // node index per axis within the set
    int pad;
};

// Layout of the even/odd Horner coefficients of one node for a padded order
// QM (8 or 16).  The one-axis equilibrium factor of Eq. (gExpanded),
//   g_k(u, T) = w_k sum_{l<Q} He_l(p_k)/l! sum_s l!/(2^s s!(l-2s)!) (T-1)^s u^(l-2s),
// regrouped by powers th^s (th = T - 1) and u^j (j = l - 2s), has the
// coefficients B_k[s][j] = w_k He_{j+2s}(p_k) / (2^s s! j!) for j + 2s < Q.
// Splitting each u-polynomial into even and odd parts, g = Ge(u^2) + u Go(u^2),
// gives the factor of the mirrored node p = -p_k as Ge - u Go for free.
// Per s (from 0): the even coefficients j = 0, 2, .. then the odd j = 1, 3, ..
template <int QM>
struct HornerLayout {
    static constexpr int S = (QM - 1) / 2;
    static constexpr int ne(int s) { return (QM - 1 - 2 * s) / 2 + 1; }
    static constexpr int no(int s) { return (QM - 2 - 2 * s) >= 0 ? (QM - 2 - 2 * s) / 2 + 1 : 0; }
    static constexpr int off(int s) {
        int o = 0;
        for (int t = 0; t < s; ++t) o += ne(t) + no(t);
        return o;
    }
    static constexpr int total() { return off(S + 1); }
};

// One entry of the plane processing order of the stage passes: planes run
// set by set, ky-major (in x-factor table groups for 2D FP32 storage), with
// each x-node followed by its mirror so that one Horner evaluation serves
// both.
struct PlaneStep {
    double px, py;            // velocity of the plane
    double m0, mx, my, me;    // moment weights (as in PlaneDesc)
    int v;                    // plane index in the state layout
    int set;                  // 0 = phi, 1 = chi
    int kx, ky;               // node indices
    int hx;                   // node whose Horner row evaluates (kx, mirror)
    int first;                // 1: evaluate the pair now; 0: use the cached mirror
    int hy;                   // node whose Horner row evaluates (ky, mirror)
    int new_group;            // 1: ky (or the set) changed -> y factor changes
    int yfirst;               // 1: evaluate the y pair now; 0: use the cached mirror
    int new_tab;              // 1: first step of an x-factor table group (tables rebuilt)
    int tcount;               // mirror pairs in the table group (2D, orders up to 8)
    int slot;                 // table slot of kx within its group
};

// PlaneStep packed for the kernels (6 dwords, prefetched into SGPRs):
// bits: set | first<<1 | new_group<<2 | yfirst<<3 | new_tab<<4 | last<<5 |
// slot<<6 | tcount<<9 | hx<<12 | hy<<17 (node indices < 32; last marks the
// final plane of the order; new_tab, slot and tcount describe the x-factor
// table group, see upload_tables).
struct PackedStep {
    double px, py;
    int v;
    int bits;
};

// Constant tables of one context, in device memory.
struct DevTables {
    PackedStep step[kMaxPlanes + 3];  // zero padding entries past the last plane (look-ahead)
    // h[set][k][l] = w_k He_l(p_k) / l!  (zero for l >= Q_set), so that the
    // one-axis equilibrium factor of Eq. (gExpanded) is g_k = sum_l h[k][l] a_l
    // with the Hermite coefficients a_l(u, T) of the local Maxwellian.
    double h[2][kQMax][kQMax];
    // Even/odd Horner coefficients per set and node (HornerLayout<8> and <16>).
    double hc8[2][kQMax][HornerLayout<8>::total()];
    double hc16[2][kQMax][HornerLayout<16>::total()];
    int q[2];                 // Q_phi, Q_chi
    int nplanes, nphi;
    PlaneDesc plane[kMaxPlanes];
    PlaneStep order[kMaxPlanes];
};

enum Kind : int { kAdvect = 0, kStage3 = 3, kStage4 = 4, kStage5 = 5 };

// Arguments of one stage pass.  See the kernel file for the stage algebra.
struct StageArgs {
    const void* src;       // plane-set advected in this pass (F^n, G3 or G4)
    const double* msrc;    // its moments (n, ux, [uy], T)
    void* out;             // output plane-set (G3, G4) or FP64 VF (advect)
    double* mout;          // output moments
    void* fbuf;            // state buffer: F^n / R / F^{n+1}
    const double* mn;      // moments of F^n (stage 4)
    const DevTables* tab;
    int nx, ny, bcx, bcy;
    int ntx, nty, tiles_per_xcd, qm;  // qm: padded Horner order (8 or 16)
    int paired;              // 2D, both orders even: planes come in x-mirror pairs
    long long plane_stride;  // cells per plane
    long long mstride;       // elements per moment field (1D kernels)
    double inv_dx, inv_dy;
    double dt, omega;
    double a_rel, b_rel;     // relax-on-read weights: F_i = a_rel G + b_rel E
    double a1, a2;           // 1/(1+c) and (1+2c)/(1+c)^2, c = alpha dt/tau
    // Combined stage coefficients (w = dt/tau):
    //  k[0] = (1 - alpha) w a2                              (pass 3)
    //  k[1] = (1 - alpha) w a2 / 4 - beta w a1 - eta w a2,
    //  k[2] = kappa w a1, k[3] = alpha w a2 / 6, k[4] = w a1 / 6   (pass 4)
    //  k[5] = 2 w a1 / 3                                    (pass 5)
    double k[6];
    double chi_fac;          // K + D - d
    double dk;               // D + K
    // (last, so that the plain passes see the fields above at the offsets
    // they were tuned with)
    void* rbuf;              // stage 4: where R goes (fbuf, or the next state
                             // buffer of an out-of-place step; read by the 1D
                             // passes and the recording 2D passes)
    void* sval_out;          // 2D passes 3 / 4 / 5: where the stage values F2 / F3 /
                             // F4 at the own cells go (recorded steps), or NULL
};

// Host helpers shared by the single-grid and batched contexts (imexlb.cpp).
bool quadrature_rule(int Q, double* p, double* w);
hipError_t upload_tables(int d, const int Q[2], const double p[2][kQMax], const double w[2][kQMax],
                         int tab_nodes, DevTables** d_tab, hipStream_t stream);
void stage_coefficients(double dt, double tau, StageArgs& a);  // dt, omega, a1, a2, k[]
// Per-pass arguments of one step from F; with Fnext the step is out of place
// (R and F^{n+1} go to Fnext, F is only read).
void pass_args(const StageArgs& a, void* F, void* G3, void* G4, double* Mn, double* M3, double* M4,
               StageArgs out[3], void* Fnext = nullptr);

// Launchers (kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_stage(int d, bool f32, int kind, const StageArgs& a, hipStream_t s);
hipError_t launch_init_equilibrium(int d, bool f32, const DevTables* tab, const double* n,
                                   const double* ux, const double* uy, const double* T,
                                   void* F, double* M, long long cells, double chi_fac,
                                   hipStream_t s);
// moments of F (plane stride cells) into M with field stride ms
hipError_t launch_moments(int d, bool f32, const DevTables* tab, const void* F, double* M,
                          long long cells, long long ms, double dk, hipStream_t s);
// Work-groups of the domain sums and the density loss (one partial each).
constexpr int kSumBlocks = 1024;

// Reductions (reduce.hip).  Moment fields M = (n, ux, [uy], T) with field
// stride ms.  The sums use nblocks work-groups whose partials (4 resp. 1
// values each) go to partial; the totals to out4 / out1 (device).
hipError_t launch_domain_sums(int d, const double* M, long long ms, long long cells, double dk,
                              double* partial, int nblocks, double* out4, hipStream_t s);
hipError_t launch_density_loss(const double* n, const double* target, long long cells, double* grad,
                               double* partial, int nblocks, double* out1, hipStream_t s);
// flag = INT_MAX; then flag = min(flag, code) when a cell is non-physical.
hipError_t launch_check_reset(int* flag, hipStream_t s);
hipError_t launch_check(int d, const double* M, long long ms, long long cells, int code, int* flag,
                        hipStream_t s);
// Adjoint building blocks (adjoint.hip): the stage value F = a src + b E(M)
// in the storage type (f32: float, else double); dM = (dE/dM)^T dE with dE
// in the storage type; out = y + (dM/dF)^T dM with y and out in the storage
// type (y NULL: zero; y may be out).  Arithmetic is FP64 throughout.
hipError_t launch_materialise(int d, int qm, bool f32, const DevTables* tab, const void* src, const double* M,
                              double a, double b, void* out, long long cells, double chi_fac,
                              hipStream_t s);
// Transposed advection: with dA = sum_j c[j] z[j] (the adjoint of the
// fluxes) and V = V^T dA at every node, writes y1 = e0 V + sum_j e[j] z[j]
// and, when y2 is not NULL, y2 = f0 V + sum_j f[j] z[j].  z[0] is an FP64
// plane-set; F (the linearisation point), z[1..], y1 and, unless y2_f64 is
// set, y2 are plane-sets of the storage type (f32: float, else double).
// The outputs must not alias F or any z[j].
struct AdvAdjIO {
    const void* z[4];
    double c[4], e[4], f[4];
    double e0, f0;
    int n;
    int y2_f64;
    void* y1;
    void* y2;
};
hipError_t launch_advect_adjoint(int d, bool f32, const DevTables* tab, int nplanes, const void* F,
                                 const AdvAdjIO& io, int nx, int ny, int bcx, int bcy, double inv_dx, double inv_dy,
                                 hipStream_t s);
hipError_t launch_eq_adjoint(int d, int qm, bool f32, const DevTables* tab, const double* M, const void* dE,
                             double* dM, long long cells, double chi_fac, hipStream_t s);
hipError_t launch_mom_adjoint(int d, bool f32, const DevTables* tab, const double* M, const double* dM,
                              const void* y, void* out, long long cells, double dk, hipStream_t s);

// Batched 1D passes: one launch covers every tile of every tube.  targs[i]
// holds tube i's arguments for this pass; tiles[j] = (tube, first cell).
hipError_t launch_stage1d_batch(bool f32, int kind, int qm, int tile, const StageArgs* targs,
                                const int2* tiles, int ntiles, hipStream_t s);

// Persistent batched steps (temporal blocking).  An item is a tube, or a
// chunk [own0, own1) of an outflow tube, stepped over the region
// [r0, r0 + len) of tube cells in a private area; its pass arguments
// (iargs[3 item + 0..2], passes 3, 4, 5) point into that area, with the
// region as the line (nx = len) and the private plane and moment strides.
struct PersistItem {
    long long soff;   // tube's first state element in the global buffers
    long long coff;   // tube's first cell in the global moment fields
    int nx;           // tube length (plane stride of the global state)
    int r0, len;      // region, in tube cells
    int own0, own1;   // cells this item writes back, in tube cells
    int pad;
};
// Global buffers of one launch: the state and moments are read from *_in
// and the items' own cells written to *_out (distinct buffers).
struct PersistIO {
    const void* f_in;
    void* f_out;
    const double* m_in;
    double* m_out;
    long long ctot;   // field stride of the global moments
    int nplanes;
};
// One launch of nsteps whole steps: block b owns the items
// bin_items[bin_start[b] .. bin_start[b + 1]).
hipError_t launch_stage1d_persist(bool f32, int qm, int tile, const StageArgs* iargs, const PersistItem* items,
                                  const int* bin_start, const int* bin_items, int nbins, const PersistIO& io,
                                  int nsteps, hipStream_t s);

// Tile shapes (cells) used by the stage kernels: 2D tiles of kTile2X x
// kTile2Y cells, kOwn2 consecutive cells per thread (kTile2X kTile2Y / kOwn2
// threads).  32 x 16 keeps one FP64 work-group under 80 KB of LDS, so two
// work-groups share a CU and one's barrier waits overlap the other's work.
#ifndef IMEXLB_TILE2Y
#define IMEXLB_TILE2Y 16
#endif
#ifndef IMEXLB_OWN2
#define IMEXLB_OWN2 2
#endif
#ifndef IMEXLB_TILE2X
#define IMEXLB_TILE2X 32
#endif
constexpr int kTile2X = IMEXLB_TILE2X, kTile2Y = IMEXLB_TILE2Y;
constexpr int kOwn2 = IMEXLB_OWN2;
constexpr int kTile1X = 1024;
// Tile widths (cells) the batched 1D passes can be launched with.
constexpr int kBatchTiles[3] = {256, 512, 1024};
// 2D tiles are visited in patches of kPatchW x kPatchH tiles (patch rows
// top to bottom, patches left to right inside a patch row, tiles row-major
// inside a patch), so that the tiles running at the same time on one XCD
// (32 CUs x 2 work-groups) form a compact block whose halos hit that XCD's
// L2.  The patch is wide in x: x-halo reads are 5-cell row segments that
// use a fraction of each cache line, y-halo reads whole rows.
#ifndef IMEXLB_PATCH_W
#define IMEXLB_PATCH_W 12
#endif
#ifndef IMEXLB_PATCH_H
#define IMEXLB_PATCH_H 6
#endif
constexpr int kPatchW = IMEXLB_PATCH_W, kPatchH = IMEXLB_PATCH_H;
// Nodes per x-factor table group of the 2D plane order (orders up to 8):
// two mirror pairs, i.e. 4 tables of one double per loaded cell in LDS
// (31 KB), small enough to sit next to the two LDS tiles of the pipelined
// and mirror-pair plane loops with two work-groups per compute unit.
constexpr int kTabNodes2D = 4;

}  // namespace imexlb
