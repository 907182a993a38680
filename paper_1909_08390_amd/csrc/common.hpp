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

// Constant tables of one context, in device memory.
struct DevTables {
    // h[set][k][l] = w_k He_l(p_k) / l!  (zero for l >= Q_set), so that the
    // one-axis equilibrium factor of Eq. (gExpanded) is g_k = sum_l h[k][l] a_l
    // with the Hermite coefficients a_l(u, T) of the local Maxwellian.
    double h[2][kQMax][kQMax];
    int q[2];                 // Q_phi, Q_chi
    int nplanes, nphi;
    PlaneDesc plane[kMaxPlanes];
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
    int ntx, nty, tiles_per_xcd, pad0;
    long long plane_stride;  // cells per plane
    double inv_dx, inv_dy;
    double dt, omega;
    double a_rel, b_rel;     // relax-on-read weights: F_i = a_rel G + b_rel E
    double a1, a2;           // 1/(1+c) and (1+2c)/(1+c)^2, c = alpha dt/tau
    double chi_fac;          // K + D - d
    double dk;               // D + K
};

// Launchers (kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_stage(int d, bool f32, int kind, const StageArgs& a, hipStream_t s);
hipError_t launch_init_equilibrium(int d, bool f32, const DevTables* tab, const double* n,
                                   const double* ux, const double* uy, const double* T,
                                   void* F, double* M, long long cells, double chi_fac,
                                   hipStream_t s);
hipError_t launch_moments(int d, bool f32, const DevTables* tab, const void* F, double* M,
                          long long cells, double dk, hipStream_t s);
hipError_t launch_domain_sums(int d, const double* M, long long cells, double dk,
                              double* partial, int nblocks, double* out4, hipStream_t s);
hipError_t launch_check(int d, const double* M, long long cells, int* flag, hipStream_t s);

// Tile shapes (cells) used by the stage kernels.
constexpr int kTile2X = 64, kTile2Y = 16;
constexpr int kTile1X = 1024;

}  // namespace imexlb
