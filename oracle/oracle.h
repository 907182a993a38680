/*
 * oracle.h -- plain FP64 CPU reference of the implicit-explicit
 * finite-difference lattice Boltzmann step of Kis & Ambrus,
 * "Implicit-Explicit Finite-Difference Lattice Boltzmann Model with Varying
 * Adiabatic Index" (arXiv:1909.08390).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The GPU library never
 * includes this header, links this code or calls it; the two share nothing.
 *
 * Layout of a state array F (all arrays are host memory, FP64):
 *   F[v][y][x], x fastest, v = plane (one discrete velocity of phi or chi).
 *   phi planes first:  v = kx + Qphi*ky           (ky = 0 when d = 1)
 *   chi planes next:   v = Qphi^d + qx + Qchi*qy  (qy = 0 when d = 1)
 *   Node indices run over the ascending Gauss-Hermite nodes.
 * Cell-field arrays (n, ux, uy, T) are [y][x].  Cell centres sit at
 * x_s = (s + 1/2) * lx/nx for s = 0 .. nx-1 (the paper's (s - 1/2) delta s
 * with 1-based s).
 */
#ifndef IMEXLB_ORACLE_H
#define IMEXLB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_OUTFLOW = 0, ORACLE_PERIODIC = 1 };

typedef struct {
    int d;            /* non-homogeneous axes: 1 or 2 */
    int nx, ny;       /* cells per axis (ny = 1 when d = 1) */
    double lx, ly;    /* domain lengths */
    int q_phi, q_chi; /* quadrature order per axis for phi and chi */
    int K;            /* internal degrees of freedom */
    double tau, dt;   /* relaxation time, time step */
    int bc_x, bc_y;   /* ORACLE_OUTFLOW or ORACLE_PERIODIC */
} oracle_cfg;

/* Number of planes Qphi^d + Qchi^d. */
int oracle_num_planes(const oracle_cfg* c);

/* Gauss-Hermite nodes (roots of He_Q, ascending) and weights
 * w_k = Q!/He_{Q+1}(p_k)^2.  Returns 0, or -1 if Q < 1 or Q > 40. */
int oracle_gauss_hermite(int Q, double* p, double* w);

/* One-axis truncated Hermite factor g_k(u, T), k = 0..Q-1. */
void oracle_g(int Q, const double* p, const double* w, double u, double T, double* g);

/* Per-plane velocity components (p_x, p_y) -- p_y = 0 when d = 1. */
void oracle_velocities(const oracle_cfg* c, double* px, double* py);

/* F = discrete equilibrium of (n, u, T) at every cell. uy ignored if d = 1. */
void oracle_equilibrium(const oracle_cfg* c, const double* n, const double* ux,
                        const double* uy, const double* T, double* F);

/* (n, u, T) of every cell.  uy may be NULL when d = 1. */
void oracle_moments(const oracle_cfg* c, const double* F, double* n, double* ux,
                    double* uy, double* T);

/* MP-9 interface value for a positive velocity from the nine values
 * F_{s-4} .. F_{s+4}. */
double oracle_mp9_face(const double* f9);

/* VF = (p . grad) F per plane, by MP-9 fluxes with 5 ghost nodes. */
void oracle_advect(const oracle_cfg* c, const double* F, double* VF);

/* Advance F by nsteps IMEX-SSP3(4,3,3) steps in place.  When stages is not
 * NULL it receives the four stage values F^(1..4) of the last step
 * (4 * planes * cells doubles).  Returns 0, or -1 on bad configuration or
 * allocation failure. */
int oracle_step(const oracle_cfg* c, double* F, int nsteps, double* stages);

#ifdef __cplusplus
}
#endif
#endif
