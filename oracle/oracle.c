/*
 * oracle.c -- plain FP64 CPU reference of the IMEX finite-difference
 * lattice Boltzmann step with MP-9 advection (Kis & Ambrus,
 * arXiv:1909.08390).
 *
 * TEST INFRASTRUCTURE ONLY: the definition the GPU library is checked
 * against.  It is deliberately plain and slow: full arrays for every stage,
 * the equilibrium written as the paper's double sum, the MP-9 limiter in the
 * paper's two-case form, the time stages taken generically from the Butcher
 * tableaux.  Nothing here is shared with the GPU library.
 *
 * Readings of the paper taken here (each one is listed with its reason in
 * the project's design notes):
 *  - Hermite polynomials are the probabilists' He_n (weight exp(-p^2/2));
 *    only these make the printed weight formula sum to one.
 *  - chi's discrete equilibrium carries the same prefactor (K + D - d) T as
 *    the continuous one: chi_eq,q = (K + D - d) T n prod_a g_{a,q_a}.
 *  - The stages follow Table I.  The printed stage-3 closed form drops the
 *    -(1 - alpha) dF^(2) term of Table I's third row and is not used.
 *  - The MP limiter's tie (the product exactly zero) takes the first case.
 *  - A negative velocity uses the mirrored stencil; a zero velocity carries
 *    no flux.
 *  - Outflow ghost nodes copy the boundary fluid node; periodic ghosts wrap.
 *    Ghosts are filled for every advected stage value.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define D_TOTAL 3   /* D = 3 momentum dimensions (Sec. II) */
#define NGHOST 5    /* ghost nodes per side (Sec. IV, last paragraph) */
#define ALPHA_MP 4.0 /* alpha_MP = 4 (Sec. IV) */

/* IMEX-SSP3(4,3,3) constants printed in the caption of Table I. */
#define TAB_ALPHA 0.24169426078821
#define TAB_BETA 0.06042356519705
#define TAB_ETA 0.12915286960590

static int cells_of(const oracle_cfg* c) { return c->nx * (c->d == 2 ? c->ny : 1); }

static int ipow(int b, int e) {
    int r = 1;
    for (int i = 0; i < e; i++) r *= b;
    return r;
}

int oracle_num_planes(const oracle_cfg* c) {
    return ipow(c->q_phi, c->d) + ipow(c->q_chi, c->d);
}

/* ------------------------------------------------------------------------
 * Sec. II, velocity-space discretisation: nodes are the roots of the
 * Hermite polynomial of order Q; weights w_k(Q) = Q!/[H_{Q+1}(p_k)]^2.
 * He_n by its three-term recurrence He_{n+1} = x He_n - n He_{n-1}.
 * ---------------------------------------------------------------------- */
static long double hermite_he(int n, long double x) {
    if (n == 0) return 1.0L;
    long double hm = 1.0L, h = x;
    for (int j = 1; j < n; j++) {
        long double hp = x * h - (long double)j * hm;
        hm = h;
        h = hp;
    }
    return h;
}

int oracle_gauss_hermite(int Q, double* p, double* w) {
    if (Q < 1 || Q > 40) return -1;
    /* All roots of He_Q lie inside |x| < 2 sqrt(Q) + 1.  Scan for sign
     * changes on a fine grid, then bisect each bracket in long double. */
    long double B = 2.0L * sqrtl((long double)Q) + 1.0L;
    long double h = 1.0e-4L;
    int found = 0;
    long double a = -B + 0.3183e-4L; /* offset keeps grid points off x = 0 */
    long double fa = hermite_he(Q, a);
    while (a < B && found < Q) {
        long double b = a + h;
        long double fb = hermite_he(Q, b);
        if (fa == 0.0L) {
            p[found++] = (double)a;
        } else if ((fa < 0.0L) != (fb < 0.0L) && fb != 0.0L) {
            long double lo = a, hi = b, flo = fa;
            for (int it = 0; it < 200; it++) {
                long double mid = 0.5L * (lo + hi);
                if (mid == lo || mid == hi) break;
                long double fm = hermite_he(Q, mid);
                if (fm == 0.0L) { lo = hi = mid; break; }
                if ((fm < 0.0L) == (flo < 0.0L)) { lo = mid; flo = fm; }
                else hi = mid;
            }
            p[found++] = (double)(0.5L * (lo + hi));
        }
        a = b;
        fa = fb;
    }
    if (found != Q) return -1;
    /* He_Q(-x) = (-1)^Q He_Q(x): the roots are symmetric about 0. */
    for (int k = 0; k < Q / 2; k++) {
        double m = 0.5 * (p[Q - 1 - k] - p[k]);
        p[k] = -m;
        p[Q - 1 - k] = m;
    }
    if (Q % 2 == 1) p[Q / 2] = 0.0;
    long double qfact = 1.0L;
    for (int j = 2; j <= Q; j++) qfact *= (long double)j;
    for (int k = 0; k < Q; k++) {
        long double hq1 = hermite_he(Q + 1, (long double)p[k]);
        w[k] = (double)(qfact / (hq1 * hq1));
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Sec. II, Eq. (gExpanded): truncated Hermite expansion of the one-axis
 * Maxwellian factor,
 *   g_k = w_k sum_{l=0}^{Q-1} (1/l!) He_l(p_k)
 *         sum_{s=0}^{floor(l/2)} l!/(2^s s! (l-2s)!) (T-1)^s u^(l-2s)
 * (m = 1).  Written literally as the double sum.
 * ---------------------------------------------------------------------- */
static double factorial(int n) {
    double r = 1.0;
    for (int j = 2; j <= n; j++) r *= (double)j;
    return r;
}

void oracle_g(int Q, const double* p, const double* w, double u, double T, double* g) {
    for (int k = 0; k < Q; k++) {
        double outer = 0.0;
        for (int l = 0; l < Q; l++) {
            double inner = 0.0;
            for (int s = 0; s <= l / 2; s++) {
                double coef = factorial(l) / (pow(2.0, s) * factorial(s) * factorial(l - 2 * s));
                inner += coef * pow(T - 1.0, s) * pow(u, l - 2 * s);
            }
            outer += (1.0 / factorial(l)) * (double)hermite_he(l, (long double)p[k]) * inner;
        }
        g[k] = w[k] * outer;
    }
}

/* Quadrature tables of one configuration. */
typedef struct {
    double pp[64], wp[64]; /* phi nodes / weights per axis */
    double pc[64], wc[64]; /* chi nodes / weights per axis */
} quad_t;

static int make_quad(const oracle_cfg* c, quad_t* q) {
    if (c->q_phi > 64 || c->q_chi > 64) return -1;
    if (oracle_gauss_hermite(c->q_phi, q->pp, q->wp)) return -1;
    if (oracle_gauss_hermite(c->q_chi, q->pc, q->wc)) return -1;
    return 0;
}

void oracle_velocities(const oracle_cfg* c, double* px, double* py) {
    quad_t q;
    if (make_quad(c, &q)) return;
    int Qp = c->q_phi, Qc = c->q_chi;
    int v = 0;
    if (c->d == 1) {
        for (int k = 0; k < Qp; k++, v++) { px[v] = q.pp[k]; py[v] = 0.0; }
        for (int k = 0; k < Qc; k++, v++) { px[v] = q.pc[k]; py[v] = 0.0; }
    } else {
        for (int ky = 0; ky < Qp; ky++)
            for (int kx = 0; kx < Qp; kx++, v++) { px[v] = q.pp[kx]; py[v] = q.pp[ky]; }
        for (int qy = 0; qy < Qc; qy++)
            for (int qx = 0; qx < Qc; qx++, v++) { px[v] = q.pc[qx]; py[v] = q.pc[qy]; }
    }
}

/* ------------------------------------------------------------------------
 * Sec. II: phi_eq,k = n prod_a g^{Qphi}_{a,k_a} (Eq. gExpanded); chi_eq is
 * the same construction with Qchi nodes, times the factor (K + D - d) T of
 * the continuous relation chi_eq = (K + D - d) T phi_eq (Eq. galpha).
 * ---------------------------------------------------------------------- */
static void eq_cell(const oracle_cfg* c, const quad_t* q, double n, double ux, double uy,
                    double T, double* out /* planes values */) {
    int Qp = c->q_phi, Qc = c->q_chi;
    double gxp[64], gyp[64], gxc[64], gyc[64];
    oracle_g(Qp, q->pp, q->wp, ux, T, gxp);
    oracle_g(Qc, q->pc, q->wc, ux, T, gxc);
    double chi_pref = (double)(c->K + D_TOTAL - c->d) * T;
    int v = 0;
    if (c->d == 1) {
        for (int k = 0; k < Qp; k++) out[v++] = n * gxp[k];
        for (int k = 0; k < Qc; k++) out[v++] = chi_pref * n * gxc[k];
    } else {
        oracle_g(Qp, q->pp, q->wp, uy, T, gyp);
        oracle_g(Qc, q->pc, q->wc, uy, T, gyc);
        for (int ky = 0; ky < Qp; ky++)
            for (int kx = 0; kx < Qp; kx++) out[v++] = n * gxp[kx] * gyp[ky];
        for (int qy = 0; qy < Qc; qy++)
            for (int qx = 0; qx < Qc; qx++) out[v++] = chi_pref * n * gxc[qx] * gyc[qy];
    }
}

void oracle_equilibrium(const oracle_cfg* c, const double* n, const double* ux,
                        const double* uy, const double* T, double* F) {
    quad_t q;
    if (make_quad(c, &q)) return;
    int P = oracle_num_planes(c), N = cells_of(c);
    double* tmp = (double*)malloc(sizeof(double) * (size_t)P);
    for (int i = 0; i < N; i++) {
        eq_cell(c, &q, n[i], ux[i], c->d == 2 ? uy[i] : 0.0, T[i], tmp);
        for (int v = 0; v < P; v++) F[(size_t)v * N + i] = tmp[v];
    }
    free(tmp);
}

/* ------------------------------------------------------------------------
 * Sec. II, Eq. (Moments_discrete) with m = 1 (rho = n):
 *   n = sum_k phi_k,  n u = sum_k p_k phi_k,
 *   (D+K)/2 n T = sum_k phi_k xi_k^2 / 2 + sum_q chi_q / 2,  xi = p - u.
 * ---------------------------------------------------------------------- */
static void moments_with(const oracle_cfg* c, const double* px, const double* py,
                         const double* F, double* n, double* ux, double* uy, double* T) {
    int N = cells_of(c);
    int Pphi = ipow(c->q_phi, c->d), P = oracle_num_planes(c);
    for (int i = 0; i < N; i++) {
        double s0 = 0.0, sx = 0.0, sy = 0.0;
        for (int v = 0; v < Pphi; v++) {
            double f = F[(size_t)v * N + i];
            s0 += f;
            sx += px[v] * f;
            sy += py[v] * f;
        }
        double u_x = sx / s0, u_y = sy / s0;
        double e = 0.0;
        for (int v = 0; v < Pphi; v++) {
            double f = F[(size_t)v * N + i];
            double xi2 = (px[v] - u_x) * (px[v] - u_x) + (py[v] - u_y) * (py[v] - u_y);
            e += f * xi2 / 2.0;
        }
        for (int v = Pphi; v < P; v++) e += F[(size_t)v * N + i] / 2.0;
        n[i] = s0;
        ux[i] = u_x;
        if (uy) uy[i] = u_y;
        T[i] = e / ((double)(D_TOTAL + c->K) / 2.0 * s0);
    }
}

void oracle_moments(const oracle_cfg* c, const double* F, double* n, double* ux,
                    double* uy, double* T) {
    int P = oracle_num_planes(c);
    double* px = (double*)malloc(sizeof(double) * (size_t)P);
    double* py = (double*)malloc(sizeof(double) * (size_t)P);
    oracle_velocities(c, px, py);
    moments_with(c, px, py, F, n, ux, uy, T);
    free(px);
    free(py);
}

/* ------------------------------------------------------------------------
 * Sec. IV: MP-9 interface value for a positive advection velocity.
 * minmod(x, y) = (1/2)[sgn x + sgn y] min(|x|, |y|); the four-argument
 * minmod is the signed smallest magnitude when all four share a sign, else 0.
 * ---------------------------------------------------------------------- */
static double sgn(double x) { return (x > 0.0) - (x < 0.0); }

static double minmod2(double x, double y) {
    return 0.5 * (sgn(x) + sgn(y)) * fmin(fabs(x), fabs(y));
}

static double minmod4(double a, double b, double c, double d) {
    if (a > 0.0 && b > 0.0 && c > 0.0 && d > 0.0) return fmin(fmin(a, b), fmin(c, d));
    if (a < 0.0 && b < 0.0 && c < 0.0 && d < 0.0) return fmax(fmax(a, b), fmax(c, d));
    return 0.0;
}

static double min3(double a, double b, double c) { return fmin(a, fmin(b, c)); }
static double max3(double a, double b, double c) { return fmax(a, fmax(b, c)); }

double oracle_mp9_face(const double* f) {
    /* f[j] = F_{s-4+j}; F_s = f[4]. */
    double Fs = f[4], Fp1 = f[5], Fm1 = f[3];
    double FL = (4.0 * f[0] - 41.0 * f[1] + 199.0 * f[2] - 641.0 * f[3] + 1879.0 * f[4] +
                 1375.0 * f[5] - 305.0 * f[6] + 55.0 * f[7] - 5.0 * f[8]) / 2520.0;
    double FMP = Fs + minmod2(Fp1 - Fs, ALPHA_MP * (Fs - Fm1));
    if ((FL - Fs) * (FL - FMP) <= 0.0) return FL;
    /* C_j = F_{j+1} - 2F_j + F_{j-1} at j = s-1, s, s+1. */
    double Cm = f[4] - 2.0 * f[3] + f[2];
    double Cs = f[5] - 2.0 * f[4] + f[3];
    double Cp = f[6] - 2.0 * f[5] + f[4];
    double FUL = Fs + ALPHA_MP * (Fs - Fm1);
    double FLC = Fs + 0.5 * (Fs - Fm1) + (4.0 / 3.0) * minmod4(4.0 * Cs - Cm, 4.0 * Cm - Cs, Cs, Cm);
    double FMD = 0.5 * (Fs + Fp1 - minmod4(4.0 * Cs - Cp, 4.0 * Cp - Cs, Cs, Cp));
    double Fmin = fmax(min3(Fs, Fp1, FMD), min3(Fs, FUL, FLC));
    double Fmax = fmin(max3(Fs, Fp1, FMD), max3(Fs, FUL, FLC));
    return FL + minmod2(Fmin - FL, Fmax - FL);
}

/* ------------------------------------------------------------------------
 * Sec. IV: (p dF/dx)_s = (Flux_{s+1/2} - Flux_{s-1/2}) / delta s, the flux
 * being p times the MP-9 interface value (the reconstruction is homogeneous
 * of degree one, so scaling by p commutes with it).  Multi-dimensional
 * advection is dimensionally unsplit: one 1D operator per axis, summed.
 * The line is extended by 5 ghost nodes per side.
 * ---------------------------------------------------------------------- */
static void advect_line(const double* line, int S, int stride, int bc, double p, double ds,
                        double* out, int out_stride) {
    /* ext[NGHOST + s] = F_s for s in [-5, S + 5). */
    double* ext = (double*)malloc(sizeof(double) * (size_t)(S + 2 * NGHOST));
    for (int s = -NGHOST; s < S + NGHOST; s++) {
        int src;
        if (s >= 0 && s < S) src = s;
        else if (bc == ORACLE_PERIODIC) src = ((s % S) + S) % S;
        else src = s < 0 ? 0 : S - 1;
        ext[NGHOST + s] = line[(size_t)src * stride];
    }
    /* Interface value at s+1/2 for s = -1 .. S-1. */
    double* face = (double*)malloc(sizeof(double) * (size_t)(S + 1));
    for (int s = -1; s < S; s++) {
        double f9[9];
        if (p > 0.0) {
            for (int j = 0; j < 9; j++) f9[j] = ext[NGHOST + s - 4 + j];
        } else {
            /* mirrored stencil: slot j holds F_{s+5-j} */
            for (int j = 0; j < 9; j++) f9[j] = ext[NGHOST + s + 5 - j];
        }
        face[s + 1] = oracle_mp9_face(f9);
    }
    for (int s = 0; s < S; s++)
        out[(size_t)s * out_stride] += p * (face[s + 1] - face[s]) / ds;
    free(face);
    free(ext);
}

static void advect_with(const oracle_cfg* c, const double* px, const double* py,
                        const double* F, double* VF) {
    int N = cells_of(c), P = oracle_num_planes(c);
    int nx = c->nx, ny = c->d == 2 ? c->ny : 1;
    double dx = c->lx / nx, dy = c->d == 2 ? c->ly / ny : 1.0;
    memset(VF, 0, sizeof(double) * (size_t)N * P);
    for (int v = 0; v < P; v++) {
        const double* Fv = F + (size_t)v * N;
        double* Vv = VF + (size_t)v * N;
        if (px[v] != 0.0)
            for (int y = 0; y < ny; y++)
                advect_line(Fv + (size_t)y * nx, nx, 1, c->bc_x, px[v], dx, Vv + (size_t)y * nx, 1);
        if (c->d == 2 && py[v] != 0.0)
            for (int x = 0; x < nx; x++)
                advect_line(Fv + x, ny, nx, c->bc_y, py[v], dy, Vv + x, nx);
    }
}

void oracle_advect(const oracle_cfg* c, const double* F, double* VF) {
    int P = oracle_num_planes(c);
    double* px = (double*)malloc(sizeof(double) * (size_t)P);
    double* py = (double*)malloc(sizeof(double) * (size_t)P);
    oracle_velocities(c, px, py);
    advect_with(c, px, py, F, VF);
    free(px);
    free(py);
}

/* ------------------------------------------------------------------------
 * Sec. III, Eq. (IMEX) with the IMEX-SSP3(4,3,3) tableaux of Table I:
 *   F^(i) = F^n - dt sum_{j<i} At_ij V F^(j) - sum_{j<=i} A_ij dF^(j),
 *   F^{n+1} = F^n - dt sum_i wt_i V F^(i) - sum_i w_i dF^(i),
 *   dF^(i) = (dt/tau) (F^(i) - F^(i)_eq).
 * F^(i)_eq is built from the moments of the explicit part S_i (everything
 * but the diagonal implicit term): dF terms carry no mass, momentum or
 * energy (Sec. III), so F^(i) and S_i share n, u and T.  The diagonal term
 * then gives F^(i) = (S_i + A_ii (dt/tau) F^(i)_eq) / (1 + A_ii dt/tau).
 * ---------------------------------------------------------------------- */
int oracle_step(const oracle_cfg* c, double* F, int nsteps, double* stages) {
    if (c->d != 1 && c->d != 2) return -1;
    if (c->tau <= 0.0 || c->dt <= 0.0) return -1;
    const double al = TAB_ALPHA, be = TAB_BETA, et = TAB_ETA;
    const double At[4][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 1, 0, 0}, {0, 0.25, 0.25, 0}};
    const double wt[4] = {0, 1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
    const double A[4][4] = {{al, 0, 0, 0},
                            {-al, al, 0, 0},
                            {0, 1.0 - al, al, 0},
                            {be, et, 0.5 - be - et - al, al}};
    const double w[4] = {0, 1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};

    int N = cells_of(c), P = oracle_num_planes(c);
    size_t tot = (size_t)N * P;
    double omega = c->dt / c->tau;
    double* px = (double*)malloc(sizeof(double) * (size_t)P);
    double* py = (double*)malloc(sizeof(double) * (size_t)P);
    double* S = (double*)malloc(sizeof(double) * tot);
    double* E = (double*)malloc(sizeof(double) * tot);
    double* Fi = (double*)malloc(sizeof(double) * tot * 4);
    double* dF = (double*)malloc(sizeof(double) * tot * 4);
    double* VFi = (double*)malloc(sizeof(double) * tot * 4);
    double* mn = (double*)malloc(sizeof(double) * (size_t)N);
    double* mux = (double*)malloc(sizeof(double) * (size_t)N);
    double* muy = (double*)malloc(sizeof(double) * (size_t)N);
    double* mT = (double*)malloc(sizeof(double) * (size_t)N);
    if (!px || !py || !S || !E || !Fi || !dF || !VFi || !mn || !mux || !muy || !mT) {
        free(px); free(py); free(S); free(E); free(Fi); free(dF); free(VFi);
        free(mn); free(mux); free(muy); free(mT);
        return -1;
    }
    oracle_velocities(c, px, py);

    for (int step = 0; step < nsteps; step++) {
        for (int i = 0; i < 4; i++) {
            /* explicit part S_i */
            for (size_t e = 0; e < tot; e++) {
                double s = F[e];
                for (int j = 0; j < i; j++) {
                    if (At[i][j] != 0.0) s -= c->dt * At[i][j] * VFi[(size_t)j * tot + e];
                    if (A[i][j] != 0.0) s -= A[i][j] * dF[(size_t)j * tot + e];
                }
                S[e] = s;
            }
            /* implicit BGK stage in closed form */
            moments_with(c, px, py, S, mn, mux, muy, mT);
            oracle_equilibrium(c, mn, mux, muy, mT, E);
            double ci = A[i][i] * omega;
            double* Fcur = Fi + (size_t)i * tot;
            double* dcur = dF + (size_t)i * tot;
            for (size_t e = 0; e < tot; e++) {
                Fcur[e] = (S[e] + ci * E[e]) / (1.0 + ci);
                dcur[e] = omega * (Fcur[e] - E[e]);
            }
            /* explicit advection of this stage, where any later row uses it */
            int used = wt[i] != 0.0;
            for (int k = i + 1; k < 4; k++) used |= At[k][i] != 0.0;
            if (used) advect_with(c, px, py, Fcur, VFi + (size_t)i * tot);
        }
        for (size_t e = 0; e < tot; e++) {
            double s = F[e];
            for (int i = 0; i < 4; i++) {
                if (wt[i] != 0.0) s -= c->dt * wt[i] * VFi[(size_t)i * tot + e];
                if (w[i] != 0.0) s -= w[i] * dF[(size_t)i * tot + e];
            }
            F[e] = s;
        }
    }
    if (stages && nsteps > 0) memcpy(stages, Fi, sizeof(double) * tot * 4);
    free(px); free(py); free(S); free(E); free(Fi); free(dF); free(VFi);
    free(mn); free(mux); free(muy); free(mT);
    return 0;
}
