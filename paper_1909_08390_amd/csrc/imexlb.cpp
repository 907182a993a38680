// Host side of the imexlb C ABI: configuration checks, Gauss-Hermite
// quadrature and equilibrium tables (Sec. II), buffer binding and the launch
// sequence of the IMEX-SSP3(4,3,3) step (Sec. III).
#include "imexlb.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <new>
#include <string>

#include "common.hpp"

using namespace imexlb;

struct imexlb_ctx {
    imexlb_config cfg;
    hipStream_t stream = nullptr;
    int device = 0;
    int nplanes = 0, nphi = 0, nf = 0;  // planes, phi planes, moment fields
    long long cells = 0;
    size_t elem = 8;
    double p[2][kQMax] = {}, w[2][kQMax] = {};
    DevTables* d_tab = nullptr;
    double* d_small = nullptr;   // reduction partials + 4 sums
    int* d_flag = nullptr;
    int nred = 0;
    void* d_state = nullptr;
    void* d_work = nullptr;
    void* d_adj = nullptr;       // adjoint workspace (caller-owned)
    bool have_state = false;
    std::string err;
};

namespace {

constexpr double kAlpha = 0.24169426078821;  // Table I

imexlb_status fail(imexlb_ctx* c, imexlb_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

imexlb_status hip_fail(imexlb_ctx* c, hipError_t e, const char* what) {
    return fail(c, IMEXLB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// He_n(x) by He_{n+1} = x He_n - n He_{n-1}.
long double he(int n, long double x) {
    long double a = 1.0L, b = x;
    if (n == 0) return a;
    for (int j = 1; j < n; ++j) {
        long double c = x * b - (long double)j * a;
        a = b;
        b = c;
    }
    return b;
}

// Gauss-Hermite rule for the weight exp(-p^2/2)/sqrt(2 pi) (Sec. II):
// eigenvalues of the symmetric Jacobi matrix of the monic recurrence
// (off-diagonal sqrt(k)) by cyclic Jacobi rotations, polished by Newton on
// He_Q; weights Q!/(Q He_{Q-1}(p))^2, which equals the paper's
// Q!/He_{Q+1}(p)^2 at a root of He_Q.
bool gauss_hermite(int Q, double* p, double* w) {
    if (Q < 1 || Q > kQMax) return false;
    long double A[kQMax][kQMax] = {};
    for (int k = 0; k + 1 < Q; ++k) A[k][k + 1] = A[k + 1][k] = sqrtl((long double)(k + 1));
    for (int sweep = 0; sweep < 100; ++sweep) {
        long double off = 0.0L;
        for (int i = 0; i < Q; ++i)
            for (int j = i + 1; j < Q; ++j) off += A[i][j] * A[i][j];
        if (off < 1e-36L) break;
        for (int i = 0; i < Q; ++i)
            for (int j = i + 1; j < Q; ++j) {
                if (A[i][j] == 0.0L) continue;
                long double th = (A[j][j] - A[i][i]) / (2.0L * A[i][j]);
                long double t = (th >= 0 ? 1.0L : -1.0L) / (fabsl(th) + sqrtl(th * th + 1.0L));
                long double c = 1.0L / sqrtl(t * t + 1.0L), s = t * c;
                for (int k = 0; k < Q; ++k) {  // A <- A R
                    long double aki = A[k][i], akj = A[k][j];
                    A[k][i] = c * aki - s * akj;
                    A[k][j] = s * aki + c * akj;
                }
                for (int k = 0; k < Q; ++k) {  // A <- R^T A
                    long double aik = A[i][k], ajk = A[j][k];
                    A[i][k] = c * aik - s * ajk;
                    A[j][k] = s * aik + c * ajk;
                }
            }
    }
    long double x[kQMax];
    for (int i = 0; i < Q; ++i) x[i] = A[i][i];
    for (int i = 1; i < Q; ++i)  // ascending
        for (int j = i; j > 0 && x[j] < x[j - 1]; --j) {
            long double t = x[j];
            x[j] = x[j - 1];
            x[j - 1] = t;
        }
    long double qf = 1.0L;
    for (int j = 2; j <= Q; ++j) qf *= (long double)j;
    for (int i = 0; i < Q; ++i) {
        for (int it = 0; it < 8; ++it) {  // He_Q' = Q He_{Q-1}
            long double f = he(Q, x[i]), df = (long double)Q * he(Q - 1, x[i]);
            if (df == 0.0L) break;
            x[i] -= f / df;
        }
    }
    for (int i = 0; i < Q / 2; ++i) {  // He_Q(-x) = (-1)^Q He_Q(x)
        long double m = 0.5L * (x[Q - 1 - i] - x[i]);
        x[i] = -m;
        x[Q - 1 - i] = m;
    }
    if (Q % 2) x[Q / 2] = 0.0L;
    for (int i = 0; i < Q; ++i) {
        long double d = (long double)Q * he(Q - 1, x[i]);
        p[i] = (double)x[i];
        w[i] = (double)(Q == 1 ? 1.0L : qf / (d * d));
    }
    return true;
}

}  // namespace

namespace imexlb {

bool quadrature_rule(int Q, double* p, double* w) { return gauss_hermite(Q, p, w); }

// Builds the constant tables of one quadrature (Sec. II) and copies them to
// a new device allocation *d_tab (synchronous on s).
hipError_t upload_tables(int d, const int Q[2], const double p[2][kQMax], const double w[2][kQMax],
                         int tab_nodes, DevTables** d_tab, hipStream_t stream) {
    *d_tab = nullptr;
    DevTables* t = new (std::nothrow) DevTables();
    if (!t) return hipErrorOutOfMemory;
    const int nphi = d == 2 ? Q[0] * Q[0] : Q[0];
    const int nplanes = nphi + (d == 2 ? Q[1] * Q[1] : Q[1]);
    std::memset(t, 0, sizeof(*t));
    for (int s = 0; s < 2; ++s) {
        t->q[s] = Q[s];
        for (int k = 0; k < Q[s]; ++k) {
            long double fact = 1.0L;
            for (int l = 0; l < Q[s]; ++l) {
                if (l > 0) fact *= (long double)l;
                t->h[s][k][l] = (double)((long double)w[s][k] * he(l, (long double)p[s][k]) / fact);
            }
        }
    }
    // Even/odd Horner rows: B_k[s][j] = w_k He_{j+2s}(p_k) / (2^s s! j!) for
    // j + 2s < Q (the regrouped double sum of Eq. gExpanded), zero beyond.
    auto horner_row = [&](int s, int k, int QM, double* row) {
        const int S = (QM - 1) / 2;
        int o = 0;
        for (int ss = 0; ss <= S; ++ss) {
            for (int par = 0; par < 2; ++par)
                for (int j = par; j <= QM - 1 - 2 * ss; j += 2) {
                    double val = 0.0;
                    if (j + 2 * ss < Q[s]) {
                        long double den = 1.0L;
                        for (int i = 1; i <= ss; ++i) den *= 2.0L * (long double)i;  // 2^s s!
                        for (int i = 2; i <= j; ++i) den *= (long double)i;          // j!
                        val = (double)((long double)w[s][k] * he(j + 2 * ss, (long double)p[s][k]) / den);
                    }
                    row[o++] = val;
                }
        }
    };
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < Q[s]; ++k) {
            horner_row(s, k, 8, t->hc8[s][k]);
            horner_row(s, k, 16, t->hc16[s][k]);
        }
    t->nplanes = nplanes;
    t->nphi = nphi;
    {   // processing order of the passes: per set, ky-major; every node (in
        // x and in y) followed by its mirror, so that one Horner evaluation
        // gives the factors of both.  2D grids of orders up to 8 take the x
        // nodes of a set in table groups of tab_nodes / 2 mirror pairs (all
        // ky of one group before the next group), so that the kernels keep
        // the x factors of one group in LDS tables.
        const bool grouped = d == 2 && Q[0] <= 8 && Q[1] <= 8;
        int j = 0;
        for (int s = 0; s < 2; ++s) {
            const int base = s ? nphi : 0;
            const int nyg = d == 2 ? Q[s] : 1;
            const int npairs = (Q[s] + 1) / 2;
            const int gpairs = grouped ? std::max(1, tab_nodes / 2) : npairs;
            for (int k0 = 0; k0 < npairs; k0 += gpairs) {
                const int kend = std::min(npairs, k0 + gpairs);
                bool tab_start = true;
                for (int ly = 0; ly < (nyg + 1) / 2; ++ly) {
                    const int ypair[2] = {ly, nyg - 1 - ly};
                    const int ycnt = ypair[0] == ypair[1] ? 1 : 2;
                    for (int ey = 0; ey < ycnt; ++ey) {
                        const int ky = ypair[ey];
                        bool group_start = true;
                        for (int k = k0; k < kend; ++k) {
                            const int pair[2] = {k, Q[s] - 1 - k};
                            const int cnt = pair[0] == pair[1] ? 1 : 2;
                            for (int e = 0; e < cnt; ++e, ++j) {
                                PlaneStep& st = t->order[j];
                                const int kx = pair[e];
                                st.v = base + kx + Q[s] * ky;
                                st.set = s;
                                st.kx = kx;
                                st.ky = ky;
                                st.hx = k;
                                st.first = e == 0;
                                st.hy = ly;
                                st.new_group = group_start;
                                st.yfirst = group_start && ey == 0;
                                st.new_tab = tab_start;
                                st.tcount = grouped ? kend - k0 : 0;
                                st.slot = grouped ? 2 * (k - k0) + e : 0;
                                group_start = false;
                                tab_start = false;
                            }
                        }
                    }
                }
            }
        }
    }
    int v = 0;
    for (int s = 0; s < 2; ++s) {
        const int ny_ = d == 2 ? Q[s] : 1;
        for (int ky = 0; ky < ny_; ++ky)
            for (int kx = 0; kx < Q[s]; ++kx, ++v) {
                PlaneDesc& pd = t->plane[v];
                pd.px = p[s][kx];
                pd.py = d == 2 ? p[s][ky] : 0.0;
                pd.set = s;
                pd.kx = kx;
                pd.ky = ky;
                if (s == 0) {
                    pd.m0 = 1.0;
                    pd.mx = pd.px;
                    pd.my = pd.py;
                    pd.me = pd.px * pd.px + pd.py * pd.py;
                } else {
                    pd.m0 = pd.mx = pd.my = 0.0;
                    pd.me = 1.0;
                }
            }
    }
    for (int j = 0; j < nplanes; ++j) {
        PlaneStep& st = t->order[j];
        const PlaneDesc& pd = t->plane[st.v];
        st.px = pd.px;
        st.py = pd.py;
        st.m0 = pd.m0;
        st.mx = pd.mx;
        st.my = pd.my;
        st.me = pd.me;
        PackedStep& ps = t->step[j];
        ps.px = st.px;
        ps.py = st.py;
        ps.v = st.v;
        ps.bits = st.set | (st.first << 1) | (st.new_group << 2) | (st.yfirst << 3) | (st.new_tab << 4) |
                  ((j == nplanes - 1) << 5) | (st.slot << 6) | (st.tcount << 9) | (st.hx << 12) |
                  (st.hy << 17);
    }
    hipError_t e = hipMalloc((void**)d_tab, sizeof(DevTables));
    if (e == hipSuccess) e = hipMemcpyAsync(*d_tab, t, sizeof(DevTables), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    delete t;
    if (e != hipSuccess && *d_tab) {
        (void)hipFree(*d_tab);
        *d_tab = nullptr;
    }
    return e;
}

void stage_coefficients(double dt, double tau, StageArgs& a) {
    a.dt = dt;
    a.omega = dt / tau;
    const double cc = kAlpha * a.omega;
    a.a1 = 1.0 / (1.0 + cc);
    a.a2 = (1.0 + 2.0 * cc) / ((1.0 + cc) * (1.0 + cc));
    constexpr double be = 0.06042356519705, et = 0.12915286960590;  // Table I
    const double ka = 0.5 - be - et - kAlpha;
    const double w = a.omega;
    a.k[0] = (1.0 - kAlpha) * w * a.a2;
    a.k[1] = 0.25 * (1.0 - kAlpha) * w * a.a2 - be * w * a.a1 - et * w * a.a2;
    a.k[2] = ka * w * a.a1;
    a.k[3] = kAlpha * w * a.a2 / 6.0;
    a.k[4] = w * a.a1 / 6.0;
    a.k[5] = 2.0 * w * a.a1 / 3.0;
}

// Pass 3 advects F2 = a2 F^n + b2 E^n; passes 4 and 5 advect
// F3 = a1 G3 + c a1 E3 and F4 = a1 G4 + c a1 E4 (relax on read).
void pass_args(const StageArgs& a, void* F, void* G3, void* G4, double* Mn, double* M3, double* M4,
               StageArgs out[3], void* Fnext) {
    if (!Fnext) Fnext = F;
    const double cc = kAlpha * a.omega;
    out[0] = out[1] = out[2] = a;
    out[0].src = F;
    out[0].msrc = Mn;
    out[0].out = G3;
    out[0].mout = M3;
    out[0].a_rel = a.a2;
    out[0].b_rel = cc * cc / ((1.0 + cc) * (1.0 + cc));
    out[1].src = G3;
    out[1].msrc = M3;
    out[1].out = G4;
    out[1].mout = M4;
    out[1].fbuf = F;
    out[1].rbuf = Fnext;
    out[1].mn = Mn;
    out[1].a_rel = a.a1;
    out[1].b_rel = cc * a.a1;
    out[2].src = G4;
    out[2].msrc = M4;
    out[2].out = Fnext;
    out[2].mout = Mn;
    out[2].fbuf = Fnext;
    out[2].a_rel = a.a1;
    out[2].b_rel = cc * a.a1;
}

}  // namespace imexlb

namespace {

imexlb_status validate(const imexlb_config* c, std::string& why) {
    if (!c) { why = "config is NULL"; return IMEXLB_EINVAL; }
    if (c->d != 1 && c->d != 2) { why = "d must be 1 or 2"; return IMEXLB_EINVAL; }
    if (c->nx < 1 || c->ny < 1) { why = "nx, ny must be >= 1"; return IMEXLB_EINVAL; }
    if (c->d == 1 && c->ny != 1) { why = "ny must be 1 when d = 1"; return IMEXLB_EINVAL; }
    if ((long long)c->nx * c->ny >= (1LL << 31)) { why = "too many cells (>= 2^31)"; return IMEXLB_EINVAL; }
    if (!(c->lx > 0.0) || (c->d == 2 && !(c->ly > 0.0))) { why = "lengths must be > 0"; return IMEXLB_EINVAL; }
    if (c->q_phi < 3 || c->q_phi > kQMax) { why = "q_phi must be in [3, 16]"; return IMEXLB_EINVAL; }
    if (c->q_chi < 1 || c->q_chi > kQMax) { why = "q_chi must be in [1, 16]"; return IMEXLB_EINVAL; }
    if (c->K < 0) { why = "K must be >= 0"; return IMEXLB_EINVAL; }
    if (!(c->tau > 0.0) || !std::isfinite(c->tau)) { why = "tau must be > 0"; return IMEXLB_EINVAL; }
    if (!(c->dt > 0.0) || !std::isfinite(c->dt)) { why = "dt must be > 0"; return IMEXLB_EINVAL; }
    if (c->bc_x != IMEXLB_OUTFLOW && c->bc_x != IMEXLB_PERIODIC) { why = "bad bc_x"; return IMEXLB_EINVAL; }
    if (c->d == 2 && c->bc_y != IMEXLB_OUTFLOW && c->bc_y != IMEXLB_PERIODIC) { why = "bad bc_y"; return IMEXLB_EINVAL; }
    if (c->storage != IMEXLB_F64 && c->storage != IMEXLB_F32) { why = "bad storage"; return IMEXLB_EINVAL; }
    {
        // planes are addressed with 32-bit byte offsets (one tile row of slack)
        const long long elem = c->storage == IMEXLB_F32 ? 4 : 8;
        if (((long long)c->ny + kTile2Y) * c->nx * elem >= (1LL << 31)) {
            why = "one plane must stay below 2 GiB";
            return IMEXLB_EINVAL;
        }
    }
    return IMEXLB_OK;
}

imexlb_status need_state(const imexlb_ctx* c) {
    if (!c->d_state || !c->d_work) return IMEXLB_ESTATE;
    if (!c->have_state) return IMEXLB_ESTATE;
    return IMEXLB_OK;
}

// Workspace: G3 | G4 | M^n | M3 | M4.
void* work_g(const imexlb_ctx* c, int i) {
    return (char*)c->d_work + (size_t)i * align256((size_t)c->nplanes * c->cells * c->elem);
}
double* work_m(const imexlb_ctx* c, int i) {
    size_t off = 2 * align256((size_t)c->nplanes * c->cells * c->elem) +
                 (size_t)i * align256((size_t)c->nf * c->cells * sizeof(double));
    return (double*)((char*)c->d_work + off);
}

StageArgs base_args(const imexlb_ctx* c) {
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    const imexlb_config& k = c->cfg;
    a.tab = c->d_tab;
    a.nx = k.nx;
    a.ny = k.d == 2 ? k.ny : 1;
    a.bcx = k.bc_x;
    a.bcy = k.d == 2 ? k.bc_y : 0;
    if (k.d == 2) {
        a.ntx = (k.nx + kTile2X - 1) / kTile2X;
        a.nty = (k.ny + kTile2Y - 1) / kTile2Y;
    } else {
        a.ntx = (k.nx + kTile1X - 1) / kTile1X;
        a.nty = 1;
    }
    a.tiles_per_xcd = (a.ntx * a.nty + 7) / 8;
    a.qm = (k.q_phi <= 8 && k.q_chi <= 8) ? 8 : 16;
    a.paired = k.d == 2 && k.q_phi % 2 == 0 && k.q_chi % 2 == 0;
    a.plane_stride = c->cells;
    a.mstride = c->cells;
    a.inv_dx = k.nx / k.lx;
    a.inv_dy = k.d == 2 ? k.ny / k.ly : 0.0;
    stage_coefficients(k.dt, k.tau, a);
    a.chi_fac = (double)(k.K + kDTotal - k.d);
    a.dk = (double)(kDTotal + k.K);
    return a;
}

}  // namespace

extern "C" {

const char* imexlb_status_string(imexlb_status s) {
    switch (s) {
        case IMEXLB_OK: return "ok";
        case IMEXLB_EINVAL: return "invalid argument";
        case IMEXLB_ENOMEM: return "out of memory";
        case IMEXLB_EHIP: return "HIP runtime error";
        case IMEXLB_ENONPHYS: return "non-physical state (n <= 0, T <= 0 or non-finite)";
        case IMEXLB_ESTATE: return "call out of order (no bound buffers or no state)";
    }
    return "unknown status";
}

const char* imexlb_last_error(const imexlb_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

imexlb_status imexlb_create(const imexlb_config* cfg, void* hip_stream, imexlb_ctx** out) {
    if (!out) return IMEXLB_EINVAL;
    *out = nullptr;
    std::string why;
    imexlb_status st = validate(cfg, why);
    if (st != IMEXLB_OK) {
        std::fprintf(stderr, "imexlb_create: %s\n", why.c_str());
        return st;
    }
    imexlb_ctx* c = new (std::nothrow) imexlb_ctx();
    if (!c) return IMEXLB_ENOMEM;
    c->cfg = *cfg;
    if (cfg->d == 1) c->cfg.ny = 1;
    c->stream = (hipStream_t)hip_stream;
    const int d = cfg->d;
    const int Q[2] = {cfg->q_phi, cfg->q_chi};
    for (int s = 0; s < 2; ++s)
        if (!gauss_hermite(Q[s], c->p[s], c->w[s])) {
            delete c;
            return IMEXLB_EINVAL;
        }
    // CFL = |p| dt / delta s <= 1 for every advection velocity (Sec. IV).
    double pmax = 0.0;
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < Q[s]; ++k) pmax = std::fmax(pmax, std::fabs(c->p[s][k]));
    const double cflx = pmax * cfg->dt * cfg->nx / cfg->lx;
    const double cfly = d == 2 ? pmax * cfg->dt * cfg->ny / cfg->ly : 0.0;
    if (cflx > 1.0 || cfly > 1.0) {
        std::fprintf(stderr, "imexlb_create: CFL %.3f > 1\n", std::fmax(cflx, cfly));
        delete c;
        return IMEXLB_EINVAL;
    }
    c->nphi = d == 2 ? Q[0] * Q[0] : Q[0];
    c->nplanes = c->nphi + (d == 2 ? Q[1] * Q[1] : Q[1]);
    c->nf = d + 2;
    c->cells = (long long)cfg->nx * c->cfg.ny;
    c->elem = cfg->storage == IMEXLB_F32 ? 4 : 8;

    hipError_t e = upload_tables(d, Q, c->p, c->w, kTabNodes2D, &c->d_tab, c->stream);
    if (e == hipErrorOutOfMemory) {
        delete c;
        return IMEXLB_ENOMEM;
    }
    if (e == hipSuccess) e = hipGetDevice(&c->device);
    c->nred = kSumBlocks;
    if (e == hipSuccess) e = hipMalloc((void**)&c->d_small, sizeof(double) * (4 * c->nred + 4));
    if (e == hipSuccess) e = hipMalloc((void**)&c->d_flag, sizeof(int) * 64);
    if (e != hipSuccess) {
        std::fprintf(stderr, "imexlb_create: %s\n", hipGetErrorString(e));
        imexlb_destroy(c);
        return IMEXLB_EHIP;
    }
    *out = c;
    return IMEXLB_OK;
}

void imexlb_destroy(imexlb_ctx* c) {
    if (!c) return;
    if (c->d_tab) (void)hipFree(c->d_tab);
    if (c->d_small) (void)hipFree(c->d_small);
    if (c->d_flag) (void)hipFree(c->d_flag);
    delete c;
}

imexlb_status imexlb_set_stream(imexlb_ctx* c, void* s) {
    if (!c) return IMEXLB_EINVAL;
    c->stream = (hipStream_t)s;
    return IMEXLB_OK;
}

size_t imexlb_state_bytes(const imexlb_ctx* c) {
    return c ? (size_t)c->nplanes * c->cells * c->elem : 0;
}

size_t imexlb_workspace_bytes(const imexlb_ctx* c) {
    if (!c) return 0;
    return 2 * align256((size_t)c->nplanes * c->cells * c->elem) +
           3 * align256((size_t)c->nf * c->cells * sizeof(double));
}

int imexlb_num_planes(const imexlb_ctx* c) { return c ? c->nplanes : 0; }

imexlb_status imexlb_bind(imexlb_ctx* c, void* d_state, void* d_work) {
    if (!c) return IMEXLB_EINVAL;
    if (!d_state || !d_work) return fail(c, IMEXLB_EINVAL, "bind: NULL buffer");
    if (((uintptr_t)d_state & 255) || ((uintptr_t)d_work & 255))
        return fail(c, IMEXLB_EINVAL, "bind: buffers must be 256-byte aligned");
    c->d_state = d_state;
    c->d_work = d_work;
    c->have_state = false;
    return IMEXLB_OK;
}

imexlb_status imexlb_quadrature(const imexlb_ctx* c, double* pp, double* wp, double* pc, double* wc) {
    if (!c) return IMEXLB_EINVAL;
    for (int k = 0; k < c->cfg.q_phi; ++k) {
        if (pp) pp[k] = c->p[0][k];
        if (wp) wp[k] = c->w[0][k];
    }
    for (int k = 0; k < c->cfg.q_chi; ++k) {
        if (pc) pc[k] = c->p[1][k];
        if (wc) wc[k] = c->w[1][k];
    }
    return IMEXLB_OK;
}

imexlb_status imexlb_set_equilibrium(imexlb_ctx* c, const double* n, const double* ux,
                                     const double* uy, const double* T) {
    if (!c) return IMEXLB_EINVAL;
    if (!c->d_state || !c->d_work) return fail(c, IMEXLB_ESTATE, "set_equilibrium: not bound");
    if (!n || !ux || !T || (c->cfg.d == 2 && !uy)) return fail(c, IMEXLB_EINVAL, "set_equilibrium: NULL field");
    const bool f32 = c->cfg.storage == IMEXLB_F32;
    hipError_t e = launch_init_equilibrium(c->cfg.d, f32, c->d_tab, n, ux, uy, T, c->d_state, nullptr,
                                           c->cells, (double)(c->cfg.K + kDTotal - c->cfg.d), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_equilibrium");
    e = launch_moments(c->cfg.d, f32, c->d_tab, c->d_state, work_m(c, 0), c->cells, c->cells,
                       (double)(kDTotal + c->cfg.K), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_equilibrium moments");
    c->have_state = true;
    return IMEXLB_OK;
}

imexlb_status imexlb_set_state(imexlb_ctx* c, const void* F) {
    if (!c) return IMEXLB_EINVAL;
    if (!c->d_state || !c->d_work) return fail(c, IMEXLB_ESTATE, "set_state: not bound");
    if (!F) return fail(c, IMEXLB_EINVAL, "set_state: NULL");
    hipError_t e = hipSuccess;
    if (F != c->d_state)
        e = hipMemcpyAsync(c->d_state, F, imexlb_state_bytes(c), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_state copy");
    e = launch_moments(c->cfg.d, c->cfg.storage == IMEXLB_F32, c->d_tab, c->d_state, work_m(c, 0),
                       c->cells, c->cells, (double)(kDTotal + c->cfg.K), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_state moments");
    c->have_state = true;
    return IMEXLB_OK;
}

imexlb_status imexlb_get_state(const imexlb_ctx* c, void* F) {
    if (!c) return IMEXLB_EINVAL;
    if (!F) return fail(const_cast<imexlb_ctx*>(c), IMEXLB_EINVAL, "get_state: NULL");
    if (need_state(c) != IMEXLB_OK) return fail(const_cast<imexlb_ctx*>(c), IMEXLB_ESTATE, "get_state: no state");
    if (F == c->d_state) return IMEXLB_OK;
    hipError_t e = hipMemcpyAsync(F, c->d_state, imexlb_state_bytes(c), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(const_cast<imexlb_ctx*>(c), e, "get_state");
    return IMEXLB_OK;
}

}  // extern "C"

namespace {

// Where a recorded step puts its stage sources and moments (caller memory,
// imexlb_step_record_bytes): G3 | G4 (storage type) | M^n | M3 | M4 (FP64),
// and in 2D | F2 | F3 | F4, the stage values the three passes swept, as
// stored at the own cells by their relax on read (storage type).
struct StepRecord {
    void *G3, *G4;
    double *Mn, *M3, *M4;
    void *F2, *F3, *F4;  // NULL in 1D
};

size_t record_ps(const imexlb_ctx* c) { return align256((size_t)c->nplanes * c->cells * c->elem); }
size_t record_ms(const imexlb_ctx* c) { return align256((size_t)c->nf * c->cells * sizeof(double)); }
int record_nsv(const imexlb_ctx* c) { return c->cfg.d == 2 ? 3 : 0; }
size_t record_bytes(const imexlb_ctx* c) { return (2 + record_nsv(c)) * record_ps(c) + 3 * record_ms(c); }

StepRecord record_of(const imexlb_ctx* c, const void* rec) {
    char* b = (char*)rec;
    const size_t ps = record_ps(c), ms = record_ms(c);
    char* f = b + 2 * ps + 3 * ms;
    const bool sv = record_nsv(c) > 0;
    return StepRecord{b, b + ps, (double*)(b + 2 * ps), (double*)(b + 2 * ps + ms), (double*)(b + 2 * ps + 2 * ms),
                      sv ? f : nullptr, sv ? f + ps : nullptr, sv ? f + 2 * ps : nullptr};
}

// The launch sequence of nsteps IMEX steps.  When ev is non-NULL it holds
// 3 * nsteps + 1 events recorded around the passes.  With rec (one step),
// the stage sources G3, G4 and the moments M3, M4 go to the record instead
// of the workspace.  With next (one step), R and F^{n+1} go to next, which
// then becomes the bound state; the buffer bound before keeps F^n.
imexlb_status run_steps(imexlb_ctx* c, int nsteps, hipEvent_t* ev, const StepRecord* rec = nullptr,
                        void* next = nullptr) {
    const int d = c->cfg.d;
    const bool f32 = c->cfg.storage == IMEXLB_F32;
    StageArgs a = base_args(c);
    void* F = c->d_state;
    void* G3 = rec ? rec->G3 : work_g(c, 0);
    void* G4 = rec ? rec->G4 : work_g(c, 1);
    double* Mn = work_m(c, 0);
    double* M3 = rec ? rec->M3 : work_m(c, 1);
    double* M4 = rec ? rec->M4 : work_m(c, 2);
    StageArgs pa[3];
    // an out-of-place step is a recorded one: in 2D only the recording
    // passes write R to a buffer other than the state they read
    if (next && !rec) return fail(c, IMEXLB_EINVAL, "step: out of place without a record");
    pass_args(a, F, G3, G4, Mn, M3, M4, pa, next);
    if (rec) {
        pa[0].sval_out = rec->F2;
        pa[1].sval_out = rec->F3;
        pa[2].sval_out = rec->F4;
    }
    const StageArgs &a3 = pa[0], &a4 = pa[1], &a5 = pa[2];
    const bool check = c->cfg.check_physical != 0;
    hipError_t e = hipSuccess;
    if (check) e = launch_check_reset(c->d_flag, c->stream);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[0], c->stream);
    for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
        e = launch_stage(d, f32, kStage3, a3, c->stream);
        if (e == hipSuccess && ev) e = hipEventRecord(ev[3 * s + 1], c->stream);
        if (e == hipSuccess) e = launch_stage(d, f32, kStage4, a4, c->stream);
        if (e == hipSuccess && ev) e = hipEventRecord(ev[3 * s + 2], c->stream);
        if (e == hipSuccess) e = launch_stage(d, f32, kStage5, a5, c->stream);
        // the moments of F^{n+1} (written by pass 5) against n > 0, T > 0, finite
        if (e == hipSuccess && check) e = launch_check(d, Mn, c->cells, c->cells, s + 1, c->d_flag, c->stream);
        if (e == hipSuccess && ev) e = hipEventRecord(ev[3 * s + 3], c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "step");
    if (next) c->d_state = next;
    return IMEXLB_OK;
}

// With check_physical set: wait for the steps and report the first step
// that produced a non-physical cell.
imexlb_status finish_check(imexlb_ctx* c) {
    if (!c->cfg.check_physical) return IMEXLB_OK;
    int h = 0;
    hipError_t e = hipMemcpyAsync(&h, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "step: physical check");
    if (h != INT_MAX)
        return fail(c, IMEXLB_ENONPHYS, "step: non-physical moments (n <= 0, T <= 0 or non-finite) after step " +
                                            std::to_string(h) + " of this call");
    return IMEXLB_OK;
}

}  // namespace

extern "C" {

imexlb_status imexlb_step(imexlb_ctx* c, int nsteps) {
    if (!c) return IMEXLB_EINVAL;
    if (nsteps < 0) return fail(c, IMEXLB_EINVAL, "step: nsteps < 0");
    if (need_state(c) != IMEXLB_OK) return fail(c, IMEXLB_ESTATE, "step: no bound state");
    imexlb_status st = run_steps(c, nsteps, nullptr);
    return st == IMEXLB_OK ? finish_check(c) : st;
}

size_t imexlb_step_record_bytes(const imexlb_ctx* c) {
    return c ? record_bytes(c) : 0;
}

}  // extern "C"

namespace {

imexlb_status step_recorded(imexlb_ctx* c, void* d_record, void* d_next, const char* what) {
    if (!c) return IMEXLB_EINVAL;
    const std::string w = what;
    if (!d_record) return fail(c, IMEXLB_EINVAL, w + ": NULL record");
    if ((uintptr_t)d_record & 255) return fail(c, IMEXLB_EINVAL, w + ": record must be 256-byte aligned");
    if (need_state(c) != IMEXLB_OK) return fail(c, IMEXLB_ESTATE, w + ": no bound state");
    const StepRecord r = record_of(c, d_record);
    // M^n before pass 5 overwrites it with M^{n+1}
    hipError_t e = hipMemcpyAsync(r.Mn, work_m(c, 0), (size_t)c->nf * c->cells * sizeof(double),
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, what);
    imexlb_status st = run_steps(c, 1, nullptr, &r, d_next);
    return st == IMEXLB_OK ? finish_check(c) : st;
}

}  // namespace

extern "C" {

imexlb_status imexlb_step_recorded(imexlb_ctx* c, void* d_record) {
    return step_recorded(c, d_record, nullptr, "step_recorded");
}

imexlb_status imexlb_step_recorded_to(imexlb_ctx* c, void* d_record, void* d_next) {
    if (!c) return IMEXLB_EINVAL;
    if (!d_next) return fail(c, IMEXLB_EINVAL, "step_recorded_to: NULL next state");
    if ((uintptr_t)d_next & 255) return fail(c, IMEXLB_EINVAL, "step_recorded_to: next state must be 256-byte aligned");
    if (need_state(c) != IMEXLB_OK) return fail(c, IMEXLB_ESTATE, "step_recorded_to: no bound state");
    // the next buffer must not overlap the bound state, the workspace or the record
    auto overlaps = [](const void* a, size_t na, const void* b, size_t nb) {
        const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
        return x < y + nb && y < x + na;
    };
    const size_t sb = imexlb_state_bytes(c);
    if (overlaps(d_next, sb, c->d_state, sb) || overlaps(d_next, sb, c->d_work, imexlb_workspace_bytes(c)) ||
        overlaps(d_next, sb, d_record, record_bytes(c)))
        return fail(c, IMEXLB_EINVAL, "step_recorded_to: next state overlaps the bound state, the workspace or the record");
    return step_recorded(c, d_record, d_next, "step_recorded_to");
}

imexlb_status imexlb_step_timed(imexlb_ctx* c, int nsteps, double ms[3]) {
    if (!c || !ms) return IMEXLB_EINVAL;
    if (nsteps < 0) return fail(c, IMEXLB_EINVAL, "step_timed: nsteps < 0");
    if (need_state(c) != IMEXLB_OK) return fail(c, IMEXLB_ESTATE, "step_timed: no bound state");
    const int ne = 3 * nsteps + 1;
    hipEvent_t* ev = new (std::nothrow) hipEvent_t[ne];
    if (!ev) return fail(c, IMEXLB_ENOMEM, "step_timed: events");
    int made = 0;
    hipError_t e = hipSuccess;
    for (; made < ne && e == hipSuccess; ++made) e = hipEventCreate(&ev[made]);
    imexlb_status st = IMEXLB_OK;
    if (e != hipSuccess) {
        --made;
        st = hip_fail(c, e, "step_timed: event create");
    } else {
        st = run_steps(c, nsteps, ev);
        if (st == IMEXLB_OK) {
            e = hipEventSynchronize(ev[ne - 1]);
            for (int s = 0; s < nsteps && e == hipSuccess; ++s)
                for (int k = 0; k < 3 && e == hipSuccess; ++k) {
                    float t = 0.0f;
                    e = hipEventElapsedTime(&t, ev[3 * s + k], ev[3 * s + k + 1]);
                    ms[k] += t;
                }
            if (e != hipSuccess) st = hip_fail(c, e, "step_timed: elapsed");
            if (st == IMEXLB_OK) st = finish_check(c);
        }
    }
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    delete[] ev;
    return st;
}

imexlb_status imexlb_moments(const imexlb_ctx* c, double* n, double* ux, double* uy, double* T) {
    if (!c) return IMEXLB_EINVAL;
    imexlb_ctx* m = const_cast<imexlb_ctx*>(c);
    if (need_state(c) != IMEXLB_OK) return fail(m, IMEXLB_ESTATE, "moments: no state");
    const double* M = work_m(c, 0);
    const size_t b = (size_t)c->cells * sizeof(double);
    double* dst[4] = {n, ux, c->cfg.d == 2 ? uy : nullptr, T};
    int src[4] = {0, 1, 2, c->nf - 1};
    for (int f = 0; f < 4; ++f) {
        if (!dst[f]) continue;
        hipError_t e = hipMemcpyAsync(dst[f], M + (size_t)src[f] * c->cells, b, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(m, e, "moments copy");
    }
    return IMEXLB_OK;
}

imexlb_status imexlb_compute_moments(const imexlb_ctx* c, const void* F, double* n, double* ux,
                                     double* uy, double* T) {
    if (!c) return IMEXLB_EINVAL;
    imexlb_ctx* m = const_cast<imexlb_ctx*>(c);
    if (!c->d_work) return fail(m, IMEXLB_ESTATE, "compute_moments: not bound");
    if (!F || !n || !ux || !T) return fail(m, IMEXLB_EINVAL, "compute_moments: NULL");
    // computed into the M3 slot of the workspace, then copied out
    double* M = work_m(c, 1);
    hipError_t e = launch_moments(c->cfg.d, c->cfg.storage == IMEXLB_F32, c->d_tab, F, M, c->cells,
                                  c->cells, (double)(kDTotal + c->cfg.K), c->stream);
    if (e != hipSuccess) return hip_fail(m, e, "compute_moments");
    const size_t b = (size_t)c->cells * sizeof(double);
    double* dst[4] = {n, ux, c->cfg.d == 2 ? uy : nullptr, T};
    int src[4] = {0, 1, 2, c->nf - 1};
    for (int f = 0; f < 4; ++f) {
        if (!dst[f]) continue;
        e = hipMemcpyAsync(dst[f], M + (size_t)src[f] * c->cells, b, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(m, e, "compute_moments copy");
    }
    return IMEXLB_OK;
}

imexlb_status imexlb_advect(const imexlb_ctx* c, const void* F, double* VF) {
    if (!c) return IMEXLB_EINVAL;
    imexlb_ctx* m = const_cast<imexlb_ctx*>(c);
    if (!F || !VF) return fail(m, IMEXLB_EINVAL, "advect: NULL");
    StageArgs a = base_args(c);
    a.src = F;
    a.out = VF;
    a.a_rel = 1.0;
    a.b_rel = 0.0;
    hipError_t e = launch_stage(c->cfg.d, c->cfg.storage == IMEXLB_F32, kAdvect, a, c->stream);
    if (e != hipSuccess) return hip_fail(m, e, "advect");
    return IMEXLB_OK;
}

imexlb_status imexlb_domain_sums(const imexlb_ctx* c, double out[4]) {
    if (!c || !out) return IMEXLB_EINVAL;
    imexlb_ctx* m = const_cast<imexlb_ctx*>(c);
    if (need_state(c) != IMEXLB_OK) return fail(m, IMEXLB_ESTATE, "domain_sums: no state");
    double* part = c->d_small;
    double* res = c->d_small + 4 * c->nred;
    hipError_t e = launch_domain_sums(c->cfg.d, work_m(c, 0), c->cells, c->cells, (double)(kDTotal + c->cfg.K),
                                      part, c->nred, res, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, res, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(m, e, "domain_sums");
    return IMEXLB_OK;
}

imexlb_status imexlb_density_loss(const imexlb_ctx* c, const double* n, const double* target, double* loss,
                                  double* grad) {
    if (!c) return IMEXLB_EINVAL;
    imexlb_ctx* m = const_cast<imexlb_ctx*>(c);
    if (!target || !loss) return fail(m, IMEXLB_EINVAL, "density_loss: NULL target or loss");
    if (!n) {
        if (need_state(c) != IMEXLB_OK) return fail(m, IMEXLB_ESTATE, "density_loss: no state");
        n = work_m(c, 0);  // field 0 of the state's moments
    }
    hipError_t e = launch_density_loss(n, target, c->cells, grad, c->d_small, c->nred, loss, c->stream);
    if (e != hipSuccess) return hip_fail(m, e, "density_loss");
    return IMEXLB_OK;
}

imexlb_status imexlb_check_state(const imexlb_ctx* c) {
    if (!c) return IMEXLB_EINVAL;
    imexlb_ctx* m = const_cast<imexlb_ctx*>(c);
    if (need_state(c) != IMEXLB_OK) return fail(m, IMEXLB_ESTATE, "check_state: no state");
    int h = 0;
    hipError_t e = launch_check_reset(c->d_flag, c->stream);
    if (e == hipSuccess) e = launch_check(c->cfg.d, work_m(c, 0), c->cells, c->cells, 1, c->d_flag, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(m, e, "check_state");
    return h != INT_MAX ? fail(m, IMEXLB_ENONPHYS, "check_state: non-physical moments") : IMEXLB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Adjoint of one IMEX step (reverse sweep through the stages of Table I).
// ---------------------------------------------------------------------------
namespace {

// Adjoint workspace: F scratch | X1 | X2 | X3 | X4 (plane-sets of the
// storage type: the step's scratch copy of F^n, then the stage adjoints
// between the kernels of the reverse sweep) | dM (FP64 moment set) | the
// record of the recomputed step (imexlb_step_record_bytes).
struct AdjLayout {
    size_t ps, ms, rec;  // bytes: storage plane-set, FP64 moment set, record
    size_t total() const { return 5 * ps + ms + rec; }
};

AdjLayout adj_layout(const imexlb_ctx* c) {
    AdjLayout L;
    L.ps = align256((size_t)c->nplanes * c->cells * c->elem);
    L.ms = align256((size_t)c->nf * c->cells * sizeof(double));
    L.rec = record_bytes(c);
    return L;
}

void* adj_s(const imexlb_ctx* c) { return c->d_adj; }
void* adj_x(const imexlb_ctx* c, int i) { return (char*)c->d_adj + (size_t)(1 + i) * adj_layout(c).ps; }
double* adj_dm(const imexlb_ctx* c) { return (double*)((char*)c->d_adj + 5 * adj_layout(c).ps); }
void* adj_rec(const imexlb_ctx* c) {
    const AdjLayout L = adj_layout(c);
    return (char*)c->d_adj + 5 * L.ps + L.ms;
}

}  // namespace

extern "C" {

size_t imexlb_adjoint_workspace_bytes(const imexlb_ctx* c) { return c ? adj_layout(c).total() : 0; }

imexlb_status imexlb_adjoint_bind(imexlb_ctx* c, void* d_adj) {
    if (!c) return IMEXLB_EINVAL;
    if (!d_adj) return fail(c, IMEXLB_EINVAL, "adjoint_bind: NULL buffer");
    if ((uintptr_t)d_adj & 255) return fail(c, IMEXLB_EINVAL, "adjoint_bind: buffer must be 256-byte aligned");
    c->d_adj = d_adj;
    return IMEXLB_OK;
}

}  // extern "C"

namespace {

// The reverse sweep of one step taken from Fn, given the step's record: the
// stage sources G3, G4, the moments M^n, M3, M4 and (2D) the stage values
// F2, F3, F4 the forward swept; without those (1D) the stage values are
// formed again from the sources and moments.
imexlb_status adjoint_core(imexlb_ctx* c, const void* Fn, const StepRecord& r, const double* lam1, double* lam0) {
    const void *G3 = r.G3, *G4 = r.G4;
    const double *Mn = r.Mn, *M3 = r.M3, *M4 = r.M4;
    const int d = c->cfg.d;
    const bool f32 = c->cfg.storage == IMEXLB_F32;
    const long long cells = c->cells;
    const double chi = (double)(c->cfg.K + kDTotal - d), dk = (double)(kDTotal + c->cfg.K);
    hipStream_t s = c->stream;
    double* dM = adj_dm(c);
    void *X1 = adj_x(c, 0), *X2 = adj_x(c, 1), *X3 = adj_x(c, 2), *X4 = adj_x(c, 3);
    const StageArgs a = base_args(c);
    hipError_t e = hipSuccess;
    // coefficients (w = dt/tau, cc = alpha w)
    const double dt = a.dt, w = a.omega, cc = kAlpha * w, a1 = a.a1, a2 = a.a2;
    const double b2 = cc * cc / ((1.0 + cc) * (1.0 + cc));
    constexpr double be = 0.06042356519705, et = 0.12915286960590;  // Table I
    const double ka = 0.5 - be - et - kAlpha;
    const int np = c->nplanes, nx = c->cfg.nx, ny = d == 2 ? c->cfg.ny : 1;
    const double idx = a.inv_dx, idy = a.inv_dy;
    const int qm = a.qm;
    // V^T with the linear combinations its two consumers read: the adjoint
    // of the fluxes dA = sum_j cs_j z_j, then y1 = e0 V + sum_j es_j z_j (the
    // equilibrium adjoint's input) and y2 = f0 V + sum_j fs_j z_j (the moment
    // adjoint's), V = V^T dA.  zs[0] is lam^{n+1} (FP64); the other stage
    // adjoints, y1 and y2 are in the storage type, except a y2 that is lam^n
    // itself (y2_f64).
    auto adv = [&](const void* F, std::initializer_list<const void*> zs, std::initializer_list<double> cs,
                   double e0, std::initializer_list<double> es, double f0, std::initializer_list<double> fs,
                   void* y1, void* y2, bool y2_f64) {
        AdvAdjIO io{};
        io.n = (int)zs.size();
        io.y2_f64 = y2_f64 ? 1 : 0;
        for (int j = 0; j < io.n; ++j) {
            io.z[j] = zs.begin()[j];
            io.c[j] = cs.begin()[j];
            io.e[j] = es.begin()[j];
            io.f[j] = fs.begin()[j];
        }
        io.e0 = e0;
        io.f0 = f0;
        io.y1 = y1;
        io.y2 = y2;
        return launch_advect_adjoint(d, f32, c->d_tab, np, F, io, nx, ny, c->cfg.bc_x, c->cfg.bc_y, idx, idy, s);
    };
    auto eqt = [&](const double* M, const void* y) {
        return launch_eq_adjoint(d, qm, f32, c->d_tab, M, y, dM, cells, chi, s);
    };
    // y and out in the storage type, or both FP64 (f64)
    auto momt = [&](const double* M, const void* y, void* out, bool f64) {
        return launch_mom_adjoint(d, f32 && !f64, c->d_tab, M, dM, y, out, cells, dk, s);
    };
    const double* L = lam1;
    // stage 4: F4 = a1 S4 + c a1 E4, dA4 = -(2/3) dt L, d(dF4) = -(2/3) L;
    // dE4 = c a1 V4 + (2/3) w a1 L, dS4 (before the moment term) = a1 V4 - (2/3) w a1 L
    const void* F4 = r.F4 ? r.F4 : X1;
    if (e == hipSuccess && !r.F4) e = launch_materialise(d, qm, f32, c->d_tab, G4, M4, a1, cc * a1, X1, cells, chi, s);
    if (e == hipSuccess)
        e = adv(F4, {L}, {-(2.0 / 3.0) * dt}, cc * a1, {(2.0 / 3.0) * w * a1}, a1, {-(2.0 / 3.0) * w * a1}, X2, X4,
                false);
    if (e == hipSuccess) e = eqt(M4, X2);
    if (e == hipSuccess) e = momt(M4, X4, X3, false);  // X3 = dS4
    // stage 3: dA3 = -(1/6) dt L - dt/4 dS4, d(dF3) = -(1/6) L - kappa dS4
    const void* F3 = r.F3 ? r.F3 : X1;
    if (e == hipSuccess && !r.F3) e = launch_materialise(d, qm, f32, c->d_tab, G3, M3, a1, cc * a1, X1, cells, chi, s);
    if (e == hipSuccess)
        e = adv(F3, {L, X3}, {-dt / 6.0, -0.25 * dt}, cc * a1, {w * a1 / 6.0, ka * w * a1}, a1,
                {-w * a1 / 6.0, -ka * w * a1}, X2, X4, false);
    if (e == hipSuccess) e = eqt(M3, X2);
    if (e == hipSuccess) e = momt(M3, X4, X1, false);  // X1 = dS3
    // stages 2 and 1: F2 = a2 F^n + b2 E^n, dA2 = -(1/6) dt L - dt/4 dS4 - dt dS3,
    // d(dF1) = -beta dS4, d(dF2) = -(1/6) L - eta dS4 - (1 - alpha) dS3; the
    // moment adjoint's input goes straight to lam0 and is completed in place
    const void* F2 = r.F2 ? r.F2 : X2;
    if (e == hipSuccess && !r.F2) e = launch_materialise(d, qm, f32, c->d_tab, Fn, Mn, a2, b2, X2, cells, chi, s);
    if (e == hipSuccess)
        e = adv(F2, {L, X3, X1}, {-dt / 6.0, -0.25 * dt, -dt}, b2,
                {w * a2 / 6.0, w * a1 * be + w * a2 * et, w * a2 * (1.0 - kAlpha)}, a2,
                {1.0 - w * a2 / 6.0, 1.0 - w * a1 * be - w * a2 * et, 1.0 - w * a2 * (1.0 - kAlpha)}, X4, lam0,
                true);
    if (e == hipSuccess) e = eqt(Mn, X4);
    if (e == hipSuccess) e = momt(Mn, lam0, lam0, true);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_step");
    return IMEXLB_OK;
}

}  // namespace

extern "C" {


imexlb_status imexlb_adjoint_step(imexlb_ctx* c, const void* Fn, const double* lam1, double* lam0) {
    if (!c) return IMEXLB_EINVAL;
    if (!c->d_adj) return fail(c, IMEXLB_ESTATE, "adjoint_step: no adjoint workspace bound");
    if (!Fn || !lam1 || !lam0) return fail(c, IMEXLB_EINVAL, "adjoint_step: NULL buffer");
    if ((const void*)lam1 == (const void*)lam0) return fail(c, IMEXLB_EINVAL, "adjoint_step: lam1 and lam0 alias");
    const int d = c->cfg.d;
    const bool f32 = c->cfg.storage == IMEXLB_F32;
    const long long cells = c->cells;
    const double dk = (double)(kDTotal + c->cfg.K);
    hipStream_t s = c->stream;
    // forward recompute of the step's record, on a scratch copy of F^n: the
    // stage sources G3 = S_3, G4 = S_4, the moments and (2D) the stage
    // values; pass 5 runs only for the stage values F4 its relax forms
    void* Fs = adj_s(c);
    const StepRecord r = record_of(c, adj_rec(c));
    StageArgs pa[3];
    pass_args(base_args(c), Fs, r.G3, r.G4, r.Mn, r.M3, r.M4, pa);
    pa[0].sval_out = r.F2;
    pa[1].sval_out = r.F3;
    pa[2].sval_out = r.F4;
    pa[2].mout = adj_dm(c);  // the moments of F^{n+1} are not needed
    hipError_t e = hipMemcpyAsync(Fs, Fn, imexlb_state_bytes(c), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_moments(d, f32, c->d_tab, Fn, r.Mn, cells, cells, dk, s);
    if (e == hipSuccess) e = launch_stage(d, f32, kStage3, pa[0], s);
    if (e == hipSuccess) e = launch_stage(d, f32, kStage4, pa[1], s);
    if (e == hipSuccess && r.F4) e = launch_stage(d, f32, kStage5, pa[2], s);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_step");
    return adjoint_core(c, Fn, r, lam1, lam0);
}

imexlb_status imexlb_adjoint_step_recorded(imexlb_ctx* c, const void* Fn, const void* d_record,
                                           const double* lam1, double* lam0) {
    if (!c) return IMEXLB_EINVAL;
    if (!c->d_adj) return fail(c, IMEXLB_ESTATE, "adjoint_step_recorded: no adjoint workspace bound");
    if (!Fn || !d_record || !lam1 || !lam0) return fail(c, IMEXLB_EINVAL, "adjoint_step_recorded: NULL buffer");
    if ((uintptr_t)d_record & 255)
        return fail(c, IMEXLB_EINVAL, "adjoint_step_recorded: record must be 256-byte aligned");
    if ((const void*)lam1 == (const void*)lam0)
        return fail(c, IMEXLB_EINVAL, "adjoint_step_recorded: lam1 and lam0 alias");
    return adjoint_core(c, Fn, record_of(c, d_record), lam1, lam0);
}

imexlb_status imexlb_advect_adjoint(const imexlb_ctx* c, const double* F, const double* dA, double* dF) {
    if (!c) return IMEXLB_EINVAL;
    imexlb_ctx* m = const_cast<imexlb_ctx*>(c);
    if (!F || !dA || !dF) return fail(m, IMEXLB_EINVAL, "advect_adjoint: NULL buffer");
    const StageArgs a = base_args(c);
    if (dF == F || dF == dA) return fail(m, IMEXLB_EINVAL, "advect_adjoint: dF aliases F or dA");
    AdvAdjIO io{};
    io.n = 1;
    io.z[0] = dA;
    io.c[0] = 1.0;
    io.e0 = 1.0;
    io.y1 = dF;
    hipError_t e = launch_advect_adjoint(c->cfg.d, false, c->d_tab, c->nplanes, F, io, c->cfg.nx,
                                         c->cfg.d == 2 ? c->cfg.ny : 1, c->cfg.bc_x, c->cfg.bc_y, a.inv_dx,
                                         a.inv_dy, c->stream);
    if (e != hipSuccess) return hip_fail(m, e, "advect_adjoint");
    return IMEXLB_OK;
}

imexlb_status imexlb_moments_adjoint(imexlb_ctx* c, const void* F, const double* dn, const double* dux,
                                     const double* duy, const double* dT, double* lam) {
    if (!c) return IMEXLB_EINVAL;
    if (!c->d_adj) return fail(c, IMEXLB_ESTATE, "moments_adjoint: no adjoint workspace bound");
    const int d = c->cfg.d;
    if (!F || !dn || !dux || !dT || (d == 2 && !duy) || !lam)
        return fail(c, IMEXLB_EINVAL, "moments_adjoint: NULL buffer");
    const long long cells = c->cells;
    const size_t fb = (size_t)cells * sizeof(double);
    double *M = record_of(c, adj_rec(c)).Mn, *dM = adj_dm(c);  // scratch
    hipStream_t s = c->stream;
    hipError_t e = launch_moments(d, c->cfg.storage == IMEXLB_F32, c->d_tab, F, M, cells, cells,
                                  (double)(kDTotal + c->cfg.K), s);
    const double* src[4] = {dn, dux, d == 2 ? duy : dT, dT};
    for (int f = 0; f < c->nf && e == hipSuccess; ++f)
        e = hipMemcpyAsync(dM + (size_t)f * cells, src[f], fb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = launch_mom_adjoint(d, false, c->d_tab, M, dM, nullptr, lam, cells, (double)(kDTotal + c->cfg.K), s);
    if (e != hipSuccess) return hip_fail(c, e, "moments_adjoint");
    return IMEXLB_OK;
}

imexlb_status imexlb_equilibrium_adjoint(imexlb_ctx* c, const double* n, const double* ux, const double* uy,
                                         const double* T, const double* lam, double* dn, double* dux,
                                         double* duy, double* dT) {
    if (!c) return IMEXLB_EINVAL;
    if (!c->d_adj) return fail(c, IMEXLB_ESTATE, "equilibrium_adjoint: no adjoint workspace bound");
    const int d = c->cfg.d;
    if (!n || !ux || !T || !lam || !dn || !dux || !dT || (d == 2 && (!uy || !duy)))
        return fail(c, IMEXLB_EINVAL, "equilibrium_adjoint: NULL buffer");
    const long long cells = c->cells;
    const size_t fb = (size_t)cells * sizeof(double);
    double *M = record_of(c, adj_rec(c)).Mn, *dM = adj_dm(c);  // scratch
    hipStream_t s = c->stream;
    const double* src[4] = {n, ux, d == 2 ? uy : T, T};
    hipError_t e = hipSuccess;
    for (int f = 0; f < c->nf && e == hipSuccess; ++f)
        e = hipMemcpyAsync(M + (size_t)f * cells, src[f], fb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = launch_eq_adjoint(d, base_args(c).qm, false, c->d_tab, M, lam, dM, cells,
                              (double)(c->cfg.K + kDTotal - d), s);
    double* dst[4] = {dn, dux, d == 2 ? duy : dT, dT};
    for (int f = 0; f < c->nf && e == hipSuccess; ++f)
        e = hipMemcpyAsync(dst[f], dM + (size_t)f * cells, fb, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(c, e, "equilibrium_adjoint");
    return IMEXLB_OK;
}

}  // extern "C"
