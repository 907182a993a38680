/*
 * imexlb.h -- C ABI of the MI355X (gfx950) IMEX finite-difference lattice
 * Boltzmann library (method of Kis & Ambrus, arXiv:1909.08390).
 *
 * The library advances the two reduced distributions phi and chi of the
 * BGK-Boltzmann equation (Sec. II) on a 1D or 2D grid with the
 * IMEX-SSP3(4,3,3) Runge-Kutta scheme of Sec. III (Table I): advection is
 * explicit, by 9th-order monotonicity-preserving (MP-9) fluxes (Sec. IV);
 * the BGK collision is implicit and solved in closed form from the stage
 * moments.
 *
 * Memory model.  All large buffers are device memory owned by the caller
 * (e.g. torch tensors): the state and a workspace, sized by
 * imexlb_state_bytes() / imexlb_workspace_bytes() and handed over with
 * imexlb_bind().  The context owns only small constant tables.  Every call
 * is issued on the context's HIP stream; calls taking device pointers are
 * asynchronous, calls taking host pointers synchronise that stream.
 *
 * State layout (the "plane-set").  F[v][y][x], x fastest, dense, element
 * type double (IMEXLB_F64) or float (IMEXLB_F32).  Plane v runs over the
 * discrete velocities: phi planes first, v = kx + Qphi*ky (ky = 0 when
 * d = 1), then chi planes, v = Qphi^d + qx + Qchi*qy; node indices follow the
 * ascending Gauss-Hermite nodes.  Cell centres sit at (i + 1/2) l/n.
 * Macroscopic fields (n, ux, uy, T) are FP64 arrays [y][x] of nx*ny values.
 *
 * Errors.  Every call returns a status; nothing is thrown across the ABI.
 * imexlb_last_error() gives a text for the last failing call of a context.
 */
#ifndef IMEXLB_H
#define IMEXLB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IMEXLB_OK = 0,
    IMEXLB_EINVAL = -1,   /* invalid argument or configuration            */
    IMEXLB_ENOMEM = -2,   /* host or small device allocation failed        */
    IMEXLB_EHIP = -3,     /* HIP runtime error (launch, copy, device)      */
    IMEXLB_ENONPHYS = -4, /* state check found n <= 0, T <= 0 or non-finite */
    IMEXLB_ESTATE = -5    /* call out of order (not bound / no state set)  */
} imexlb_status;

typedef enum { IMEXLB_OUTFLOW = 0, IMEXLB_PERIODIC = 1 } imexlb_bc;
typedef enum { IMEXLB_F64 = 0, IMEXLB_F32 = 1 } imexlb_storage;

/* Problem definition.  Sec. II fixes D = 3 momentum dimensions, of which the
 * first d are non-homogeneous; K internal degrees of freedom give the
 * adiabatic index gamma = (D + K + 2)/(D + K).  Units: m = k_B = 1, lengths
 * in units of the domain size (Sec. II, non-dimensionalisation). */
typedef struct {
    int d;              /* 1 or 2                                              */
    int nx, ny;         /* cells per axis; ny must be 1 when d = 1; one plane
                           ((ny + 16) nx elements) must stay below 2 GiB       */
    double lx, ly;      /* domain lengths (> 0); ly ignored when d = 1         */
    int q_phi, q_chi;   /* Gauss-Hermite order per axis: 3 <= q_phi <= 16,
                           1 <= q_chi <= 16 (energy is exact only from q_phi = 3,
                           Sec. II exactness up to order Q - 1)                */
    int K;              /* internal degrees of freedom, >= 0                   */
    double tau;         /* BGK relaxation time, > 0                            */
    double dt;          /* time step, > 0, with max|p| dt / (l/n) <= 1 per axis
                           (the CFL condition of Sec. IV)                      */
    int bc_x, bc_y;     /* imexlb_bc per axis: outflow (ghost nodes copy the
                           boundary node, Sec. IV) or periodic                 */
    int storage;        /* imexlb_storage of the plane-sets                    */
    int check_physical; /* nonzero: imexlb_step checks the moments after every
                           step and returns IMEXLB_ENONPHYS when some cell has
                           n <= 0, T <= 0 or a non-finite moment (the step
                           call then synchronises the stream)                  */
} imexlb_config;

typedef struct imexlb_ctx imexlb_ctx;

/* Validate cfg, build the Gauss-Hermite quadrature and the equilibrium
 * tables (Sec. II) and upload them.  hip_stream is a hipStream_t (NULL for
 * the default stream).  On success *out owns the context. */
imexlb_status imexlb_create(const imexlb_config* cfg, void* hip_stream, imexlb_ctx** out);
void imexlb_destroy(imexlb_ctx* ctx);

/* Change the stream later calls are issued on. */
imexlb_status imexlb_set_stream(imexlb_ctx* ctx, void* hip_stream);

/* Bytes of one plane-set (planes * cells * element size). */
size_t imexlb_state_bytes(const imexlb_ctx* ctx);
/* Bytes of the workspace: two stage plane-sets and three FP64 moment sets. */
size_t imexlb_workspace_bytes(const imexlb_ctx* ctx);
/* Number of planes Qphi^d + Qchi^d. */
int imexlb_num_planes(const imexlb_ctx* ctx);

/* Hand over caller-owned device memory: d_state (imexlb_state_bytes) and
 * d_workspace (imexlb_workspace_bytes), both 256-byte aligned.  The library
 * never frees them.  Rebinding invalidates the stored state. */
imexlb_status imexlb_bind(imexlb_ctx* ctx, void* d_state, void* d_workspace);

/* Host copies of the per-axis nodes and weights (q_phi resp. q_chi values):
 * nodes are the roots of He_Q, weights Q!/He_{Q+1}(p)^2 (Sec. II). */
imexlb_status imexlb_quadrature(const imexlb_ctx* ctx, double* p_phi, double* w_phi,
                                double* p_chi, double* w_chi);

/* Set the state to the discrete equilibrium of the device fields
 * (n, ux, uy, T) (Sec. II, Eq. gExpanded and chi_eq = (K + D - d) T phi_eq).
 * d_uy is ignored when d = 1. */
imexlb_status imexlb_set_equilibrium(imexlb_ctx* ctx, const double* d_n, const double* d_ux,
                                     const double* d_uy, const double* d_T);

/* Copy a raw plane-set (device, state layout) into the bound state and
 * recompute its moments. */
imexlb_status imexlb_set_state(imexlb_ctx* ctx, const void* d_F);
/* Copy the bound state into d_F (device, state layout). */
imexlb_status imexlb_get_state(const imexlb_ctx* ctx, void* d_F);

/* Advance the bound state by nsteps IMEX-SSP3(4,3,3) steps (Sec. III):
 * three fused stage passes per step, asynchronous on the stream.  With
 * cfg.check_physical set, the moments are checked on the device after every
 * step and the call synchronises at the end: IMEXLB_ENONPHYS (the message
 * names the first step that produced a non-physical cell) or IMEXLB_OK.  The
 * steps are taken in either case. */
imexlb_status imexlb_step(imexlb_ctx* ctx, int nsteps);

/* imexlb_step with per-pass timing: adds to ms[0], ms[1], ms[2] the summed
 * durations (milliseconds, HIP events recorded on the context's stream
 * between the launches) of the stage-3, stage-4 and stage-5 passes of all
 * nsteps steps.  Same results and status as imexlb_step (with
 * cfg.check_physical set, each step's check kernel falls in its stage-5
 * interval); synchronises the stream at the end.  For measurement. */
imexlb_status imexlb_step_timed(imexlb_ctx* ctx, int nsteps, double ms[3]);

/* Device fields (n, ux, uy, T) of the current state (Sec. II, discrete
 * moments); d_uy is neither read nor written when d = 1 (may be NULL). */
imexlb_status imexlb_moments(const imexlb_ctx* ctx, double* d_n, double* d_ux,
                             double* d_uy, double* d_T);

/* Device FP64 fields of an arbitrary plane-set d_F (state layout, storage
 * type of the context): the moments reduction on its own. */
imexlb_status imexlb_compute_moments(const imexlb_ctx* ctx, const void* d_F, double* d_n,
                                     double* d_ux, double* d_uy, double* d_T);

/* Device FP64 plane-set d_VF = (p . grad) F of the plane-set d_F by MP-9
 * fluxes with ghost nodes (Sec. IV), the advection operator on its own. */
imexlb_status imexlb_advect(const imexlb_ctx* ctx, const void* d_F, double* d_VF);

/* Host sums over all cells of the current state: out[0] = mass, out[1..2] =
 * momentum (x, y; y is 0 when d = 1), out[3] = total energy
 * (D+K)/2 n T + n |u|^2 / 2 (Sec. II, Eq. Moments), sums of cell values
 * (multiply by the cell volume for integrals).  On periodic grids the step
 * conserves all four (the MP-9 fluxes telescope, Sec. IV; the BGK terms
 * carry no moments, Sec. III).  Deterministic: wavefront shuffle sums in a
 * fixed order.  Synchronises the stream. */
imexlb_status imexlb_domain_sums(const imexlb_ctx* ctx, double out[4]);

/* Density loss L = 1/2 sum over cells of (n - n*)^2 and its gradient
 * dL/dn = n - n*, for the adjoint workloads.  d_n: device FP64 density field
 * (nx*ny values), or NULL for the density of the current state; d_target:
 * device FP64 field n*; d_loss: device, one double (written); d_grad: device
 * field (written) or NULL.  Deterministic, as imexlb_domain_sums.
 * Asynchronous.  Errors: EINVAL for NULL d_target or d_loss, ESTATE for
 * d_n = NULL without a state. */
imexlb_status imexlb_density_loss(const imexlb_ctx* ctx, const double* d_n, const double* d_target,
                                  double* d_loss, double* d_grad);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sums
 * of imexlb_domain_sums, same kernels and bitwise the same results, of
 * caller-given moment fields, with no context, no allocation and no memset.
 * d_M: device FP64 fields (n, ux, [uy], T) of `cells` values each, field
 * after field (d + 2 fields); d_out: device, 4 doubles (written): mass,
 * momentum x, y (0 when d = 1), energy with D + K = 3 + K.  Asynchronous on
 * hip_stream (NULL: the null stream).  The per-work-group partials live in
 * a 32 KiB static device array that each GPU holds for the life of the
 * process; calls that overlap in time on one GPU (other streams, other
 * threads) share it and race, so issue them in one stream order.
 * Errors (checked before any device work): IMEXLB_EINVAL for d not 1 or 2,
 * K < 0, NULL buffers, or cells outside [1, 2^31 - 1]; IMEXLB_EHIP for a HIP
 * failure.  Messages go to stderr. */
imexlb_status imexlb_domain_sums_noalloc(int d, int K, const double* d_M, long long cells,
                                         double* d_out, void* hip_stream);

/* Scan the current moments for n <= 0, T <= 0 or non-finite values:
 * IMEXLB_OK or IMEXLB_ENONPHYS.  Synchronises the stream. */
imexlb_status imexlb_check_state(const imexlb_ctx* ctx);

/* ------------------------------------------------------------------------
 * Adjoint (reverse mode) of the step, for gradients of a loss of the
 * final state with respect to an earlier state or to initial fields.
 *
 * Adjoint variables are FP64 plane-sets lam[v][y][x] (the derivative of the
 * loss with respect to each population), whatever the storage type; the
 * stage adjoints inside a step are held in the storage type (arithmetic
 * FP64 throughout).  The
 * adjoint step recomputes the stage sources of the step from its input
 * state (Sec. III, Table I) in a caller-owned adjoint workspace and then
 * runs the stages backwards: MP-9 advection transposed (a face that the
 * monotonicity test clips takes the derivative of the clip branch, Sec. IV),
 * equilibrium and moment Jacobians transposed (Sec. II), and the relaxation
 * weights.  It is exact (up to rounding) wherever the limiter decisions are
 * locally constant; at a decision boundary it returns one one-sided
 * derivative.
 * ------------------------------------------------------------------------ */

/* Size of, and binding of, the adjoint workspace (256-byte aligned device
 * buffer): five plane-sets of the storage type, one FP64 moment set and
 * the record of one step (imexlb_step_record_bytes), in which the adjoint
 * step recomputes the step it reverses. */
size_t imexlb_adjoint_workspace_bytes(const imexlb_ctx* ctx);
imexlb_status imexlb_adjoint_bind(imexlb_ctx* ctx, void* d_adj_workspace);

/* lam_n = (dF^{n+1}/dF^n)^T lam_np1 for one step taken from the state d_Fn
 * (storage type, ABI layout; not modified).  lam_np1 and lam_n are distinct
 * FP64 plane-sets.  Asynchronous.  Errors: ESTATE without an adjoint
 * workspace, EINVAL for NULL or aliased buffers. */
imexlb_status imexlb_adjoint_step(imexlb_ctx* ctx, const void* d_Fn, const double* d_lam_np1,
                                  double* d_lam_n);

/* Recorded steps, for reverse sweeps that walk a segment of steps again:
 * the stage sources G3, G4 of Table I's third and fourth stages (storage
 * type, ABI layout) and the moments M^n, M3, M4 of one step (FP64, fields
 * (n, u_x, [u_y], T)), laid out G3 | G4 | M^n | M3 | M4, each part 256-byte
 * aligned; in 2D followed by F2 | F3 | F4, the stage values (Table I) at
 * every cell as the three stage passes formed them on read and advected
 * them (storage type), so that the adjoint linearises the advection at the
 * very values the forward swept.  imexlb_step_record_bytes: size of one
 * record. */
size_t imexlb_step_record_bytes(const imexlb_ctx* ctx);

/* One IMEX step, as imexlb_step(ctx, 1), that also leaves the step's stage
 * sources, moments and (2D) stage values in d_record (device, 256-byte aligned,
 * imexlb_step_record_bytes; caller-owned).  Asynchronous unless
 * check_physical is set.  Errors: as imexlb_step; EINVAL for a NULL or
 * misaligned record. */
imexlb_status imexlb_step_recorded(imexlb_ctx* ctx, void* d_record);

/* imexlb_step_recorded out of place (Sec. III, Table I): the step reads the
 * bound state F^n without modifying it, writes F^{n+1} (and, in between,
 * the stage-4 combination R) into d_next, and then binds d_next as the
 * state, so a reverse sweep keeps every state of a segment without copies.
 * d_next: caller-owned device buffer of imexlb_state_bytes, 256-byte
 * aligned, distinct from the bound state, the workspace and the record; the
 * buffer bound before the call stays the caller's and keeps F^n.
 * Asynchronous unless check_physical is set.  Errors: as
 * imexlb_step_recorded; EINVAL for a NULL or misaligned d_next or one that
 * overlaps the bound state, the workspace or the record (nothing is launched
 * and the binding is unchanged). */
imexlb_status imexlb_step_recorded_to(imexlb_ctx* ctx, void* d_record, void* d_next);

/* imexlb_adjoint_step for the step that imexlb_step_recorded (or
 * imexlb_step_recorded_to) took from d_Fn, reading the step's stage sources,
 * moments and, in 2D, stage values from its record instead of recomputing
 * the step.  Bit for bit the result of imexlb_adjoint_step when the
 * recorded step started from the moments imexlb_set_state takes of d_Fn;
 * after a step the moments come from that step's last pass and agree with
 * those to rounding.  Errors: as imexlb_adjoint_step; EINVAL for a NULL or
 * misaligned record. */
imexlb_status imexlb_adjoint_step_recorded(imexlb_ctx* ctx, const void* d_Fn, const void* d_record,
                                           const double* d_lam_np1, double* d_lam_n);

/* dF = V^T dA: the transpose of the MP-9 advection operator of
 * imexlb_advect at the FP64 plane-set d_F (Sec. IV), for an FP64 plane-set
 * dA; the linearisation follows the limiter decisions at d_F.  d_dF must not
 * alias d_F or d_dA (EINVAL). */
imexlb_status imexlb_advect_adjoint(const imexlb_ctx* ctx, const double* d_F, const double* d_dA,
                                    double* d_dF);

/* lam = (dM/dF)^T dM: the adjoint of the moments (n, u_x, u_y, T) of the
 * plane-set d_F (Sec. II, Eq. Moments_discrete) for given moment adjoints
 * (FP64 fields; d_duy ignored when d = 1). */
imexlb_status imexlb_moments_adjoint(imexlb_ctx* ctx, const void* d_F, const double* d_dn,
                                     const double* d_dux, const double* d_duy, const double* d_dT,
                                     double* d_lam);

/* Adjoint of imexlb_set_equilibrium: (dn, du_x, du_y, dT) = (dE/d(n,u,T))^T lam
 * for the equilibrium of the fields (n, u_x, u_y, T) (Sec. II, Eq. gExpanded). */
imexlb_status imexlb_equilibrium_adjoint(imexlb_ctx* ctx, const double* d_n, const double* d_ux,
                                         const double* d_uy, const double* d_T, const double* d_lam,
                                         double* d_dn, double* d_dux, double* d_duy, double* d_dT);

/* Static text for a status; the context's last error message. */
const char* imexlb_status_string(imexlb_status s);
const char* imexlb_last_error(const imexlb_ctx* ctx);

/* ------------------------------------------------------------------------
 * Batches of independent 1D problems (shock tubes) of uneven size.
 *
 * Every tube is a d = 1 problem of the model above with its own cell count,
 * length, K (so its own adiabatic index, Sec. II), tau, dt and boundary
 * rule; all tubes share one velocity quadrature and one storage type.  The
 * batch runs under one of imexlb_batch_plan_count() execution plans, chosen
 * by imexlb_batch_tune() or set directly:
 *  - per-pass launches (mode 0): one IMEX step is three launches, one per
 *    fused pass, each covering every tile of every tube;
 *  - persistent launches (mode 1): one launch covers up to `steps` whole
 *    steps.  Each work-group owns a bin of items, a tube or a chunk of an
 *    outflow tube longer than `chunk` cells, and separates the passes with
 *    work-group barriers only; a chunk is stepped over its cells extended
 *    by 15 cells per step on each side (three passes of the 5-cell MP-9
 *    reach, Sec. IV), at most `chunk` cells in all, so the results are
 *    those of the whole tube.
 * Every plan gives bitwise the same results.
 *
 * Layout.  Tube i's plane-set starts at element state_offset[i] of the
 * state buffer (multiples of 64 elements) and holds Q planes of nx_i cells,
 * F_i[v][x], Q = q_phi + q_chi, plane order as above.  Macroscopic fields
 * are FP64 arrays over all cells of all tubes: tube i's cells sit at
 * cell_offset[i] .. cell_offset[i] + nx_i - 1 of an array of
 * imexlb_batch_cells() values.
 * ------------------------------------------------------------------------ */
typedef struct {
    int nx;             /* cells (>= 1)                                        */
    int K;              /* internal degrees of freedom (>= 0)                  */
    double lx;          /* length (> 0)                                        */
    double tau, dt;     /* relaxation time and time step (> 0; CFL <= 1)       */
    int bc;             /* imexlb_bc at both ends                              */
} imexlb_tube;

typedef struct imexlb_batch imexlb_batch;

/* Validate the tubes (same rules as imexlb_create per tube), build the
 * shared quadrature tables and the tile table.  q_phi, q_chi and storage as
 * in imexlb_config.  On success *out owns the batch.  Errors: EINVAL
 * (count < 1, a bad tube, bad orders or storage), ENOMEM, EHIP. */
imexlb_status imexlb_batch_create(const imexlb_tube* tubes, int count, int q_phi, int q_chi,
                                  int storage, void* hip_stream, imexlb_batch** out);
void imexlb_batch_destroy(imexlb_batch* b);
imexlb_status imexlb_batch_set_stream(imexlb_batch* b, void* hip_stream);

/* Sizes in bytes of the state and workspace buffers (the workspace holds the
 * stage and moment buffers and the private areas of the persistent plans),
 * the total cell count and the per-tube offsets (host arrays of count
 * elements, either may be NULL). */
size_t imexlb_batch_state_bytes(const imexlb_batch* b);
size_t imexlb_batch_workspace_bytes(const imexlb_batch* b);
long long imexlb_batch_cells(const imexlb_batch* b);
imexlb_status imexlb_batch_layout(const imexlb_batch* b, long long* state_offset, long long* cell_offset);

/* Hand over caller-owned device buffers (256-byte aligned). */
imexlb_status imexlb_batch_bind(imexlb_batch* b, void* d_state, void* d_workspace);

/* Every tube at its local equilibrium of the given fields (device arrays of
 * imexlb_batch_cells() doubles): n, u, T. */
imexlb_status imexlb_batch_set_equilibrium(imexlb_batch* b, const double* d_n, const double* d_u,
                                           const double* d_T);
/* Recompute the moments after the caller wrote the state buffer directly. */
imexlb_status imexlb_batch_state_changed(imexlb_batch* b);

/* nsteps IMEX steps of every tube (each with its own dt).  Asynchronous.
 * The timed form synchronises and adds the milliseconds of passes 3, 4, 5
 * (HIP events around each batched launch) to ms[0..2]; under a persistent
 * plan the passes share launches, and the whole time goes to ms[0]. */
imexlb_status imexlb_batch_step(imexlb_batch* b, int nsteps);
imexlb_status imexlb_batch_step_timed(imexlb_batch* b, int nsteps, double ms[3]);

/* Moments (n, u, T) of the current state, device arrays of
 * imexlb_batch_cells() doubles. */
imexlb_status imexlb_batch_moments(const imexlb_batch* b, double* d_n, double* d_u, double* d_T);

/* Execution plans.  imexlb_batch_plan_info writes info[0..5] = mode (0
 * per-pass launches, 1 persistent), tile (cells per tile: 256, 512 or 1024;
 * work-groups of tile/4 threads), order (mode 0: 0 tube by tube, 1 longest
 * tubes first; mode 1: 1), chunk (mode 1: outflow tubes longer than this
 * are split into chunks whose extended regions hold at most this many
 * cells), steps (mode 1: steps per launch) and bins (mode 1: at most
 * this many work-groups, items assigned longest first to the least-loaded
 * one); EINVAL for a plan outside [0, imexlb_batch_plan_count()). */
int imexlb_batch_plan_count(void);
imexlb_status imexlb_batch_plan_info(int plan, int info[6]);
imexlb_status imexlb_batch_set_plan(imexlb_batch* b, int plan);
int imexlb_batch_get_plan(const imexlb_batch* b);

/* The per-pass plan with this tile width (cells per work-group: 256, 512 or
 * 1024) and tile order (0: tube by tube, 1: longest tubes first); the tile
 * width and order of the current plan. */
imexlb_status imexlb_batch_set_tiling(imexlb_batch* b, int tile, int order);
imexlb_status imexlb_batch_get_tiling(const imexlb_batch* b, int* tile, int* order);

/* Autotuner: time every plan over nsteps steps (after one untimed step) on
 * the current state and keep the fastest.  The state and its moments are
 * saved first and restored after each plan, so the call leaves them
 * unchanged; it allocates and frees a device copy of them.  ms_out
 * (optional, host, imexlb_batch_plan_count() values) receives the time per
 * step of each plan in plan order.  Requires a bound state.  Synchronises. */
imexlb_status imexlb_batch_tune(imexlb_batch* b, int nsteps, double* ms_out);

const char* imexlb_batch_last_error(const imexlb_batch* b);

/* ------------------------------------------------------------------------
 * Measurement helper (not a step of the method).
 *
 * Achievable HBM rate of a plain device copy: the practical ceiling that the
 * bandwidth of the stage passes is set against, next to the spec-sheet peak.
 * Copies `bytes` from d_src to d_dst (device memory owned by the caller,
 * 16-byte aligned, not overlapping; bytes a positive multiple of 16, at most
 * 2^40) once untimed and then `reps` times on hip_stream (NULL: the null
 * stream), one 16-byte load and store per thread, each copy timed with HIP
 * events, and writes the best rate in GB/s (bytes read plus bytes written,
 * per second) to *gbs (host).  d_dst ends up equal to d_src.  Synchronises.
 * IMEXLB_EINVAL for NULL or misaligned pointers, a bad size or reps < 1
 * (checked before any HIP call); IMEXLB_EHIP for a HIP failure. */
imexlb_status imexlb_copy_probe(const void* d_src, void* d_dst, size_t bytes, int reps,
                                void* hip_stream, double* gbs);

#ifdef __cplusplus
}
#endif
#endif
