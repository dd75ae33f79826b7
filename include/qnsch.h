/*
 * qnsch.h -- C ABI of the MI355X (gfx950) solver for one time step of the
 * primitive-variable scheme for the quasi-incompressible
 * Navier-Stokes-Cahn-Hilliard system.
 *
 * Reference: Guo, Lin, Lowengrub, Wise, "Mass conservative and energy stable
 * finite difference methods for the quasi-incompressible Navier-Stokes-Cahn-
 * Hilliard system: primitive variable and projection-type schemes".
 *
 * The discrete problem (sec. 6.1, eqs. (pm-num-mx), (pm-num-mass),
 * (pm-num-phase), (pm-num-chem) with the advection and surface-tension forms of
 * App. A.5-A.6 and the boundary conditions of App. A.4): given the state at
 * time n, find w = (c, mubar, pbar, u, v) at time n+1 with N(w) = 0.  It is
 * solved by the nonlinear FAS multigrid of sec. 7.1 (pointwise Newton update of
 * (c, mubar) and Vanka box update of (u, v, pbar), or the two in one coupled
 * box, red-black order, V-cycles).
 *
 * Precision.  QNSCH_FP64: every phase in FP64.  QNSCH_MIXED: defect
 * correction; the residual r = -N(w), the update w += delta, the stop test and
 * the mass and energy sums are FP64, and delta comes from one FP32 multigrid
 * V-cycle per outer iteration on the linearisation J(w) delta = r (same
 * smoother, colour order and transfers, applied to the correction).  Both
 * stop on the same FP64 residual norms, so both return a solution of the same
 * discrete system to the same tolerance.
 *
 * Grid and host array layout (all host arrays are double, m1*m2 entries,
 * row-major with x fastest, index j*m1 + i):
 *   cell (i,j): 0 <= i < m1, 0 <= j < m2, centre ((i+1/2)h, (j+1/2)h),
 *               h = Lx/m1 = Ly/m2 (square cells, sec. 5);
 *   c, mu (mubar), p (pbar): cell values;
 *   u[j*m1+i]: x-velocity on the west face of cell (i,j), at (i h, (j+1/2)h);
 *              with walls in x the entries i = 0 are the wall (zero) and the
 *              east wall face x = Lx is not stored; periodic in x: face i = 0
 *              is also the face x = Lx;
 *   v[j*m1+i]: y-velocity on the south face of cell (i,j), at ((i+1/2)h, j h),
 *              with the same convention in y.
 *
 * Ownership: the caller owns every host buffer; calls copy synchronously on the
 * context's stream.  The library owns all device memory of a context (taken
 * from hipMalloc, or from the caller's allocator: qnsch_set_allocator).  A
 * context must be used from one host thread at a time.
 *
 * Errors: functions return QNSCH_OK (0) or a negative code; qnsch_last_error()
 * gives a message.  A step that fails leaves the state at time n.
 */
#ifndef QNSCH_H
#define QNSCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    QNSCH_OK = 0,
    QNSCH_EINVAL = -1,    /* bad argument (dims, parameters, NULL) */
    QNSCH_ENOMEM = -2,    /* device allocation failed */
    QNSCH_ENOCONV = -3,   /* max_vcycles reached above tol */
    QNSCH_EDIVERGED = -4, /* non-finite residual, or c past the density pole */
    QNSCH_EDEVICE = -5,   /* HIP runtime error */
    QNSCH_EBUSY = -6      /* call not allowed in the current phase */
};

enum { QNSCH_BC_WALL = 0, QNSCH_BC_PERIODIC = 1 };
enum { QNSCH_FP64 = 0, QNSCH_MIXED = 1 };
/* Smoother of the V-cycle (sec. 7.1).  SEGREGATED: the two steps of sec. 7.1,
 * a pointwise Newton step on (c, mubar) of the cell, then the Vanka box of its
 * four faces and pbar.  COUPLED (default): one Newton step on the seven
 * unknowns of the cell (four faces, pbar, c, mubar) with the five cell and
 * face equations plus the phase and chemical-potential equations of the cell;
 * the faces and pbar take the vanka_omega-relaxed step, c and mubar the full
 * one.  Both have the same fixed point, the solution of sec. 6.1; the coupled
 * box keeps the V-cycle factor bounded under refinement at density ratios
 * where the segregated one degrades. */
enum { QNSCH_SMOOTH_SEGREGATED = 0, QNSCH_SMOOTH_COUPLED = 1 };
/* Scheme.  PRIMITIVE (default): the primitive-variable scheme of sec. 6.1.
 * PROJECTION: the projection scheme of sec. 6.2, eqs. (pj-num-mx)-(pj-num-chem):
 * an intermediate velocity u~ from the momentum equation without pressure,
 * surface tension and gravity, the velocity of time n+1 from the projection
 * equation (pj-num-pjx) (gravity acting there, as in the time-discrete scheme
 * (pj-pj)), and the mass, phase and chemical-potential equations with it
 * (rho^n in the time derivative of c and in rho^n mubar, the advection of c at
 * time n+1).  The velocity of time n+1 is eliminated, so the unknowns are c,
 * mubar, pbar and u~; the smoother is the one of sec. 7.2 (per cell a Newton
 * step on (c, mubar) with the velocity of time n+1 held, the Vanka box of the
 * four u~ faces, a Newton step in pbar on the mass equation), whatever
 * `smoother` says.  During a step the velocity arguments and results of the
 * phase calls are u~; after a completed step (qnsch_step, or qnsch_end_step
 * after phases) they are the velocity of time n+1.  FP64 only; the server
 * accepts primitive requests only. */
enum { QNSCH_PRIMITIVE = 0, QNSCH_PROJECTION = 1 };

typedef struct {
    int32_t m1, m2;     /* cells in x and y; both even, divisible by 2^levels */
    double Lx, Ly;      /* domain size; Lx/m1 must equal Ly/m2 */
    int32_t bc_x, bc_y; /* QNSCH_BC_WALL (no-slip u, Neumann c, mu, p) or PERIODIC */
    int32_t levels;     /* multigrid levels; 0 = coarsen while the coarsest level has > 32 cells */
} qnsch_grid;

/* Interface ratio parameter eta of sec. 8.1, which matches the phase-field
 * surface tension to the sharp-interface one for the density pair:
 *   eta = (rho2 - rho1)^3 / (2 sqrt2 rho1 rho2 (rho2^2 - rho1^2 - 2 rho1 rho2 ln(rho2/rho1))),
 * evaluated through a series in x = rho2/rho1 - 1 for |x| < 0.05 (the direct
 * form cancels there), with the equal-density limit 3/(2 sqrt2 rho1).
 * Host-only; returns NaN unless both densities are positive. */
double qnsch_default_eta(double rho1, double rho2);

/* Non-dimensional parameters of sec. 2.2; fluid 1 is c = 1 (rho(1) = rho1). */
typedef struct {
    double rho1, rho2;   /* densities, > 0 */
    double visc1, visc2; /* viscosities, > 0 */
    double Re, We;       /* Reynolds and Weber numbers, > 0 */
    double inv_Fr;       /* 1/Fr, gravity along -y; 0 = no gravity */
    double Pe, M;        /* Peclet number and the Mach-like number M, > 0 */
    double eps;          /* interface thickness parameter, > 0 */
    double eta;          /* interface ratio parameter; <= 0 takes qnsch_default_eta(rho1, rho2) */
    double mob_reg;      /* constant under the square root of the mobility (sec. 6.1), >= 0;
                            < 0 takes eps, the paper's choice */
    double rho_ref;      /* density the gravity force is measured against (0 with walls in y) */
} qnsch_params;

typedef struct {
    int32_t precision;   /* QNSCH_FP64 or QNSCH_MIXED (see above) */
    double tol;          /* stop when every per-equation norm sqrt(h^2 sum r^2) <= tol */
    int32_t max_vcycles; /* error QNSCH_ENOCONV beyond this */
    int32_t nu1, nu2;    /* pre/post smoothing sweeps (one sweep = red + black), 0..15 */
    int32_t nu_coarse;   /* sweeps on the coarsest level; 0 = automatic (4 for the
                            primitive scheme on 6 levels or more, else 6) */
    double vanka_omega;  /* relaxation factor of the box update (1 = exact box solve) */
    int32_t smoother;    /* QNSCH_SMOOTH_COUPLED or QNSCH_SMOOTH_SEGREGATED */
    int32_t scheme;      /* QNSCH_PRIMITIVE or QNSCH_PROJECTION */
    double coarse_omega; /* relaxation factor of the velocity and pressure updates on the
                            coarsest level (the primitive box's faces and pbar; the
                            projection scheme's pressure step); in (0, 2), or 0 =
                            automatic (1.75 where nu_coarse's automatic value is 4,
                            else 1.6) */
    int32_t accel;       /* depth m (0..3) of the acceleration of the cycle iteration
                            below; 0 = plain cycles */
    int32_t blocking;    /* temporal blocking of the smoothing (below): 0 = off,
                            1 = coarse levels, and the finest level where it has at
                            most one 16 x 16 tile per compute unit, 2 = the finest
                            level also with two */
} qnsch_opts;

/* Temporal blocking (a performance variant of the smoother of sec. 7.1; the
 * iterates are those of the plain half-sweeps up to rounding).  On the levels
 * that are smoothed by launches over many workgroups (not those resident in
 * one workgroup's LDS) and have at most two 16 x 16 tiles per compute unit
 * (one on the finest level unless blocking is 2), where a launch's fixed
 * cost is as large as its relaxation, a red and the following black
 * half-sweep run in one launch: each tile relaxes the red
 * cells of its tile widened by two cells on every side in LDS, then its own
 * black cells.  Sweeps go in pairs (an odd last sweep takes two half-sweep
 * launches).  Needs a second set of
 * c, mubar, pbar per level (24 bytes per cell of every level), in mixed
 * precision of the FP32 corrections dc, dmu, dp (12 bytes), whose smoother is
 * fused the same way, as is the projection scheme's smoother of sec. 7.2; a
 * level with a periodic axis shorter than 19 cells keeps the half-sweep
 * launches. */

/* Acceleration of the cycle iteration (not part of the paper, whose sec. 7.1
 * asks only for a standard FAS V-cycle; the discrete system, its root and the
 * stop test are unchanged).  The cycle results w_k (after the pbar mean
 * removal) and their residuals r_k = -N(w_k) are kept for the last m + 1
 * cycles of a step, from its second cycle on (the first result's residual
 * is dominated by the change of the time-n data).  Before the next cycle
 * the iterate becomes
 *   w = w_k + sum_i g_i (w_k - w_{k-i}),  i = 1..n,
 * with g minimising the linearised residual || r_k + sum_i g_i (r_k - r_{k-i}) ||
 * (plain sum of squares over the five fields; normal equations solved by
 * Cholesky), the nonlinear Krylov acceleration of multigrid of Washio and
 * Oosterlee (ETNA 6, 1997).  n = min(m, number of earlier results), cut to
 * the leading block whose Cholesky pivots exceed 1e-12 times the diagonal;
 * a result whose largest residual norm is not below that of the result
 * before it starts a new history (n = 0 next).  In mixed precision the next
 * correction cycle solves for the same combination of the residuals at the
 * combined iterate. */

/* Statistics of the last qnsch_step (a step run by phases fills vcycles
 * only).  Residual norms are the per-equation sqrt(h^2 sum r^2) of the stop
 * test, in the order (c, mu, p, u, v). */
#define QNSCH_HIST 128
typedef struct {
    int32_t vcycles;        /* V-cycles (mixed: outer iterations) of the last step */
    double res[5];          /* final per-equation residual norms (c, mu, p, u, v) */
    double res0[5];         /* residual norms before the first V-cycle */
    double step_ms;         /* wall time of the last step */
    int32_t hist_len;       /* entries of hist: min(vcycles + 1, QNSCH_HIST) */
    double hist[QNSCH_HIST][5]; /* hist[0] = res0, hist[k] = norms of the result of
                                   cycle k (before an acceleration combines it) */
    double dissipation[5];  /* dissipation of the last step, as qnsch_dissipation
                               returned it for that step; NaN until it was asked for */
} qnsch_step_stats;

typedef struct qnsch_ctx qnsch_ctx;

/* Defaults: FP64, tol 1e-10, 50 V-cycles, V(2,2), the coarsest solve's
 * automatic settings (nu_coarse = coarse_omega = 0: 4 sweeps over-relaxed by
 * 1.75 in the primitive scheme on hierarchies of 6 levels or more, else 6 by
 * 1.6; as many or fewer V-cycles than 30 plain sweeps on the workloads of
 * sec. 8), omega 1, coupled smoother, primitive scheme, acceleration depth
 * 2, temporal blocking (1: the coarse levels, and the finest level where it
 * has at most one 16 x 16 tile per compute unit). */
void qnsch_default_opts(qnsch_opts *opts);

/* Create a context on the current HIP device.  hip_stream: a hipStream_t to
 * run on, or NULL for the default stream.  opts NULL = defaults.  Allocates its
 * device memory in two blocks, the level descriptors and the fields of every
 * level, from hipMalloc or the allocator of qnsch_set_allocator (qnsch_footprint: roughly 150 bytes per
 * finest cell in FP64, 182 in mixed precision, plus 80 (accel + 1) for the
 * acceleration's history and 32 (16 in mixed precision) for the second cell
 * set of temporal blocking).  Returns
 * QNSCH_EINVAL for grids or parameters outside the ranges stated above, and
 * QNSCH_EDEVICE if the device check that the first creation on a device runs
 * fails (the kernels read their workgroup size from the dispatch's implicit
 * kernel arguments; a library built for another layout of them refuses to
 * run; the check's reason goes to stderr). */
int qnsch_create(const qnsch_grid *grid, const qnsch_params *params, const qnsch_opts *opts,
                 void *hip_stream, qnsch_ctx **out);
void qnsch_destroy(qnsch_ctx *ctx);
const char *qnsch_last_error(const qnsch_ctx *ctx);
int qnsch_levels(const qnsch_ctx *ctx);

/* State at time n (host arrays, layout above).  mu, p, u, v may be NULL (zero).
 * Wall faces are forced to zero.  Ends any step in progress. */
int qnsch_set_state(qnsch_ctx *ctx, const double *c, const double *mu, const double *p,
                    const double *u, const double *v);
/* During a step (after qnsch_begin_step): overwrite the current iterate with
 * host arrays, keeping the time-n data; for inspection of single phases. */
int qnsch_set_iterate(qnsch_ctx *ctx, const double *c, const double *mu, const double *p,
                      const double *u, const double *v);
/* Current iterate (after a successful step: the state at time n+1).  NULL
 * pointers are skipped. */
int qnsch_get_state(qnsch_ctx *ctx, double *c, double *mu, double *p, double *u, double *v);

/* One time step of size dt (sec. 6.1 solved by sec. 7.1): V-cycles until every
 * residual norm is <= tol.  On failure the state stays at time n. */
int qnsch_step(qnsch_ctx *ctx, double dt);

/* Phases of a step, for inspection: begin_step fixes the time-n data (the
 * current state) on every level; vcycle runs one V-cycle, fixes the mean of
 * pbar to zero and (accel > 0, from the second call of the step on) records
 * the result and its residual for the acceleration; accelerate replaces the
 * iterate by the combination of the recorded results (see above; no change
 * before two results are recorded or with accel = 0; a combination not
 * applied before the next vcycle is dropped); a step is vcycle, then
 * accelerate and vcycle until the tolerance is met.  residual returns r = -N(w) of the current iterate (5
 * fields of m1*m2, order c, mu, p, u, v; NULL to skip) and its norms;
 * halfsweep runs one colour half-sweep (colour 0: (i+j) even) on the finest
 * level; end_step commits the iterate as the new state (projection scheme:
 * replaces u~ by the velocity of time n+1). */
int qnsch_begin_step(qnsch_ctx *ctx, double dt);
int qnsch_vcycle(qnsch_ctx *ctx);
int qnsch_accelerate(qnsch_ctx *ctx);
int qnsch_residual(qnsch_ctx *ctx, double *r_out, double norms[5]);
int qnsch_halfsweep(qnsch_ctx *ctx, int colour);
int qnsch_end_step(qnsch_ctx *ctx);
/* Mixed-precision contexts, during a step: the FP32 linearisation used by the
 * correction cycle, applied to a host correction dw (5 fields of m1*m2 in the
 * order and layout of qnsch_residual): out = J(w) dw at the current iterate w
 * (its FP32 rounding), 5 fields, FP32 arithmetic returned as double.  Faces on
 * walls are not unknowns: their entries of dw are ignored and of out are 0.
 * QNSCH_EINVAL on an FP64 context; halfsweep is QNSCH_EINVAL on a mixed one. */
int qnsch_lin_apply(qnsch_ctx *ctx, const double *dw, double *out);

/* Mass of the two components of the current state (Theorem of sec. 6.1):
 * out = {h^2 sum rho(c) c, h^2 sum rho(c) (1-c)}.  FP64, deterministic. */
int qnsch_mass(qnsch_ctx *ctx, double out[2]);
/* Discrete energy of the current state (Theorem of sec. 6.1 with the norms of
 * App. A.7): out = {E, kinetic, gradient, bulk (double well), potential}. */
int qnsch_energy(qnsch_ctx *ctx, double out[5]);
/* Dissipation of the step just taken (Theorem of sec. 6.1, norms of App.
 * A.7), from the new state and the time-n data of that step:
 *   out[0] = dt/Re ||sqrt(mu) grad_d u||^2,  out[1] = dt/(3Re) ||sqrt(mu) div_d u||^2,
 *   out[2] = dt/(M Pe) ||sqrt(m) grad_D mu_c||^2 (mu_c = mubar + alpha pbar),
 *   out[3] = 1/2 ||sqrt(rho^n)(u^{n+1} - u^n)||^2,  out[4] = 0;
 * mu, m, rho at c^n; the vertex norm weights each vertex by a quarter of
 * each adjacent cell.  Projection scheme (Theorem of sec. 6.2): out[0], out[1]
 * and out[3] on the intermediate velocity u~ in place of u^{n+1}, and
 * out[4] = 1/2 ||sqrt(rho(c^{n+1}))(u^{n+1} - u~)||^2.  With walls in y the
 * energy law reads E^{n+1} - E^n + sum(out) = 0 at the converged solution.
 * QNSCH_EBUSY before the first step. */
int qnsch_dissipation(qnsch_ctx *ctx, double out[5]);
/* Physical diagnostics of the current state (sec. 8):
 *   out[0] = V_c = sum(c v) / sum(c), v at the cell the mean of its south and
 *            north faces (rising velocity of the c = 1 phase);
 *   out[1] = h^2 sum c;  out[2] = max |div_d u|;  out[3] = ||div_d u||_{2,h};
 *   out[4] / out[5] = highest / lowest height of a c = 1/2 crossing between
 *            vertically adjacent cells (linear interpolation; the tips of
 *            the rising and the falling fluid), NaN if none;
 *   out[6] = highest crossing in the first column x = h/2 (the interface
 *            height of a capillary wave at its crest), NaN if none;
 *   out[7] = h^2 sum div_d u (zero with walls or periodic boundaries). */
int qnsch_diagnostics(qnsch_ctx *ctx, double out[8]);
/* Device memory of contexts.  By default a context takes its device arrays
 * (one block for the level descriptors, one for every level's fields, and
 * the residual fields qnsch_residual returns, at its first call) from
 * hipMalloc and returns them with hipFree at qnsch_destroy.  For callers
 * whose framework owns device memory: after qnsch_set_allocator(alloc,
 * free_fn, user), contexts created from then on (server contexts included)
 * take every such block from alloc(bytes, user) and return it with
 * free_fn(ptr, bytes, user) when destroyed; a context keeps the functions it
 * was created with.  alloc must return memory of the current device that this
 * library's HIP runtime can address, aligned to 256 bytes, or NULL (the call
 * that needed it then fails with QNSCH_ENOMEM and frees what it took).
 * qnsch_set_allocator(NULL, NULL, NULL) restores hipMalloc / hipFree.  Pinned
 * host staging buffers always come from hipHostMalloc.  Process-wide and
 * thread-safe; QNSCH_EINVAL if exactly one of the functions is NULL. */
typedef void *(*qnsch_alloc_fn)(size_t bytes, void *user);
typedef void (*qnsch_free_fn)(void *ptr, size_t bytes, void *user);
int qnsch_set_allocator(qnsch_alloc_fn alloc, qnsch_free_fn free_fn, void *user);

/* Launches of a cycle (qnsch_step, qnsch_vcycle): with enable != 0 the
 * operations of a cycle before its residual reduction are captured once into
 * an executable HIP graph (per pattern of the levels' double-buffered faces,
 * on a stream of the context's own) and replayed on the context's stream, one
 * host call per cycle instead of one per kernel; the acceleration's
 * combination and the residual reduction, whose arguments change from cycle
 * to cycle, are launched directly.  The kernels, their arguments and their
 * order are those of the direct launches, so results are bitwise the same.
 * Cycles run with launches timed by qnsch_profile or qnsch_profile_ops are
 * launched directly.  Off (enable = 0) by default: the kernels of a cycle run
 * long enough that the device takes the next directly launched kernel
 * without a longer gap than from a graph (the step times of the benchmark
 * workloads agree within 1 %).  QNSCH_EINVAL on a NULL context; a failed
 * capture is reported by the step that needed it. */
int qnsch_graphs(qnsch_ctx *ctx, int enable);
/* Statistics of the last step (above); launches nothing. */
int qnsch_stats(qnsch_ctx *ctx, qnsch_step_stats *out);
/* Block until all work of the context's stream has finished. */
int qnsch_synchronize(qnsch_ctx *ctx);

/* Measurement support.  qnsch_profile(ctx, mode) resets the counters and
 * times launches with HIP events on the context's stream: mode 1 every launch
 * of the finest-level smoothing kernel (FP64 half-sweep, or FP32 in mixed
 * precision; the fused sweep kernel where blocking covers the finest level),
 * mode 2 every launch, 0 none.  qnsch_profile_ops(ctx, op_mask) resets them
 * and times every launch of the operations whose bit is set in op_mask (bit =
 * the library's operation number, as in the breakdown below), on every
 * level.  Launches timed by mode 1 or by op_mask carry the events themselves
 * (the kernel's own start and end; an operation that launches several
 * kernels, a residual or step-end reduction, is bracketed by event records
 * instead); mode 2 brackets every launch.  qnsch_profile_read returns
 * {finest smoothing launches timed, their total milliseconds}.
 * qnsch_profile_breakdown returns the number of timed classes and writes up
 * to cap of them: kinds[k] = 16 * operation + level, out[2k] = launches,
 * out[2k+1] = total milliseconds. */
int qnsch_profile(qnsch_ctx *ctx, int mode);
int qnsch_profile_ops(qnsch_ctx *ctx, uint64_t op_mask);
int qnsch_profile_read(qnsch_ctx *ctx, double out[2]);
int qnsch_profile_breakdown(qnsch_ctx *ctx, int32_t *kinds, double *out, int32_t cap);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call the allocator): the residual
 * norms of qnsch_residual for an iterate and time-n data held in the
 * caller's device memory, without a context.  c, mu, p, u, v (the iterate)
 * and cn, un, vn (the state at time n) are device arrays of m1*m2 doubles
 * in the host layout above (wall faces zero); norms (host) receives the five
 * per-equation norms sqrt(h^2 sum r^2) of r = -N(w) for the step dt.  The
 * reduction's partial sums and the level descriptor go to a static device
 * array of the library (about 2.6 MB on every device it runs on, held until
 * the process ends), so the call allocates nothing; grids of more than
 * 4194304 cells or more than 20480 tiles of 16 x 16 cells are rejected
 * (QNSCH_EINVAL).  Runs on hip_stream (NULL: the
 * default stream) and returns when the norms are on the host.  Calls that
 * overlap on one device race on that array.  QNSCH_EINVAL for NULL
 * arguments, dt <= 0 or a grid or parameters qnsch_create would reject;
 * QNSCH_EDEVICE on a HIP error; qnsch_residual_noalloc_error() gives the
 * message of the last failure. */
int qnsch_residual_noalloc(const qnsch_grid *grid, const qnsch_params *params, double dt, const double *c,
                           const double *mu, const double *p, const double *u, const double *v, const double *cn,
                           const double *un, const double *vn, void *hip_stream, double norms[5]);
const char *qnsch_residual_noalloc_error(void);

/* Copy-kernel probe on the current device: copies n doubles reps times
 * between two buffers it allocates and frees; out = {GB/s counting read and
 * write, milliseconds per copy}. */
int qnsch_copy_probe(size_t n, int reps, double out[2]);

/* ---------------------------------------------------------------------------
 * Serving: many independent simulations with continuous batching.
 *
 * A server owns a queue of requests (each a grid, parameters, options, an
 * initial concentration and a number of steps of size dt).  qnsch_server_
 * progress admits queued requests first come, first served while a slot is
 * free and their device footprint fits the HBM budget, keeps every admitted
 * hierarchy resident, and issues the next operation of every running request;
 * operations of the same kind (a colour half-sweep at whatever level, a
 * restriction, ...) are merged into one work-list launch.  A request's result
 * does not depend on which other requests share its launches.  The caller
 * submits requests whenever they arrive and calls progress in a loop.
 * Requests, results and histories are host memory owned by the server until
 * it is destroyed.
 */
typedef struct qnsch_server qnsch_server;

/* Device bytes a context of this grid allocates (0 if the grid is invalid);
 * the server admits requests by this footprint. */
size_t qnsch_footprint(const qnsch_grid *grid, const qnsch_opts *opts);

/* The serving calls differ from a minimal request loop in two deliberate
 * ways: qnsch_server_create takes the number of lanes (HIP streams the
 * requests are spread over, so that one lane's latency-bound phases overlap
 * another's), and qnsch_server_result returns the whole final state and the
 * per-step vcycles and timings besides the mass and energy histories, so
 * that a served result can be compared field by field with the same request
 * run alone.
 *
 * hbm_budget: device bytes the admitted requests may hold together (idle
 * contexts kept for reuse count too and are released first when a new shape
 * needs room); max_slots: most requests in flight; lanes: number of HIP
 * streams the requests are spread over (1..16; each admitted request joins the
 * least loaded lane and stays there; launches of different lanes overlap on
 * the device); hip_stream: used as the first lane if not NULL (the others are
 * created non-blocking). */
int qnsch_server_create(size_t hbm_budget, int32_t max_slots, int32_t lanes, void *hip_stream, qnsch_server **out);
void qnsch_server_destroy(qnsch_server *srv);
const char *qnsch_server_last_error(const qnsch_server *srv);
/* Queue a request; c0 (m1*m2, host) is copied.  QNSCH_ENOMEM if its footprint
 * exceeds the whole budget; QNSCH_EINVAL as for qnsch_create.  opts.blocking
 * is ignored (0): the server's merged launches already fill the device. */
int qnsch_server_submit(qnsch_server *srv, const qnsch_grid *grid, const qnsch_params *params,
                        const qnsch_opts *opts, const double *c0, int32_t nsteps, double dt, uint64_t *id);
/* Run up to max_ticks scheduler ticks; returns the number of unfinished
 * requests (queued + running) or a negative error. */
int qnsch_server_progress(qnsch_server *srv, int32_t max_ticks);
/* state: 0 queued, 1 running, 2 done; status: QNSCH_OK or the request's error. */
int qnsch_server_poll(qnsch_server *srv, uint64_t id, int32_t *state, int32_t *status);
/* Results of a finished request (NULL pointers are skipped): final state
 * (layout as qnsch_get_state), per step {mass 2, energy 5, wall ms, V-cycles},
 * times = {queue wait ms, submit-to-done ms}.  Returns the request's status
 * (QNSCH_EBUSY while it is not finished). */
int qnsch_server_result(qnsch_server *srv, uint64_t id, double *c, double *mu, double *p, double *u, double *v,
                        double *mass_hist, double *energy_hist, double *step_ms, int32_t *vcycles, double *times);
/* out = {p50 step ms, p99 step ms, cell-steps done, seconds from first
 * admission to last completion, cell-steps/s, steps done, launches, ticks,
 * host ms in admission, host ms in result download, host ms blocked waiting
 * for the device, contexts allocated (the rest were recycled)}. */
int qnsch_server_stats(qnsch_server *srv, double out[12]);
/* Step latency and throughput of the server so far: p50 and p99 of the wall
 * time of every finished step of every request (ms, from the step's start to
 * its end, time spent waiting for the device or the scheduler inside the
 * server included), and cell-steps per second from the first admission to
 * the last completion.  NULL pointers are skipped; 0 before any step ends. */
int qnsch_server_latency(qnsch_server *srv, double *p50_ms, double *p99_ms, double *cell_steps_per_s);

#ifdef __cplusplus
}
#endif
#endif
