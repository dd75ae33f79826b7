/*
 * qnsch_oracle.c -- FP64 CPU oracle for the primitive-variable q-NSCH time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only tests/, the smoke check and the benchmark's CPU-baseline leg do.
 * It shares no source with the GPU library.
 *
 * What it computes (Guo, Lin, Lowengrub, Wise, "Mass conservative and energy
 * stable finite difference methods for the quasi-incompressible
 * Navier-Stokes-Cahn-Hilliard system", sec. 6.1, eqs. (pm-num-mx)-(pm-num-chem)
 * with the special forms (e1e1-1), (e1e1-2), (e1e1), (e1e2), App. A):
 *
 *   N(w) = 0,  w = (c, mubar, pbar, u, v) at time n+1,
 *
 * every equation written as "left side minus right side" of the paper, so the
 * discrete solution is the root of N.  The solver is the paper's nonlinear FAS
 * multigrid (sec. 7.1): per cell a pointwise Newton (Gauss-Seidel) update of
 * (c, mubar) on the phase and chemical-potential equations, then a Vanka box
 * update of the four faces and the pressure of the cell on the momentum and
 * mass equations (or, by default, one Newton step on all seven unknowns of the
 * cell), in red-black order, inside a V-cycle.  The paper leaves the
 * V-cycle, transfers and sweep semantics to its references; the readings used
 * here are stated where they are implemented.
 *
 * Obviously-correct choices:
 *   - every discrete operator is a separate small function named as in App. A;
 *   - local Jacobians (smoothers, dense Newton) come from complex-step
 *     differentiation of the very residual functions below, so there is no
 *     second, hand-derived copy of any derivative (exact to rounding: no
 *     subtraction is involved);
 *   - everything is FP64, single-threaded, sequential sums.
 *
 * Storage: interior cells only, row-major, x fastest, index j*m1+i,
 *   cell (i,j), 0<=i<m1, 0<=j<m2, centre ((i+1/2)h, (j+1/2)h);
 *   u(i,j) = x-velocity on the west face of cell (i,j), at (i h, (j+1/2)h);
 *   v(i,j) = y-velocity on the south face of cell (i,j), at ((i+1/2)h, j h).
 * Ghost values are never stored: the accessors apply the boundary conditions of
 * App. A.4 (Neumann/periodic cells; no-slip/periodic edges).
 *
 * The projection scheme (sec. 6.2, eqs. (pj-num-mx)-(pj-num-chem)) is the
 * second option (opts.scheme).  Its unknowns are c, mubar, pbar and the
 * intermediate velocity u~ (stored in the face fields during a step); the
 * velocity of time n+1 is eliminated through the projection equation
 * (pj-num-pjx), which gives it face by face from u~ and the cell unknowns
 * (ufin, vfin).  Its smoother is the four steps of sec. 7.2 (see halfsweep).
 * After a converged step the face fields hold the velocity of time n+1.
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "qnsch_oracle.h"
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cx;

enum { F_C = 0, F_MU, F_P, F_U, F_V, F_CN, F_UN, F_VN, NFIELD };
#define NSTATE 5 /* c, mu, p, u, v */

typedef struct {
    int m1, m2;
    double h;
    double *f[NFIELD];   /* iterate (0..4) and time-n data (5..7) */
    double *rhs[NSTATE]; /* FAS right-hand side; zero on the finest level */
    double *w0[NSTATE];  /* restricted iterate R w, kept for the correction */
    double *r[NSTATE];   /* residual work array */
} Level;

struct orc_ctx {
    orc_grid g;
    orc_params p;
    orc_opts o;
    double alpha, K1, K2, K3;
    double dt;
    int nlev;
    Level lev[ORC_MAXLEV];
    /* committed state at time n (restored on failure) */
    double *save[NSTATE];
    /* projection scheme: the velocity of time n+1 frozen on level fzlev
     * (during the point update of c, mubar), and the intermediate velocity of
     * the last completed step on the finest level */
    const Level *fzlev;
    double *ufz, *vfz;
    double *ut_save[2];
    /* set while the coarsest-level solve of a V-cycle runs */
    int in_coarse;
    /* acceleration of the cycle iteration: the last nh cycle results of the
     * step (hw) and their residuals (hr), index 0 the newest; the pending
     * combination uses acc_use of the earlier ones with coefficients acc_g */
    double *hw[ORC_MAXACC + 1][NSTATE], *hr[ORC_MAXACC + 1][NSTATE];
    int nh, acc_use, acc_pending, ncycle;
    double acc_g[ORC_MAXACC], acc_last, acc_nr[NSTATE];
    /* statistics of the last step */
    int nv;
    double hist[ORC_MAXV + 1][NSTATE];
    int in_step;
};

/* The complex-step perturbation of the thread evaluating a residual: on
 * level plev, either one unknown (pf, pi, pj) or, when pdir[0] is set, every
 * unknown along the direction pdir; thaw set = the frozen velocity of the
 * projection scheme is not used (its pressure column).  Per thread, so that
 * the cells of one colour may be relaxed by several threads (they are
 * independent: see halfsweep); the arithmetic does not depend on it. */
typedef struct {
    const Level *plev;
    int pf, pi, pj;
    double ph;
    const double *pdir[NSTATE];
    int thaw;
} Pert;
static __thread Pert tp = { NULL, -1, 0, 0, 0.0, { NULL }, 0 };

/* ------------------------------------------------------------------------- */
/* material laws, sec. 2.1 and eq. (def-rhoal), g of sec. 4.1, m of sec. 6.1 */

static cx rho_of(const orc_ctx *o, cx c)
{
    return o->p.rho1 * o->p.rho2 / ((o->p.rho2 - o->p.rho1) * c + o->p.rho1);
}
static cx visc_of(const orc_ctx *o, cx c)
{
    return o->p.visc1 * o->p.visc2 / ((o->p.visc2 - o->p.visc1) * c + o->p.visc1);
}
/* regularised mobility m(c) = sqrt(c^2 (1-c)^2 + reg), evaluated on time-n data */
static cx mob_of(const orc_ctx *o, cx c)
{
    return csqrt(c * c * (1.0 - c) * (1.0 - c) + o->p.mob_reg);
}
static cx Fdw(cx c) { return c * c * (c - 1.0) * (c - 1.0) / 4.0; }
static cx gsec(cx a, cx b) { return 0.25 * (a * (a - 1.0) + b * (b - 1.0)) * (a + b - 1.0); }
static cx rsec(const orc_ctx *o, cx a, cx b) { return -o->alpha * rho_of(o, a) * rho_of(o, b); }

/* ------------------------------------------------------------------------- */
/* accessors with boundary conditions (App. A.4)                              */

static int wrap(int k, int n) { return ((k % n) + n) % n; }

static cx raw(const orc_ctx *o, const Level *L, int fld, int i, int j)
{
    size_t k = (size_t)j * L->m1 + i;
    cx v = L->f[fld][k];
    (void)o;
    if (L == tp.plev && tp.ph != 0.0) {
        if (tp.pdir[0]) {
            if (fld < NSTATE) v += I * tp.ph * tp.pdir[fld][k];
        } else if (fld == tp.pf && i == tp.pi && j == tp.pj) {
            v += I * tp.ph;
        }
    }
    return v;
}

static int projection(const orc_ctx *o) { return o->o.scheme == ORC_PROJECTION; }

static void die(const char *msg, int a, int b)
{
    fprintf(stderr, "qnsch oracle: %s (%d,%d)\n", msg, a, b);
    abort();
}

/* cell-centred field with one ghost layer: Neumann mirror or periodic wrap,
 * x resolved first, then y (corners) */
static cx cellv(const orc_ctx *o, const Level *L, int fld, int i, int j)
{
    if (i < -1 || i > L->m1 || j < -1 || j > L->m2) die("cell ghost depth", i, j);
    if (i < 0 || i >= L->m1) i = o->g.bcx == ORC_PERIODIC ? wrap(i, L->m1) : (i < 0 ? 0 : L->m1 - 1);
    if (j < 0 || j >= L->m2) j = o->g.bcy == ORC_PERIODIC ? wrap(j, L->m2) : (j < 0 ? 0 : L->m2 - 1);
    return raw(o, L, fld, i, j);
}

/* east-west edge field at face x = i h, row j.  No-slip: normal velocity zero
 * on x-walls; tangential ghost rows reflected (u_ghost = -u) so that the
 * average a_y u vanishes on the y-walls. */
static cx uv(const orc_ctx *o, const Level *L, int fld, int i, int j)
{
    if (i < -1 || i > L->m1 + 1 || j < -1 || j > L->m2) die("u index", i, j);
    if (o->g.bcx == ORC_PERIODIC) {
        i = wrap(i, L->m1);
    } else if (i == 0 || i == L->m1) {
        return 0.0;
    } else if (i < 0 || i > L->m1) {
        die("u beyond an x-wall", i, j);
    }
    if (j < 0 || j >= L->m2) {
        if (o->g.bcy == ORC_PERIODIC) return raw(o, L, fld, i, wrap(j, L->m2));
        return -raw(o, L, fld, i, j < 0 ? 0 : L->m2 - 1);
    }
    return raw(o, L, fld, i, j);
}

/* north-south edge field at column i, face y = j h */
static cx vv(const orc_ctx *o, const Level *L, int fld, int i, int j)
{
    if (j < -1 || j > L->m2 + 1 || i < -1 || i > L->m1) die("v index", i, j);
    if (o->g.bcy == ORC_PERIODIC) {
        j = wrap(j, L->m2);
    } else if (j == 0 || j == L->m2) {
        return 0.0;
    } else if (j < 0 || j > L->m2) {
        die("v beyond a y-wall", i, j);
    }
    if (i < 0 || i >= L->m1) {
        if (o->g.bcx == ORC_PERIODIC) return raw(o, L, fld, wrap(i, L->m1), j);
        return -raw(o, L, fld, i < 0 ? 0 : L->m1 - 1, j);
    }
    return raw(o, L, fld, i, j);
}

static int u_unknown(const orc_ctx *o, const Level *L, int i)
{
    return o->g.bcx == ORC_PERIODIC ? 1 : (i >= 1 && i <= L->m1 - 1);
}
static int v_unknown(const orc_ctx *o, const Level *L, int j)
{
    return o->g.bcy == ORC_PERIODIC ? 1 : (j >= 1 && j <= L->m2 - 1);
}

/* ------------------------------------------------------------------------- */
/* cell functions of the concentration                                        */

static cx rho_c(const orc_ctx *o, const Level *L, int fld, int i, int j) { return rho_of(o, cellv(o, L, fld, i, j)); }
static cx visc_n(const orc_ctx *o, const Level *L, int i, int j) { return visc_of(o, cellv(o, L, F_CN, i, j)); }
static cx mob_n(const orc_ctx *o, const Level *L, int i, int j) { return mob_of(o, cellv(o, L, F_CN, i, j)); }

/* ------------------------------------------------------------------------- */
/* difference and average operators of App. A.2 (h = L->h)                    */

/* edge-to-centre, at cell (i,j) */
static cx a_x(const orc_ctx *o, const Level *L, int fu, int i, int j) { return 0.5 * (uv(o, L, fu, i + 1, j) + uv(o, L, fu, i, j)); }
static cx d_x(const orc_ctx *o, const Level *L, int fu, int i, int j) { return (uv(o, L, fu, i + 1, j) - uv(o, L, fu, i, j)) / L->h; }
static cx a_y(const orc_ctx *o, const Level *L, int fv, int i, int j) { return 0.5 * (vv(o, L, fv, i, j + 1) + vv(o, L, fv, i, j)); }
static cx d_y(const orc_ctx *o, const Level *L, int fv, int i, int j) { return (vv(o, L, fv, i, j + 1) - vv(o, L, fv, i, j)) / L->h; }

/* centre-to-edge of a concentration-derived cell function.  kind selects the
 * cell function: 0 = the field itself, 1 = rho(field) */
static cx cfun(const orc_ctx *o, const Level *L, int fld, int kind, int i, int j)
{
    cx c = cellv(o, L, fld, i, j);
    return kind ? rho_of(o, c) : c;
}
/* A_x, D_x at the east-west face (i,j), between cells i-1 and i */
static cx A_xc(const orc_ctx *o, const Level *L, int fld, int kind, int i, int j) { return 0.5 * (cfun(o, L, fld, kind, i, j) + cfun(o, L, fld, kind, i - 1, j)); }
static cx D_xc(const orc_ctx *o, const Level *L, int fld, int i, int j) { return (cellv(o, L, fld, i, j) - cellv(o, L, fld, i - 1, j)) / L->h; }
/* A_y, D_y at the north-south face (i,j), between cells j-1 and j */
static cx A_yc(const orc_ctx *o, const Level *L, int fld, int kind, int i, int j) { return 0.5 * (cfun(o, L, fld, kind, i, j) + cfun(o, L, fld, kind, i, j - 1)); }
static cx D_yc(const orc_ctx *o, const Level *L, int fld, int i, int j) { return (cellv(o, L, fld, i, j) - cellv(o, L, fld, i, j - 1)) / L->h; }

/* centre-to-vertex average (calligraphic A) at vertex (i h, j h) of rho^n and
 * of the viscosity mu(c^n) */
static cx Av_rho_n(const orc_ctx *o, const Level *L, int i, int j)
{
    return 0.25 * (rho_c(o, L, F_CN, i, j) + rho_c(o, L, F_CN, i - 1, j) + rho_c(o, L, F_CN, i, j - 1) + rho_c(o, L, F_CN, i - 1, j - 1));
}
static cx Av_visc_n(const orc_ctx *o, const Level *L, int i, int j)
{
    return 0.25 * (visc_n(o, L, i, j) + visc_n(o, L, i - 1, j) + visc_n(o, L, i, j - 1) + visc_n(o, L, i - 1, j - 1));
}
/* edge-to-vertex: calligraphic A_x, D_x of a north-south field; A_y, D_y of an
 * east-west field, at vertex (i,j) */
static cx cA_x(const orc_ctx *o, const Level *L, int fv, int i, int j) { return 0.5 * (vv(o, L, fv, i, j) + vv(o, L, fv, i - 1, j)); }
static cx cD_x(const orc_ctx *o, const Level *L, int fv, int i, int j) { return (vv(o, L, fv, i, j) - vv(o, L, fv, i - 1, j)) / L->h; }
static cx cA_y(const orc_ctx *o, const Level *L, int fu, int i, int j) { return 0.5 * (uv(o, L, fu, i, j) + uv(o, L, fu, i, j - 1)); }
static cx cD_y(const orc_ctx *o, const Level *L, int fu, int i, int j) { return (uv(o, L, fu, i, j) - uv(o, L, fu, i, j - 1)) / L->h; }

/* ------------------------------------------------------------------------- */
/* vertex functions that the momentum equation differences (vertex-to-edge)  */

/* x-row: calA rho^n * calA_x v^n * calD_y u   and   calA rho^n * calA_x v^n */
static cx vx_adv(const orc_ctx *o, const Level *L, int i, int j) { return Av_rho_n(o, L, i, j) * cA_x(o, L, F_VN, i, j) * cD_y(o, L, F_U, i, j); }
static cx vx_flux(const orc_ctx *o, const Level *L, int i, int j) { return Av_rho_n(o, L, i, j) * cA_x(o, L, F_VN, i, j); }
static cx vx_visc(const orc_ctx *o, const Level *L, int i, int j) { return Av_visc_n(o, L, i, j) * cD_y(o, L, F_U, i, j); }
/* y-row: calA rho^n * calA_y u^n * calD_x v   and   calA rho^n * calA_y u^n */
static cx vy_adv(const orc_ctx *o, const Level *L, int i, int j) { return Av_rho_n(o, L, i, j) * cA_y(o, L, F_UN, i, j) * cD_x(o, L, F_V, i, j); }
static cx vy_flux(const orc_ctx *o, const Level *L, int i, int j) { return Av_rho_n(o, L, i, j) * cA_y(o, L, F_UN, i, j); }
static cx vy_visc(const orc_ctx *o, const Level *L, int i, int j) { return Av_visc_n(o, L, i, j) * cD_x(o, L, F_V, i, j); }

/* cell functions used by the momentum rows */
static cx cell_rho_ax_un(const orc_ctx *o, const Level *L, int i, int j) { return rho_c(o, L, F_CN, i, j) * a_x(o, L, F_UN, i, j); }
static cx cell_rho_ay_vn(const orc_ctx *o, const Level *L, int i, int j) { return rho_c(o, L, F_CN, i, j) * a_y(o, L, F_VN, i, j); }
static cx theta(const orc_ctx *o, const Level *L, int i, int j) { return d_x(o, L, F_U, i, j) + d_y(o, L, F_V, i, j); }

/* ------------------------------------------------------------------------- */
/* projection scheme: velocity of time n+1 from the projection equation       */
/* (pj-num-pjx), A rho (u - u~)/dt = -D pbar/M + A(rho_ew mubar) D c/M, with   */
/* rho = rho(c) and c, mubar of the iterate (time n+1) in the surface-tension */
/* form of App. A.6, and gravity in the projection equation as in the         */
/* time-discrete scheme (pj-pj), -(1/Fr)(A_y rho - rho_ref) on north-south     */
/* faces.  Zero on wall faces (normal velocity, (pj-dis-bc3)); only faces of  */
/* interior rows are asked for.                                                */

/* east-west face (i,j), 0 <= i <= m1 */
static cx ufin(const orc_ctx *o, const Level *L, int i, int j)
{
    if (o->g.bcx == ORC_PERIODIC) i = wrap(i, L->m1);
    else if (i <= 0 || i >= L->m1) return 0.0;
    if (L == o->fzlev && !tp.thaw) return o->ufz[(size_t)j * L->m1 + i];
    cx Ar = A_xc(o, L, F_C, 1, i, j);
    cx st = 0.5 * (rho_c(o, L, F_C, i, j) * cellv(o, L, F_MU, i - 1, j) + rho_c(o, L, F_C, i - 1, j) * cellv(o, L, F_MU, i, j))
          * D_xc(o, L, F_C, i, j);
    return uv(o, L, F_U, i, j) + o->dt / Ar * (st - D_xc(o, L, F_P, i, j)) / o->p.M;
}
/* north-south face (i,j), 0 <= j <= m2 */
static cx vfin(const orc_ctx *o, const Level *L, int i, int j)
{
    if (o->g.bcy == ORC_PERIODIC) j = wrap(j, L->m2);
    else if (j <= 0 || j >= L->m2) return 0.0;
    if (L == o->fzlev && !tp.thaw) return o->vfz[(size_t)j * L->m1 + i];
    cx Ar = A_yc(o, L, F_C, 1, i, j);
    cx st = 0.5 * (rho_c(o, L, F_C, i, j) * cellv(o, L, F_MU, i, j - 1) + rho_c(o, L, F_C, i, j - 1) * cellv(o, L, F_MU, i, j))
          * D_yc(o, L, F_C, i, j);
    cx grav = o->p.inv_Fr * (Ar - o->p.rho_ref);
    return vv(o, L, F_V, i, j) + o->dt / Ar * ((st - D_yc(o, L, F_P, i, j)) / o->p.M - grav);
}

/* ------------------------------------------------------------------------- */
/* residuals: left side minus right side of each equation                      */

/* x-momentum (pm-num-mx), first row, at the east-west face (i,j) */
static cx res_u(const orc_ctx *o, const Level *L, int i, int j)
{
    const double h = L->h, dt = o->dt;
    cx u = uv(o, L, F_U, i, j), un = uv(o, L, F_UN, i, j);
    cx Arn = A_xc(o, L, F_CN, 1, i, j); /* A_x rho^n */
    cx Ars = A_xc(o, L, F_C, 1, i, j);  /* A_x rho^{n+1} */
    /* rho^n u^n . grad u^{n+1}, (e1e1-1): A_x(rho a_x u^n d_x u) + frakA_y(calA rho calA_x v^n calD_y u) */
    cx adv = 0.5 * (cell_rho_ax_un(o, L, i, j) * d_x(o, L, F_U, i, j) + cell_rho_ax_un(o, L, i - 1, j) * d_x(o, L, F_U, i - 1, j))
           + 0.5 * (vx_adv(o, L, i, j + 1) + vx_adv(o, L, i, j));
    /* (1/2) div(rho^n u^n) u^{n+1}, (e1e1-2): D_x(rho a_x u^n) + frakD_y(calA rho calA_x v^n) */
    cx div = (cell_rho_ax_un(o, L, i, j) - cell_rho_ax_un(o, L, i - 1, j)) / h + (vx_flux(o, L, i, j + 1) - vx_flux(o, L, i, j)) / h;
    /* surface tension, (e1e1) with App. A.6 */
    cx st = 0.5 * (rho_c(o, L, F_CN, i, j) * cellv(o, L, F_MU, i - 1, j) + rho_c(o, L, F_CN, i - 1, j) * cellv(o, L, F_MU, i, j)) * D_xc(o, L, F_CN, i, j);
    /* viscous: D_x(mu d_x u) + frakD_y(calA mu calD_y u) */
    cx visc = (visc_n(o, L, i, j) * d_x(o, L, F_U, i, j) - visc_n(o, L, i - 1, j) * d_x(o, L, F_U, i - 1, j)) / h + (vx_visc(o, L, i, j + 1) - vx_visc(o, L, i, j)) / h;
    /* D_x(mu div_d u) */
    cx gd = (visc_n(o, L, i, j) * theta(o, L, i, j) - visc_n(o, L, i - 1, j) * theta(o, L, i - 1, j)) / h;
    cx N = Arn * (u - un) / dt + adv + (Ars - Arn) / (2.0 * dt) * u + 0.5 * div * u - visc / o->p.Re - gd / (3.0 * o->p.Re);
    /* (pj-num-mx) for the intermediate velocity has neither pressure nor
     * surface tension; they act in the projection equation */
    if (!projection(o)) N += D_xc(o, L, F_P, i, j) / o->p.M - st / o->p.M;
    return N;
}

/* y-momentum (pm-num-mx), second row, at the north-south face (i,j) */
static cx res_v(const orc_ctx *o, const Level *L, int i, int j)
{
    const double h = L->h, dt = o->dt;
    cx v = vv(o, L, F_V, i, j), vn = vv(o, L, F_VN, i, j);
    cx Arn = A_yc(o, L, F_CN, 1, i, j);
    cx Ars = A_yc(o, L, F_C, 1, i, j);
    /* frakA_x(calA rho calA_y u^n calD_x v) + A_y(rho a_y v^n d_y v) */
    cx adv = 0.5 * (vy_adv(o, L, i + 1, j) + vy_adv(o, L, i, j))
           + 0.5 * (cell_rho_ay_vn(o, L, i, j) * d_y(o, L, F_V, i, j) + cell_rho_ay_vn(o, L, i, j - 1) * d_y(o, L, F_V, i, j - 1));
    /* frakD_x(calA rho calA_y u^n) + D_y(rho a_y v^n) */
    cx div = (vy_flux(o, L, i + 1, j) - vy_flux(o, L, i, j)) / h + (cell_rho_ay_vn(o, L, i, j) - cell_rho_ay_vn(o, L, i, j - 1)) / h;
    cx st = 0.5 * (rho_c(o, L, F_CN, i, j) * cellv(o, L, F_MU, i, j - 1) + rho_c(o, L, F_CN, i, j - 1) * cellv(o, L, F_MU, i, j)) * D_yc(o, L, F_CN, i, j);
    cx visc = (vy_visc(o, L, i + 1, j) - vy_visc(o, L, i, j)) / h + (visc_n(o, L, i, j) * d_y(o, L, F_V, i, j) - visc_n(o, L, i, j - 1) * d_y(o, L, F_V, i, j - 1)) / h;
    cx gd = (visc_n(o, L, i, j) * theta(o, L, i, j) - visc_n(o, L, i, j - 1) * theta(o, L, i, j - 1)) / h;
    /* gravity -(1/Fr) A_y rho^n j, measured against a reference density */
    cx grav = o->p.inv_Fr * (Arn - o->p.rho_ref);
    cx N = Arn * (v - vn) / dt + adv + (Ars - Arn) / (2.0 * dt) * v + 0.5 * div * v - visc / o->p.Re - gd / (3.0 * o->p.Re);
    if (!projection(o)) N += D_yc(o, L, F_P, i, j) / o->p.M - st / o->p.M + grav;
    return N;
}

/* variable-coefficient diffusion div_d(A k grad_D phi) at cell (i,j); the
 * coefficient k is a cell function selected by kc:
 *   0 = m(c^n),  1 = rho^{n+1/2} = (rho(c)+rho(c^n))/2;
 * phi is a cell field, or (fld = -1) c^{n+1/2} = (c+c^n)/2 */
static cx kcoef(const orc_ctx *o, const Level *L, int kc, int i, int j)
{
    if (kc == 0) return mob_n(o, L, i, j);
    return 0.5 * (rho_c(o, L, F_C, i, j) + rho_c(o, L, F_CN, i, j));
}
static cx phival(const orc_ctx *o, const Level *L, int fld, int i, int j)
{
    if (fld >= 0) return cellv(o, L, fld, i, j);
    return 0.5 * (cellv(o, L, F_C, i, j) + cellv(o, L, F_CN, i, j));
}
static cx divAkgrad(const orc_ctx *o, const Level *L, int kc, int fld, int i, int j)
{
    const double h = L->h;
    cx k0 = kcoef(o, L, kc, i, j), p0 = phival(o, L, fld, i, j);
    cx fe = 0.5 * (kcoef(o, L, kc, i + 1, j) + k0) * (phival(o, L, fld, i + 1, j) - p0) / h;
    cx fw = 0.5 * (k0 + kcoef(o, L, kc, i - 1, j)) * (p0 - phival(o, L, fld, i - 1, j)) / h;
    cx fn = 0.5 * (kcoef(o, L, kc, i, j + 1) + k0) * (phival(o, L, fld, i, j + 1) - p0) / h;
    cx fs = 0.5 * (k0 + kcoef(o, L, kc, i, j - 1)) * (p0 - phival(o, L, fld, i, j - 1)) / h;
    return (fe - fw) / h + (fn - fs) / h;
}

/* mass equation (pm-num-mass) at cell (i,j); projection scheme (pj-num-mass)
 * with the velocity of time n+1 */
static cx res_p(const orc_ctx *o, const Level *L, int i, int j)
{
    double a = o->alpha, Pe = o->p.Pe;
    cx div = projection(o) ? (ufin(o, L, i + 1, j) - ufin(o, L, i, j)) / L->h + (vfin(o, L, i, j + 1) - vfin(o, L, i, j)) / L->h
                           : d_x(o, L, F_U, i, j) + d_y(o, L, F_V, i, j);
    return div - a / Pe * divAkgrad(o, L, 0, F_MU, i, j) - a * a / Pe * divAkgrad(o, L, 0, F_P, i, j);
}

/* phase equation (pm-num-phase) with the advection form (e1e2), App. A.5 */
static cx res_c(const orc_ctx *o, const Level *L, int i, int j)
{
    const double h = L->h;
    double a = o->alpha, Pe = o->p.Pe;
    cx c = cellv(o, L, F_C, i, j), cn = cellv(o, L, F_CN, i, j);
    if (projection(o)) {
        /* (pj-num-phase): rho^n (c - c^n)/dt + rho^{n+1} u^{n+1} . grad c^{n+1} in
         * the form (e1e2) of App. A.5 with every factor at time n+1 */
        cx ax = 0.5 * (rho_c(o, L, F_C, i + 1, j) * (cellv(o, L, F_C, i + 1, j) - c) / h * ufin(o, L, i + 1, j)
                     + rho_c(o, L, F_C, i - 1, j) * (c - cellv(o, L, F_C, i - 1, j)) / h * ufin(o, L, i, j));
        cx ay = 0.5 * (rho_c(o, L, F_C, i, j + 1) * (cellv(o, L, F_C, i, j + 1) - c) / h * vfin(o, L, i, j + 1)
                     + rho_c(o, L, F_C, i, j - 1) * (c - cellv(o, L, F_C, i, j - 1)) / h * vfin(o, L, i, j));
        return rho_of(o, cn) * (c - cn) / o->dt + ax + ay
             - divAkgrad(o, L, 0, F_MU, i, j) / Pe - a / Pe * divAkgrad(o, L, 0, F_P, i, j);
    }
    cx advx = 0.5 * (rho_c(o, L, F_CN, i + 1, j) * (cellv(o, L, F_CN, i + 1, j) - cn) / h * uv(o, L, F_U, i + 1, j)
                   + rho_c(o, L, F_CN, i - 1, j) * (cn - cellv(o, L, F_CN, i - 1, j)) / h * uv(o, L, F_U, i, j));
    cx advy = 0.5 * (rho_c(o, L, F_CN, i, j + 1) * (cellv(o, L, F_CN, i, j + 1) - cn) / h * vv(o, L, F_V, i, j + 1)
                   + rho_c(o, L, F_CN, i, j - 1) * (cn - cellv(o, L, F_CN, i, j - 1)) / h * vv(o, L, F_V, i, j));
    return rho_of(o, c) * (c - cn) / o->dt + advx + advy
         - divAkgrad(o, L, 0, F_MU, i, j) / Pe - a / Pe * divAkgrad(o, L, 0, F_P, i, j);
}

/* pointwise |grad_D phi|^2 at a cell: a_x((D_x phi)^2) + a_y((D_y phi)^2) */
static cx gradsq(const orc_ctx *o, const Level *L, int fld, int i, int j)
{
    cx e = D_xc(o, L, fld, i + 1, j), w = D_xc(o, L, fld, i, j);
    cx n = D_yc(o, L, fld, i, j + 1), s = D_yc(o, L, fld, i, j);
    return 0.5 * (e * e + w * w) + 0.5 * (n * n + s * s);
}

/* chemical-potential equation (pm-num-chem) at cell (i,j) */
static cx res_mu(const orc_ctx *o, const Level *L, int i, int j)
{
    cx c = cellv(o, L, F_C, i, j), cn = cellv(o, L, F_CN, i, j), mu = cellv(o, L, F_MU, i, j);
    cx rs = rho_of(o, c), rn = rho_of(o, cn);
    cx rhalf = 0.5 * (rs + rn), Fhalf = 0.5 * (Fdw(c) + Fdw(cn));
    cx Ghalf = 0.5 * (gradsq(o, L, F_C, i, j) + gradsq(o, L, F_CN, i, j));
    cx r = rsec(o, c, cn);
    /* (pj-num-chem) has rho^n mubar where (pm-num-chem) has rho^{n+1} mubar */
    cx rm = projection(o) ? rn : rs;
    return rm * mu - o->K1 * (rhalf * gsec(c, cn) + Fhalf * r) - o->K2 * Ghalf * r + o->K3 * divAkgrad(o, L, 1, -1, i, j);
}

/* ------------------------------------------------------------------------- */
/* whole-level residual r = rhs - N(w) at every unknown, zero elsewhere       */

static void residual_level(orc_ctx *o, Level *L, double *r[NSTATE])
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            size_t k = (size_t)j * L->m1 + i;
            r[0][k] = L->rhs[0][k] - creal(res_c(o, L, i, j));
            r[1][k] = L->rhs[1][k] - creal(res_mu(o, L, i, j));
            r[2][k] = L->rhs[2][k] - creal(res_p(o, L, i, j));
            r[3][k] = u_unknown(o, L, i) ? L->rhs[3][k] - creal(res_u(o, L, i, j)) : 0.0;
            r[4][k] = v_unknown(o, L, j) ? L->rhs[4][k] - creal(res_v(o, L, i, j)) : 0.0;
        }
}

/* per-equation discrete L2 norm sqrt(h^2 sum r^2) over the unknowns */
static void norms_level(const Level *L, double *r[NSTATE], double out[NSTATE])
{
    size_t n = (size_t)L->m1 * L->m2;
    for (int e = 0; e < NSTATE; e++) {
        double s = 0.0;
        for (size_t k = 0; k < n; k++) s += r[e][k] * r[e][k];
        out[e] = sqrt(L->h * L->h * s);
    }
}

/* ------------------------------------------------------------------------- */
/* local solves                                                                */

/* Gaussian elimination with partial pivoting on an n x n system, in place */
static int gepp(int n, double A[7][7], double b[7])
{
    for (int k = 0; k < n; k++) {
        int piv = k;
        for (int r = k + 1; r < n; r++)
            if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
        if (A[piv][k] == 0.0) return -1;
        if (piv != k) {
            for (int c = 0; c < n; c++) { double t = A[k][c]; A[k][c] = A[piv][c]; A[piv][c] = t; }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int r = k + 1; r < n; r++) {
            double l = A[r][k] / A[k][k];
            for (int c = k; c < n; c++) A[r][c] -= l * A[k][c];
            b[r] -= l * b[k];
        }
    }
    for (int k = n - 1; k >= 0; k--) {
        double s = b[k];
        for (int c = k + 1; c < n; c++) s -= A[k][c] * b[c];
        b[k] = s / A[k][k];
    }
    return 0;
}

#define CSTEP 1e-30

static void perturb(orc_ctx *o, const Level *L, int fld, int i, int j)
{
    (void)o;
    tp.plev = L; tp.pf = fld; tp.pi = i; tp.pj = j; tp.ph = CSTEP; tp.pdir[0] = NULL;
}
static void unperturb(orc_ctx *o) { (void)o; tp.plev = NULL; tp.pf = -1; tp.ph = 0.0; tp.pdir[0] = NULL; }

/* Step 1 of sec. 7.1 at cell (i,j): one Newton step on the phase and chemical-
 * potential equations in the two unknowns c_ij, mubar_ij, all else frozen. */
static void ch_point(orc_ctx *o, Level *L, int i, int j)
{
    size_t k = (size_t)j * L->m1 + i;
    double J[7][7], b[7];
    int fl[2] = { F_C, F_MU };
    for (int col = 0; col < 2; col++) {
        perturb(o, L, fl[col], i, j);
        cx rc = res_c(o, L, i, j), rm = res_mu(o, L, i, j);
        J[0][col] = cimag(rc) / CSTEP;
        J[1][col] = cimag(rm) / CSTEP;
        if (col == 0) { b[0] = L->rhs[0][k] - creal(rc); b[1] = L->rhs[1][k] - creal(rm); }
    }
    unperturb(o);
    if (gepp(2, J, b) != 0) return;
    L->f[F_C][k] += b[0];
    L->f[F_MU][k] += b[1];
}

/* Step 2 of sec. 7.1 at cell (i,j): Vanka box on the two east-west faces, the
 * two north-south faces and the pressure of the cell.  The box equations are
 * linear in these unknowns, so one Newton step with the exact (complex-step)
 * Jacobian is the exact box solve.  Velocities are read from the snapshot
 * (the field arrays) and the corrections are written to unew/vnew.
 * Coupled smoother (the default; a reading, see halfsweep): the cell's c and
 * mubar join the box with the phase and chemical-potential equations of the
 * cell, and one Newton step on the seven equations replaces step 1. */
static void vanka_box(orc_ctx *o, Level *L, int i, int j, double *unew, double *vnew)
{
    int fld[7], ci[7], cj[7], n = 0;
    int ie = (i + 1 == L->m1) ? (o->g.bcx == ORC_PERIODIC ? 0 : -1) : i + 1;
    int jn = (j + 1 == L->m2) ? (o->g.bcy == ORC_PERIODIC ? 0 : -1) : j + 1;
    if (u_unknown(o, L, i)) { fld[n] = F_U; ci[n] = i; cj[n] = j; n++; }
    if (ie >= 0 && u_unknown(o, L, ie)) { fld[n] = F_U; ci[n] = ie; cj[n] = j; n++; }
    if (v_unknown(o, L, j)) { fld[n] = F_V; ci[n] = i; cj[n] = j; n++; }
    if (jn >= 0 && v_unknown(o, L, jn)) { fld[n] = F_V; ci[n] = i; cj[n] = jn; n++; }
    /* projection scheme (sec. 7.2, step 2): the four intermediate-velocity
     * faces alone, on the momentum equations (pj-num-mx) */
    if (!projection(o)) { fld[n] = F_P; ci[n] = i; cj[n] = j; n++; }
    if (!projection(o) && o->o.smoother == ORC_SMOOTH_COUPLED) {
        fld[n] = F_C; ci[n] = i; cj[n] = j; n++;
        fld[n] = F_MU; ci[n] = i; cj[n] = j; n++;
    }
    double J[7][7], b[7];
    for (int col = 0; col < n; col++) {
        perturb(o, L, fld[col], ci[col], cj[col]);
        for (int row = 0; row < n; row++) {
            size_t kr = (size_t)cj[row] * L->m1 + ci[row];
            cx r;
            /* the equation attached to each unknown: momentum at a face, mass,
             * phase and chemical potential at the cell */
            int rf;
            if (fld[row] == F_U) { r = res_u(o, L, ci[row], cj[row]); rf = 3; }
            else if (fld[row] == F_V) { r = res_v(o, L, ci[row], cj[row]); rf = 4; }
            else if (fld[row] == F_C) { r = res_c(o, L, ci[row], cj[row]); rf = 0; }
            else if (fld[row] == F_MU) { r = res_mu(o, L, ci[row], cj[row]); rf = 1; }
            else { r = res_p(o, L, ci[row], cj[row]); rf = 2; }
            J[row][col] = cimag(r) / CSTEP;
            if (col == 0) b[row] = L->rhs[rf][kr] - creal(r);
        }
    }
    unperturb(o);
    if (gepp(n, J, b) != 0) return;
    /* faces and pbar take the relaxed step: vanka_omega, or coarse_omega on
     * the coarsest-level solve of the primitive scheme (over-relaxation; a
     * reading: the cycle is left to the multigrid references of sec. 7);
     * c and mubar the full Newton step */
    double om = (!projection(o) && o->in_coarse) ? o->o.coarse_omega : o->o.vanka_omega;
    for (int q = 0; q < n; q++) {
        size_t kq = (size_t)cj[q] * L->m1 + ci[q];
        double d = om * b[q];
        if (fld[q] == F_U) unew[kq] = L->f[F_U][kq] + d;
        else if (fld[q] == F_V) vnew[kq] = L->f[F_V][kq] + d;
        else if (fld[q] == F_C) L->f[F_C][kq] += b[q];
        else if (fld[q] == F_MU) L->f[F_MU][kq] += b[q];
        else L->f[F_P][kq] += d;
    }
}

/* Projection scheme, step 3 of sec. 7.2 at cell (i,j): one Newton step on the
 * mass equation (pj-num-mass) in pbar of the cell, the velocity of time n+1
 * taken from the projection of the current unknowns (through which pbar acts
 * on the four faces); exact, the equation being linear in pbar. */
static void p_point(orc_ctx *o, Level *L, int i, int j)
{
    size_t k = (size_t)j * L->m1 + i;
    perturb(o, L, F_P, i, j);
    cx r = res_p(o, L, i, j);
    unperturb(o);
    double J = cimag(r) / CSTEP;
    if (J == 0.0) return;
    /* over-relaxed by coarse_omega in the coarsest-level solve (as the
     * primitive box's pressure and velocity there) */
    double om = o->in_coarse ? o->o.coarse_omega : 1.0;
    L->f[F_P][k] += om * (L->rhs[2][k] - creal(r)) / J;
}

/* Projection scheme, coupled form of step 1 (a reading, see halfsweep_pj):
 * one Newton step on (N_c, N_mu, N_p) in (c, mubar, pbar) of the cell.  The
 * c and mubar columns of the local Jacobian take the velocity of time n+1
 * held (as step 1 of sec. 7.2), the pbar column lets it follow pbar through
 * the projection equation (pj-num-pjx); the residuals are those of the
 * current iterate.  Complex-step derivatives as everywhere. */
static void cmp_point(orc_ctx *o, Level *L, int i, int j)
{
    size_t k = (size_t)j * L->m1 + i;
    double J[7][7], b[7];
    int fl[3] = { F_C, F_MU, F_P };
    for (int col = 0; col < 3; col++) {
        tp.thaw = col == 2;
        perturb(o, L, fl[col], i, j);
        cx rc = res_c(o, L, i, j), rm = res_mu(o, L, i, j), rp = res_p(o, L, i, j);
        J[0][col] = cimag(rc) / CSTEP;
        J[1][col] = cimag(rm) / CSTEP;
        J[2][col] = cimag(rp) / CSTEP;
        if (col == 0) { b[0] = L->rhs[0][k] - creal(rc); b[1] = L->rhs[1][k] - creal(rm); b[2] = L->rhs[2][k] - creal(rp); }
    }
    unperturb(o);
    tp.thaw = 0;
    if (gepp(3, J, b) != 0) return;
    L->f[F_C][k] += b[0];
    L->f[F_MU][k] += b[1];
    L->f[F_P][k] += b[2];
}

/* Projection scheme, one colour (sec. 7.2, steps per cell of the colour):
 *   1. one Newton step on (N_c, N_mu) in (c, mubar), the velocity of time n+1
 *      frozen at its value before the half-sweep (the stored velocity of the
 *      paper's sequential sweep); with the coupled smoother (the default, a
 *      reading) the step also takes pbar with the mass equation (cmp_point):
 *      held apart, mubar and pbar are updated in turn although the phase and
 *      mass equations see them together (through mubar + alpha pbar), which
 *      stalls the cycles under refinement (58 V-cycles on the 256 x 256
 *      convergence case of sec. 9 against 10 coupled);
 *   2. the Vanka box of the four intermediate-velocity faces (exact: the
 *      momentum equations are linear in u~), Jacobi within the colour as in
 *      the primitive scheme;
 *   3. the pbar update above, with the new u~, c and mubar;
 *   4. the velocity of time n+1 is not stored: it is the projection of the
 *      current unknowns wherever it is used.
 * Steps 2 and 3 of one cell read only its own box faces and cells of the
 * other colour besides its own c, mubar, pbar, so all boxes of the colour
 * may take step 2 before any takes step 3. */
static void halfsweep_pj(orc_ctx *o, int l, int colour)
{
    Level *L = &o->lev[l];
    size_t n = (size_t)L->m1 * L->m2;
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            size_t k = (size_t)j * L->m1 + i;
            o->ufz[k] = u_unknown(o, L, i) ? creal(ufin(o, L, i, j)) : 0.0;
            o->vfz[k] = v_unknown(o, L, j) ? creal(vfin(o, L, i, j)) : 0.0;
        }
    o->fzlev = L;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++)
            if (((i + j) & 1) == colour) {
                if (o->o.smoother == ORC_SMOOTH_COUPLED) cmp_point(o, L, i, j);
                else ch_point(o, L, i, j);
            }
    o->fzlev = NULL;
    double *unew = malloc(n * sizeof(double)), *vnew = malloc(n * sizeof(double));
    memcpy(unew, L->f[F_U], n * sizeof(double));
    memcpy(vnew, L->f[F_V], n * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++)
            if (((i + j) & 1) == colour) vanka_box(o, L, i, j, unew, vnew);
    memcpy(L->f[F_U], unew, n * sizeof(double));
    memcpy(L->f[F_V], vnew, n * sizeof(double));
    free(unew);
    free(vnew);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++)
            if (((i + j) & 1) == colour) p_point(o, L, i, j);
}

/* One colour half-sweep (reading of sec. 7.1): colour = (i+j) mod 2.
 * Segregated smoother (the paper's two steps): first the pointwise CH update
 * at every cell of the colour (these are independent: their stencils only
 * reach cells of the other colour), then the Vanka box of every cell of the
 * colour.  Coupled smoother: the box alone, with c and mubar of the cell in
 * it (the phase and mass equations depend on mubar and pbar only through
 * mubar + alpha pbar, which the segregated steps update in turn).  All boxes
 * read the same velocity snapshot (Jacobi within a colour, Gauss-Seidel
 * across colours); c, mubar and pbar of a box are read by no other box of
 * its colour and are updated in place. */
static void halfsweep(orc_ctx *o, int l, int colour)
{
    if (projection(o)) { halfsweep_pj(o, l, colour); return; }
    Level *L = &o->lev[l];
    size_t n = (size_t)L->m1 * L->m2;
    if (o->o.smoother == ORC_SMOOTH_SEGREGATED) {
#pragma omp parallel for schedule(static)
        for (int j = 0; j < L->m2; j++)
            for (int i = 0; i < L->m1; i++)
                if (((i + j) & 1) == colour) ch_point(o, L, i, j);
    }
    double *unew = malloc(n * sizeof(double)), *vnew = malloc(n * sizeof(double));
    memcpy(unew, L->f[F_U], n * sizeof(double));
    memcpy(vnew, L->f[F_V], n * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++)
            if (((i + j) & 1) == colour) vanka_box(o, L, i, j, unew, vnew);
    memcpy(L->f[F_U], unew, n * sizeof(double));
    memcpy(L->f[F_V], vnew, n * sizeof(double));
    free(unew);
    free(vnew);
}

static void sweep(orc_ctx *o, int l)
{
    halfsweep(o, l, 0);
    halfsweep(o, l, 1);
}

/* ------------------------------------------------------------------------- */
/* grid transfers (the paper defers them to its multigrid references; reading:
 * cell quantities by the mean of the four children and piecewise-constant
 * interpolation; face quantities by the mean of the two coincident fine faces
 * and interpolation linear across the coarse cell, constant along the face) */

static void restrict_cell(const Level *F, const Level *C, const double *f, double *c)
{
    for (int J = 0; J < C->m2; J++)
        for (int Ii = 0; Ii < C->m1; Ii++) {
            int i = 2 * Ii, j = 2 * J;
            c[(size_t)J * C->m1 + Ii] = 0.25 * (f[(size_t)j * F->m1 + i] + f[(size_t)j * F->m1 + i + 1]
                                              + f[(size_t)(j + 1) * F->m1 + i] + f[(size_t)(j + 1) * F->m1 + i + 1]);
        }
}
static void restrict_u(const Level *F, const Level *C, const double *f, double *c)
{
    for (int J = 0; J < C->m2; J++)
        for (int Ii = 0; Ii < C->m1; Ii++)
            c[(size_t)J * C->m1 + Ii] = 0.5 * (f[(size_t)(2 * J) * F->m1 + 2 * Ii] + f[(size_t)(2 * J + 1) * F->m1 + 2 * Ii]);
}
static void restrict_v(const Level *F, const Level *C, const double *f, double *c)
{
    for (int J = 0; J < C->m2; J++)
        for (int Ii = 0; Ii < C->m1; Ii++)
            c[(size_t)J * C->m1 + Ii] = 0.5 * (f[(size_t)(2 * J) * F->m1 + 2 * Ii] + f[(size_t)(2 * J) * F->m1 + 2 * Ii + 1]);
}
static void restrict_fields(const orc_ctx *o, const Level *F, const Level *C, double *const f[NSTATE], double *const c[NSTATE])
{
    (void)o;
    restrict_cell(F, C, f[0], c[0]);
    restrict_cell(F, C, f[1], c[1]);
    restrict_cell(F, C, f[2], c[2]);
    restrict_u(F, C, f[3], c[3]);
    restrict_v(F, C, f[4], c[4]);
}

/* w_fine += P(w_coarse - w0) */
static void prolong_correct(const orc_ctx *o, Level *F, const Level *C)
{
    size_t nc = (size_t)C->m1 * C->m2;
    double *e[NSTATE];
    for (int q = 0; q < NSTATE; q++) {
        e[q] = malloc(nc * sizeof(double));
        for (size_t k = 0; k < nc; k++) e[q][k] = C->f[q][k] - C->w0[q][k];
    }
    /* coarse face corrections beyond the last column/row: periodic image or wall (0) */
    for (int j = 0; j < F->m2; j++)
        for (int i = 0; i < F->m1; i++) {
            size_t k = (size_t)j * F->m1 + i;
            int Ii = i / 2, J = j / 2;
            size_t kc = (size_t)J * C->m1 + Ii;
            for (int q = 0; q < 3; q++) F->f[q][k] += e[q][kc];
            if (u_unknown(o, F, i)) {
                double du;
                if ((i & 1) == 0) du = e[3][kc];
                else {
                    double east = (Ii + 1 < C->m1) ? e[3][(size_t)J * C->m1 + Ii + 1] : (o->g.bcx == ORC_PERIODIC ? e[3][(size_t)J * C->m1] : 0.0);
                    du = 0.5 * (e[3][kc] + east);
                }
                F->f[F_U][k] += du;
            }
            if (v_unknown(o, F, j)) {
                double dv;
                if ((j & 1) == 0) dv = e[4][kc];
                else {
                    double north = (J + 1 < C->m2) ? e[4][(size_t)(J + 1) * C->m1 + Ii] : (o->g.bcy == ORC_PERIODIC ? e[4][Ii] : 0.0);
                    dv = 0.5 * (e[4][kc] + north);
                }
                F->f[F_V][k] += dv;
            }
        }
    for (int q = 0; q < NSTATE; q++) free(e[q]);
}

/* ------------------------------------------------------------------------- */
/* FAS V-cycle                                                                 */

static void residual_at(orc_ctx *o, int l, double *r[NSTATE])
{
    residual_level(o, &o->lev[l], r);
}

static void vcycle(orc_ctx *o, int l)
{
    if (l == o->nlev - 1) {
        o->in_coarse = 1;
        for (int s = 0; s < o->o.nu_coarse; s++) sweep(o, l);
        o->in_coarse = 0;
        return;
    }
    Level *F = &o->lev[l], *C = &o->lev[l + 1];
    for (int s = 0; s < o->o.nu1; s++) sweep(o, l);
    residual_at(o, l, F->r);
    restrict_fields(o, F, C, F->f, C->f);       /* w_H = R w_h */
    size_t nc = (size_t)C->m1 * C->m2;
    for (int q = 0; q < NSTATE; q++) memcpy(C->w0[q], C->f[q], nc * sizeof(double));
    /* f_H = N_H(R w_h) + R(f_h - N_h(w_h)):  with rhs_H = 0, residual_at gives -N_H(R w) */
    double *Rr[NSTATE];
    for (int q = 0; q < NSTATE; q++) { Rr[q] = malloc(nc * sizeof(double)); memset(C->rhs[q], 0, nc * sizeof(double)); }
    restrict_fields(o, F, C, F->r, Rr);
    residual_at(o, l + 1, C->r);
    for (int q = 0; q < NSTATE; q++) {
        for (size_t k = 0; k < nc; k++) C->rhs[q][k] = -C->r[q][k] + Rr[q][k];
        free(Rr[q]);
    }
    /* rhs only lives on unknowns: wall faces carry no equation */
    for (int J = 0; J < C->m2; J++)
        for (int Ii = 0; Ii < C->m1; Ii++) {
            size_t k = (size_t)J * C->m1 + Ii;
            if (!u_unknown(o, C, Ii)) C->rhs[3][k] = 0.0;
            if (!v_unknown(o, C, J)) C->rhs[4][k] = 0.0;
        }
    vcycle(o, l + 1);
    prolong_correct(o, F, C);
    for (int s = 0; s < o->o.nu2; s++) sweep(o, l);
}

/* pbar is determined up to a constant (it enters only through differences):
 * fix its mean to zero after every cycle */
static void remove_p_mean(orc_ctx *o)
{
    Level *L = &o->lev[0];
    size_t n = (size_t)L->m1 * L->m2;
    double s = 0.0;
    for (size_t k = 0; k < n; k++) s += L->f[F_P][k];
    s /= (double)n;
    for (size_t k = 0; k < n; k++) L->f[F_P][k] -= s;
}

/* ------------------------------------------------------------------------- */
/* Acceleration of the cycle iteration.  Not in the paper (sec. 7.1 asks only  */
/* for a standard FAS V-cycle): the nonlinear Krylov acceleration of          */
/* multigrid of Washio and Oosterlee (ETNA 6, 1997).  With results w_0 (the    */
/* newest), w_1, ... and residuals r_k = rhs - N(w_k), the next cycle starts   */
/* from w_0 + sum_a g_a (w_0 - w_{a+1}), g minimising the linearised residual  */
/* || r_0 + sum_a g_a (r_0 - r_{a+1}) ||_2 (plain sum over all fields).        */

/* g from the normal equations H g = -b, H_ab = (e_a, e_b), b_a = (e_a, r_0),
 * e_a = r_0 - r_{a+1}, by Cholesky; only the leading block whose pivots stay
 * above 1e-12 of their diagonal entry is used.  Returns its size. */
static int acc_coefficients(const orc_ctx *o, int n, double g[ORC_MAXACC])
{
    const Level *L = &o->lev[0];
    size_t nc = (size_t)L->m1 * L->m2;
    double H[ORC_MAXACC][ORC_MAXACC] = { { 0 } }, b[ORC_MAXACC] = { 0 };
    for (int a = 0; a < n; a++) {
        for (int c = 0; c < n; c++) {
            double s = 0.0;
            for (int q = 0; q < NSTATE; q++)
                for (size_t k = 0; k < nc; k++)
                    s += (o->hr[0][q][k] - o->hr[a + 1][q][k]) * (o->hr[0][q][k] - o->hr[c + 1][q][k]);
            H[a][c] = s;
        }
        double s = 0.0;
        for (int q = 0; q < NSTATE; q++)
            for (size_t k = 0; k < nc; k++) s += (o->hr[0][q][k] - o->hr[a + 1][q][k]) * o->hr[0][q][k];
        b[a] = s;
    }
    /* H = C C^T, C lower triangular */
    double C[ORC_MAXACC][ORC_MAXACC] = { { 0 } };
    int use = 0;
    for (int c = 0; c < n; c++) {
        double piv = H[c][c];
        for (int k = 0; k < c; k++) piv -= C[c][k] * C[c][k];
        if (!(piv > 1e-12 * H[c][c]) || !isfinite(piv)) break;
        C[c][c] = sqrt(piv);
        for (int r = c + 1; r < n; r++) {
            double s = H[r][c];
            for (int k = 0; k < c; k++) s -= C[r][k] * C[c][k];
            C[r][c] = s / C[c][c];
        }
        use = c + 1;
    }
    double y[ORC_MAXACC] = { 0 };
    for (int a = 0; a < ORC_MAXACC; a++) g[a] = 0.0;
    for (int a = 0; a < use; a++) {
        double s = -b[a];
        for (int k = 0; k < a; k++) s -= C[a][k] * y[k];
        y[a] = s / C[a][a];
    }
    for (int a = use - 1; a >= 0; a--) {
        double s = y[a];
        for (int k = a + 1; k < use; k++) s -= C[k][a] * g[k];
        g[a] = s / C[a][a];
    }
    return use;
}

/* record the cycle result just computed (iterate of the finest level, its
 * residual in lev[0].r with norms nr) and fix the pending combination; a
 * result whose largest norm is not below the previous one's starts a new
 * history */
static void acc_record(orc_ctx *o, const double nr[NSTATE])
{
    const int m = o->o.accel;
    Level *L = &o->lev[0];
    size_t nb = (size_t)L->m1 * L->m2 * sizeof(double);
    double mx = 0.0;
    for (int q = 0; q < NSTATE; q++) mx = nr[q] > mx ? nr[q] : mx;
    int keep = o->nh < m + 1 ? o->nh + 1 : m + 1;
    if (o->nh > 0 && !(mx < o->acc_last)) keep = 1;
    /* the buffers of the oldest result take the new one */
    for (int q = 0; q < NSTATE; q++) {
        double *tw = o->hw[m][q], *tr = o->hr[m][q];
        for (int k = m; k > 0; k--) { o->hw[k][q] = o->hw[k - 1][q]; o->hr[k][q] = o->hr[k - 1][q]; }
        o->hw[0][q] = tw;
        o->hr[0][q] = tr;
        memcpy(o->hw[0][q], L->f[q], nb);
        memcpy(o->hr[0][q], L->r[q], nb);
    }
    o->nh = keep;
    o->acc_use = acc_coefficients(o, keep - 1, o->acc_g);
    o->acc_pending = 1;
    o->acc_last = mx;
}

/* the pending combination replaces the iterate of the finest level */
static void acc_apply(orc_ctx *o)
{
    if (!o->acc_pending) return;
    o->acc_pending = 0;
    Level *L = &o->lev[0];
    size_t nc = (size_t)L->m1 * L->m2;
    for (int q = 0; q < NSTATE; q++)
        for (size_t k = 0; k < nc; k++) {
            double w = o->hw[0][q][k];
            for (int a = 0; a < o->acc_use; a++) w += o->acc_g[a] * (o->hw[0][q][k] - o->hw[a + 1][q][k]);
            L->f[q][k] = w;
        }
}

/* ------------------------------------------------------------------------- */
/* public API                                                                  */

static double *zalloc(size_t n)
{
    double *p = calloc(n, sizeof(double));
    if (!p) { fprintf(stderr, "qnsch oracle: out of memory\n"); abort(); }
    return p;
}

orc_ctx *orc_create(const orc_grid *g, const orc_params *p, const orc_opts *opt)
{
    if (g->m1 < 2 || g->m2 < 2 || (g->m1 & 1) || (g->m2 & 1)) return NULL;
    double hx = g->Lx / g->m1, hy = g->Ly / g->m2;
    if (fabs(hx - hy) > 1e-12 * hx) return NULL;
    orc_ctx *o = calloc(1, sizeof(orc_ctx));
    o->g = *g;
    o->p = *p;
    o->o = *opt;
    o->alpha = (p->rho2 - p->rho1) / (p->rho1 * p->rho2);
    o->K1 = p->M * p->eta / (p->eps * p->We);
    o->K2 = p->eps * p->eta * p->M / (2.0 * p->We);
    o->K3 = p->eps * p->eta * p->M / p->We;
    /* levels: each level halves both dimensions, every level keeps even
     * dimensions (the red-black colouring needs them); auto = coarsen while the
     * coarsest level has more than 32 cells */
    int nl = g->levels;
    if (nl <= 0) {
        nl = 1;
        while (nl < ORC_MAXLEV && g->m1 % (1 << (nl + 1)) == 0 && g->m2 % (1 << (nl + 1)) == 0
               && (g->m1 >> (nl - 1)) * (g->m2 >> (nl - 1)) > 32)
            nl++;
    }
    if (nl > ORC_MAXLEV || g->m1 % (1 << nl) != 0 || g->m2 % (1 << nl) != 0) { free(o); return NULL; }
    o->nlev = nl;
    /* the coarsest solve's automatic settings (a reading of the multigrid
     * that sec. 7 defers to its references): 4 sweeps over-relaxed by 1.75
     * in the primitive scheme on hierarchies of 6 levels or more, else 6
     * sweeps by 1.6 */
    {
        const int deep = opt->scheme != ORC_PROJECTION && nl >= 6;
        if (o->o.nu_coarse <= 0) o->o.nu_coarse = deep ? 4 : 6;
        if (o->o.coarse_omega <= 0.0) o->o.coarse_omega = deep ? 1.75 : 1.6;
    }
    for (int l = 0; l < nl; l++) {
        Level *L = &o->lev[l];
        L->m1 = g->m1 >> l;
        L->m2 = g->m2 >> l;
        L->h = hx * (double)(1 << l);
        size_t n = (size_t)L->m1 * L->m2;
        for (int q = 0; q < NFIELD; q++) L->f[q] = zalloc(n);
        for (int q = 0; q < NSTATE; q++) { L->rhs[q] = zalloc(n); L->w0[q] = zalloc(n); L->r[q] = zalloc(n); }
    }
    size_t n0 = (size_t)g->m1 * g->m2;
    for (int q = 0; q < NSTATE; q++) o->save[q] = zalloc(n0);
    o->ufz = zalloc(n0);
    o->vfz = zalloc(n0);
    o->ut_save[0] = zalloc(n0);
    o->ut_save[1] = zalloc(n0);
    if (opt->accel < 0 || opt->accel > ORC_MAXACC) { orc_destroy(o); return NULL; }
    for (int k = 0; k <= opt->accel; k++)
        for (int q = 0; q < NSTATE; q++) { o->hw[k][q] = zalloc(n0); o->hr[k][q] = zalloc(n0); }
    return o;
}

void orc_destroy(orc_ctx *o)
{
    if (!o) return;
    for (int l = 0; l < o->nlev; l++) {
        Level *L = &o->lev[l];
        for (int q = 0; q < NFIELD; q++) free(L->f[q]);
        for (int q = 0; q < NSTATE; q++) { free(L->rhs[q]); free(L->w0[q]); free(L->r[q]); }
    }
    for (int q = 0; q < NSTATE; q++) free(o->save[q]);
    free(o->ufz); free(o->vfz); free(o->ut_save[0]); free(o->ut_save[1]);
    for (int k = 0; k <= ORC_MAXACC; k++)
        for (int q = 0; q < NSTATE; q++) { free(o->hw[k][q]); free(o->hr[k][q]); }
    free(o);
}

int orc_levels(const orc_ctx *o) { return o->nlev; }

/* host arrays: m1*m2 each, layout as described at the top */
void orc_set_state(orc_ctx *o, const double *c, const double *mu, const double *p, const double *u, const double *v)
{
    Level *L = &o->lev[0];
    size_t n = (size_t)L->m1 * L->m2;
    const double *src[NSTATE] = { c, mu, p, u, v };
    for (int q = 0; q < NSTATE; q++) {
        if (src[q]) memcpy(L->f[q], src[q], n * sizeof(double));
        else memset(L->f[q], 0, n * sizeof(double));
    }
    /* wall faces are not unknowns: they hold zero */
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            if (!u_unknown(o, L, i)) L->f[F_U][(size_t)j * L->m1 + i] = 0.0;
            if (!v_unknown(o, L, j)) L->f[F_V][(size_t)j * L->m1 + i] = 0.0;
        }
    o->in_step = 0;
}

void orc_get_state(const orc_ctx *o, double *c, double *mu, double *p, double *u, double *v)
{
    const Level *L = &o->lev[0];
    size_t n = (size_t)L->m1 * L->m2;
    double *dst[NSTATE] = { c, mu, p, u, v };
    for (int q = 0; q < NSTATE; q++)
        if (dst[q]) memcpy(dst[q], L->f[q], n * sizeof(double));
}

/* time-n data of every level, from the current iterate of the finest level;
 * coarse levels take the restriction of c^n, u^n, v^n (their own h) */
void orc_begin_step(orc_ctx *o, double dt)
{
    o->dt = dt;
    Level *L0 = &o->lev[0];
    size_t n0 = (size_t)L0->m1 * L0->m2;
    for (int q = 0; q < NSTATE; q++) memcpy(o->save[q], L0->f[q], n0 * sizeof(double));
    memcpy(L0->f[F_CN], L0->f[F_C], n0 * sizeof(double));
    memcpy(L0->f[F_UN], L0->f[F_U], n0 * sizeof(double));
    memcpy(L0->f[F_VN], L0->f[F_V], n0 * sizeof(double));
    for (int q = 0; q < NSTATE; q++) memset(L0->rhs[q], 0, n0 * sizeof(double));
    for (int l = 1; l < o->nlev; l++) {
        Level *F = &o->lev[l - 1], *C = &o->lev[l];
        restrict_cell(F, C, F->f[F_CN], C->f[F_CN]);
        restrict_u(F, C, F->f[F_UN], C->f[F_UN]);
        restrict_v(F, C, F->f[F_VN], C->f[F_VN]);
    }
    o->nv = 0;
    o->in_step = 1;
    o->nh = 0;
    o->acc_use = 0;
    o->acc_pending = 0;
    o->acc_last = 0.0;
    o->ncycle = 0;
}

void orc_residual(orc_ctx *o, double *r_out /* 5*m1*m2 or NULL */, double norms[5])
{
    Level *L = &o->lev[0];
    residual_level(o, L, L->r);
    norms_level(L, L->r, norms);
    if (r_out) {
        size_t n = (size_t)L->m1 * L->m2;
        for (int q = 0; q < NSTATE; q++) memcpy(r_out + q * n, L->r[q], n * sizeof(double));
    }
}

void orc_halfsweep(orc_ctx *o, int colour) { halfsweep(o, 0, colour & 1); }

/* one cycle: V-cycle, pbar mean removal and, with acceleration, from the
 * second cycle of the step on, the record of the result (a pending
 * combination that was not applied is dropped) */
void orc_vcycle(orc_ctx *o)
{
    o->acc_pending = 0;
    vcycle(o, 0);
    remove_p_mean(o);
    if (o->o.accel > 0 && o->ncycle++ > 0) {
        Level *L = &o->lev[0];
        residual_level(o, L, L->r);
        norms_level(L, L->r, o->acc_nr);
        acc_record(o, o->acc_nr);
    }
}

void orc_accelerate(orc_ctx *o) { acc_apply(o); }

/* coefficients of the pending combination; returns how many are used */
int orc_accel_coeffs(const orc_ctx *o, double g[ORC_MAXACC])
{
    for (int a = 0; a < ORC_MAXACC; a++) g[a] = o->acc_g[a];
    return o->acc_pending ? o->acc_use : 0;
}

static int state_ok(const orc_ctx *o)
{
    const Level *L = &o->lev[0];
    size_t n = (size_t)L->m1 * L->m2;
    for (size_t k = 0; k < n; k++) {
        for (int q = 0; q < NSTATE; q++)
            if (!isfinite(L->f[q][k])) return 0;
        double c = L->f[F_C][k];
        double den = (o->p.rho2 - o->p.rho1) * c + o->p.rho1;
        if (!(den > 0.0)) return 0;
    }
    return 1;
}

static void restore(orc_ctx *o)
{
    Level *L = &o->lev[0];
    size_t n = (size_t)L->m1 * L->m2;
    for (int q = 0; q < NSTATE; q++) memcpy(L->f[q], o->save[q], n * sizeof(double));
}

/* projection scheme, end of a converged step: the face fields take the
 * velocity of time n+1; the intermediate velocity is kept for the
 * dissipation */
static void project_final(orc_ctx *o)
{
    Level *L = &o->lev[0];
    size_t n = (size_t)L->m1 * L->m2;
    double *uf = zalloc(n), *vf = zalloc(n);
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            size_t k = (size_t)j * L->m1 + i;
            if (u_unknown(o, L, i)) uf[k] = creal(ufin(o, L, i, j));
            if (v_unknown(o, L, j)) vf[k] = creal(vfin(o, L, i, j));
        }
    memcpy(o->ut_save[0], L->f[F_U], n * sizeof(double));
    memcpy(o->ut_save[1], L->f[F_V], n * sizeof(double));
    memcpy(L->f[F_U], uf, n * sizeof(double));
    memcpy(L->f[F_V], vf, n * sizeof(double));
    free(uf);
    free(vf);
}

/* projection scheme: the velocity of time n+1 from the current iterate of
 * the finest level (zero on wall faces; u(i,j) on the west face of cell
 * (i,j), v(i,j) on its south face) */
void orc_velocity_np1(orc_ctx *o, double *u, double *v)
{
    Level *L = &o->lev[0];
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            size_t k = (size_t)j * L->m1 + i;
            u[k] = u_unknown(o, L, i) ? creal(ufin(o, L, i, j)) : 0.0;
            v[k] = v_unknown(o, L, j) ? creal(vfin(o, L, i, j)) : 0.0;
        }
}

int orc_solve(orc_ctx *o)
{
    double nr[NSTATE];
    orc_residual(o, NULL, nr);
    for (int e = 0; e < NSTATE; e++) o->hist[0][e] = nr[e];
    int it = 0;
    for (;;) {
        double mx = 0.0;
        for (int e = 0; e < NSTATE; e++) mx = nr[e] > mx ? nr[e] : mx;
        if (!isfinite(mx) || !state_ok(o)) { restore(o); return ORC_EDIVERGED; }
        if (mx <= o->o.tol) break;
        if (it >= o->o.max_vcycles) { restore(o); return ORC_ENOCONV; }
        if (it > 0) orc_accelerate(o);
        orc_vcycle(o);
        it++;
        if (o->o.accel > 0 && it > 1) memcpy(nr, o->acc_nr, sizeof(nr));
        else orc_residual(o, NULL, nr);
        for (int e = 0; e < NSTATE; e++) o->hist[it][e] = nr[e];
        o->nv = it;
    }
    if (projection(o)) project_final(o);
    o->in_step = 0;
    return ORC_OK;
}

int orc_step(orc_ctx *o, double dt)
{
    orc_begin_step(o, dt);
    return orc_solve(o);
}

int orc_stats(const orc_ctx *o, double *hist /* (ORC_MAXV+1)*5 */)
{
    if (hist) memcpy(hist, o->hist, sizeof(o->hist));
    return o->nv;
}

/* ------------------------------------------------------------------------- */
/* diagnostics: mass (Theorem of sec. 6.1) and discrete energy                */

void orc_mass(orc_ctx *o, double out[2])
{
    Level *L = &o->lev[0];
    double s1 = 0.0, s2 = 0.0, h2 = L->h * L->h;
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            double c = L->f[F_C][(size_t)j * L->m1 + i];
            double r = creal(rho_of(o, c));
            s1 += r * c;
            s2 += r * (1.0 - c);
        }
    out[0] = h2 * s1;
    out[1] = h2 * s2;
}

/* E_h = kinetic + gradient + bulk + potential (Theorem of sec. 6.1, App. A.7):
 *   kinetic   = 1/2 ||sqrt(rho) u||^2 = h^2/2 (sum_ew A_x rho u^2 + sum_ns A_y rho v^2)
 *   gradient  = eps eta/(2 We) ||sqrt(rho) grad_D c||^2
 *   bulk      = eta/(eps We) h^2 (rho F(c), 1)
 *   potential = (1/Fr) h^2 (rho (y - 0), 1) relative to the reference density
 * out = {E, kinetic, gradient, bulk, potential} */
void orc_energy(orc_ctx *o, double out[5])
{
    Level *L = &o->lev[0];
    double h = L->h, h2 = h * h;
    double kin = 0.0, grad = 0.0, bulk = 0.0, pot = 0.0;
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            if (u_unknown(o, L, i)) {
                double A = creal(A_xc(o, L, F_C, 1, i, j)), u = L->f[F_U][(size_t)j * L->m1 + i];
                kin += 0.5 * A * u * u;
            }
            if (v_unknown(o, L, j)) {
                double A = creal(A_yc(o, L, F_C, 1, i, j)), v = L->f[F_V][(size_t)j * L->m1 + i];
                kin += 0.5 * A * v * v;
            }
            /* gradient energy as face sums: [rho D_x c, D_x c]_ew + [rho D_y c, D_y c]_ns */
            double dx = creal(D_xc(o, L, F_C, i, j)), dy = creal(D_yc(o, L, F_C, i, j));
            if (i > 0 || o->g.bcx == ORC_PERIODIC) grad += creal(A_xc(o, L, F_C, 1, i, j)) * dx * dx;
            if (j > 0 || o->g.bcy == ORC_PERIODIC) grad += creal(A_yc(o, L, F_C, 1, i, j)) * dy * dy;
            double c = L->f[F_C][(size_t)j * L->m1 + i];
            double r = creal(rho_of(o, c));
            bulk += r * creal(Fdw(c));
            pot += (r - o->p.rho_ref) * (j + 0.5) * h;
        }
    kin *= h2;
    grad *= o->p.eps * o->p.eta / (2.0 * o->p.We) * h2;
    bulk *= o->p.eta / (o->p.eps * o->p.We) * h2;
    pot *= o->p.inv_Fr * h2;
    out[0] = kin + grad + bulk + pot;
    out[1] = kin;
    out[2] = grad;
    out[3] = bulk;
    out[4] = pot;
}

/* Dissipation of the step just taken, from the norms of App. A.7 evaluated on
 * the new iterate with the time-n coefficients (Theorem of sec. 6.1):
 *   out[0] = dt/Re ||sqrt(mu) grad_d u||^2
 *   out[1] = dt/(3Re) ||sqrt(mu) div_d u||^2
 *   out[2] = dt/(M Pe) ||sqrt(m) grad_D mu_c||^2,  mu_c = mubar + alpha pbar
 *   out[3] = 1/2 ||sqrt(rho^n)(u^{n+1} - u^n)||^2
 *   out[4] = 0
 * with the vertex inner product <phi f, g>_vc = (phi, calA(f g))_2, i.e. each
 * vertex weighted by a quarter of each adjacent interior cell.  Projection
 * scheme (Theorem of sec. 6.2): out[0], out[1], out[3] on the intermediate
 * velocity u~ in place of u^{n+1}, and
 *   out[4] = 1/2 ||sqrt(rho^{n+1})(u^{n+1} - u~)||^2  (face weights A rho(c^{n+1})). */
static void dissipation_of(orc_ctx *o, double out[4]);
void orc_dissipation(orc_ctx *o, double out[5])
{
    Level *L = &o->lev[0];
    out[4] = 0.0;
    if (!projection(o)) { dissipation_of(o, out); return; }
    double *uf = L->f[F_U], *vf = L->f[F_V];
    L->f[F_U] = o->ut_save[0];
    L->f[F_V] = o->ut_save[1];
    dissipation_of(o, out);
    L->f[F_U] = uf;
    L->f[F_V] = vf;
    double g5 = 0.0;
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            size_t k = (size_t)j * L->m1 + i;
            if (u_unknown(o, L, i)) {
                double d = uf[k] - o->ut_save[0][k];
                g5 += creal(A_xc(o, L, F_C, 1, i, j)) * d * d;
            }
            if (v_unknown(o, L, j)) {
                double d = vf[k] - o->ut_save[1][k];
                g5 += creal(A_yc(o, L, F_C, 1, i, j)) * d * d;
            }
        }
    out[4] = 0.5 * L->h * L->h * g5;
}
static void dissipation_of(orc_ctx *o, double out[4])
{
    Level *L = &o->lev[0];
    double h = L->h, h2 = h * h;
    double g1 = 0.0, g2 = 0.0, g3 = 0.0, g4 = 0.0;
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            double mu = creal(visc_n(o, L, i, j));
            double dxu = creal(d_x(o, L, F_U, i, j)), dyv = creal(d_y(o, L, F_V, i, j));
            /* cell part of ||sqrt(mu) grad_d u||^2 and ||sqrt(mu) div_d u||^2 */
            g1 += mu * (dxu * dxu + dyv * dyv);
            g2 += mu * (dxu + dyv) * (dxu + dyv);
            /* vertex parts: calA of (calD_y u)^2 and (calD_x v)^2 over the four corners */
            double s = 0.0;
            for (int a = 0; a <= 1; a++)
                for (int b = 0; b <= 1; b++) {
                    double dyu = creal(cD_y(o, L, F_U, i + a, j + b));
                    double dxv = creal(cD_x(o, L, F_V, i + a, j + b));
                    s += dyu * dyu + dxv * dxv;
                }
            g1 += mu * 0.25 * s;
            /* mobility part on faces: [m D mu_c, D mu_c] */
            if (i > 0 || o->g.bcx == ORC_PERIODIC) {
                double m = 0.5 * (creal(mob_n(o, L, i, j)) + creal(mob_n(o, L, i - 1, j)));
                double d = creal(D_xc(o, L, F_MU, i, j)) + o->alpha * creal(D_xc(o, L, F_P, i, j));
                g3 += m * d * d;
            }
            if (j > 0 || o->g.bcy == ORC_PERIODIC) {
                double m = 0.5 * (creal(mob_n(o, L, i, j)) + creal(mob_n(o, L, i, j - 1)));
                double d = creal(D_yc(o, L, F_MU, i, j)) + o->alpha * creal(D_yc(o, L, F_P, i, j));
                g3 += m * d * d;
            }
            size_t k = (size_t)j * L->m1 + i;
            if (u_unknown(o, L, i)) {
                double du = L->f[F_U][k] - L->f[F_UN][k];
                g4 += creal(A_xc(o, L, F_CN, 1, i, j)) * du * du;
            }
            if (v_unknown(o, L, j)) {
                double dv = L->f[F_V][k] - L->f[F_VN][k];
                g4 += creal(A_yc(o, L, F_CN, 1, i, j)) * dv * dv;
            }
        }
    out[0] = o->dt / o->p.Re * h2 * g1;
    out[1] = o->dt / (3.0 * o->p.Re) * h2 * g2;
    out[2] = o->dt / (o->p.M * o->p.Pe) * h2 * g3;
    out[3] = 0.5 * h2 * g4;
}

/* Physical diagnostics of the current state (sec. 8), by their definitions:
 *   out[0] rising velocity V_c = int(v c) / int(c), v at a cell centre the
 *          mean of the cell's two v faces;
 *   out[1] int(c);  out[2] max |div_d u|;  out[3] ||div_d u||_{2,h};
 *   out[4], out[5] highest and lowest height where c crosses 1/2 between two
 *          vertically adjacent cells (linear interpolation between centres;
 *          across a periodic y boundary too), NaN if none;
 *   out[6] highest such crossing in the first column, NaN if none;
 *   out[7] int(div_d u). */
void orc_diagnostics(orc_ctx *o, double out[8])
{
    Level *L = &o->lev[0];
    double h = L->h, cv = 0.0, cs = 0.0, dmax = 0.0, d2 = 0.0, dsum = 0.0;
    double top = -INFINITY, bot = INFINITY, col0 = -INFINITY;
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            double c = creal(cellv(o, L, F_C, i, j));
            double vc = 0.5 * (creal(vv(o, L, F_V, i, j)) + creal(vv(o, L, F_V, i, j + 1)));
            cv += c * vc;
            cs += c;
            double div = creal(d_x(o, L, F_U, i, j)) + creal(d_y(o, L, F_V, i, j));
            if (fabs(div) > dmax) dmax = fabs(div);
            d2 += div * div;
            dsum += div;
            if (j + 1 < L->m2 || o->g.bcy == ORC_PERIODIC) {
                double c2 = creal(cellv(o, L, F_C, i, j + 1));
                if ((c - 0.5) * (c2 - 0.5) < 0.0) {
                    double y = (j + 0.5) * h + h * (0.5 - c) / (c2 - c);
                    if (y > top) top = y;
                    if (y < bot) bot = y;
                    if (i == 0 && y > col0) col0 = y;
                }
            }
        }
    out[0] = cs != 0.0 ? cv / cs : NAN;
    out[1] = h * h * cs;
    out[2] = dmax;
    out[3] = sqrt(h * h * d2);
    out[4] = isinf(top) ? NAN : top;
    out[5] = isinf(bot) ? NAN : bot;
    out[6] = isinf(col0) ? NAN : col0;
    out[7] = h * h * dsum;
}

/* ------------------------------------------------------------------------- */
/* dense pieces for small grids and unit tests                                 */

/* number and ordering of unknowns/equations: for each cell in storage order:
 * c, mu, p, then u (if an unknown), v (if an unknown) */
static int unk_list(const orc_ctx *o, int *fld, int *ii, int *jj)
{
    const Level *L = &o->lev[0];
    int n = 0;
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            int f[5] = { F_C, F_MU, F_P, F_U, F_V };
            for (int q = 0; q < 5; q++) {
                if (q == 3 && !u_unknown(o, L, i)) continue;
                if (q == 4 && !v_unknown(o, L, j)) continue;
                if (fld) { fld[n] = f[q]; ii[n] = i; jj[n] = j; }
                n++;
            }
        }
    return n;
}

int orc_num_unknowns(const orc_ctx *o) { return unk_list(o, NULL, NULL, NULL); }

static cx res_any(orc_ctx *o, int fld, int i, int j)
{
    Level *L = &o->lev[0];
    switch (fld) {
    case F_C: return res_c(o, L, i, j);
    case F_MU: return res_mu(o, L, i, j);
    case F_P: return res_p(o, L, i, j);
    case F_U: return res_u(o, L, i, j);
    default: return res_v(o, L, i, j);
    }
}

/* N(w) as a vector in unknown order, and (optionally) its dense Jacobian by
 * complex-step columns (n*n, row-major) */
int orc_dense(orc_ctx *o, double *Nvec, double *Jmat)
{
    int n = unk_list(o, NULL, NULL, NULL);
    int *fld = malloc(n * sizeof(int)), *ii = malloc(n * sizeof(int)), *jj = malloc(n * sizeof(int));
    unk_list(o, fld, ii, jj);
    if (Nvec)
        for (int r = 0; r < n; r++) Nvec[r] = creal(res_any(o, fld[r], ii[r], jj[r]));
    if (Jmat) {
        for (int c = 0; c < n; c++) {
            perturb(o, &o->lev[0], fld[c], ii[c], jj[c]);
            for (int r = 0; r < n; r++) Jmat[(size_t)r * n + c] = cimag(res_any(o, fld[r], ii[r], jj[r])) / CSTEP;
        }
        unperturb(o);
    }
    free(fld); free(ii); free(jj);
    return n;
}

/* add a vector in unknown order to the iterate */
void orc_add_unknowns(orc_ctx *o, const double *dx)
{
    int n = unk_list(o, NULL, NULL, NULL);
    int *fld = malloc(n * sizeof(int)), *ii = malloc(n * sizeof(int)), *jj = malloc(n * sizeof(int));
    unk_list(o, fld, ii, jj);
    Level *L = &o->lev[0];
    for (int r = 0; r < n; r++) L->f[fld[r]][(size_t)jj[r] * L->m1 + ii[r]] += dx[r];
    free(fld); free(ii); free(jj);
}

/* directional derivative J(w) d of N at the current iterate of the finest
 * level, by one complex step along d (d and out: 5 fields of m1*m2, order
 * c, mu, p, u, v); entries at non-unknown faces of d are ignored */
void orc_jvp(orc_ctx *o, const double *d, double *out)
{
    Level *L = &o->lev[0];
    size_t n = (size_t)L->m1 * L->m2;
    tp.plev = L; tp.ph = CSTEP; tp.pf = -1;
    for (int q = 0; q < NSTATE; q++) tp.pdir[q] = d + q * n;
    for (int j = 0; j < L->m2; j++)
        for (int i = 0; i < L->m1; i++) {
            size_t k = (size_t)j * L->m1 + i;
            out[0 * n + k] = cimag(res_c(o, L, i, j)) / CSTEP;
            out[1 * n + k] = cimag(res_mu(o, L, i, j)) / CSTEP;
            out[2 * n + k] = cimag(res_p(o, L, i, j)) / CSTEP;
            out[3 * n + k] = u_unknown(o, L, i) ? cimag(res_u(o, L, i, j)) / CSTEP : 0.0;
            out[4 * n + k] = v_unknown(o, L, j) ? cimag(res_v(o, L, i, j)) / CSTEP : 0.0;
        }
    unperturb(o);
}

/* The grid transfers of the V-cycle between levels l and l+1, exposed for
 * unit tests.  orc_restrict: fine = 5 fields (c, mu, p, u, v) of level l,
 * packed m1_l*m2_l each; coarse = the same 5 fields of level l+1, as the
 * V-cycle restricts the iterate and the residual.  orc_prolong: fine += P e
 * for a coarse correction e (5 fields of level l+1), as the V-cycle corrects
 * the iterate; faces that are not unknowns of level l are left unchanged. */
void orc_restrict(const orc_ctx *o, int l, const double *fine, double *coarse)
{
    const Level *F = &o->lev[l], *C = &o->lev[l + 1];
    size_t nf = (size_t)F->m1 * F->m2, nc = (size_t)C->m1 * C->m2;
    double *f[NSTATE], *c[NSTATE];
    for (int q = 0; q < NSTATE; q++) { f[q] = (double *)fine + q * nf; c[q] = coarse + q * nc; }
    restrict_fields(o, F, C, f, c);
}
void orc_prolong(orc_ctx *o, int l, const double *e, double *fine)
{
    Level F = o->lev[l], C = o->lev[l + 1];
    size_t nf = (size_t)F.m1 * F.m2, nc = (size_t)C.m1 * C.m2;
    double *zero = zalloc(nc);
    for (int q = 0; q < NSTATE; q++) {
        F.f[q] = fine + q * nf;
        C.f[q] = (double *)e + q * nc;
        C.w0[q] = zero;
    }
    prolong_correct(o, &F, &C);
    free(zero);
}

/* Threads that relax the cells of one colour and evaluate residuals (the
 * cells are independent, every result is the same with any number; sums stay
 * sequential).  n <= 0 leaves the setting; returns the number in use. */
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* material laws at a pair (c1, c0), for identity checks:
 * out = {rho(c1), visc(c1), m(c1), F(c1), g(c1,c0), r(c1,c0)} */
void orc_material(const orc_ctx *o, double c1, double c0, double out[6])
{
    out[0] = creal(rho_of(o, c1));
    out[1] = creal(visc_of(o, c1));
    out[2] = creal(mob_of(o, c1));
    out[3] = creal(Fdw(c1));
    out[4] = creal(gsec(c1, c0));
    out[5] = creal(rsec(o, c1, c0));
}
