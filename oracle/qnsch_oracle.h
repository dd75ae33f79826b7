/*
 * qnsch_oracle.h -- FP64 CPU oracle of the primitive-variable q-NSCH time step.
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
 * CPU-baseline leg; never by the GPU library.  Array layout and equations are
 * described at the top of qnsch_oracle.c.
 */
#ifndef QNSCH_ORACLE_H
#define QNSCH_ORACLE_H

#define ORC_MAXLEV 12
#define ORC_MAXV 200
#define ORC_MAXACC 3

enum { ORC_WALL = 0, ORC_PERIODIC = 1 };
enum { ORC_OK = 0, ORC_ENOCONV = -3, ORC_EDIVERGED = -4 };

typedef struct {
    int m1, m2;
    double Lx, Ly;
    int bcx, bcy;
    int levels; /* 0 = automatic */
} orc_grid;

typedef struct {
    double rho1, rho2, visc1, visc2; /* fluid 1 is c = 1 */
    double Re, We, inv_Fr, Pe, M, eps, eta;
    double mob_reg; /* the constant under the square root of the mobility */
    double rho_ref; /* density the gravity term is measured against */
} orc_params;

enum { ORC_SMOOTH_SEGREGATED = 0, ORC_SMOOTH_COUPLED = 1 };
enum { ORC_PRIMITIVE = 0, ORC_PROJECTION = 1 };

typedef struct {
    double tol;
    int max_vcycles, nu1, nu2, nu_coarse; /* nu_coarse 0: automatic (4 primitive with 6 levels or more, else 6) */
    double vanka_omega;
    int smoother; /* ORC_SMOOTH_COUPLED (default) or ORC_SMOOTH_SEGREGATED; projection scheme: step 1 with or without pbar */
    int scheme;   /* ORC_PRIMITIVE (sec. 6.1) or ORC_PROJECTION (sec. 6.2) */
    double coarse_omega; /* relaxation of the velocity/pressure updates on the coarsest level;
                            0: automatic (1.75 with 4 automatic sweeps, else 1.6) */
    int accel;           /* depth (0..ORC_MAXACC) of the acceleration of the cycle iteration; 0 = off */
} orc_opts;

typedef struct orc_ctx orc_ctx;

orc_ctx *orc_create(const orc_grid *, const orc_params *, const orc_opts *);
void orc_destroy(orc_ctx *);
int orc_levels(const orc_ctx *);
void orc_set_state(orc_ctx *, const double *c, const double *mu, const double *p, const double *u, const double *v);
void orc_get_state(const orc_ctx *, double *c, double *mu, double *p, double *u, double *v);
void orc_begin_step(orc_ctx *, double dt);
void orc_residual(orc_ctx *, double *r_out, double norms[5]);
void orc_halfsweep(orc_ctx *, int colour);
void orc_vcycle(orc_ctx *);
void orc_accelerate(orc_ctx *);
int orc_accel_coeffs(const orc_ctx *, double g[ORC_MAXACC]);
int orc_solve(orc_ctx *);
int orc_step(orc_ctx *, double dt);
int orc_stats(const orc_ctx *, double *hist);
void orc_mass(orc_ctx *, double out[2]);
void orc_energy(orc_ctx *, double out[5]);
void orc_dissipation(orc_ctx *, double out[5]);
void orc_diagnostics(orc_ctx *, double out[8]);
int orc_num_unknowns(const orc_ctx *);
int orc_dense(orc_ctx *, double *Nvec, double *Jmat);
void orc_add_unknowns(orc_ctx *, const double *dx);
void orc_jvp(orc_ctx *, const double *d, double *out);
void orc_velocity_np1(orc_ctx *, double *u, double *v);
void orc_restrict(const orc_ctx *, int l, const double *fine, double *coarse);
void orc_prolong(orc_ctx *, int l, const double *e, double *fine);
int orc_threads(int n);
void orc_material(const orc_ctx *, double c1, double c0, double out[6]);

#endif
