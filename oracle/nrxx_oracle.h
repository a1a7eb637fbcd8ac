/*
 * nrxx_oracle.h -- FP64 CPU reference ("oracle") for the steady-state NRxx
 * moment solver with fast sweeping and the FAS (nonlinear multigrid) V-cycle
 * of Hu & Li, "An efficient nonlinear multigrid solver for the simulation of
 * rarefied gas cavity flow" (arXiv 2206.13164).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a plain, slow, obviously correct implementation.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant with the HIP library.
 *
 * Data layout (oracle only): a level is an array of cell records in row-major
 * order, record (i, j) at offset (j*nx + i) * (N + 3), where N = C(M+3, 3).
 * A record is [u1, u2, theta, f_0, ..., f_{N-1}]: the Hermite basis
 * parameters (u, theta) of the expansion (u3 == 0) followed by the expansion
 * coefficients in the graded order: |alpha| = 0..M; within one degree, alpha1
 * descending, then alpha2 descending, alpha3 = rest.
 */
#ifndef NRXX_ORACLE_H
#define NRXX_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Problem description (dimensionless: m = 1, reference density and
 * temperature 1, velocities in units of sqrt(theta_0)). */
typedef struct {
  int nx, ny;           /* finest grid */
  double lx, ly;        /* domain size */
  int M;                /* expansion order, >= 3 */
  int collision;        /* 0 = BGK, 1 = Shakhov, 2 = ES-BGK */
  double Pr, Kn, omega, beta; /* nu = beta sqrt(pi/2) rho theta^(1-omega) / Kn */
  int order;            /* 1 or 2 (spatial reconstruction) */
  int limiter;          /* 0 = minmod, 1 = central slopes */
  double cfl;           /* local CFL number */
  double nu_dt_cap;     /* > 0: cap dt so that nu*dt <= nu_dt_cap; <= 0: no cap */
  double wall_u[4];     /* tangential wall speed, walls S, E, N, W */
  double wall_theta[4]; /* wall temperature, walls S, E, N, W */
  int levels, s1, s2, s3, gamma; /* multigrid: levels (finest = 0), smoothing steps, cycle index */
  double mass0;         /* > 0: total mass restored after every cycle; <= 0: no mass fix */
} orc_problem;

/* ---- index set and constants ---- */
int orc_nalpha(int M);
void orc_alpha_list(int M, int *out /* N x 3 */);
double orc_cmax(int n);   /* largest root of He_n */

/* ---- Hermite algebra (one coefficient vector) ---- */
void orc_basis_change(int M, const double *f, const double *from /*u1,u2,th*/,
                      const double *to, double *out);
void orc_xi_mult(int M, int d /*0,1,2*/, const double *f, const double *basis, double *out);
int orc_normalise(int M, double *rec /* N+3, in place */);
void orc_macro(int M, const double *rec, double *out /* rho,u1,u2,th,s11,s12,s22,s33,q1,q2,q3 */);
void orc_collision(const orc_problem *P, const double *rec, double *Q);
void orc_regularisation(int M, int d, const double *f, double du1, double du2, double dth, double *G);
void orc_wall_flux(const orc_problem *P, int wall /*0 S,1 E,2 N,3 W*/, const double *rec, double *phi);
void orc_face_flux(const orc_problem *P, int d, const double *recL, const double *recR,
                   const double *basis, double *F, double *g, double *wm, double *wp);

/* ---- level operators ---- */
void orc_level_shape(const orc_problem *P, int level, int *nx, int *ny);
int orc_cell_residual(const orc_problem *P, int level, const double *st, int i, int j, double *R);
double orc_local_dt(const orc_problem *P, int level, const double *rec);
int orc_residual(const orc_problem *P, int level, const double *st, const double *rhs,
                 double *Rbar /* r - R(f), may be NULL */, double *norm /* may be NULL */);
double orc_norm(const orc_problem *P, int level, const double *Rrec);
double orc_mass(const orc_problem *P, int level, const double *st);
int orc_sweep(const orc_problem *P, int level, double *st, const double *rhs, int dir_mask,
              int nsteps, int wavefront);
int orc_restrict(const orc_problem *P, int level_fine, const double *fine, const double *fineR,
                 double *coarse, double *coarseR);
int orc_correct(const orc_problem *P, int level_fine, double *fine, const double *coarse_new,
                const double *coarse_old);
int orc_fas_rhs(const orc_problem *P, int level_coarse, const double *coarse, const double *coarseRbar,
                double *rhs);
int orc_vcycle(const orc_problem *P, int level, double *st, const double *rhs);
int orc_mass_fix(const orc_problem *P, double *st);
int orc_solve(const orc_problem *P, double *st, double tol, int max_cycles, double ref_norm,
              int *cycles, double *hist);
int orc_euler_step(const orc_problem *P, int level, double *st, double *dt_used);
void orc_set_threads(int n);
/* 1: V-cycles sweep in anti-diagonal order (OpenMP), 0: serial order. */
void orc_set_vcycle_wavefront(int on);

#ifdef __cplusplus
}
#endif
#endif
