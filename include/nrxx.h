/*
 * nrxx.h -- C ABI of the MI355X (gfx950) steady-state solver for the
 * Boltzmann equation with BGK-type collisions in the numerical regularized
 * moment (NRxx) discretisation, with fast sweeping and the FAS nonlinear
 * multigrid V-cycle of Hu & Li, "An efficient nonlinear multigrid solver for
 * the simulation of rarefied gas cavity flow" (arXiv 2206.13164).
 *
 * Problem solved (Sec. 3, eq. (19) and (21)): on a rectangle of nx x ny
 * uniform cells, find cell distributions f_ij in F_M^[u_ij, theta_ij]
 * (Sec. 2.2, eq. (11)) with R_ij(f) = r_ij, where R_ij is the finite-volume
 * operator of eq. (13) and r = 0 on the finest level.
 *
 * ---------------------------------------------------------------------------
 * Memory layout of every per-cell object ("record"): device memory, FP64,
 * cells in row-major order (cell (i, j) = column i, row j, i fastest, row
 * j = 0 at y = 0), `nrxx_record_stride(M)` doubles per cell:
 *     [u1, u2, theta, f_0, ..., f_{N-1}, padding]
 * with N = (M+1)(M+2)(M+3)/6 coefficients in the graded order: |alpha| = 0..M;
 * within one degree alpha_1 descending, then alpha_2 descending, alpha_3 =
 * rest (so f_1, f_2, f_3 are f_{e_1}, f_{e_2}, f_{e_3}).  (u1, u2, theta) are
 * the parameters of the Hermite basis the coefficients are expressed in.
 * A state record satisfies eq. (10): f_0 = rho > 0, f_{e_i} = 0,
 * f_{2e_1} + f_{2e_2} + f_{2e_3} = 0, theta > 0.  Coefficients with odd
 * alpha_3 vanish for this two-dimensional, xi_3-even problem; the library
 * treats them as zero on input and writes zeros.  Residual and right-hand
 * side records use the same layout; their (u1, u2, theta) name the basis
 * of their coefficients.  Padding entries are never read and are left as is.
 *
 * Walls are indexed S = 0 (y = 0), E = 1 (x = lx), N = 2 (y = ly),
 * W = 3 (x = 0); all are fully diffuse (Sec. 4).
 *
 * Ownership: the caller owns every pointer passed in (state, residual and
 * right-hand-side buffers, e.g. torch tensors' data pointers).  The context
 * owns the coarse levels and scratch it allocates in nrxx_create and frees in
 * nrxx_destroy.
 *
 * Ordering: all device work is enqueued on the stream given to nrxx_create.
 * Calls that return host values (norm_out, mass_out, cycles_out, ...)
 * synchronise that stream; the others return after enqueueing.
 *
 * Errors: every call returns an nrxx_status; nothing throws.  A call given
 * invalid arguments changes nothing.  Non-physical states found by a kernel
 * (rho <= 0, theta <= 0 or non-finite values) are reported by the next call
 * that synchronises; the offending cell keeps its previous value.  The text
 * of the last error is available from nrxx_last_error.  A context is not
 * thread-safe; use one context per host thread and stream.
 * ---------------------------------------------------------------------------
 */
#ifndef NRXX_H
#define NRXX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nrxx_ctx nrxx_ctx;

typedef enum {
  NRXX_OK = 0,
  NRXX_EINVAL = -1,    /* bad argument: see nrxx_last_error */
  NRXX_ENONPHYS = -2,  /* rho <= 0 or theta <= 0 produced by an update */
  NRXX_EDIVERGED = -3, /* non-finite residual norm */
  NRXX_ENOMEM = -4,    /* device allocation failed */
  NRXX_EHIP = -5,      /* HIP runtime error */
  NRXX_EMAXIT = -6     /* nrxx_solve reached max_cycles (state is valid) */
} nrxx_status;

/* Problem description; dimensionless units (molecular mass 1, velocities in
 * sqrt(theta_0)).  Sec. 4 fixes cfl = 0.9, s1 = s2 = 2, s3 = 4, omega = 0.81,
 * beta = 1 (Shakhov and BGK), Pr = 2/3 (argon). */
typedef struct {
  int32_t nx, ny;         /* finest grid; both divisible by 2^(levels-1) */
  double lx, ly;          /* domain size */
  int32_t M;              /* expansion order, 3 <= M <= 10; M > 8 runs FP64 (precision 0)
                             with the work-queue schedule (0 or 3) only */
  int32_t collision;      /* 0 = BGK (eq. (6)), 1 = Shakhov (eq. (8)), 2 = ES-BGK (eq. (7):
                             Gaussian of covariance theta I + (1 - 1/Pr) sigma / rho; Sec. 4
                             takes beta = Pr for it) */
  double Pr, Kn, omega, beta; /* nu = beta sqrt(pi/2) rho theta^(1-omega) / Kn, eq. (29) */
  int32_t order;          /* 1 or 2: spatial reconstruction, eq. (15) */
  int32_t limiter;        /* order 2 only: 0 = minmod, 1 = central slopes */
  double cfl;             /* CFL number of eq. (18) */
  double nu_dt_cap;       /* > 0: the local step also obeys nu*dt <= nu_dt_cap */
  double wall_u[4];       /* tangential wall speed (x for S/N, y for E/W) */
  double wall_theta[4];   /* wall temperature */
  int32_t levels;         /* multigrid levels K+1; level 0 = finest, levels-1 = coarsest */
  int32_t s1, s2, s3;     /* pre-, post-smoothing and coarsest FS steps (Alg. 2) */
  int32_t gamma;          /* 1 = V-cycle, 2 = W-cycle */
  double mass0;           /* > 0: total mass restored after every cycle (Sec. 4); <= 0: off */
  int32_t precision;      /* 0 = FP64 throughout.  1 = FP32 smoothing blocks with FP64 defect
                             correction: each block computes d = r - R(f) in FP64, runs its
                             fast-sweeping steps in FP32 on the scaled problem
                             R32(g) = R32(g0) + s d (g0 = fp32(f), s >= 1 chosen so that g - g0
                             stays near 1e-2 of the level's first correction), and adds
                             (g - g0) / s to f in FP64; residuals, restriction, coarse
                             right-hand sides, corrections and the mass fix stay FP64, so the
                             fixed point is the FP64 steady state.  Other values: NRXX_EINVAL. */
  int32_t schedule;       /* sweep schedule (all give the serial Gauss-Seidel result bit for bit):
                             0 = automatic (= 3), 1 = one launch per anti-diagonal,
                             2 = static persistent: one workgroup per grid column, all resident
                                 at once (NRXX_EINVAL if the device cannot hold them),
                             3 = work queue: persistent workgroups take (column, sweep) units in
                                 dependency order; consecutive sweeps overlap, each cell waiting
                                 only for its own stencil in the previous sweep */
} nrxx_problem;

/* Doubles per cell record for order M (N + 3 rounded up to a multiple of 8). */
int32_t nrxx_record_stride(int32_t M);

/* Create a context for `p` whose work is enqueued on `hip_stream` (a
 * hipStream_t, NULL = the null stream).  Validates `p` (NRXX_EINVAL), builds
 * the level hierarchy of Sec. 3.2.2 (coarse cell (I,J) = fine cells 2I..2I+1
 * x 2J..2J+1) and allocates coarse levels and scratch (NRXX_ENOMEM).  On
 * success *out is a new context; on failure *out is NULL. */
int nrxx_create(const nrxx_problem *p, void *hip_stream, nrxx_ctx **out);

/* Synchronise and free everything the context owns.  NULL is accepted. */
int nrxx_destroy(nrxx_ctx *ctx);

/* Text of the last error of this context ("" if none); valid until the next
 * call on the context.  NULL gives the text of the last failed nrxx_create. */
const char *nrxx_last_error(const nrxx_ctx *ctx);

/* Cells of `level` (0 = finest). */
int nrxx_level_shape(const nrxx_ctx *ctx, int level, int32_t *nx, int32_t *ny);

/* Sweep schedule used on `level`: 1 = one launch per anti-diagonal,
 * 2 = static persistent, 3 = work queue (see nrxx_problem.schedule).  All
 * give the serial Gauss-Seidel result.  Negative: NRXX_EINVAL. */
int nrxx_level_schedule(const nrxx_ctx *ctx, int level);

/* Fill `state` (a level-`level` record array) with the global Maxwellian of
 * density rho, velocity (u1, u2) and temperature theta (Sec. 4.1). */
int nrxx_init_maxwellian(nrxx_ctx *ctx, int level, double *state, double rho, double u1,
                         double u2, double theta);

/* Defect of eq. (21)/(22) on `level`: R_out = r - R(f) per cell, expressed in
 * the cell's current basis (Alg. 2, line "compute the fine grid residual"),
 * with r projected from its own basis into the cell's.  rhs == NULL means
 * r = 0.  R_out may be NULL.  If norm_out != NULL, writes the weighted L2
 * norm of eq. (28) (per-cell weight alpha! theta^-|alpha|, area weighted,
 * divided by lx*ly) and synchronises. */
int nrxx_residual(nrxx_ctx *ctx, int level, const double *state, const double *rhs,
                  double *R_out, double *norm_out);

/* `nsteps` steps of the fast sweeping iteration, Alg. 1, in place on `state`
 * (level `level`), for the right-hand side `rhs` (NULL: r = 0).  dir_mask bit
 * k enables sweep direction D(k+1) of Sec. 3.1 (15 = the full step
 * D1, D2, D3, D4).  Each cell update uses the local step of eq. (18) from the
 * cell's current state, f <- f + dt (R_ij(f) - r_ij), then re-expands the
 * cell in its new (u, theta) (Sec. 2.4).  The result equals the serial
 * cell-by-cell order of the paper exactly: cells are updated along the
 * anti-diagonals of each direction's order.  With precision 1 the call is one
 * FP32 smoothing block of `nsteps` steps (see nrxx_problem.precision); the
 * block's scale reference is the defect of the context's first block on that
 * level. */
int nrxx_sweep(nrxx_ctx *ctx, int level, double *state, const double *rhs, int dir_mask, int nsteps);

/* Restriction of Sec. 3.2.2: from level `level_fine` to level_fine + 1.
 * (u_H, theta_H) by conservation of mass, momentum and energy (eq. (24)),
 * coefficients averaged after projection into that basis (eq. (25)).  If
 * fineR and coarseR are both non-NULL the residual records are restricted
 * into the same basis. */
int nrxx_restrict(nrxx_ctx *ctx, int level_fine, const double *fine, const double *fineR,
                  double *coarse, double *coarseR);

/* Coarse right-hand side of eq. (22): rhs = R_H(coarse) + coarseR, stored in
 * the basis of `coarse` (level `level_coarse`). */
int nrxx_fas_rhs(nrxx_ctx *ctx, int level_coarse, const double *coarse, const double *coarseR,
                 double *rhs);

/* Coarse-grid correction with injection as prolongation, eq. (26): each fine
 * cell of level `level_fine` gets f + T(coarse_new - coarse_old) projected
 * into its basis and re-expanded.  A cell that would become non-physical
 * keeps its value. */
int nrxx_correct(nrxx_ctx *ctx, int level_fine, double *fine, const double *coarse_new,
                 const double *coarse_old);

/* Total mass sum_ij rho_ij dx dy of `state` (synchronises). */
int nrxx_mass(nrxx_ctx *ctx, int level, const double *state, double *mass_out);

/* Explicit time marching (Sec. 2.4), the baseline fast sweeping and NMG are
 * compared with (Sec. 3, 4): `nsteps` forward Euler
 * steps of eq. (16) on level `level` with r = 0, each with the global time
 * step of eq. (17) (the smallest local step of eq. (18) over the level, with
 * the relaxation cap of the problem): every cell is updated from the same old
 * state, f <- normalise(f + dt R(f)).  `state` (device, the level's records)
 * is updated in place.  dt_out (host, may be NULL) gets the step of the last
 * step (0 when nsteps = 0).  Allocates one level-sized scratch buffer on the
 * first call (owned by the context).  Synchronises; NRXX_ENONPHYS if an
 * update made a cell non-physical (the state is then partly updated). */
int nrxx_euler(nrxx_ctx *ctx, int level, double *state, int nsteps, double *dt_out);

/* One NMG iteration NMG_K(f, 0) of Alg. 2 on the finest-level `state`
 * (gamma recursive calls, s1/s2 smoothing, s3 coarsest steps), followed by
 * the mass correction of Sec. 4 when mass0 > 0.  If norm_out != NULL, writes
 * ||R(f)|| of the result (eq. (28)) and synchronises. */
int nrxx_fas_vcycle(nrxx_ctx *ctx, double *state, double *norm_out);

/* NMG solver of Sec. 3.2.3: repeat nrxx_fas_vcycle until
 * ||R(f)|| <= tol * ref_norm (eq. (28)); ref_norm <= 0 means the norm of the
 * input state.  Writes the number of cycles to *cycles_out and, if hist_out is
 * non-NULL (max_cycles + 1 doubles), the norm history (entry 0 = input).
 * Returns NRXX_OK on convergence, NRXX_EMAXIT if max_cycles was reached. */
int nrxx_solve(nrxx_ctx *ctx, double *state, double tol, int max_cycles, double ref_norm,
               int *cycles_out, double *hist_out);

/* Cumulative device time (ms, from HIP events recorded around each group of
 * sweep kernels), the number of cell updates and the number of sweep kernel
 * launches since the context was created or last reset; any output may be
 * NULL; `reset` != 0 zeroes the counts after reading.  Synchronises. */
int nrxx_sweep_stats(nrxx_ctx *ctx, double *ms_out, double *cell_updates_out,
                     double *launches_out, int reset);

/* Bound (seconds, 1e-8 .. 3600; default 2) on any single wait of a
 * persistent sweep kernel for a neighbouring column.  A wait that exceeds it
 * makes every workgroup of the launch give up, so the kernel always ends; the
 * next synchronising call returns NRXX_EHIP and the state then holds a
 * partially completed sweep.  The context stays usable. */
int nrxx_set_wait_limit(nrxx_ctx *ctx, double seconds);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the defect
 * and norm of nrxx_residual without a context.  `p` describes the problem
 * (validated as by nrxx_create: NRXX_EINVAL), `level` selects its level
 * (0 = finest); state, rhs (NULL: r = 0) and R_out (may be NULL) are device
 * record arrays of that level, owned by the caller, in the layout above.
 * Results equal nrxx_residual's on a context of `p`, bit for bit.
 * norm_dev (device, one double, may be NULL) receives the eq. (28) norm
 * without synchronising; norm_host (host, may be NULL) receives it after
 * the call synchronises the stream.  Work is enqueued on hip_stream
 * (a hipStream_t, NULL = the null stream).
 * The call allocates nothing: the per-cell scratch of the norm lives in a
 * fixed device array of the library, NRXX_NOALLOC_MAX_CELLS + 64 doubles
 * (2 MiB) per GPU, held by each GPU it runs on until the process ends; a
 * norm of a level with more cells is refused (NRXX_EINVAL).  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (different
 * streams or host threads) race and must be serialised by the caller.
 * Errors: text via nrxx_last_error(NULL). */
#define NRXX_NOALLOC_MAX_CELLS 262144
int nrxx_residual_noalloc(const nrxx_problem *p, int32_t level, const double *state,
                          const double *rhs, double *R_out, double *norm_dev, double *norm_host,
                          void *hip_stream);

/* ---------------------------------------------------------------------------
 * Batches: many independent problems solved together on one device.
 *
 * A batch holds n problem descriptions that share s1, s2, s3 and gamma
 * (precision must be 0); grids, level counts, M, order, Kn, walls,
 * collision model and Pr may differ (a problem takes its s3 coarsest steps on
 * its own coarsest level while the others recurse further).  Problems with the same (M, order) form a group; each
 * group runs its V-cycles on a stream of its own (created by the batch, at
 * the default priority), with persistent work-queue sweep kernels whose
 * units are (problem, grid column, sweep direction): every cell is updated in
 * the serial order of Alg. 1, so each problem's result is bitwise the one
 * nrxx_sweep / nrxx_fas_vcycle give for it alone.  Each problem stops
 * independently when its residual norm (eq. (28)) falls to tol times its
 * initial norm; converged problems are masked off on the device.
 *
 * `states` arguments are host arrays of n device pointers, problem i's
 * finest-level record array (layout of the single-problem calls); the caller
 * owns them.  Calls are enqueued on the batch streams and synchronise with
 * the stream given to nrxx_batch_create before returning.
 * ------------------------------------------------------------------------- */
typedef struct nrxx_batch nrxx_batch;

/* Execution choice of one group (see nrxx_batch_autotune). */
typedef struct {
  int32_t M, order;      /* the group (read only) */
  int32_t problems;      /* problems in the group (read only) */
  int32_t team_width;    /* wavefronts per cell team: 8 (M <= 5 only), 4, 2 or 1 */
  int32_t grid;          /* persistent sweep workgroups (>= 1) */
  int32_t unit_order;    /* 0: units ordered by column position, then problem;
                            1: by problem (largest first), then column position */
  int32_t split;         /* 1: each cell team evaluates its own-column terms before the waits
                            on neighbouring columns (shorter latency); 0: waits first, then an
                            unsplit team (fewer registers, more teams per CU) */
  double block_ms;       /* last autotune: time of one s1-step block on level 0 */
  int32_t kernel;        /* 0: cell-team sweep kernel (team_width wavefronts per cell, split);
                            1: wavefront-per-cell sweep kernel (each wavefront updates the cells
                            of its own units alone: longer latency per cell, many more cells in
                            flight per CU; team_width and split are ignored).  Both give the
                            same results bit for bit. */
  int32_t rows_per_sync; /* kernel 1: rows of a column updated per set of waits on neighbouring
                            columns and per acquire/release (>= 1; larger: fewer cache
                            invalidations, later start of the downstream column) */
} nrxx_batch_tuning;

/* Validates every problem as nrxx_create does, plus the shared fields; builds
 * the groups, their level tables and coarse levels.  Initial tuning: the
 * default team width, every resident workgroup, unit_order 0. */
int nrxx_batch_create(const nrxx_problem *problems, int32_t n, void *hip_stream,
                      nrxx_batch **out);
int nrxx_batch_destroy(nrxx_batch *b);
const char *nrxx_batch_last_error(const nrxx_batch *b);
int nrxx_batch_groups(const nrxx_batch *b);
int nrxx_batch_get_tuning(const nrxx_batch *b, int group, nrxx_batch_tuning *out);
/* Sets kernel, team_width, split, grid and unit_order of a group (NRXX_EINVAL if
 * invalid). */
int nrxx_batch_set_tuning(nrxx_batch *b, int group, const nrxx_batch_tuning *t);
/* Times every candidate (cell-team kernel: split x team width x grid {all
 * resident, half} x unit order; wavefront-per-cell kernel with rows_per_sync 1:
 * grid x unit order)
 * on one s1-step smoothing block of the finest level of `states`, keeps the
 * fastest per group; then, with two or more groups (which run at once and
 * share the device), times one NMG iteration of all groups at once for each
 * combination of per-group grids of 1, 3/4, 1/2 and 1/4 times the group's
 * choice (up to 64 combinations, else one group at a time), times the four
 * fastest three more times interleaved with the own grids, and keeps the
 * lowest median if it beats the own grids' median by at least 1.5 %.
 * Restores `states` bit for bit. */
int nrxx_batch_autotune(nrxx_batch *b, double *const *states);
/* Global Maxwellian in every problem. */
int nrxx_batch_init_maxwellian(nrxx_batch *b, double *const *states, double rho, double u1,
                               double u2, double theta);
/* Residual norm of eq. (28) of every problem (norms_out: n doubles). */
int nrxx_batch_residual_norms(nrxx_batch *b, double *const *states, double *norms_out);
/* `nsteps` fast-sweeping steps (all four directions) on every problem's
 * finest level, r = 0 (as nrxx_sweep with dir_mask 15). */
int nrxx_batch_sweep(nrxx_batch *b, double *const *states, int nsteps);
/* One NMG iteration (Alg. 2 + mass fix) on every problem, as
 * nrxx_fas_vcycle; norms_out (n doubles, may be NULL) gets the new norms. */
int nrxx_batch_vcycle(nrxx_batch *b, double *const *states, double *norms_out);
/* Solve every problem to ||R|| <= tol * ||R(initial)|| or max_cycles
 * V-cycles.  use_graph != 0 replays each group's cycle from a HIP graph
 * captured on first use (re-captured after a tuning change).  Outputs (n
 * each, may be NULL): cycles taken, final and initial norms.  NRXX_OK when
 * every problem converged, NRXX_EMAXIT otherwise (states valid). */
int nrxx_batch_solve(nrxx_batch *b, double *const *states, double tol, int32_t max_cycles,
                     int32_t use_graph, int32_t *cycles_out, double *norms_out, double *ref_out);
/* As nrxx_set_wait_limit, for the batch's sweep kernels (drops captured
 * graphs). */
int nrxx_batch_set_wait_limit(nrxx_batch *b, double seconds);
/* Device time (ms) of the batch's V-cycles and the cell updates their sweeps
 * made since creation or the last reset. */
int nrxx_batch_stats(nrxx_batch *b, double *ms_out, double *cell_updates_out, int reset);
/* on = 1: record a HIP event pair on the group's stream around every sweep
 * kernel launch enqueued directly (captured graphs carry no timing events:
 * time with use_graph = 0); 0: off (default).  Autotuning is never timed. */
int nrxx_batch_set_timing(nrxx_batch *b, int32_t on);
/* Sweep-kernel statistics of one group while timing is on, since the last
 * reset: summed launch durations (ms), launches, and the cell updates those
 * launches made on the finest level and on coarse levels (problems masked
 * off by convergence are not counted).  Groups run concurrently on their
 * own streams, so durations of different groups overlap in time. */
int nrxx_batch_kernel_stats(nrxx_batch *b, int32_t group, double *ms_out, double *launches_out,
                            double *cell_updates_fine_out, double *cell_updates_coarse_out,
                            int32_t reset);

/* ---------------------------------------------------------------------------
 * Warm start from macroscopic fields, and the warm-start network.
 * ------------------------------------------------------------------------- */

/* Fill the finest-level `state` from macroscopic fields given on an
 * fnx x fny grid that divides the finest grid (each cell takes the fields of
 * the field cell it lies in).  fields: device, fny x fnx x 9 floats,
 * (rho, u1, u2, theta, sigma11, sigma12, sigma22, q1, q2) per cell; the
 * record is the Grad-type closure in the basis [u, theta]: f_0 = rho,
 * f_{e_i+e_j} = sigma_ij / (1 + delta_ij) with sigma33 = -(sigma11 +
 * sigma22), f_{3e_i} = f_{e_i+2e_d} = q_i / 5 (d != i), all else 0, which
 * reproduces rho, u, theta, sigma and q (eq. (10) relations).  Synchronises;
 * NRXX_ENONPHYS if some rho or theta is not positive (the state is then
 * unusable and the caller should start from a Maxwellian). */
int nrxx_init_fields(nrxx_ctx *ctx, double *state, const float *fields, int32_t fnx, int32_t fny);

/* The nine fields above for every cell of `state` on `level` (device output,
 * ny x nx x 9 floats): rho = f_0, (u, theta) of the basis,
 * sigma_ij = (1 + delta_ij) f_{e_i+e_j}, q_i = 2 f_{3e_i} + sum_d f_{2e_d+e_i}. */
int nrxx_state_fields(nrxx_ctx *ctx, int level, const double *state, float *fields);

/* A fully connected network y = L_n(s(... s(L_1(x)))) with affine layers L_k
 * (W_k: widths[k+1] x widths[k], b_k), SiLU s(z) = z / (1 + e^-z), inputs
 * standardised ((x - in_mean) / in_std) and outputs de-standardised
 * (y * out_std + out_mean).  Products use BF16 operands with FP32
 * accumulation on the matrix cores; weights keep FP32 masters.  Training
 * minimises the mean over rows and outputs of the squared error in
 * standardised output units with Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * X, Y, T are device row-major float arrays (rows x widths[0], rows x
 * widths[n]); parameters on the host are, per layer, W row-major then b. */
typedef struct nrxx_mlp nrxx_mlp;
int nrxx_mlp_create(const int32_t *widths, int32_t nlayers, int32_t max_rows, void *hip_stream,
                    nrxx_mlp **out);
int nrxx_mlp_destroy(nrxx_mlp *m);
const char *nrxx_mlp_last_error(const nrxx_mlp *m);
int64_t nrxx_mlp_param_count(const nrxx_mlp *m);
/* Loads parameters (host floats) and resets the optimiser state. */
int nrxx_mlp_set_params(nrxx_mlp *m, const float *params);
int nrxx_mlp_get_params(const nrxx_mlp *m, float *params);
/* Host arrays of widths[0] and widths[n] floats; standard deviations > 0. */
int nrxx_mlp_set_scaling(nrxx_mlp *m, const float *in_mean, const float *in_std,
                         const float *out_mean, const float *out_std);
int nrxx_mlp_forward(nrxx_mlp *m, const float *X, int32_t rows, float *Y);
/* Gradients of the loss on (X, T) with respect to every parameter, written
 * to host `grads` in the parameter layout; loss_out (may be NULL) gets the
 * loss.  Synchronises. */
int nrxx_mlp_gradients(nrxx_mlp *m, const float *X, const float *T, int32_t rows, float *grads,
                       double *loss_out);
/* One Adam step of learning rate lr on the batch (X, T); loss_out (may be
 * NULL; synchronises if not) gets the loss before the step. */
int nrxx_mlp_train_step(nrxx_mlp *m, const float *X, const float *T, int32_t rows, float lr,
                        double *loss_out);

#ifdef __cplusplus
}
#endif
#endif
