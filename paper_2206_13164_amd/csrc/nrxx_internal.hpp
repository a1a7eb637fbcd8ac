// nrxx_internal.hpp -- declarations shared by the HIP kernels and the host
// side of the C ABI.  Not part of the public interface (include/nrxx.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nrxx {

constexpr int MMIN = 3;
// Largest expansion order: the wavefront-per-cell kernels and the light
// per-cell kernels take M up to MMAX; the cell-team kernels (whose LDS holds
// eight dense coefficient cubes) and the FP32 blocks stop at MTEAM.
constexpr int MMAX = 10;
constexpr int MTEAM = 8;

__host__ __device__ constexpr int nalpha(int M) { return (M + 1) * (M + 2) * (M + 3) / 6; }
__host__ __device__ constexpr int record_stride(int M) { return (nalpha(M) + 3 + 7) / 8 * 8; }

// Per-level constants handed to every kernel by value.
struct LevelArgs {
  int nx, ny, stride;
  int collision, order, limiter;
  double dx, dy, idx, idy, ds, inv_area;  // cell size, its inverse, cell area, 1 / (lx ly)
  double Kn, Pr, omega, beta, cfl, nu_cap, C;  // C = largest root of He_{M+1}
  double wall_u[4], wall_th[4];                // S, E, N, W
  double jminus[MMAX + 1];                     // J^-_{k0}(0) / k!, entering wall half-range
};

// Launchers (host functions defined in nrxx_kernels.hip).  All enqueue on
// `s` and return hipSuccess or the launch error.
hipError_t launch_sweep_diag(int M, const LevelArgs &A, double *st, const double *rhs, int dir,
                             int t, int *err, hipStream_t s);
// Persistent sweeps: `nsweep` directions (2 bits each in dirs) in one launch,
// one workgroup per grid column; cnt[nx] are monotone progress counters that
// hold `base` for every column at launch; waits give up after `limit` ticks
// of the 100 MHz wall clock and set *abort_flag and bit 2 of *err.
hipError_t launch_sweep_persist(int M, const LevelArgs &A, double *st, const double *rhs,
                                int nsweep, unsigned dirs, int *cnt, int base, int *err,
                                int *abort_flag, unsigned long long limit, hipStream_t s);
// Columns (workgroups) of the persistent sweep kernel that can be resident at
// once on the current device (0 if unknown).
int persist_max_columns(int M, int order);
// FP32 smoothing blocks: sweeps on FP32 records, the effective FP32
// right-hand side R32(g0) + d32 (k_residual in MODE_FAS), conversion of the
// FP64 state to FP32 working copies and the FP64 write-back of the block's
// increment.
hipError_t launch_sweep_diag32(int M, const LevelArgs &A, float *st, const float *rhs, int dir,
                               int t, int *err, hipStream_t s);
hipError_t launch_sweep_persist32(int M, const LevelArgs &A, float *st, const float *rhs,
                                  int nsweep, unsigned dirs, int *cnt, int base, int *err,
                                  int *abort_flag, unsigned long long limit, hipStream_t s);
int persist_max_columns32(int M, int order);
hipError_t launch_fas32(int M, const LevelArgs &A, const float *g0, const float *d32, float *out,
                        hipStream_t s);
// g (and g0 if non-null) = fp32 copy of src, coefficients times *scale
// (scale == nullptr: 1)
hipError_t launch_to32(int M, const LevelArgs &A, const double *src, float *g, float *g0,
                       const double *scale, hipStream_t s);
// f0 <- normalise(f0 + (g - g0) / *scale), the difference formed in g0's basis
hipError_t launch_from32(int M, const LevelArgs &A, double *f0, const float *g, const float *g0,
                         const double *scale, int *err, hipStream_t s);
// scale = max(1, tau dref / ||d||) from the per-cell weighted squares of d;
// dref <- ||d|| when it is still zero
hipError_t launch_block_scale(const LevelArgs &A, const double *part, double tau, double *dref,
                              double *scale, hipStream_t s);
hipError_t launch_residual(int M, const LevelArgs &A, const double *st, const double *rhs,
                           const double *Radd, double *out, double *norm_part, int mode,
                           hipStream_t s);
// Forward Euler: *dt_out <- the global step (smallest local step of the
// level); st <- normalise(st - dt d) per cell, d = -R(st) in the cell basis.
hipError_t launch_euler_dt(int M, const LevelArgs &A, const double *st, double *dt_out,
                           hipStream_t s);
hipError_t launch_euler_update(int M, const LevelArgs &A, double *st, const double *d,
                               const double *dt, int *err, hipStream_t s);
hipError_t launch_restrict(int M, const LevelArgs &Afine, const double *fine, const double *fineR,
                           double *coarse, double *coarseR, int *err, hipStream_t s);
hipError_t launch_correct(int M, const LevelArgs &Afine, double *fine, const double *cnew,
                          const double *cold, int *err, hipStream_t s);
hipError_t launch_init_maxwellian(int M, const LevelArgs &A, double *st, double rho, double u1,
                                  double u2, double th, hipStream_t s);
hipError_t launch_cell_sum(const LevelArgs &A, const double *src, int src_stride, int src_offset,
                           double scale, double *dst, hipStream_t s);
hipError_t launch_mass_scale(int M, const LevelArgs &A, double *st, const double *mass,
                             double mass0, hipStream_t s);


// Records of a level from macroscopic fields on a coarser fnx x fny grid
// (injection; bit 0 of *err for rho or theta not positive), and the nine
// fields of every cell of a level.
hipError_t launch_init_fields(int M, const LevelArgs &A, double *st, const float *fields, int fnx,
                              int fny, int *err, hipStream_t s);
hipError_t launch_state_fields(int M, const LevelArgs &A, const double *st, float *fields,
                               hipStream_t s);

// ---- batched instances (nrxx_batch.hip) ------------------------------------
// One instance at one level of a group (device table entry).  Level 0 `st`
// is the caller's state; coarse `st` is f~_H.  cell0 = first cell of the
// instance in the group's cell numbering of the level (entries sorted by it).
// Problems may have different level counts: on levels a problem does not
// have, its entry has no cells (ncell = 0, nx = ny = 0, no buffers); `cont`
// is 1 where the problem continues to a coarser level (0 on its coarsest).
struct BLevel {
  LevelArgs A;
  double *st, *rhs, *Rbar, *fbar, *RH;
  int *cnt;  // nx progress counters of the sweep kernel
  int cell0, ncell, inst, cont;
  double mass0;
};
bool batch_width_ok(int M, int nw);
int batch_default_width(int M);
// Persistent work-queue sweeps: units[U] = (slot << 16 | column position),
// nsweep <= 8 sweeps (2 direction bits each in dirs).  Counters: a problem's
// entry `cnt` points at its first column's counter of sweep 0; sweep s's are
// cstride further (cstride = columns of the whole group); *queue and all
// counters must be zero at launch.
// st_ovr / rhs_ovr (non-null: a one-problem table) replace the table's
// state and right-hand side; launch_bsweep32 sweeps FP32 records that way.
constexpr int kMaxSweepsPerLaunch = 8;
// split = 1: cell team split around the cross-column waits (shorter latency);
// 0: all waits first, unsplit team (fewer registers, more teams per CU).
hipError_t launch_bsweep(int M, int order, int nw, int split, int grid, const BLevel *tab,
                         const int *units, int U, int nsweep, unsigned dirs, int *queue,
                         int cstride, const int *active, int *err, int *abort_flag,
                         unsigned long long limit, hipStream_t s, double *st_ovr = nullptr,
                         const double *rhs_ovr = nullptr);
hipError_t launch_bsweep32(int M, int order, int nw, int grid, const BLevel *tab, const int *units,
                           int U, int nsweep, unsigned dirs, int *queue, int cstride,
                           const int *active, int *err, int *abort_flag, unsigned long long limit,
                           hipStream_t s, float *st, const float *rhs);
int bsweep_resident(int M, int order, int nw, int split);
// The wavefront-per-cell form of the same work-queue sweep (nrxx_wsweep.hip):
// same units, order, counters and waits; every wavefront of a workgroup
// takes its own units.  FP64 only.
// kb: rows of a column taken per wait/acquire/release (>= 1).  st_ovr /
// rhs_ovr (non-null: a one-problem table) replace the table's state and
// right-hand side.
hipError_t launch_wsweep(int M, int order, int grid, const BLevel *tab, const int *units, int U,
                         int nsweep, unsigned dirs, int *queue, int cstride, const int *active,
                         int *err, int *abort_flag, unsigned long long limit, int kb,
                         hipStream_t s, double *st_ovr = nullptr, const double *rhs_ovr = nullptr);
// One problem's residual with one wavefront per cell (modes of
// launch_residual); used for M > MTEAM.
hipError_t launch_wresidual1(int M, const LevelArgs &A, const double *st, const double *rhs,
                             const double *Radd, double *out, double *norm_part, int mode,
                             hipStream_t s);
int wsweep_resident(int M, int order);  // workgroups resident at once (0 if unknown)
// Batched residuals with one wavefront per cell.  role 0: Rbar = rhs - R(st)
// (problems that continue to a coarser level); 1: rhs = R(fbar) + RH
// (eq. (22)); 2: partial = weighted squares (eq. (28)).  Bit-identical to the
// cell-team residual.
hipError_t launch_wresidual(int M, int order, int ncell, const BLevel *tab, int nslot,
                            const int *active, int role, double *partial, hipStream_t s);
int wsweep_wavefronts_per_group(int M);
int bsweep_resident32(int M, int order, int nw);
hipError_t launch_brestrict(int M, int ncell_coarse, const BLevel *tabF, const BLevel *tabC,
                            int nslot, const int *active, int *err, hipStream_t s);
hipError_t launch_bcopy(int M, int ncell, const BLevel *tab, int nslot, const int *active,
                        hipStream_t s);
hipError_t launch_bcorrect(int M, int ncell_coarse, const BLevel *tabF, const BLevel *tabC,
                           int nslot, const int *active, int *err, hipStream_t s);
// what 0: out[inst] = norm from partial; 1: out[inst] = mass of st
hipError_t launch_bsum(const BLevel *tab, int nslot, int stride, const int *active,
                       const double *partial, int what, double *out, hipStream_t s);
hipError_t launch_bmass_scale(int M, int ncell, const BLevel *tab, int nslot, const int *active,
                              const double *mass, hipStream_t s);
hipError_t launch_bstatus(const BLevel *tab, int nslot, const double *norms, const double *ref,
                          const double *tol, int *active, int *cycles, int *err, hipStream_t s);
hipError_t launch_bfill(int *p, int n, int v, hipStream_t s);

}  // namespace nrxx
