// nrxx_api.cpp -- host side of the C ABI declared in include/nrxx.h: the
// context, the level hierarchy of Sec. 3.2.2, the V-cycle of Alg. 2, the
// mass correction of Sec. 4 and the solver loop of Sec. 3.2.3.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/nrxx.h"
#include "nrxx_host.hpp"

using namespace nrxx;

namespace {

// text of the last failed call that has no context (nrxx_create, the
// context-free entry points); a fixed buffer, so setting it allocates nothing
thread_local char g_create_error[512];

// Largest root of He_n: largest eigenvalue of the symmetric tridiagonal
// (Jacobi) matrix of the probabilists' Hermite recurrence (off-diagonal
// sqrt(k)), by Sturm-sequence bisection.
double largest_hermite_root(int n) {
  if (n <= 1) return 0.0;
  auto count_below = [n](double x) {
    int cnt = 0;
    double d = -x;
    if (d < 0) ++cnt;
    for (int k = 1; k < n; ++k) {
      if (d == 0.0) d = 1e-300;
      d = -x - (double)k / d;
      if (d < 0) ++cnt;
    }
    return cnt;
  };
  double lo = 0.0, hi = 2.0 * sqrt((double)n) + 2.0;
  for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (count_below(mid) >= n) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// J^-_{k0}(0) / k!: entering half-range of a wall Maxwellian at rest along
// the normal, (2 pi)^-1/2 int_{-inf}^0 He_k(w) w e^{-w^2/2} dw / k!.
// int_{-inf}^0 w He_k(w) e^{-w^2/2} = int_{-inf}^0 (He_{k+1} + k He_{k-1}) e^{-w^2/2},
// and int_{-inf}^0 He_m e^{-w^2/2} = (-1)^m int_0^inf He_m e^{-w^2/2}, with
// int_0^inf He_0 = sqrt(pi/2) and int_0^inf He_m = He_{m-1}(0) for m >= 1.
void wall_entering_constants(int M, double *out) {
  double h0[MMAX + 3];  // He_m(0), m <= M + 2 (fixed size: no allocation)
  h0[0] = 1.0;
  h0[1] = 0.0;
  for (int m = 1; m + 1 < M + 3; ++m) h0[m + 1] = -m * h0[m - 1];
  auto neg_half = [&](int m) {  // (2 pi)^-1/2 int_{-inf}^0 He_m e^{-w^2/2}
    double pos = m == 0 ? 0.5 : h0[m - 1] / sqrt(2.0 * M_PI);
    return (m % 2 == 0) ? pos : -pos;
  };
  double fact = 1.0;
  for (int k = 0; k <= M; ++k) {
    if (k > 0) fact *= k;
    double v = neg_half(k + 1) + (k > 0 ? k * neg_half(k - 1) : 0.0);
    out[k] = v / fact;
  }
}

}  // namespace

struct nrxx_ctx {
  nrxx_problem P;
  hipStream_t stream = nullptr;
  int M = 0, stride = 0, L = 0;
  std::vector<LevelArgs> lv;
  // per level k: Rbar (k < L-1); fbar, ftil, rhs, RH (k >= 1)
  std::vector<double *> Rbar, fbar, ftil, rhs, RH;
  double *partial = nullptr;  // per-cell scalars of the finest level
  double *dscal = nullptr;    // device scalars
  double *hscal = nullptr;    // pinned host copies
  int *derr = nullptr;
  int *dabort = nullptr;                 // abort flag of persistent sweeps
  std::vector<int *> cnt;                // per level: column progress counters
  std::vector<long long> pbase;          // per level: counter value at the next launch
  std::vector<int> persist;              // per level: 1 = static persistent sweeps
  std::vector<int> persist32;            // per level: 1 = static persistent FP32 sweeps
  // queue schedule (overlapping sweeps through the work-queue kernel), per
  // level: a one-problem table, its units and its counters
  std::vector<int> queue;                // per level: 1 = queue schedule
  std::vector<BLevel *> qtab;
  std::vector<int *> qunits, qcnt;
  int *qactive = nullptr;
  int qnw = 0, qgrid = 0, qgrid32 = 0;
  unsigned long long wait_ticks = 200000000ULL;  // bound of one cross-column wait: 2 s at 100 MHz
  // FP32 smoothing blocks (precision 1), per level: working copy g, its
  // start g0, effective right-hand side r32, FP64 defect d64
  std::vector<float *> g32, g0_32, r32;
  std::vector<double *> d64;
  double *dblk = nullptr;                // per level: block scale, reference defect norm
  double *ebuf = nullptr;                // forward Euler: -R of a level (finest-level size)
  std::string err;
  struct Timed { hipEvent_t a, b; double cells, launches; };
  std::vector<Timed> timed;                               // recorded, not yet read
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;  // read event pairs, for reuse
  double sweep_ms = 0.0, sweep_cells = 0.0, sweep_launches = 0.0;
};

namespace {

// Size of an FP32 block's unknowns' change relative to the level's first
// correction (precision 1).
constexpr double kBlockTau = 1e-2;

int fail(nrxx_ctx *c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  else snprintf(g_create_error, sizeof g_create_error, "%s", buf);
  return code;
}

int hipchk(nrxx_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return NRXX_OK;
  return fail(c, NRXX_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define CHK(expr)                                   \
  do {                                              \
    int rc_ = hipchk(c, (expr), #expr);             \
    if (rc_) return rc_;                            \
  } while (0)

bool level_ok(const nrxx_ctx *c, int level) { return c && level >= 0 && level < c->L; }

size_t level_doubles(const nrxx_ctx *c, int k) {
  return (size_t)c->lv[k].nx * c->lv[k].ny * c->stride;
}

// Read and clear the device error word; map it to a status.
int check_device(nrxx_ctx *c) {
  CHK(hipMemcpyAsync(c->hscal + 7, c->derr, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  CHK(hipStreamSynchronize(c->stream));
  int e;
  memcpy(&e, c->hscal + 7, sizeof(int));
  if (e & 4) {
    // a persistent sweep gave up waiting: counters are inconsistent, reset
    CHK(hipMemsetAsync(c->derr, 0, sizeof(int), c->stream));
    CHK(hipMemsetAsync(c->dabort, 0, sizeof(int), c->stream));
    for (int k = 0; k < c->L; ++k) {
      CHK(hipMemsetAsync(c->cnt[k], 0, sizeof(int) * c->lv[k].nx, c->stream));
      c->pbase[k] = 0;
    }
    CHK(hipStreamSynchronize(c->stream));
    return fail(c, NRXX_EHIP, "persistent sweep timed out waiting for a neighbouring column");
  }
  if (e & 1) {
    CHK(hipMemsetAsync(c->derr, 0, sizeof(int), c->stream));
    return fail(c, NRXX_ENONPHYS, "non-physical state (rho <= 0 or theta <= 0) in an update");
  }
  return NRXX_OK;
}

// Sweep timing: an event pair around each smoothing call, taken from the
// context's pool; finished pairs are read into the running totals and go
// back to the pool (every 4096 calls, and on nrxx_sweep_stats).
int timing_begin(nrxx_ctx *c, nrxx_ctx::Timed &tm) {
  if (!c->ev_free.empty()) {
    tm.a = c->ev_free.back().first;
    tm.b = c->ev_free.back().second;
    c->ev_free.pop_back();
  } else {
    CHK(hipEventCreate(&tm.a));
    if (hipEventCreate(&tm.b) != hipSuccess) {
      (void)hipEventDestroy(tm.a);
      return fail(c, NRXX_EHIP, "hipEventCreate failed");
    }
  }
  CHK(hipEventRecord(tm.a, c->stream));
  return NRXX_OK;
}

int fold_timings(nrxx_ctx *c) {
  for (auto &x : c->timed) {
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, x.a, x.b));
    c->sweep_ms += ms;
    c->sweep_cells += x.cells;
    c->sweep_launches += x.launches;
    c->ev_free.emplace_back(x.a, x.b);
  }
  c->timed.clear();
  return NRXX_OK;
}

int timing_end(nrxx_ctx *c, nrxx_ctx::Timed &tm, double cells, double launches) {
  CHK(hipEventRecord(tm.b, c->stream));
  tm.cells = cells;
  tm.launches = launches;
  c->timed.push_back(tm);
  if (c->timed.size() > 4096) {
    CHK(hipEventSynchronize(c->timed.back().b));
    return fold_timings(c);
  }
  return NRXX_OK;
}

// Directional sweeps of a level through the work-queue kernel: up to
// kMaxSweepsPerLaunch sweeps per launch, counters cleared by a fill kernel.
template <typename Real>
int queue_sweeps(nrxx_ctx *c, int level, Real *st, const Real *rhs, const std::vector<int> &dirs,
                 double *launches) {
  const LevelArgs &A = c->lv[level];
  const int ncnt = 1 + kMaxSweepsPerLaunch * A.nx;
  for (size_t s0 = 0; s0 < dirs.size(); s0 += kMaxSweepsPerLaunch) {
    const int nsw = (int)std::min<size_t>(kMaxSweepsPerLaunch, dirs.size() - s0);
    unsigned bits = 0;
    for (int q = 0; q < nsw; ++q) bits |= (unsigned)dirs[s0 + q] << (2 * q);
    CHK(launch_bfill(c->qcnt[level], ncnt, 0, c->stream));
    const int full = sizeof(Real) == 8 ? c->qgrid : c->qgrid32;
    const int grid = std::max(1, std::min(full, nsw * A.nx));
    if constexpr (sizeof(Real) == 8) {
      if (c->M > MTEAM)  // one wavefront per cell past the cell team's largest M
        CHK(launch_wsweep(c->M, A.order, grid, c->qtab[level], c->qunits[level], A.nx, nsw, bits,
                          c->qcnt[level], A.nx, c->qactive, c->derr, c->dabort, c->wait_ticks, 1,
                          c->stream, st, rhs));
      else
        CHK(launch_bsweep(c->M, A.order, c->qnw, 1, grid, c->qtab[level], c->qunits[level], A.nx,
                          nsw, bits, c->qcnt[level], A.nx, c->qactive, c->derr, c->dabort,
                          c->wait_ticks, c->stream, st, rhs));
    }
    else
      CHK(launch_bsweep32(c->M, A.order, c->qnw, grid, c->qtab[level], c->qunits[level], A.nx, nsw,
                          bits, c->qcnt[level], A.nx, c->qactive, c->derr, c->dabort, c->wait_ticks,
                          c->stream, st, rhs));
    *launches += 1.0;
  }
  return NRXX_OK;
}

int sweep_impl(nrxx_ctx *c, int level, double *st, const double *rhs, int mask, int nsteps) {
  const LevelArgs &A = c->lv[level];
  nrxx_ctx::Timed tm;
  int trc = timing_begin(c, tm);
  if (trc) return trc;
  int ndir = 0;
  std::vector<int> dirs;
  for (int s = 0; s < nsteps; ++s)
    for (int k = 0; k < 4; ++k)
      if (mask & (1 << k)) dirs.push_back(k);
  ndir = (int)dirs.size();
  double launches = 0.0;
  if (c->queue[level]) {
    int rc = queue_sweeps<double>(c, level, st, rhs, dirs, &launches);
    if (rc) return rc;
  } else if (c->persist[level]) {
    // up to 16 directional sweeps per launch (2 bits per direction)
    for (size_t s0 = 0; s0 < dirs.size(); s0 += 16) {
      const int nsw = (int)std::min<size_t>(16, dirs.size() - s0);
      unsigned bits = 0;
      for (int q = 0; q < nsw; ++q) bits |= (unsigned)dirs[s0 + q] << (2 * q);
      if (c->pbase[level] + (long long)nsw * A.ny > (1LL << 30)) {
        CHK(hipMemsetAsync(c->cnt[level], 0, sizeof(int) * A.nx, c->stream));
        c->pbase[level] = 0;
      }
      CHK(launch_sweep_persist(c->M, A, st, rhs, nsw, bits, c->cnt[level], (int)c->pbase[level],
                               c->derr, c->dabort, c->wait_ticks, c->stream));
      c->pbase[level] += (long long)nsw * A.ny;
      launches += 1.0;
    }
  } else {
    for (int k : dirs)
      for (int t = 0; t <= A.nx + A.ny - 2; ++t) {
        CHK(launch_sweep_diag(c->M, A, st, rhs, k, t, c->derr, c->stream));
        launches += 1.0;
      }
  }
  return timing_end(c, tm, (double)ndir * A.nx * A.ny, launches);
}

// One FP32 smoothing block (precision 1).  The FP64 defect d = r - R64(f0)
// is computed once; the sweeps run in FP32 on g (starting at g0 = fp32(f0))
// for the right-hand side R32(g0) + s d, and (g - g0) / s is added to the FP64
// state, which is re-expanded in FP64.  The fixed point of the FP32 sweeps
// satisfies R32(g) - R32(g0) = s d, so (g - g0) / s approximates the Newton
// correction J^-1 d; the scale s keeps g - g0 at about kBlockTau times the
// level's first correction, so neither FP32 rounding of the state nor the
// rounding noise of R32 (about 2^-24 of the flux terms) stops the FP64
// defect from falling to FP64 levels, while s d stays small enough for the
// nonlinearity of R to change the correction by only about that fraction.
int sweep32_impl(nrxx_ctx *c, int level, double *st, const double *rhs, int mask, int nsteps) {
  const LevelArgs &A = c->lv[level];
  std::vector<int> dirs;
  for (int s = 0; s < nsteps; ++s)
    for (int k = 0; k < 4; ++k)
      if (mask & (1 << k)) dirs.push_back(k);
  if (dirs.empty()) return NRXX_OK;
  nrxx_ctx::Timed tm;
  int trc = timing_begin(c, tm);
  if (trc) return trc;
  float *g = c->g32[level], *g0 = c->g0_32[level], *r = c->r32[level];
  // d = r - R64(f0) and its norm; s = block scale; s d -> g as a temporary
  // FP32 copy; r32 = R32(g0) + s d; then g = g0
  double *scale = c->dblk + 2 * level;
  CHK(launch_residual(c->M, A, st, rhs, nullptr, c->d64[level], c->partial, 0, c->stream));
  CHK(launch_block_scale(A, c->partial, kBlockTau, scale + 1, scale, c->stream));
  CHK(launch_to32(c->M, A, c->d64[level], g, nullptr, scale, c->stream));
  CHK(launch_to32(c->M, A, st, g0, nullptr, nullptr, c->stream));
  CHK(launch_fas32(c->M, A, g0, g, r, c->stream));
  CHK(launch_to32(c->M, A, st, g, nullptr, nullptr, c->stream));
  double launches = 0.0;
  if (c->queue[level]) {
    int rc = queue_sweeps<float>(c, level, g, r, dirs, &launches);
    if (rc) return rc;
  } else if (c->persist32[level]) {
    for (size_t s0 = 0; s0 < dirs.size(); s0 += 16) {
      const int nsw = (int)std::min<size_t>(16, dirs.size() - s0);
      unsigned bits = 0;
      for (int q = 0; q < nsw; ++q) bits |= (unsigned)dirs[s0 + q] << (2 * q);
      if (c->pbase[level] + (long long)nsw * A.ny > (1LL << 30)) {
        CHK(hipMemsetAsync(c->cnt[level], 0, sizeof(int) * A.nx, c->stream));
        c->pbase[level] = 0;
      }
      CHK(launch_sweep_persist32(c->M, A, g, r, nsw, bits, c->cnt[level], (int)c->pbase[level],
                                 c->derr, c->dabort, c->wait_ticks, c->stream));
      c->pbase[level] += (long long)nsw * A.ny;
      launches += 1.0;
    }
  } else {
    for (int k : dirs)
      for (int t = 0; t <= A.nx + A.ny - 2; ++t) {
        CHK(launch_sweep_diag32(c->M, A, g, r, k, t, c->derr, c->stream));
        launches += 1.0;
      }
  }
  CHK(launch_from32(c->M, A, st, g, g0, scale, c->derr, c->stream));
  return timing_end(c, tm, (double)dirs.size() * A.nx * A.ny, launches);
}

int smooth_impl(nrxx_ctx *c, int level, double *st, const double *rhs, int mask, int nsteps) {
  return c->P.precision == 1 ? sweep32_impl(c, level, st, rhs, mask, nsteps)
                             : sweep_impl(c, level, st, rhs, mask, nsteps);
}

int residual_impl(nrxx_ctx *c, int level, const double *st, const double *rhs, double *out,
                  double *norm_out) {
  const LevelArgs &A = c->lv[level];
  CHK(launch_residual(c->M, A, st, rhs, nullptr, out, norm_out ? c->partial : nullptr, 0, c->stream));
  if (norm_out) {
    CHK(launch_cell_sum(A, c->partial, 1, 0, A.inv_area, c->dscal, c->stream));
    CHK(hipMemcpyAsync(c->hscal, c->dscal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CHK(hipStreamSynchronize(c->stream));
    *norm_out = sqrt(c->hscal[0]);
  }
  return NRXX_OK;
}

int vcycle_impl(nrxx_ctx *c, int k, double *st, const double *rhs) {
  const nrxx_problem &P = c->P;
  if (k == c->L - 1) return smooth_impl(c, k, st, rhs, 15, P.s3);
  int rc = smooth_impl(c, k, st, rhs, 15, P.s1);
  if (rc) return rc;
  const LevelArgs &A = c->lv[k];
  CHK(launch_residual(c->M, A, st, rhs, nullptr, c->Rbar[k], nullptr, 0, c->stream));
  CHK(launch_restrict(c->M, A, st, c->Rbar[k], c->fbar[k + 1], c->RH[k + 1], c->derr, c->stream));
  CHK(launch_residual(c->M, c->lv[k + 1], c->fbar[k + 1], nullptr, c->RH[k + 1], c->rhs[k + 1],
                      nullptr, 1, c->stream));
  CHK(hipMemcpyAsync(c->ftil[k + 1], c->fbar[k + 1], level_doubles(c, k + 1) * sizeof(double),
                     hipMemcpyDeviceToDevice, c->stream));
  for (int g = 0; g < P.gamma; ++g) {
    rc = vcycle_impl(c, k + 1, c->ftil[k + 1], c->rhs[k + 1]);
    if (rc) return rc;
  }
  CHK(launch_correct(c->M, A, st, c->ftil[k + 1], c->fbar[k + 1], c->derr, c->stream));
  return smooth_impl(c, k, st, rhs, 15, P.s2);
}

int mass_fix_impl(nrxx_ctx *c, double *st) {
  if (!(c->P.mass0 > 0.0)) return NRXX_OK;
  const LevelArgs &A = c->lv[0];
  CHK(launch_cell_sum(A, st, c->stride, 3, A.ds, c->dscal + 1, c->stream));
  CHK(launch_mass_scale(c->M, A, st, c->dscal + 1, c->P.mass0, c->stream));
  return NRXX_OK;
}

}  // namespace

namespace nrxx {

namespace {
struct MsgBuf {
  char *p;
  size_t n;
};
bool bad(MsgBuf msg, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  if (msg.p && msg.n) vsnprintf(msg.p, msg.n, fmt, ap);
  va_end(ap);
  return false;
}
}  // namespace

int set_context_free_error(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_create_error, sizeof g_create_error, fmt, ap);
  va_end(ap);
  return code;
}

bool validate_problem(const nrxx_problem &P, std::string &msg) {
  char buf[512] = {0};
  const bool ok = validate_problem(P, buf, sizeof buf);
  if (!ok) msg = buf;
  return ok;
}

bool validate_problem(const nrxx_problem &P, char *msg_buf, size_t cap) {
  const MsgBuf msg{msg_buf, cap};
  if (P.M < MMIN || P.M > MMAX) return bad(msg, "M = %d outside [%d, %d]", P.M, MMIN, MMAX);
  if (P.levels < 1 || P.levels > 16) return bad(msg, "levels = %d", P.levels);
  if (P.nx < 1 || P.ny < 1) return bad(msg, "grid %d x %d", P.nx, P.ny);
  const int f = 1 << (P.levels - 1);
  if (P.nx % f || P.ny % f) return bad(msg, "grid %d x %d not divisible by 2^(levels-1) = %d", P.nx, P.ny, f);
  if (P.nx / f < 2 || P.ny / f < 2) return bad(msg, "coarsest grid below 2 x 2");
  if (P.collision < 0 || P.collision > 2) return bad(msg, "collision = %d", P.collision);
  if (P.collision == 2 && !(P.Pr > 0)) return bad(msg, "ES-BGK needs Pr > 0");
  if (P.order != 1 && P.order != 2) return bad(msg, "order = %d", P.order);
  if (P.limiter != 0 && P.limiter != 1) return bad(msg, "limiter = %d", P.limiter);
  if (!(P.lx > 0) || !(P.ly > 0) || !(P.Kn > 0) || !(P.cfl > 0) || !(P.beta > 0))
    return bad(msg, "lx, ly, Kn, cfl and beta must be positive");
  for (int w = 0; w < 4; ++w)
    if (!(P.wall_theta[w] > 0)) return bad(msg, "wall_theta[%d] <= 0", w);
  if (P.s1 < 0 || P.s2 < 0 || P.s3 < 0 || P.gamma < 1 || P.gamma > 2)
    return bad(msg, "bad smoothing steps or gamma");
  if (P.precision != 0 && P.precision != 1)
    return bad(msg, "precision = %d not supported", P.precision);
  if (P.schedule < 0 || P.schedule > 3) return bad(msg, "schedule = %d", P.schedule);
  if (P.M > MTEAM && P.precision != 0)
    return bad(msg, "M = %d > %d needs precision 0 (FP64 sweeps)", P.M, MTEAM);
  if (P.M > MTEAM && P.schedule != 0 && P.schedule != 3)
    return bad(msg, "M = %d > %d needs the work-queue schedule (0 or 3)", P.M, MTEAM);
  if ((long long)P.nx * P.ny > (1LL << 26)) return bad(msg, "grid too large");

  return true;
}

LevelArgs make_level(const nrxx_problem &P, int k) {
  double jm[MMAX + 1] = {0};
  wall_entering_constants(P.M, jm);
  LevelArgs A{};
  A.nx = P.nx >> k;
  A.ny = P.ny >> k;
  A.stride = record_stride(P.M);
  A.collision = P.collision;
  A.order = P.order;
  A.limiter = P.limiter;
  A.dx = P.lx / A.nx;
  A.dy = P.ly / A.ny;
  A.idx = 1.0 / A.dx;
  A.idy = 1.0 / A.dy;
  A.ds = A.dx * A.dy;
  A.inv_area = 1.0 / (P.lx * P.ly);
  A.Kn = P.Kn;
  A.Pr = P.Pr;
  A.omega = P.omega;
  A.beta = P.beta;
  A.cfl = P.cfl;
  A.nu_cap = P.nu_dt_cap;
  A.C = largest_hermite_root(P.M + 1);
  for (int w = 0; w < 4; ++w) {
    A.wall_u[w] = P.wall_u[w];
    A.wall_th[w] = P.wall_theta[w];
  }
  for (int q = 0; q <= MMAX; ++q) A.jminus[q] = jm[q];
  return A;
}

}  // namespace nrxx

extern "C" {

int32_t nrxx_record_stride(int32_t M) { return (M >= MMIN && M <= MMAX) ? record_stride(M) : -1; }

int nrxx_create(const nrxx_problem *p, void *hip_stream, nrxx_ctx **out) {
  if (!out) return fail(nullptr, NRXX_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return fail(nullptr, NRXX_EINVAL, "problem is NULL");
  const nrxx_problem &P = *p;
  {
    std::string msg;
    if (!validate_problem(P, msg)) return fail(nullptr, NRXX_EINVAL, "%s", msg.c_str());
  }
  nrxx_ctx *c = new nrxx_ctx();
  c->P = P;
  c->stream = (hipStream_t)hip_stream;
  c->M = P.M;
  c->stride = record_stride(P.M);
  c->L = P.levels;
  for (int k = 0; k < c->L; ++k) {
    LevelArgs A = make_level(P, k);
    c->lv.push_back(A);
  }
  c->Rbar.assign(c->L, nullptr);
  c->fbar.assign(c->L, nullptr);
  c->ftil.assign(c->L, nullptr);
  c->rhs.assign(c->L, nullptr);
  c->RH.assign(c->L, nullptr);
  auto alloc = [&](double **ptr, size_t n) {
    return hipMalloc((void **)ptr, n * sizeof(double)) == hipSuccess;
  };
  bool ok = true;
  for (int k = 0; k < c->L && ok; ++k) {
    const size_t n = level_doubles(c, k);
    if (k < c->L - 1) ok = ok && alloc(&c->Rbar[k], n);
    if (k >= 1) ok = ok && alloc(&c->fbar[k], n) && alloc(&c->ftil[k], n) && alloc(&c->rhs[k], n) && alloc(&c->RH[k], n);
  }
  ok = ok && alloc(&c->partial, (size_t)P.nx * P.ny) && alloc(&c->dscal, 16);
  ok = ok && hipMalloc((void **)&c->derr, sizeof(int)) == hipSuccess;
  ok = ok && hipMalloc((void **)&c->dabort, sizeof(int)) == hipSuccess;
  c->cnt.assign(c->L, nullptr);
  c->pbase.assign(c->L, 0);
  c->persist.assign(c->L, 0);
  c->persist32.assign(c->L, 0);
  c->queue.assign(c->L, 0);
  c->qtab.assign(c->L, nullptr);
  c->qunits.assign(c->L, nullptr);
  c->qcnt.assign(c->L, nullptr);
  c->g32.assign(c->L, nullptr);
  c->g0_32.assign(c->L, nullptr);
  c->r32.assign(c->L, nullptr);
  c->d64.assign(c->L, nullptr);
  if (P.precision == 1) {
    ok = ok && alloc(&c->dblk, 2 * (size_t)c->L);
    if (ok) ok = hipMemsetAsync(c->dblk, 0, sizeof(double) * 2 * c->L, c->stream) == hipSuccess;
  }
  if (P.precision == 1)
    for (int k = 0; k < c->L && ok; ++k) {
      const size_t n = level_doubles(c, k);
      ok = hipMalloc((void **)&c->g32[k], n * sizeof(float)) == hipSuccess &&
           hipMalloc((void **)&c->g0_32[k], n * sizeof(float)) == hipSuccess &&
           hipMalloc((void **)&c->r32[k], n * sizeof(float)) == hipSuccess && alloc(&c->d64[k], n);
    }
  for (int k = 0; k < c->L && ok; ++k)
    ok = hipMalloc((void **)&c->cnt[k], sizeof(int) * c->lv[k].nx) == hipSuccess;
  ok = ok && hipHostMalloc((void **)&c->hscal, 16 * sizeof(double), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    nrxx_destroy(c);
    return fail(nullptr, NRXX_ENOMEM, "device allocation failed");
  }
  bool zero_ok = hipMemsetAsync(c->derr, 0, sizeof(int), c->stream) == hipSuccess &&
                 hipMemsetAsync(c->dabort, 0, sizeof(int), c->stream) == hipSuccess;
  for (int k = 0; k < c->L && zero_ok; ++k)
    zero_ok = hipMemsetAsync(c->cnt[k], 0, sizeof(int) * c->lv[k].nx, c->stream) == hipSuccess;
  if (!zero_ok || hipStreamSynchronize(c->stream) != hipSuccess) {
    nrxx_destroy(c);
    return fail(nullptr, NRXX_EHIP, "stream unusable");
  }
  // sweep schedule per level: the work-queue kernel with overlapping
  // sweeps (automatic or 3), static persistent (one workgroup per column,
  // all resident at once; 2) or one launch per anti-diagonal (1)
  if (P.schedule == 0 || P.schedule == 3) {
    // wavefronts per cell team: one problem keeps few cells in flight, so
    // wider teams (shorter cell updates) win; at M >= 6 a team of eight
    // does not fit the LDS, and four beat two on the 256^2 M = 8 solves
    c->qnw = P.M <= 5 ? 8 : 4;
    c->qgrid = P.M > MTEAM ? wsweep_resident(P.M, P.order) : bsweep_resident(P.M, P.order, c->qnw, 1);
    c->qgrid32 = P.precision == 1 ? bsweep_resident32(P.M, P.order, c->qnw) : 1;
    bool qok = c->qgrid >= 1 && c->qgrid32 >= 1 &&
               hipMalloc((void **)&c->qactive, sizeof(int)) == hipSuccess;
    const int one = 1;
    if (qok) qok = hipMemcpy(c->qactive, &one, sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    for (int k = 0; k < c->L && qok; ++k) {
      const LevelArgs &A = c->lv[k];
      qok = hipMalloc((void **)&c->qtab[k], sizeof(BLevel)) == hipSuccess &&
            hipMalloc((void **)&c->qunits[k], sizeof(int) * A.nx) == hipSuccess &&
            hipMalloc((void **)&c->qcnt[k], sizeof(int) * (1 + kMaxSweepsPerLaunch * A.nx)) == hipSuccess;
      if (!qok) break;
      BLevel e{};
      e.A = A;
      e.cnt = c->qcnt[k] + 1;
      e.ncell = A.nx * A.ny;
      e.cont = k < c->L - 1 ? 1 : 0;
      e.mass0 = P.mass0;
      std::vector<int> u(A.nx);
      for (int p = 0; p < A.nx; ++p) u[p] = p;  // slot 0, position p
      qok = hipMemcpy(c->qtab[k], &e, sizeof(BLevel), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->qunits[k], u.data(), sizeof(int) * A.nx, hipMemcpyHostToDevice) == hipSuccess;
      c->queue[k] = 1;
    }
    if (!qok) {
      nrxx_destroy(c);
      return fail(nullptr, NRXX_ENOMEM, "queue schedule set-up failed");
    }
  }
  const bool static_ok = P.schedule == 2;
  const int maxcols = static_ok ? persist_max_columns(P.M, P.order) : 0;
  const int maxcols32 = (static_ok && P.precision == 1) ? persist_max_columns32(P.M, P.order) : 0;
  for (int k = 0; k < c->L; ++k) {
    c->persist[k] = static_ok && c->lv[k].nx <= maxcols;
    c->persist32[k] = P.precision == 1 && static_ok && c->lv[k].nx <= maxcols32;
    if (P.schedule == 2 && P.precision == 1 && !c->persist32[k]) {
      nrxx_destroy(c);
      return fail(nullptr, NRXX_EINVAL, "persistent FP32 sweeps do not fit on the device");
    }
    if (P.schedule == 2 && !c->persist[k]) {
      nrxx_destroy(c);
      return fail(nullptr, NRXX_EINVAL, "persistent sweeps need %d resident workgroups, device holds %d",
                  c->lv[k].nx, maxcols);
    }
  }
  *out = c;
  return NRXX_OK;
}

int nrxx_destroy(nrxx_ctx *c) {
  if (!c) return NRXX_OK;
  (void)hipStreamSynchronize(c->stream);
  for (auto &x : c->timed) {
    (void)hipEventDestroy(x.a);
    (void)hipEventDestroy(x.b);
  }
  for (auto &x : c->ev_free) {
    (void)hipEventDestroy(x.first);
    (void)hipEventDestroy(x.second);
  }
  for (auto *v : {&c->Rbar, &c->fbar, &c->ftil, &c->rhs, &c->RH})
    for (double *p : *v)
      if (p) (void)hipFree(p);
  if (c->partial) (void)hipFree(c->partial);
  if (c->dscal) (void)hipFree(c->dscal);
  if (c->derr) (void)hipFree(c->derr);
  if (c->dabort) (void)hipFree(c->dabort);
  for (int *p : c->cnt)
    if (p) (void)hipFree(p);
  for (auto *v : {&c->g32, &c->g0_32, &c->r32})
    for (float *p : *v)
      if (p) (void)hipFree(p);
  for (double *p : c->d64)
    if (p) (void)hipFree(p);
  if (c->dblk) (void)hipFree(c->dblk);
  if (c->ebuf) (void)hipFree(c->ebuf);
  for (auto *v : {&c->qunits, &c->qcnt})
    for (int *p : *v)
      if (p) (void)hipFree(p);
  for (BLevel *p : c->qtab)
    if (p) (void)hipFree(p);
  if (c->qactive) (void)hipFree(c->qactive);
  if (c->hscal) (void)hipHostFree(c->hscal);
  delete c;
  return NRXX_OK;
}

const char *nrxx_last_error(const nrxx_ctx *c) { return c ? c->err.c_str() : g_create_error; }

int nrxx_level_shape(const nrxx_ctx *c, int level, int32_t *nx, int32_t *ny) {
  if (!level_ok(c, level) || !nx || !ny) return NRXX_EINVAL;
  *nx = c->lv[level].nx;
  *ny = c->lv[level].ny;
  return NRXX_OK;
}

int nrxx_level_schedule(const nrxx_ctx *c, int level) {
  if (!level_ok(c, level)) return NRXX_EINVAL;
  return c->queue[level] ? 3 : c->persist[level] ? 2 : 1;
}

int nrxx_init_maxwellian(nrxx_ctx *c, int level, double *state, double rho, double u1, double u2,
                         double theta) {
  if (!c) return NRXX_EINVAL;
  if (!level_ok(c, level) || !state) return fail(c, NRXX_EINVAL, "bad level or NULL state");
  if (!(rho > 0) || !(theta > 0)) return fail(c, NRXX_EINVAL, "rho and theta must be positive");
  CHK(launch_init_maxwellian(c->M, c->lv[level], state, rho, u1, u2, theta, c->stream));
  return NRXX_OK;
}

int nrxx_residual(nrxx_ctx *c, int level, const double *state, const double *rhs, double *R_out,
                  double *norm_out) {
  if (!c) return NRXX_EINVAL;
  if (!level_ok(c, level) || !state) return fail(c, NRXX_EINVAL, "bad level or NULL state");
  int rc = residual_impl(c, level, state, rhs, R_out, norm_out);
  if (rc) return rc;
  if (norm_out) {
    rc = check_device(c);
    if (rc) return rc;
    if (!isfinite(*norm_out)) return fail(c, NRXX_EDIVERGED, "residual norm not finite");
  }
  return NRXX_OK;
}

int nrxx_sweep(nrxx_ctx *c, int level, double *state, const double *rhs, int dir_mask, int nsteps) {
  if (!c) return NRXX_EINVAL;
  if (!level_ok(c, level) || !state) return fail(c, NRXX_EINVAL, "bad level or NULL state");
  if (dir_mask < 0 || dir_mask > 15 || nsteps < 0) return fail(c, NRXX_EINVAL, "bad dir_mask or nsteps");
  return smooth_impl(c, level, state, rhs, dir_mask, nsteps);
}

int nrxx_restrict(nrxx_ctx *c, int level_fine, const double *fine, const double *fineR,
                  double *coarse, double *coarseR) {
  if (!c) return NRXX_EINVAL;
  if (!level_ok(c, level_fine) || level_fine + 1 >= c->L || !fine || !coarse)
    return fail(c, NRXX_EINVAL, "bad level or NULL buffer");
  const double *fr = (fineR && coarseR) ? fineR : nullptr;
  CHK(launch_restrict(c->M, c->lv[level_fine], fine, fr, coarse, fr ? coarseR : nullptr, c->derr, c->stream));
  return NRXX_OK;
}

int nrxx_fas_rhs(nrxx_ctx *c, int level_coarse, const double *coarse, const double *coarseR,
                 double *rhs) {
  if (!c) return NRXX_EINVAL;
  if (!level_ok(c, level_coarse) || !coarse || !coarseR || !rhs)
    return fail(c, NRXX_EINVAL, "bad level or NULL buffer");
  CHK(launch_residual(c->M, c->lv[level_coarse], coarse, nullptr, coarseR, rhs, nullptr, 1, c->stream));
  return NRXX_OK;
}

int nrxx_correct(nrxx_ctx *c, int level_fine, double *fine, const double *coarse_new,
                 const double *coarse_old) {
  if (!c) return NRXX_EINVAL;
  if (!level_ok(c, level_fine) || level_fine + 1 >= c->L || !fine || !coarse_new || !coarse_old)
    return fail(c, NRXX_EINVAL, "bad level or NULL buffer");
  CHK(launch_correct(c->M, c->lv[level_fine], fine, coarse_new, coarse_old, c->derr, c->stream));
  return NRXX_OK;
}

int nrxx_mass(nrxx_ctx *c, int level, const double *state, double *mass_out) {
  if (!c) return NRXX_EINVAL;
  if (!level_ok(c, level) || !state || !mass_out) return fail(c, NRXX_EINVAL, "bad argument");
  const LevelArgs &A = c->lv[level];
  CHK(launch_cell_sum(A, state, c->stride, 3, A.ds, c->dscal + 2, c->stream));
  CHK(hipMemcpyAsync(c->hscal + 2, c->dscal + 2, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  CHK(hipStreamSynchronize(c->stream));
  *mass_out = c->hscal[2];
  return NRXX_OK;
}

int nrxx_euler(nrxx_ctx *c, int level, double *state, int nsteps, double *dt_out) {
  if (!c) return NRXX_EINVAL;
  if (!level_ok(c, level) || !state || nsteps < 0) return fail(c, NRXX_EINVAL, "bad argument");
  if (!c->ebuf) {
    const size_t n = (size_t)c->lv[0].nx * c->lv[0].ny * c->stride;
    if (hipMalloc((void **)&c->ebuf, n * sizeof(double)) != hipSuccess) {
      c->ebuf = nullptr;
      return fail(c, NRXX_ENOMEM, "hipMalloc failed");
    }
  }
  const LevelArgs &A = c->lv[level];
  for (int k = 0; k < nsteps; ++k) {
    CHK(launch_euler_dt(c->M, A, state, c->dscal + 3, c->stream));
    CHK(launch_residual(c->M, A, state, nullptr, nullptr, c->ebuf, nullptr, 0, c->stream));
    CHK(launch_euler_update(c->M, A, state, c->ebuf, c->dscal + 3, c->derr, c->stream));
  }
  if (dt_out) {
    CHK(hipMemcpyAsync(c->hscal + 3, c->dscal + 3, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  }
  int rc = check_device(c);
  if (rc) return rc;
  if (dt_out) *dt_out = nsteps > 0 ? c->hscal[3] : 0.0;
  return NRXX_OK;
}

int nrxx_fas_vcycle(nrxx_ctx *c, double *state, double *norm_out) {
  if (!c) return NRXX_EINVAL;
  if (!state) return fail(c, NRXX_EINVAL, "NULL state");
  int rc = vcycle_impl(c, 0, state, nullptr);
  if (rc) return rc;
  rc = mass_fix_impl(c, state);
  if (rc) return rc;
  if (norm_out) {
    rc = residual_impl(c, 0, state, nullptr, nullptr, norm_out);
    if (rc) return rc;
    rc = check_device(c);
    if (rc) return rc;
    if (!isfinite(*norm_out)) return fail(c, NRXX_EDIVERGED, "residual norm not finite");
  }
  return NRXX_OK;
}

int nrxx_solve(nrxx_ctx *c, double *state, double tol, int max_cycles, double ref_norm,
               int *cycles_out, double *hist_out) {
  if (!c) return NRXX_EINVAL;
  if (!state || !cycles_out || max_cycles < 0 || !(tol >= 0))
    return fail(c, NRXX_EINVAL, "bad argument");
  // FP32 blocks: every solve takes its own first block of each level as
  // the reference of the block scale, so that equal solves are equal
  if (c->P.precision == 1)
    CHK(hipMemsetAsync(c->dblk, 0, sizeof(double) * 2 * c->L, c->stream));
  double nrm;
  int rc = residual_impl(c, 0, state, nullptr, nullptr, &nrm);
  if (rc) return rc;
  if (!(ref_norm > 0)) ref_norm = nrm;
  if (hist_out) hist_out[0] = nrm;
  int n = 0;
  *cycles_out = 0;
  while (n < max_cycles && !(nrm <= tol * ref_norm)) {
    rc = nrxx_fas_vcycle(c, state, &nrm);
    if (rc) {
      *cycles_out = n;
      return rc;
    }
    ++n;
    *cycles_out = n;
    if (hist_out) hist_out[n] = nrm;
  }
  return nrm <= tol * ref_norm ? NRXX_OK : NRXX_EMAXIT;
}

int nrxx_set_wait_limit(nrxx_ctx *c, double seconds) {
  if (!c) return NRXX_EINVAL;
  if (!(seconds >= 1e-8) || seconds > 3600.0) return fail(c, NRXX_EINVAL, "wait limit %g s", seconds);
  c->wait_ticks = (unsigned long long)(seconds * 1e8);
  return NRXX_OK;
}

int nrxx_sweep_stats(nrxx_ctx *c, double *ms_out, double *cells_out, double *launches_out,
                     int reset) {
  if (!c) return NRXX_EINVAL;
  CHK(hipStreamSynchronize(c->stream));
  int rc = fold_timings(c);
  if (rc) return rc;
  if (ms_out) *ms_out = c->sweep_ms;
  if (cells_out) *cells_out = c->sweep_cells;
  if (launches_out) *launches_out = c->sweep_launches;
  if (reset) c->sweep_ms = c->sweep_cells = c->sweep_launches = 0.0;
  return NRXX_OK;
}

int nrxx_init_fields(nrxx_ctx *c, double *state, const float *fields, int32_t fnx, int32_t fny) {
  if (!c) return NRXX_EINVAL;
  const LevelArgs &A = c->lv[0];
  if (!state || !fields || fnx < 1 || fny < 1 || A.nx % fnx || A.ny % fny)
    return fail(c, NRXX_EINVAL, "NULL buffer or field grid %d x %d does not divide %d x %d", fnx, fny,
                A.nx, A.ny);
  CHK(launch_init_fields(c->M, A, state, fields, fnx, fny, c->derr, c->stream));
  return check_device(c);
}

int nrxx_state_fields(nrxx_ctx *c, int level, const double *state, float *fields) {
  if (!c) return NRXX_EINVAL;
  if (!level_ok(c, level) || !state || !fields) return fail(c, NRXX_EINVAL, "bad level or NULL buffer");
  CHK(launch_state_fields(c->M, c->lv[level], state, fields, c->stream));
  return NRXX_OK;
}

}  // extern "C"
