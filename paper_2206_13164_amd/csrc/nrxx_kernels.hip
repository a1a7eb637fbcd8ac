// nrxx_kernels.hip -- gfx950 kernels of the NRxx steady-state solver
// (Hu & Li, arXiv 2206.13164): the finite-volume operator R_ij of eq. (13)
// evaluated per cell, the fast-sweeping cell update of Alg. 1, restriction
// (eq. (24)-(25)), coarse-grid correction (eq. (26)) and reductions.
//
// The device-side building blocks (cell team, basis change, fluxes) are in
// nrxx_device.hpp.
#include "nrxx_device.hpp"

namespace nrxx {
namespace {

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// One anti-diagonal t of sweep direction `dir` (0..3 = D1..D4 of Sec. 3.1):
// cell a of the diagonal is (a0 + blockIdx.x, t - a) in the direction's
// coordinates.  Cells of one diagonal never read each other (cross-shaped
// stencil of radius <= 2), earlier diagonals are already updated and later
// ones are not: the serial Gauss-Seidel order of Alg. 1 exactly.
template <typename Real, int M, int ORDER, int NW>
__global__ __launch_bounds__(NW * WAVE) void k_sweep_diag(LevelArgs A, Real *__restrict__ st,
                                                                const Real *__restrict__ rhs,
                                                                int dir, int t, int a0, int *err) {
  __shared__ Real lds[Lay<M, NW>::TOTAL];
  const int a = a0 + blockIdx.x, b = t - a;
  const bool irev = dir == 1 || dir == 2, jrev = dir == 2 || dir == 3;
  const int i = irev ? A.nx - 1 - a : a, j = jrev ? A.ny - 1 - b : b;
  cell_team<Real, M, ORDER, NW, MODE_SWEEP>(A, lds, st, rhs, nullptr, nullptr, nullptr, i, j, err);
}


// Persistent fast sweeping: `nsweep` directional sweeps (directions taken
// from dirs[], 2 bits each) in one launch.  Workgroup g owns grid column
// i = g and updates its cells in the order of each sweep.  Cell (i, j) of
// sweep s may start when (a) the previous column in this sweep's order has
// finished row j (so the cells before it in the serial order are final) and
// (b) the columns i-2 .. i+2 have finished row j of sweep s-1 (so nothing
// still reads the cell's old value and its stencil holds final values).
// Progress counters only grow: column i has finished base + s * ny + b + 1
// cells after row b of sweep s.  Every wait is bounded (abort flag + wall
// clock), so the grid always drains.
template <typename Real, int M, int ORDER, int NW>
__global__ __launch_bounds__(NW * WAVE) void k_sweep_persist(
    LevelArgs A, Real *__restrict__ st, const Real *__restrict__ rhs, int nsweep,
    unsigned dirs, int *cnt, int base, int *err, int *abort_flag, unsigned long long limit) {
  using L = Lay<M, NW>;
  __shared__ Real lds[L::TOTAL];
  const int i = blockIdx.x;
  const int nx = A.nx, ny = A.ny;
  // the lane's slot map, read from the constant tables once, outside the
  // loops (kept in registers only at one slot per lane; more spill)
  constexpr bool HOIST_SLOTS = G<M>::SL == 1;
  Slots<M> slots;
  slots.init(threadIdx.x % WAVE);
  for (int s = 0; s < nsweep; ++s) {
    const int dir = (dirs >> (2 * s)) & 3;
    const bool irev = dir == 1 || dir == 2, jrev = dir == 2 || dir == 3;
    const int prev = irev ? i + 1 : i - 1;
    const bool hasPrev = irev ? i < nx - 1 : i > 0;
    const int pdir = s > 0 ? (dirs >> (2 * (s - 1))) & 3 : 0;
    const bool pjrev = pdir == 2 || pdir == 3;
    const int sbase = base + s * ny;
    for (int b = 0; b < ny; ++b) {
      const int j = jrev ? ny - 1 - b : b;
      // the cross-column waits run between the team's own-column half and
      // its x-direction half (the own column is this workgroup's alone)
      auto wait = [&]() -> bool {
        bool ok = true;
        if (hasPrev) ok = wait_at_least(cnt + prev, sbase + b + 1, abort_flag, limit);
        if (ok && s > 0) {
          const int bp = pjrev ? ny - 1 - j : j;  // row j in the previous sweep's order
          for (int d = -2; d <= 2 && ok; ++d) {
            const int ii = i + d;
            if (d == 0 || ii < 0 || ii >= nx) continue;
            ok = wait_at_least(cnt + ii, sbase - ny + bp + 1, abort_flag, limit);
          }
        }
        if (ok) acquire_agent();
        return ok;
      };
      if (!cell_team<Real, M, ORDER, NW, MODE_SWEEP, true>(A, lds, st, rhs, nullptr, nullptr,
                                                           nullptr, i, j, err, wait, HOIST_SLOTS ? &slots : nullptr)) {
        if (threadIdx.x == 0) atomicOr(err, 4);
        return;  // uniform across the team
      }
      if (threadIdx.x == 0) {
        // wavefront 0 stored the cell; publish it
        publish(cnt + i, sbase + b + 1);
      }
      __syncthreads();
    }
  }
}

// Residual over all cells (MODE_DEFECT) or the coarse right-hand side
// (MODE_FAS), one team per cell.
template <typename Real, int M, int ORDER, int NW, int MODE>
__global__ __launch_bounds__(NW * WAVE) void k_residual(LevelArgs A, const Real *__restrict__ st,
                                                              const Real *__restrict__ rhs,
                                                              const Real *__restrict__ Radd,
                                                              Real *__restrict__ out,
                                                              Real *__restrict__ norm_part) {
  __shared__ Real lds[Lay<M, NW>::TOTAL];
  const int cell = blockIdx.x;
  cell_team<Real, M, ORDER, NW, MODE>(A, lds, const_cast<Real *>(st), rhs, Radd, out, norm_part,
                                cell % A.nx, cell / A.nx, nullptr);
}

template <int M>
__global__ __launch_bounds__(WAVE) void k_restrict(LevelArgs Af, const double *__restrict__ fine,
                                                   const double *__restrict__ fineR,
                                                   double *__restrict__ coarse,
                                                   double *__restrict__ coarseR, int *err) {
  __shared__ double lds[RestrictLds<M>::N];
  const int cnx = Af.nx / 2;
  restrict_cell<M>(Af, fine, fineR, coarse, coarseR, blockIdx.x % cnx, blockIdx.x / cnx,
                   blockIdx.x, lds, err);
}

template <int M>
__global__ __launch_bounds__(WAVE) void k_correct(LevelArgs Af, double *__restrict__ fine,
                                                  const double *__restrict__ cnew,
                                                  const double *__restrict__ cold, int *err) {
  __shared__ double lds[CorrectLds<M>::N];
  const int cnx = Af.nx / 2;
  correct_cell<M>(Af, fine, cnew, cold, blockIdx.x % cnx, blockIdx.x / cnx, blockIdx.x, lds, err);
}

// FP32 smoothing blocks (FP32 sweeps, FP64 defect correction).
// Working copies: g = g0 = fp32(f0) for every record entry; with `scale`,
// the coefficients (not the basis parameters) are multiplied by *scale first.
template <int M>
__global__ void k_to32(int ncell, const double *__restrict__ src, float *__restrict__ g,
                       float *__restrict__ g0, const double *__restrict__ scale) {
  using g_ = G<M>;
  const size_t tot = (size_t)ncell * g_::STRIDE;
  const double sc = scale ? *scale : 1.0;
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < tot;
       x += (size_t)gridDim.x * blockDim.x) {
    const int v = (int)(x % g_::STRIDE);
    if (v >= g_::NR) continue;
    const float y = (float)(v < 3 ? src[x] : src[x] * sc);
    g[x] = y;
    if (g0) g0[x] = y;
  }
}

// f0 <- normalise(f0 + T(g0 -> f0)[T(g -> g0) g - g0] / scale) in FP64: the
// FP32 increment of the block, formed exactly (g0 is the FP32 copy of f0),
// divided by the block's defect scale and added to the FP64 state.  One
// wavefront per cell.
template <int M>
__global__ __launch_bounds__(WAVE) void k_from32(LevelArgs A, double *__restrict__ f0,
                                                 const float *__restrict__ g,
                                                 const float *__restrict__ g0,
                                                 const double *__restrict__ scale, int *err) {
  using g_ = G<M>;
  __shared__ double lds[3 * g_::CUBE + g_::MISC];
  Wave<double, M> W;
  W.init(lds, threadIdx.x);
  const size_t off = (size_t)blockIdx.x * g_::STRIDE;
  Cell<double, M> a, b, f;
  a.u1 = g[off]; a.u2 = g[off + 1]; a.th = g[off + 2];
  b.u1 = g0[off]; b.u2 = g0[off + 1]; b.th = g0[off + 2];
#pragma unroll
  for (int r = 0; r < g_::SL; ++r) {
    a.f[r] = W.S.ok[r] ? (double)g[off + 3 + W.S.ci[r]] : 0.0;
    b.f[r] = W.S.ok[r] ? (double)g0[off + 3 + W.S.ci[r]] : 0.0;
  }
  load_cell<double, M>(f0 + off, W.S, f);
  double d[g_::SL];
  put<double, M>(W.bX, W.S, a.f);
  wsync();
  bchange<double, M>(W.bX, W.bA, W.bB, b.u1 - a.u1, b.u2 - a.u2, b.th - a.th, W.S, d);
  const double inv = 1.0 / *scale;
#pragma unroll
  for (int r = 0; r < g_::SL; ++r) d[r] = (d[r] - b.f[r]) * inv;
  double t[g_::SL];
  if (b.u1 == f.u1 && b.u2 == f.u2 && b.th == f.th) {
#pragma unroll
    for (int r = 0; r < g_::SL; ++r) t[r] = d[r];
  } else {
    put<double, M>(W.bX, W.S, d);
    wsync();
    bchange<double, M>(W.bX, W.bA, W.bB, f.u1 - b.u1, f.u2 - b.u2, f.th - b.th, W.S, t);
  }
  double fs[g_::SL];
#pragma unroll
  for (int r = 0; r < g_::SL; ++r) fs[r] = f.f[r] + t[r];
  Cell<double, M> nc;
  if (normalise<double, M>(f.u1, f.u2, f.th, fs, W, nc))
    store_record<double, M>(f0 + off, nc.u1, nc.u2, nc.th, W.bA, W.lane);
  else if (W.lane == 0)
    atomicOr(err, 1);
}

// Graded-order positions of the coefficients a Grad-type closure sets:
// 0 (000), 1 (200), 2 (020), 3 (002), 4 (110), 5 (300), 6 (120), 7 (102),
// 8 (210), 9 (030), 10 (012).
struct FieldIdx {
  int k[11];
};

// Cell records from macroscopic fields (rho, u1, u2, theta, sigma11,
// sigma12, sigma22, q1, q2) given on a coarser fnx x fny grid (injection):
// basis [u, theta], f_0 = rho, f_{e_i+e_j} = sigma_ij / (1 + delta_ij) with a
// traceless stress, f_{3e_i} = f_{e_i+2e_d} = q_i / 5, everything else 0.
// A cell whose rho or theta is not positive and finite sets bit 0 of *err.
template <int M>
__global__ void k_init_fields(int nx, int ny, double *__restrict__ st, const float *__restrict__ F,
                              int fnx, int fny, FieldIdx ix, int *err) {
  using g = G<M>;
  const size_t tot = (size_t)nx * ny * g::STRIDE;
  const int rx = nx / fnx, ry = ny / fny;
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < tot;
       x += (size_t)gridDim.x * blockDim.x) {
    const int v = (int)(x % g::STRIDE);
    if (v >= g::NR) continue;
    const int cell = (int)(x / g::STRIDE);
    const int i = cell % nx, j = cell / nx;
    const float *f = F + ((size_t)(j / ry) * fnx + i / rx) * 9;
    double val = 0.0;
    if (v < 3) {
      val = f[1 + v];
      if (v == 2 && !(val > 0.0 && isfinite(val))) atomicOr(err, 1);
    } else {
      const int a = v - 3;
      const double s11 = f[4], s12 = f[5], s22 = f[6], q1 = f[7], q2 = f[8];
      if (a == ix.k[0]) {
        val = f[0];
        if (!(val > 0.0 && isfinite(val))) atomicOr(err, 1);
      } else if (a == ix.k[1]) val = s11 / 2.0;
      else if (a == ix.k[2]) val = s22 / 2.0;
      else if (a == ix.k[3]) val = -(s11 + s22) / 2.0;
      else if (a == ix.k[4]) val = s12;
      else if (a == ix.k[5] || a == ix.k[6] || a == ix.k[7]) val = q1 / 5.0;
      else if (a == ix.k[8] || a == ix.k[9] || a == ix.k[10]) val = q2 / 5.0;
    }
    st[x] = val;
  }
}

// Macroscopic fields of every cell (eq. (10) relations): rho = f_0, u,
// theta from the basis, sigma_ij = (1 + delta_ij) f_{e_i+e_j},
// q_i = 2 f_{3e_i} + sum_d f_{2e_d+e_i}; nine floats per cell.
template <int M>
__global__ void k_state_fields(int ncell, const double *__restrict__ st, FieldIdx ix,
                               float *__restrict__ F) {
  using g = G<M>;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x) {
    const double *r = st + (size_t)c * g::STRIDE;
    const double *f = r + 3;
    float *o = F + (size_t)c * 9;
    o[0] = (float)f[ix.k[0]];
    o[1] = (float)r[0];
    o[2] = (float)r[1];
    o[3] = (float)r[2];
    o[4] = (float)(2.0 * f[ix.k[1]]);
    o[5] = (float)f[ix.k[4]];
    o[6] = (float)(2.0 * f[ix.k[2]]);
    o[7] = (float)(3.0 * f[ix.k[5]] + f[ix.k[6]] + f[ix.k[7]]);
    o[8] = (float)(3.0 * f[ix.k[9]] + f[ix.k[8]] + f[ix.k[10]]);
  }
}

template <int M>
__global__ void k_init_maxwellian(int ncell, double *__restrict__ st, double rho, double u1,
                                  double u2, double th) {
  using g = G<M>;
  const size_t tot = (size_t)ncell * g::STRIDE;
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < tot;
       x += (size_t)gridDim.x * blockDim.x) {
    const int v = (int)(x % g::STRIDE);
    if (v >= g::NR) continue;
    st[x] = v == 0 ? u1 : v == 1 ? u2 : v == 2 ? th : v == 3 ? rho : 0.0;
  }
}

// Deterministic single-block sum of scale * src[c * stride + offset] over
// all cells (fixed partition and tree order).
__global__ __launch_bounds__(1024) void k_cell_sum(int ncell, const double *__restrict__ src,
                                                   int stride, int offset, double scale,
                                                   double *__restrict__ dst) {
  __shared__ double part[1024];
  double s = 0.0;
  for (int c = threadIdx.x; c < ncell; c += 1024) s += src[(size_t)c * stride + offset];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *dst = part[0] * scale;
}

// Defect scale of an FP32 smoothing block.  `part` holds the per-cell
// weighted squares of the FP64 defect d; n = ||d|| (eq. (28)).  The first
// block on a level records dref = n; later blocks use
// scale = max(1, tau dref / n), so that the FP32 unknowns of the block move by
// about tau times the level's first correction however small d has become.
__global__ __launch_bounds__(1024) void k_block_scale(int ncell, const double *__restrict__ part,
                                                      double inv_area, double tau,
                                                      double *__restrict__ dref,
                                                      double *__restrict__ scale) {
  __shared__ double sh[1024];
  double s = 0.0;
  for (int c = threadIdx.x; c < ncell; c += 1024) s += part[c];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n = sqrt(sh[0] * inv_area);
    double r = *dref;
    if (!(r > 0.0)) {
      r = n;
      *dref = n;
    }
    double k = 1.0;
    if (n > 0.0 && r > 0.0 && isfinite(n)) k = fmax(1.0, tau * r / n);
    *scale = k;
  }
}

// Mass correction of Sec. 4: scale every coefficient by mass0 / mass.
template <int M>
__global__ void k_mass_scale(int ncell, double *__restrict__ st, const double *__restrict__ mass,
                             double mass0) {
  using g = G<M>;
  const double kappa = mass0 / *mass;
  const size_t tot = (size_t)ncell * g::STRIDE;
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < tot;
       x += (size_t)gridDim.x * blockDim.x) {
    const int v = (int)(x % g::STRIDE);
    if (v >= 3 && v < g::NR) st[x] *= kappa;
  }
}

// Forward Euler (explicit time marching, eq. (16)) with the global step of
// eq. (17): the smallest local step (eq. (18), with the relaxation cap) over
// the level's cells.  One workgroup; the minimum does not depend on the
// reduction order.
template <int M>
__global__ __launch_bounds__(1024) void k_euler_dt(LevelArgs A, const double *__restrict__ st,
                                                   double *__restrict__ dt_out) {
  using g = G<M>;
  __shared__ double part[1024];
  const int ncell = A.nx * A.ny;
  double m = INFINITY;
  for (int c = threadIdx.x; c < ncell; c += 1024) {
    const double *r = st + (size_t)c * g::STRIDE;
    const double nu = A.beta * sqrt(M_PI / 2.0) * r[3] * pow(r[2], 1.0 - A.omega) / A.Kn;
    m = fmin(m, local_dt<double>(A, r[0], r[1], r[2], nu));
  }
  part[threadIdx.x] = m;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] = fmin(part[threadIdx.x], part[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *dt_out = part[0];
}

// The Euler update of every cell from the same old state: f <- normalise(f
// + dt R(f)) (Sec. 2.4), given d = -R(f) in the cell's basis (the defect
// with a zero right-hand side).  One wavefront per cell, EW per workgroup
// (four; one above MTEAM, where the dense cubes are large); a wavefront
// without a cell returns before any wavefront-level sync.
template <int M>
struct EulerW {
  static constexpr int W = M <= MTEAM ? 4 : 1;
};
template <int M>
__global__ __launch_bounds__(EulerW<M>::W * WAVE) void k_euler_update(
    LevelArgs A, double *__restrict__ st, const double *__restrict__ d,
    const double *__restrict__ dt, int *err) {
  using g = G<M>;
  constexpr int WSZ = 3 * g::CUBE + g::MISC;
  constexpr int EW = EulerW<M>::W;
  __shared__ double lds[EW * WSZ];
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int cell = blockIdx.x * EW + wv;
  if (cell >= A.nx * A.ny) return;
  Wave<double, M> W;
  W.init(lds + wv * WSZ, lane);
  Cell<double, M> c, r;
  load_cell<double, M>(st + (size_t)cell * g::STRIDE, W.S, c);
  load_cell<double, M>(d + (size_t)cell * g::STRIDE, W.S, r);
  const double h = *dt;
  double fs[g::SL];
#pragma unroll
  for (int q = 0; q < g::SL; ++q) fs[q] = c.f[q] - h * r.f[q];
  Cell<double, M> nc;
  if (normalise<double, M>(c.u1, c.u2, c.th, fs, W, nc))
    store_record<double, M>(st + (size_t)cell * g::STRIDE, nc.u1, nc.u2, nc.th, W.bA, lane);
  else if (lane == 0)
    atomicOr(err, 1);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_euler_dt(int M, const LevelArgs &A, const double *st, double *dt_out,
                           hipStream_t s) {
  NRXX_DISPATCH_MW(M, hipLaunchKernelGGL((k_euler_dt<MM>), dim3(1), dim3(1024), 0, s, A, st, dt_out));
  return hipGetLastError();
}

hipError_t launch_euler_update(int M, const LevelArgs &A, double *st, const double *d,
                               const double *dt, int *err, hipStream_t s) {
  NRXX_DISPATCH_MW(M, {
    constexpr int EW = EulerW<MM>::W;
    const int blocks = (A.nx * A.ny + EW - 1) / EW;
    hipLaunchKernelGGL((k_euler_update<MM>), dim3(blocks), dim3(EW * WAVE), 0, s, A, st, d, dt, err);
  });
  return hipGetLastError();
}

hipError_t launch_sweep_diag(int M, const LevelArgs &A, double *st, const double *rhs, int dir,
                             int t, int *err, hipStream_t s) {
  const int a0 = t - (A.ny - 1) > 0 ? t - (A.ny - 1) : 0;
  const int a1 = t < A.nx - 1 ? t : A.nx - 1;
  const int ncell = a1 - a0 + 1;
  if (ncell <= 0) return hipSuccess;
  NRXX_DISPATCH_M(M, {
    constexpr int NW = TeamWidth<MM>::NW;
    if (A.order == 1)
      hipLaunchKernelGGL((k_sweep_diag<double, MM, 1, NW>), dim3(ncell), dim3(NW * WAVE), 0, s, A, st, rhs, dir, t, a0, err);
    else
      hipLaunchKernelGGL((k_sweep_diag<double, MM, 2, NW>), dim3(ncell), dim3(NW * WAVE), 0, s, A, st, rhs, dir, t, a0, err);
  });
  return hipGetLastError();
}

hipError_t launch_sweep_persist(int M, const LevelArgs &A, double *st, const double *rhs,
                                int nsweep, unsigned dirs, int *cnt, int base, int *err,
                                int *abort_flag, unsigned long long limit, hipStream_t s) {
  NRXX_DISPATCH_M(M, {
    constexpr int NW = TeamWidth<MM>::NW;
    if (A.order == 1)
      hipLaunchKernelGGL((k_sweep_persist<double, MM, 1, NW>), dim3(A.nx), dim3(NW * WAVE), 0, s, A, st, rhs, nsweep, dirs, cnt, base, err, abort_flag, limit);
    else
      hipLaunchKernelGGL((k_sweep_persist<double, MM, 2, NW>), dim3(A.nx), dim3(NW * WAVE), 0, s, A, st, rhs, nsweep, dirs, cnt, base, err, abort_flag, limit);
  });
  return hipGetLastError();
}

int persist_max_columns(int M, int order) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e = hipErrorInvalidValue;
  switch (M) {
#define NRXX_OCC(MM)                                                                              \
    case MM: {                                                                                    \
      constexpr int NW = TeamWidth<MM>::NW;                                                       \
      e = order == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep_persist<double, MM, 1, NW>, NW * WAVE, 0) \
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep_persist<double, MM, 2, NW>, NW * WAVE, 0); \
    } break;
    NRXX_OCC(3) NRXX_OCC(4) NRXX_OCC(5) NRXX_OCC(6) NRXX_OCC(7) NRXX_OCC(8)
#undef NRXX_OCC
    default: return 0;
  }
  if (e != hipSuccess) return 0;
  return per * ncu;
}

hipError_t launch_sweep_diag32(int M, const LevelArgs &A, float *st, const float *rhs, int dir,
                               int t, int *err, hipStream_t s) {
  const int a0 = t - (A.ny - 1) > 0 ? t - (A.ny - 1) : 0;
  const int a1 = t < A.nx - 1 ? t : A.nx - 1;
  const int ncell = a1 - a0 + 1;
  if (ncell <= 0) return hipSuccess;
  NRXX_DISPATCH_M(M, {
    constexpr int NW = TeamWidth<MM>::NW;
    if (A.order == 1)
      hipLaunchKernelGGL((k_sweep_diag<float, MM, 1, NW>), dim3(ncell), dim3(NW * WAVE), 0, s, A, st, rhs, dir, t, a0, err);
    else
      hipLaunchKernelGGL((k_sweep_diag<float, MM, 2, NW>), dim3(ncell), dim3(NW * WAVE), 0, s, A, st, rhs, dir, t, a0, err);
  });
  return hipGetLastError();
}

hipError_t launch_sweep_persist32(int M, const LevelArgs &A, float *st, const float *rhs,
                                  int nsweep, unsigned dirs, int *cnt, int base, int *err,
                                  int *abort_flag, unsigned long long limit, hipStream_t s) {
  NRXX_DISPATCH_M(M, {
    constexpr int NW = TeamWidth<MM>::NW;
    if (A.order == 1)
      hipLaunchKernelGGL((k_sweep_persist<float, MM, 1, NW>), dim3(A.nx), dim3(NW * WAVE), 0, s, A, st, rhs, nsweep, dirs, cnt, base, err, abort_flag, limit);
    else
      hipLaunchKernelGGL((k_sweep_persist<float, MM, 2, NW>), dim3(A.nx), dim3(NW * WAVE), 0, s, A, st, rhs, nsweep, dirs, cnt, base, err, abort_flag, limit);
  });
  return hipGetLastError();
}

hipError_t launch_fas32(int M, const LevelArgs &A, const float *g0, const float *d32, float *out,
                        hipStream_t s) {
  const int ncell = A.nx * A.ny;
  NRXX_DISPATCH_M(M, {
    constexpr int NW = TeamWidth<MM>::NW;
    if (A.order == 1)
      hipLaunchKernelGGL((k_residual<float, MM, 1, NW, MODE_FAS>), dim3(ncell), dim3(NW * WAVE), 0, s, A, g0, (const float *)nullptr, d32, out, (float *)nullptr);
    else
      hipLaunchKernelGGL((k_residual<float, MM, 2, NW, MODE_FAS>), dim3(ncell), dim3(NW * WAVE), 0, s, A, g0, (const float *)nullptr, d32, out, (float *)nullptr);
  });
  return hipGetLastError();
}

hipError_t launch_to32(int M, const LevelArgs &A, const double *src, float *g, float *g0,
                       const double *scale, hipStream_t s) {
  const int ncell = A.nx * A.ny;
  NRXX_DISPATCH_M(M, {
    const size_t tot = (size_t)ncell * G<MM>::STRIDE;
    int blocks = (int)((tot + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_to32<MM>), dim3(blocks), dim3(256), 0, s, ncell, src, g, g0, scale);
  });
  return hipGetLastError();
}

hipError_t launch_from32(int M, const LevelArgs &A, double *f0, const float *g, const float *g0,
                         const double *scale, int *err, hipStream_t s) {
  NRXX_DISPATCH_M(M, {
    hipLaunchKernelGGL((k_from32<MM>), dim3(A.nx * A.ny), dim3(WAVE), 0, s, A, f0, g, g0, scale, err);
  });
  return hipGetLastError();
}

int persist_max_columns32(int M, int order) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e = hipErrorInvalidValue;
  switch (M) {
#define NRXX_OCC(MM)                                                                              \
    case MM: {                                                                                    \
      constexpr int NW = TeamWidth<MM>::NW;                                                       \
      e = order == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep_persist<float, MM, 1, NW>, NW * WAVE, 0) \
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep_persist<float, MM, 2, NW>, NW * WAVE, 0); \
    } break;
    NRXX_OCC(3) NRXX_OCC(4) NRXX_OCC(5) NRXX_OCC(6) NRXX_OCC(7) NRXX_OCC(8)
#undef NRXX_OCC
    default: return 0;
  }
  if (e != hipSuccess) return 0;
  return per * ncu;
}

hipError_t launch_residual(int M, const LevelArgs &A, const double *st, const double *rhs,
                           const double *Radd, double *out, double *norm_part, int mode,
                           hipStream_t s) {
  const int ncell = A.nx * A.ny;
  if (M > MTEAM) return launch_wresidual1(M, A, st, rhs, Radd, out, norm_part, mode, s);
  NRXX_DISPATCH_M(M, {
    constexpr int NW = TeamWidth<MM>::NW;
    if (mode == 0) {
      if (A.order == 1)
        hipLaunchKernelGGL((k_residual<double, MM, 1, NW, MODE_DEFECT>), dim3(ncell), dim3(NW * WAVE), 0, s, A, st, rhs, Radd, out, norm_part);
      else
        hipLaunchKernelGGL((k_residual<double, MM, 2, NW, MODE_DEFECT>), dim3(ncell), dim3(NW * WAVE), 0, s, A, st, rhs, Radd, out, norm_part);
    } else {
      if (A.order == 1)
        hipLaunchKernelGGL((k_residual<double, MM, 1, NW, MODE_FAS>), dim3(ncell), dim3(NW * WAVE), 0, s, A, st, rhs, Radd, out, norm_part);
      else
        hipLaunchKernelGGL((k_residual<double, MM, 2, NW, MODE_FAS>), dim3(ncell), dim3(NW * WAVE), 0, s, A, st, rhs, Radd, out, norm_part);
    }
  });
  return hipGetLastError();
}

hipError_t launch_restrict(int M, const LevelArgs &Af, const double *fine, const double *fineR,
                           double *coarse, double *coarseR, int *err, hipStream_t s) {
  const int nc = (Af.nx / 2) * (Af.ny / 2);
  NRXX_DISPATCH_MW(M, {
    hipLaunchKernelGGL((k_restrict<MM>), dim3(nc), dim3(WAVE), 0, s, Af, fine, fineR, coarse, coarseR, err);
  });
  return hipGetLastError();
}

hipError_t launch_correct(int M, const LevelArgs &Af, double *fine, const double *cnew,
                          const double *cold, int *err, hipStream_t s) {
  const int nc = (Af.nx / 2) * (Af.ny / 2);
  NRXX_DISPATCH_MW(M, {
    hipLaunchKernelGGL((k_correct<MM>), dim3(nc), dim3(WAVE), 0, s, Af, fine, cnew, cold, err);
  });
  return hipGetLastError();
}

hipError_t launch_init_maxwellian(int M, const LevelArgs &A, double *st, double rho, double u1,
                                  double u2, double th, hipStream_t s) {
  const int ncell = A.nx * A.ny;
  NRXX_DISPATCH_MW(M, {
    const size_t tot = (size_t)ncell * G<MM>::STRIDE;
    int blocks = (int)((tot + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_init_maxwellian<MM>), dim3(blocks), dim3(256), 0, s, ncell, st, rho, u1, u2, th);
  });
  return hipGetLastError();
}

hipError_t launch_cell_sum(const LevelArgs &A, const double *src, int src_stride, int src_offset,
                           double scale, double *dst, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_sum, dim3(1), dim3(1024), 0, s, A.nx * A.ny, src, src_stride,
                     src_offset, scale, dst);
  return hipGetLastError();
}

hipError_t launch_block_scale(const LevelArgs &A, const double *part, double tau, double *dref,
                              double *scale, hipStream_t s) {
  hipLaunchKernelGGL(k_block_scale, dim3(1), dim3(1024), 0, s, A.nx * A.ny, part, A.inv_area, tau,
                     dref, scale);
  return hipGetLastError();
}

hipError_t launch_mass_scale(int M, const LevelArgs &A, double *st, const double *mass,
                             double mass0, hipStream_t s) {
  const int ncell = A.nx * A.ny;
  NRXX_DISPATCH_MW(M, {
    const size_t tot = (size_t)ncell * G<MM>::STRIDE;
    int blocks = (int)((tot + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_mass_scale<MM>), dim3(blocks), dim3(256), 0, s, ncell, st, mass, mass0);
  });
  return hipGetLastError();
}


namespace {
// position of alpha in the graded order (|alpha| ascending; alpha_1, then
// alpha_2 descending within a degree)
int graded_index(int a1, int a2, int a3) {
  const int n = a1 + a2 + a3;
  int pos = n * (n + 1) * (n + 2) / 6;
  for (int b1 = n; b1 > a1; --b1) pos += n - b1 + 1;
  return pos + (n - a1 - a2);
}
FieldIdx field_idx() {
  static const int A[11][3] = {{0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {3, 0, 0},
                               {1, 2, 0}, {1, 0, 2}, {2, 1, 0}, {0, 3, 0}, {0, 1, 2}};
  FieldIdx ix;
  for (int q = 0; q < 11; ++q) ix.k[q] = graded_index(A[q][0], A[q][1], A[q][2]);
  return ix;
}
}  // namespace

hipError_t launch_init_fields(int M, const LevelArgs &A, double *st, const float *fields, int fnx,
                              int fny, int *err, hipStream_t s) {
  const FieldIdx ix = field_idx();
  NRXX_DISPATCH_MW(M, {
    const size_t tot = (size_t)A.nx * A.ny * G<MM>::STRIDE;
    int blocks = (int)((tot + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_init_fields<MM>), dim3(blocks), dim3(256), 0, s, A.nx, A.ny, st, fields, fnx, fny, ix, err);
  });
  return hipGetLastError();
}

hipError_t launch_state_fields(int M, const LevelArgs &A, const double *st, float *fields,
                               hipStream_t s) {
  const FieldIdx ix = field_idx();
  const int ncell = A.nx * A.ny;
  NRXX_DISPATCH_MW(M, {
    int blocks = (ncell + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_state_fields<MM>), dim3(blocks), dim3(256), 0, s, ncell, st, ix, fields);
  });
  return hipGetLastError();
}

}  // namespace nrxx
