// nrxx_batch.hip -- gfx950 kernels that run many independent cavity problems
// ("instances") of one expansion order and spatial order together.
//
// A group of instances shares M and the spatial order; grids, Kn, walls,
// collision model and Pr may differ.  Every instance at every level is one
// entry of a device table (BLevel): its constants, its buffers and its place
// in the group's cell numbering.  Cell-parallel kernels (residual, FAS
// right-hand side, restriction, correction, mass fix) run one workgroup per
// cell of the whole group and find their instance by a binary search over the
// table.  Converged instances are masked off by a per-instance flag that the
// kernels read, so a captured V-cycle needs no host decisions.
//
// The sweep kernel is persistent with a work queue.  A unit is one grid
// column of one instance in one directional sweep; units are ordered by
// (sweep, position of the column in the sweep's order, table slot) or by
// (sweep, slot, position), and workgroups take them in that order from an
// atomic counter.  A unit only waits for units earlier in the order (the
// previous column in the same sweep, and the neighbouring columns and the
// column itself in the previous sweep), and a unit is taken only by a running
// workgroup, so the waits always end however many workgroups are resident.
// Each cell is updated by the same cell team as the single-problem kernels,
// in the same serial Gauss-Seidel order of Alg. 1.  (The batched residuals
// run one wavefront per cell: nrxx_wsweep.hip.)
#include "nrxx_device.hpp"

namespace nrxx {
namespace {


// Copies a problem's level constants into LDS once per workgroup: the cell
// team reads them many times, and reading them through the table in global
// memory puts a dependent scalar load on every use.
__device__ __forceinline__ void stage_args(const LevelArgs &src, LevelArgs &dst) {
  constexpr int n = (int)(sizeof(LevelArgs) / sizeof(uint32_t));
  const uint32_t *s = reinterpret_cast<const uint32_t *>(&src);
  uint32_t *d = reinterpret_cast<uint32_t *>(&dst);
  for (int x = threadIdx.x; x < n; x += blockDim.x) d[x] = s[x];
  __syncthreads();
}

// Progress counters: cnt[s * cstride + c] = rows of column c finished in
// sweep s of this launch (zero at launch).  Cell (i, j) of sweep s waits for
//  (own) rows j-2 .. j+2 of its own column finished in sweep s-1: its own
//        stencil holds their final values and nothing still reads its old one
//        -- the column's previous sweep may still be running in another
//        workgroup, so consecutive sweeps overlap instead of waiting for
//        whole columns;
//  (up)  the previous column of sweep s finished row j;
//  (nb)  columns i-2 .. i+2 finished row j in sweep s-1.
// These are exactly the serial order's requirements for a radius-2
// cross-shaped stencil.  The own-column wait comes first (the team then reads
// its own column), the others between the two halves of the cell team.
// With st_ovr non-null (one problem, the single-problem library), its state
// and right-hand side replace the table's pointers; this is also how FP32
// records (Real = float) are swept.  SPLIT = false takes all waits of a cell
// (one acquire) before an unsplit cell team: longer per-cell latency, but a
// much smaller register footprint, so more teams fit on a CU -- the better
// trade when many problems supply independent columns.
template <typename Real, int M, int ORDER, int NW, bool SPLIT>
__global__ __launch_bounds__(NW * WAVE) void k_bsweep(const BLevel *__restrict__ tab,
                                                      const int *__restrict__ units, int U,
                                                      int nsweep, unsigned dirs, int *queue,
                                                      int cstride, const int *__restrict__ active,
                                                      int *err, int *abort_flag,
                                                      unsigned long long limit, Real *st_ovr,
                                                      const Real *rhs_ovr) {
  using L = Lay<M, NW>;
  __shared__ Real lds[L::TOTAL];
  __shared__ int su;
  __shared__ int sknown;  // rows of the own column known finished in sweep s-1
  __shared__ LevelArgs sA;
  Real *sc = lds + L::S;
  const int total = nsweep * U;
  // the lane's slot map, read from the constant tables once: inside the
  // loops every cell would re-read them from memory after its acquire (kept
  // in registers only at one slot per lane; more spill)
  constexpr bool HOIST_SLOTS = G<M>::SL == 1;
  Slots<M> slots;
  slots.init(threadIdx.x % WAVE);
  for (;;) {
    if (threadIdx.x == 0) {
      int u = atomicAdd(queue, 1);
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) u = total;
      su = u;
      sknown = 0;
    }
    __syncthreads();
    const int u = su;
    __syncthreads();
    if (u >= total) return;
    const int s = u / U, e = units[u % U];
    const int slot = e >> 16, p = e & 0xffff;
    const BLevel &B = tab[slot];
    if (!active[B.inst]) continue;
    stage_args(B.A, sA);
    Real *const st = st_ovr ? st_ovr : reinterpret_cast<Real *>(B.st);
    const Real *const rhs = st_ovr ? rhs_ovr : reinterpret_cast<const Real *>(B.rhs);
    const int nx = sA.nx, ny = sA.ny;
    int *cs = B.cnt + s * cstride;                 // this sweep's counters
    int *cp = s > 0 ? cs - cstride : nullptr;      // previous sweep's
    const int dir = (dirs >> (2 * s)) & 3;
    const bool irev = dir == 1 || dir == 2, jrev = dir == 2 || dir == 3;
    const int i = irev ? nx - 1 - p : p;
    const int prev = irev ? i + 1 : i - 1;
    const int pdir = s > 0 ? (dirs >> (2 * (s - 1))) & 3 : 0;
    const bool pjrev = pdir == 2 || pdir == 3;
    for (int b = 0; b < ny; ++b) {
      const int j = jrev ? ny - 1 - b : b;
      if (!SPLIT) {
        if (threadIdx.x == 0) {
          bool ok = true;
          if (s > 0) {
            const int need = pjrev ? ny - (j - 2 > 0 ? j - 2 : 0) : (j + 2 < ny - 1 ? j + 2 : ny - 1) + 1;
            ok = wait_at_least(cp + i, need, abort_flag, limit);
            const int bp = pjrev ? ny - 1 - j : j;
            for (int d = -2; d <= 2 && ok; ++d) {
              const int ii = i + d;
              if (d == 0 || ii < 0 || ii >= nx) continue;
              ok = wait_at_least(cp + ii, bp + 1, abort_flag, limit);
            }
          }
          if (ok && p > 0) ok = wait_at_least(cs + prev, b + 1, abort_flag, limit);
          if (ok) acquire_agent();
          sc[L::SAB] = ok ? Real(0.0) : Real(1.0);
        }
        __syncthreads();
        if (sc[L::SAB] != Real(0.0)) {
          if (threadIdx.x == 0) atomicOr(err, 4);
          return;  // uniform across the team
        }
        cell_team<Real, M, ORDER, NW, MODE_SWEEP>(sA, lds, st, rhs, nullptr, nullptr, nullptr, i, j,
                                                  err, NoWait(), HOIST_SLOTS ? &slots : nullptr);
        if (threadIdx.x == 0)
          publish(cs + i, b + 1);  // wavefront 0 stored the cell
        __syncthreads();
        continue;
      }
      if (s > 0) {
        // rows j - 2 .. j + 2 of the own column.  sknown changes only after
        // the barrier below and is read again only after the row's last
        // barrier, so the test is uniform and a row whose rows are already
        // known takes no barrier and no acquire.
        const int need = pjrev ? ny - (j - 2 > 0 ? j - 2 : 0) : (j + 2 < ny - 1 ? j + 2 : ny - 1) + 1;
        if (sknown < need) {
          int seen = need;
          if (threadIdx.x == 0) {
            const bool ok = wait_at_least(cp + i, need, abort_flag, limit, &seen);
            if (ok) acquire_agent();
            sc[L::SAB] = ok ? Real(0.0) : Real(1.0);
          }
          __syncthreads();
          if (sc[L::SAB] != Real(0.0)) {
            if (threadIdx.x == 0) atomicOr(err, 4);
            return;  // uniform across the team
          }
          if (threadIdx.x == 0) sknown = seen;
        }
      }
      auto wait = [&]() -> bool {
        bool ok = true;
        if (p > 0) ok = wait_at_least(cs + prev, b + 1, abort_flag, limit);
        if (ok && s > 0) {
          const int bp = pjrev ? ny - 1 - j : j;
          for (int d = -2; d <= 2 && ok; ++d) {
            const int ii = i + d;
            if (d == 0 || ii < 0 || ii >= nx) continue;
            ok = wait_at_least(cp + ii, bp + 1, abort_flag, limit);
          }
        }
        if (ok) acquire_agent();
        return ok;
      };
      if (!cell_team<Real, M, ORDER, NW, MODE_SWEEP, true>(sA, lds, st, rhs, nullptr, nullptr,
                                                           nullptr, i, j, err, wait, HOIST_SLOTS ? &slots : nullptr)) {
        if (threadIdx.x == 0) atomicOr(err, 4);
        return;  // uniform across the team
      }
      if (threadIdx.x == 0)
        publish(cs + i, b + 1);  // wavefront 0 stored the cell
      __syncthreads();
    }
  }
}

// Restriction of level k (tabF) into level k+1 (tabC), one wavefront per
// coarse cell of the group.
template <int M>
__global__ __launch_bounds__(WAVE) void k_brestrict(const BLevel *__restrict__ tabF,
                                                    const BLevel *__restrict__ tabC, int nslot,
                                                    const int *__restrict__ active, int *err) {
  __shared__ double lds[RestrictLds<M>::N];
  const int slot = find_slot(tabC, nslot, blockIdx.x);
  const BLevel &C = tabC[slot], &F = tabF[slot];
  if (!active[C.inst]) return;
  const int cell = blockIdx.x - C.cell0;
  restrict_cell<M>(F.A, F.st, F.Rbar, C.fbar, C.RH, cell % C.A.nx, cell / C.A.nx, cell, lds, err);
}

// Coarse state f~_H = f-bar_H before the coarse cycle.
template <int M>
__global__ __launch_bounds__(WAVE) void k_bcopy(const BLevel *__restrict__ tab, int nslot,
                                                const int *__restrict__ active) {
  const int slot = find_slot(tab, nslot, blockIdx.x);
  const BLevel &B = tab[slot];
  if (!active[B.inst]) return;
  const size_t off = (size_t)(blockIdx.x - B.cell0) * G<M>::STRIDE;
  for (int v = threadIdx.x; v < G<M>::NR; v += WAVE) B.st[off + v] = B.fbar[off + v];
}

// Coarse-grid correction of level k (tabF) from level k+1 (tabC), eq. (26).
template <int M>
__global__ __launch_bounds__(WAVE) void k_bcorrect(const BLevel *__restrict__ tabF,
                                                   const BLevel *__restrict__ tabC, int nslot,
                                                   const int *__restrict__ active, int *err) {
  __shared__ double lds[CorrectLds<M>::N];
  const int slot = find_slot(tabC, nslot, blockIdx.x);
  const BLevel &C = tabC[slot], &F = tabF[slot];
  if (!active[C.inst]) return;
  const int cell = blockIdx.x - C.cell0;
  correct_cell<M>(F.A, F.st, C.st, C.fbar, cell % C.A.nx, cell / C.A.nx, cell, lds, err);
}

// Per-instance sums over the instance's cells, one workgroup per slot, in
// the summation order of the single-problem reduction (k_cell_sum):
// what = 0: norms[inst] = sqrt(sum partial * inv_area) (eq. (28));
// what = 1: mass[inst] = sum rho * ds.
__global__ __launch_bounds__(1024) void k_bsum(const BLevel *__restrict__ tab, int stride,
                                               const int *__restrict__ active,
                                               const double *__restrict__ partial, int what,
                                               double *__restrict__ out) {
  __shared__ double sh[1024];
  const BLevel &B = tab[blockIdx.x];
  if (!active[B.inst]) return;
  double s = 0.0;
  for (int c = threadIdx.x; c < B.ncell; c += 1024)
    s += what == 0 ? partial[B.cell0 + c] : B.st[(size_t)c * stride + 3];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[B.inst] = what == 0 ? sqrt(sh[0] * B.A.inv_area) : sh[0] * B.A.ds;
}

// Mass correction of Sec. 4 per instance (mass0 > 0): coefficients times
// mass0 / mass.  One wavefront per cell of the group.
template <int M>
__global__ __launch_bounds__(WAVE) void k_bmass_scale(const BLevel *__restrict__ tab, int nslot,
                                                      const int *__restrict__ active,
                                                      const double *__restrict__ mass) {
  const int slot = find_slot(tab, nslot, blockIdx.x);
  const BLevel &B = tab[slot];
  if (!active[B.inst] || !(B.mass0 > 0.0)) return;
  const double kappa = B.mass0 / mass[B.inst];
  const size_t off = (size_t)(blockIdx.x - B.cell0) * G<M>::STRIDE;
  for (int v = 3 + threadIdx.x; v < G<M>::NR; v += WAVE) B.st[off + v] *= kappa;
}

// After a cycle: count it for every instance that took part, then keep an
// instance active while its norm is above tol * ref (a non-finite norm stops
// the instance and sets bit 3 of *err).
__global__ void k_bstatus(const BLevel *__restrict__ tab, int nslot,
                          const double *__restrict__ norms, const double *__restrict__ ref,
                          const double *__restrict__ tol, int *active, int *cycles, int *err) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslot) return;
  const int inst = tab[slot].inst;
  if (!active[inst]) return;
  cycles[inst] += 1;
  const double n = norms[inst];
  if (!isfinite(n)) {
    active[inst] = 0;
    atomicOr(err, 8);
    return;
  }
  active[inst] = n > *tol * ref[inst] ? 1 : 0;
}

__global__ void k_bfill(int *p, int n, int v) {
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) p[x] = v;
}

}  // namespace

// Team widths the batched sweep is built for: 8, 4, 2, 1 wavefronts per cell
// at M <= 5 and 4, 2, 1 at M >= 6 (the LDS of an 8-wavefront team at M >= 6
// is too large).  Fewer wavefronts per cell means a longer per-cell latency
// but more cells in flight per CU, which pays when many problems supply
// independent columns.
bool batch_width_ok(int M, int nw) {
  if (M < MMIN || M > MTEAM) return false;
  return nw == 4 || nw == 2 || nw == 1 || (nw == 8 && M <= 5);
}

int batch_default_width(int M) { return M <= 5 ? 8 : 4; }

#define NRXX_BSWEEP(MM, OO, NWV)                                                                   \
  do {                                                                                             \
    if (split)                                                                                     \
      hipLaunchKernelGGL((k_bsweep<Real, MM, OO, NWV, true>), dim3(grid), dim3(NWV * WAVE), 0, s,  \
                         tab, units, U, nsweep, dirs, queue, cstride, active, err, abort_flag,    \
                         limit, st_ovr, rhs_ovr);                                                  \
    else if constexpr (sizeof(Real) == 8)                                                          \
      hipLaunchKernelGGL((k_bsweep<Real, MM, OO, NWV, false>), dim3(grid), dim3(NWV * WAVE), 0, s, \
                         tab, units, U, nsweep, dirs, queue, cstride, active, err, abort_flag,    \
                         limit, st_ovr, rhs_ovr);                                                  \
  } while (0)
#define NRXX_BSWEEP_W(MM, OO)                   \
  switch (nw) {                                 \
    case 1: NRXX_BSWEEP(MM, OO, 1); break;      \
    case 2: NRXX_BSWEEP(MM, OO, 2); break;      \
    case 4: NRXX_BSWEEP(MM, OO, 4); break;      \
    default: NRXX_BSWEEP(MM, OO, BigW<MM>::W);  \
  }

namespace {
// the widest team of order M (8 at M <= 5; at M >= 6 nw = 8 is refused
// before dispatch and this instance aliases width 4)
template <int M>
struct BigW {
  static constexpr int W = M <= 5 ? 8 : 4;
};

template <typename Real, int M, int ORDER, bool SP>
int occupancy_of(int nw, int *per) {
  hipError_t e;
  switch (nw) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_bsweep<Real, M, ORDER, 1, SP>, WAVE, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_bsweep<Real, M, ORDER, 2, SP>, 2 * WAVE, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_bsweep<Real, M, ORDER, 4, SP>, 4 * WAVE, 0); break;
    default:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_bsweep<Real, M, ORDER, BigW<M>::W, SP>,
                                                       BigW<M>::W * WAVE, 0);
  }
  return e == hipSuccess ? 0 : -1;
}

template <typename Real>
hipError_t launch_bsweep_t(int M, int order, int nw, int split, int grid, const BLevel *tab,
                           const int *units, int U, int nsweep, unsigned dirs, int *queue,
                           int cstride, const int *active, int *err, int *abort_flag,
                           unsigned long long limit, hipStream_t s, Real *st_ovr,
                           const Real *rhs_ovr) {
  if (!batch_width_ok(M, nw) || grid < 1 || (!split && sizeof(Real) != 8))
    return hipErrorInvalidValue;
  NRXX_DISPATCH_M(M, {
    if (order == 1) {
      NRXX_BSWEEP_W(MM, 1);
    } else {
      NRXX_BSWEEP_W(MM, 2);
    }
  });
  return hipGetLastError();
}

template <typename Real, bool SP>
int resident_t(int M, int order, int nw) {
  int dev = 0, ncu = 0, per = 0;
  if (!batch_width_ok(M, nw)) return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  int rc = -1;
  switch (M) {
#define NRXX_OCC(MM) \
    case MM: rc = order == 1 ? occupancy_of<Real, MM, 1, SP>(nw, &per) : occupancy_of<Real, MM, 2, SP>(nw, &per); break;
    NRXX_OCC(3) NRXX_OCC(4) NRXX_OCC(5) NRXX_OCC(6) NRXX_OCC(7) NRXX_OCC(8)
#undef NRXX_OCC
    default: return 0;
  }
  if (rc) return 0;
  return per * ncu;
}
}  // namespace
#undef NRXX_BSWEEP_W
#undef NRXX_BSWEEP

hipError_t launch_bsweep(int M, int order, int nw, int split, int grid, const BLevel *tab,
                         const int *units, int U, int nsweep, unsigned dirs, int *queue,
                         int cstride, const int *active, int *err, int *abort_flag,
                         unsigned long long limit, hipStream_t s, double *st_ovr,
                         const double *rhs_ovr) {
  return launch_bsweep_t<double>(M, order, nw, split, grid, tab, units, U, nsweep, dirs, queue,
                                 cstride, active, err, abort_flag, limit, s, st_ovr, rhs_ovr);
}

hipError_t launch_bsweep32(int M, int order, int nw, int grid, const BLevel *tab, const int *units,
                           int U, int nsweep, unsigned dirs, int *queue, int cstride,
                           const int *active, int *err, int *abort_flag, unsigned long long limit,
                           hipStream_t s, float *st, const float *rhs) {
  return launch_bsweep_t<float>(M, order, nw, 1, grid, tab, units, U, nsweep, dirs, queue, cstride,
                                active, err, abort_flag, limit, s, st, rhs);
}

int bsweep_resident(int M, int order, int nw, int split) {
  return split ? resident_t<double, true>(M, order, nw) : resident_t<double, false>(M, order, nw);
}
int bsweep_resident32(int M, int order, int nw) { return resident_t<float, true>(M, order, nw); }

hipError_t launch_brestrict(int M, int ncell_coarse, const BLevel *tabF, const BLevel *tabC,
                            int nslot, const int *active, int *err, hipStream_t s) {
  if (ncell_coarse <= 0) return hipSuccess;
  NRXX_DISPATCH_MW(M, {
    hipLaunchKernelGGL((k_brestrict<MM>), dim3(ncell_coarse), dim3(WAVE), 0, s, tabF, tabC, nslot, active, err);
  });
  return hipGetLastError();
}

hipError_t launch_bcopy(int M, int ncell, const BLevel *tab, int nslot, const int *active,
                        hipStream_t s) {
  if (ncell <= 0) return hipSuccess;
  NRXX_DISPATCH_MW(M, {
    hipLaunchKernelGGL((k_bcopy<MM>), dim3(ncell), dim3(WAVE), 0, s, tab, nslot, active);
  });
  return hipGetLastError();
}

hipError_t launch_bcorrect(int M, int ncell_coarse, const BLevel *tabF, const BLevel *tabC,
                           int nslot, const int *active, int *err, hipStream_t s) {
  if (ncell_coarse <= 0) return hipSuccess;
  NRXX_DISPATCH_MW(M, {
    hipLaunchKernelGGL((k_bcorrect<MM>), dim3(ncell_coarse), dim3(WAVE), 0, s, tabF, tabC, nslot, active, err);
  });
  return hipGetLastError();
}

hipError_t launch_bsum(const BLevel *tab, int nslot, int stride, const int *active,
                       const double *partial, int what, double *out, hipStream_t s) {
  if (nslot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bsum, dim3(nslot), dim3(1024), 0, s, tab, stride, active, partial, what, out);
  return hipGetLastError();
}

hipError_t launch_bmass_scale(int M, int ncell, const BLevel *tab, int nslot, const int *active,
                              const double *mass, hipStream_t s) {
  if (ncell <= 0) return hipSuccess;
  NRXX_DISPATCH_MW(M, {
    hipLaunchKernelGGL((k_bmass_scale<MM>), dim3(ncell), dim3(WAVE), 0, s, tab, nslot, active, mass);
  });
  return hipGetLastError();
}

hipError_t launch_bstatus(const BLevel *tab, int nslot, const double *norms, const double *ref,
                          const double *tol, int *active, int *cycles, int *err, hipStream_t s) {
  if (nslot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bstatus, dim3((nslot + 63) / 64), dim3(64), 0, s, tab, nslot, norms, ref, tol,
                     active, cycles, err);
  return hipGetLastError();
}

hipError_t launch_bfill(int *p, int n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_bfill, dim3(blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace nrxx
