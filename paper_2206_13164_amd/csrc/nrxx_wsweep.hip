// nrxx_wsweep.hip -- batched fast-sweeping kernel with one wavefront per cell
// (nrxx_wave.hpp): the throughput form of the work-queue sweep of
// nrxx_batch.hip for many problems in flight.
//
// Units and their order are those of k_bsweep (a unit is one grid column of
// one problem in one directional sweep; units are taken from an atomic
// counter in an order in which a unit only waits for earlier units), but
// every wavefront of a workgroup takes its own units and updates the cells
// of its column alone, so a CU holds as many columns in flight as its LDS
// and registers allow instead of one or two cell teams.  Cell (i, j) of
// sweep s waits for exactly what the serial Gauss-Seidel order of Alg. 1
// needs: rows j-2 .. j+2 of its own column in sweep s-1, the previous column
// of sweep s at row j, and columns i-2 .. i+2 at row j of sweep s-1.  A
// wavefront may take its column's rows in blocks of kb rows with one set of
// waits and one acquire/release per block: fewer cache invalidations, at the
// price of a downstream column starting kb rows later.  Results are
// bit-identical to the cell-team kernels for every kb.
#include <algorithm>
#include <atomic>

#include "nrxx_wave.hpp"

namespace nrxx {
namespace {

template <int M, int WPG>
struct WSweepLds {
  WTabs<M> tabs;
  LevelArgs args[WPG];
  double buf[WPG][WLay<M>::TOTAL];
};

// Wavefronts per SIMD the register allocation of the kernel must allow
// (more cells in flight against spilled registers).
#ifndef NRXX_WOCC_SMALL
#define NRXX_WOCC_SMALL 3
#endif
#ifndef NRXX_WOCC_LARGE
#define NRXX_WOCC_LARGE 2
#endif
template <int M>
struct WOcc {
  static constexpr int W = M <= 6 ? NRXX_WOCC_SMALL : M <= 8 ? NRXX_WOCC_LARGE : 1;
};

template <int M, int ORDER, int WPG>
__global__ __launch_bounds__(WPG * WAVE) __attribute__((amdgpu_waves_per_eu(WOcc<M>::W)))
void k_wsweep(const BLevel *__restrict__ tab, const int *__restrict__ units, int U, int nsweep,
              unsigned dirs, int *queue, int cstride, const int *__restrict__ active, int *err,
              int *abort_flag, unsigned long long limit, int kb, double *st_ovr,
              const double *rhs_ovr) {
  __shared__ WSweepLds<M, WPG> sh;
  load_tabs<M>(sh.tabs);
  __syncthreads();
  // from here on the wavefronts of the workgroup are independent: no
  // workgroup barrier follows
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  LevelArgs &A = sh.args[wv];
  double *lw = sh.buf[wv];
  wzero<double, M>(lw, lane);
  WSlot<M> S;
  S.init(lane);
  const int total = nsweep * U;
  for (;;) {
    int u = 0;
    if (lane == 0) {
      u = atomicAdd(queue, 1);
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) u = total;
    }
    u = __shfl(u, 0);
    if (u >= total) return;
    const int s = u / U, e = units[u % U];
    const int slot = e >> 16, p = e & 0xffff;
    const BLevel &B = tab[slot];
    if (!active[B.inst]) continue;
    {
      // the problem's level constants, staged in this wavefront's LDS
      constexpr int n32 = (int)(sizeof(LevelArgs) / sizeof(uint32_t));
      const uint32_t *src = reinterpret_cast<const uint32_t *>(&B.A);
      uint32_t *dst = reinterpret_cast<uint32_t *>(&A);
      for (int x = lane; x < n32; x += WAVE) dst[x] = src[x];
      wsync();
    }
    double *const st = st_ovr ? st_ovr : B.st;
    const double *const rhs = st_ovr ? rhs_ovr : B.rhs;
    const int nx = A.nx, ny = A.ny;
    int *cs = B.cnt + s * cstride;             // this sweep's counters
    int *cp = s > 0 ? cs - cstride : nullptr;  // previous sweep's
    const int dir = (dirs >> (2 * s)) & 3;
    const bool irev = dir == 1 || dir == 2, jrev = dir == 2 || dir == 3;
    const int i = irev ? nx - 1 - p : p;
    const int prev = irev ? i + 1 : i - 1;
    const int pdir = s > 0 ? (dirs >> (2 * (s - 1))) & 3 : 0;
    const bool pjrev = pdir == 2 || pdir == 3;
    int known = 0;  // rows of the own column known finished in sweep s-1
    // rows are taken in blocks of kb: one set of waits (covering every row
    // of the block) and one acquire per block, one release after it
    for (int b0 = 0; b0 < ny; b0 += kb) {
      const int b1 = b0 + kb - 1 < ny - 1 ? b0 + kb - 1 : ny - 1;
      const int ja = jrev ? ny - 1 - b0 : b0, jb = jrev ? ny - 1 - b1 : b1;
      const int jlo = ja < jb ? ja : jb, jhi = ja < jb ? jb : ja;
      int ok = 1;
      if (lane == 0) {
        bool good = true;
        if (s > 0) {
          // own column, sweep s-1: rows jlo-2 .. jhi+2
          const int need = pjrev ? ny - (jlo - 2 > 0 ? jlo - 2 : 0) : (jhi + 2 < ny - 1 ? jhi + 2 : ny - 1) + 1;
          if (known < need) {
            int seen = need;
            good = wait_at_least(cp + i, need, abort_flag, limit, &seen);
            known = seen;
          }
          // columns i-2 .. i+2, sweep s-1: rows jlo .. jhi
          const int bp = pjrev ? ny - 1 - jlo : jhi;
          for (int d = -2; d <= 2 && good; ++d) {
            const int ii = i + d;
            if (d == 0 || ii < 0 || ii >= nx) continue;
            good = wait_at_least(cp + ii, bp + 1, abort_flag, limit);
          }
        }
        // previous column of sweep s: rows b0 .. b1 of the sweep order
        if (good && p > 0) good = wait_at_least(cs + prev, b1 + 1, abort_flag, limit);
        if (good) acquire_agent();
        ok = good ? 1 : 0;
      }
      ok = __shfl(ok, 0);
      if (!ok) {
        if (lane == 0) atomicOr(err, 4);
        return;  // uniform across the wavefront
      }
      for (int b = b0; b <= b1; ++b) {
        const int j = jrev ? ny - 1 - b : b;
        wave_cell<double, M, ORDER>(A, lw, sh.tabs, S, lane, st, rhs, i, j, err);
      }
      if (lane == 0) publish(cs + i, b1 + 1);
    }
  }
}

// Batched residuals with one wavefront per cell, one kernel per role
// (each inlines one copy of the cell update, which keeps its registers
// down): ROLE 0: Rbar = rhs - R(st) for the problems that continue to a
// coarser level; 1: rhs = R(fbar) + RH (eq. (22)); 2: partial[cell0 + cell]
// = weighted |rhs - R(st)|^2 ds (eq. (28)).  Every cell is independent: the
// wavefronts stride over the group's cells and look their problem up only
// when a cell leaves the problem of the previous one.
template <int M, int ORDER, int WPG, int ROLE>
__global__ __launch_bounds__(WPG * WAVE) __attribute__((amdgpu_waves_per_eu(WOcc<M>::W)))
void k_wresidual(const BLevel *__restrict__ tab, int nslot, int ncell,
                 const int *__restrict__ active, double *partial) {
  __shared__ WSweepLds<M, WPG> sh;
  load_tabs<M>(sh.tabs);
  __syncthreads();
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  LevelArgs &A = sh.args[wv];
  double *lw = sh.buf[wv];
  wzero<double, M>(lw, lane);
  WSlot<M> S;
  S.init(lane);
  int slot = -1, lo = 0, hi = 0;
  bool skip = true;
  for (int cell = blockIdx.x * WPG + wv; cell < ncell; cell += gridDim.x * WPG) {
    if (cell < lo || cell >= hi) {
      slot = uni(find_slot(tab, nslot, cell));
      const BLevel &B = tab[slot];
      lo = uni(B.cell0);
      hi = lo + uni(B.ncell);
      skip = !active[B.inst] || (ROLE == 0 && !B.cont);
      if (!skip) {
        constexpr int n32 = (int)(sizeof(LevelArgs) / sizeof(uint32_t));
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&B.A);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&A);
        wsync();
        for (int x = lane; x < n32; x += WAVE) dst[x] = src[x];
        wsync();
      }
    }
    if (skip) continue;
    const BLevel &B = tab[slot];
    const int c = cell - lo;
    const int i = c % A.nx, j = c / A.nx;
    if constexpr (ROLE == 1)
      wave_cell<double, M, ORDER, MODE_FAS>(A, lw, sh.tabs, S, lane, B.fbar, nullptr, i, j, nullptr,
                                            B.RH, B.rhs, nullptr);
    else if constexpr (ROLE == 0)
      wave_cell<double, M, ORDER, MODE_DEFECT>(A, lw, sh.tabs, S, lane, B.st, B.rhs, i, j, nullptr,
                                               nullptr, B.Rbar, nullptr);
    else
      wave_cell<double, M, ORDER, MODE_DEFECT>(A, lw, sh.tabs, S, lane, B.st, B.rhs, i, j, nullptr,
                                               nullptr, nullptr, partial + lo);
  }
}

// Wavefronts per workgroup of the kernels (each works alone; the workgroup
// only shares the layout maps): 4, or 2 at M >= 7 (the LDS of a workgroup
// stays within 64 KiB).
template <int M>
struct Wpg {
  static constexpr int W = M >= 7 ? 2 : 4;
};

// One problem's residual with one wavefront per cell (modes of
// launch_residual: MODE_DEFECT out = r - R(f) and the norm parts, MODE_FAS
// out = R(f) + Radd); the wavefronts stride over the level's cells.
template <int M, int ORDER, int WPG, int MODE>
__global__ __launch_bounds__(WPG * WAVE) __attribute__((amdgpu_waves_per_eu(WOcc<M>::W)))
void k_wres1(LevelArgs A, const double *__restrict__ st, const double *__restrict__ rhs,
             const double *__restrict__ Radd, double *__restrict__ out,
             double *__restrict__ norm_part) {
  __shared__ WSweepLds<M, WPG> sh;
  load_tabs<M>(sh.tabs);
  __syncthreads();
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  double *lw = sh.buf[wv];
  wzero<double, M>(lw, lane);
  WSlot<M> S;
  S.init(lane);
  const int ncell = A.nx * A.ny;
  for (int cell = blockIdx.x * WPG + wv; cell < ncell; cell += gridDim.x * WPG)
    wave_cell<double, M, ORDER, MODE>(A, lw, sh.tabs, S, lane, const_cast<double *>(st), rhs,
                                      cell % A.nx, cell / A.nx, nullptr, Radd, out, norm_part);
}

template <int M, int ORDER, int ROLE>
int wresidual_occupancy() {
  // workgroups per CU of this instance: a property of the kernel and the
  // architecture, asked once (threads racing here store the same value)
  static std::atomic<int> per{-1};
  int v = per.load(std::memory_order_relaxed);
  if (v < 0) {
    int p = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p, k_wresidual<M, ORDER, Wpg<M>::W, ROLE>,
                                                     Wpg<M>::W * WAVE, 0) != hipSuccess)
      return 0;
    per.store(p, std::memory_order_relaxed);
    v = p;
  }
  return v;
}

template <int M, int ORDER>
int wsweep_occupancy() {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_wsweep<M, ORDER, Wpg<M>::W>,
                                                   Wpg<M>::W * WAVE, 0) != hipSuccess)
    return 0;
  return per;
}

}  // namespace

hipError_t launch_wsweep(int M, int order, int grid, const BLevel *tab, const int *units, int U,
                         int nsweep, unsigned dirs, int *queue, int cstride, const int *active,
                         int *err, int *abort_flag, unsigned long long limit, int kb,
                         hipStream_t s, double *st_ovr, const double *rhs_ovr) {
  if (grid < 1 || kb < 1 || (order != 1 && order != 2)) return hipErrorInvalidValue;
  NRXX_DISPATCH_MW(M, {
    constexpr int W = Wpg<MM>::W;
    if (order == 1)
      hipLaunchKernelGGL((k_wsweep<MM, 1, W>), dim3(grid), dim3(W * WAVE), 0, s, tab, units, U,
                         nsweep, dirs, queue, cstride, active, err, abort_flag, limit, kb, st_ovr,
                         rhs_ovr);
    else
      hipLaunchKernelGGL((k_wsweep<MM, 2, W>), dim3(grid), dim3(W * WAVE), 0, s, tab, units, U,
                         nsweep, dirs, queue, cstride, active, err, abort_flag, limit, kb, st_ovr,
                         rhs_ovr);
  });
  return hipGetLastError();
}

template <int M, int ORDER, int ROLE>
static void wresidual_launch_r(int ncell, const BLevel *tab, int nslot, const int *active,
                               double *partial, int ncu, hipStream_t s) {
  constexpr int W = Wpg<M>::W;
  const int per = wresidual_occupancy<M, ORDER, ROLE>();
  const int need = (ncell + W - 1) / W;
  const int grid = std::max(1, std::min(need, std::max(per, 1) * ncu));
  hipLaunchKernelGGL((k_wresidual<M, ORDER, W, ROLE>), dim3(grid), dim3(W * WAVE), 0, s, tab, nslot,
                     ncell, active, partial);
}

template <int M>
static void wresidual_launch(int order, int role, int ncell, const BLevel *tab, int nslot,
                             const int *active, double *partial, int ncu, hipStream_t s) {
  if (order == 1) {
    if (role == 0) wresidual_launch_r<M, 1, 0>(ncell, tab, nslot, active, partial, ncu, s);
    else if (role == 1) wresidual_launch_r<M, 1, 1>(ncell, tab, nslot, active, partial, ncu, s);
    else wresidual_launch_r<M, 1, 2>(ncell, tab, nslot, active, partial, ncu, s);
  } else {
    if (role == 0) wresidual_launch_r<M, 2, 0>(ncell, tab, nslot, active, partial, ncu, s);
    else if (role == 1) wresidual_launch_r<M, 2, 1>(ncell, tab, nslot, active, partial, ncu, s);
    else wresidual_launch_r<M, 2, 2>(ncell, tab, nslot, active, partial, ncu, s);
  }
}

hipError_t launch_wresidual(int M, int order, int ncell, const BLevel *tab, int nslot,
                            const int *active, int role, double *partial, hipStream_t s) {
  if (ncell <= 0) return hipSuccess;
  if (order != 1 && order != 2) return hipErrorInvalidValue;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorInvalidDevice;
  if (role < 0 || role > 2) return hipErrorInvalidValue;
  NRXX_DISPATCH_MW(M, { wresidual_launch<MM>(order, role, ncell, tab, nslot, active, partial, ncu, s); });
  return hipGetLastError();
}

template <int M>
static void wres1_launch(const LevelArgs &A, const double *st, const double *rhs,
                         const double *Radd, double *out, double *norm_part, int mode, int ncu,
                         hipStream_t s) {
  constexpr int W = Wpg<M>::W;
  const int ncell = A.nx * A.ny;
  const int grid = std::max(1, std::min((ncell + W - 1) / W, 4 * ncu));
  const dim3 g(grid), b(W * WAVE);
  if (mode == 0) {
    if (A.order == 1)
      hipLaunchKernelGGL((k_wres1<M, 1, W, MODE_DEFECT>), g, b, 0, s, A, st, rhs, Radd, out, norm_part);
    else
      hipLaunchKernelGGL((k_wres1<M, 2, W, MODE_DEFECT>), g, b, 0, s, A, st, rhs, Radd, out, norm_part);
  } else {
    if (A.order == 1)
      hipLaunchKernelGGL((k_wres1<M, 1, W, MODE_FAS>), g, b, 0, s, A, st, rhs, Radd, out, norm_part);
    else
      hipLaunchKernelGGL((k_wres1<M, 2, W, MODE_FAS>), g, b, 0, s, A, st, rhs, Radd, out, norm_part);
  }
}

hipError_t launch_wresidual1(int M, const LevelArgs &A, const double *st, const double *rhs,
                             const double *Radd, double *out, double *norm_part, int mode,
                             hipStream_t s) {
  if (A.nx * A.ny <= 0) return hipSuccess;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorInvalidDevice;
  // M <= MTEAM takes the cell-team residual kernel
  if (M == 9) wres1_launch<9>(A, st, rhs, Radd, out, norm_part, mode, ncu, s);
  else if (M == 10) wres1_launch<10>(A, st, rhs, Radd, out, norm_part, mode, ncu, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// Resident workgroups of the wavefront-per-cell sweep on the current device
// (Wpg<M> wavefronts each), 0 if unknown.
int wsweep_resident(int M, int order) {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  int per = 0;
  switch (M) {
#define NRXX_WOCC(MM) \
    case MM: per = order == 1 ? wsweep_occupancy<MM, 1>() : wsweep_occupancy<MM, 2>(); break;
    NRXX_WOCC(3) NRXX_WOCC(4) NRXX_WOCC(5) NRXX_WOCC(6) NRXX_WOCC(7) NRXX_WOCC(8) NRXX_WOCC(9)
    NRXX_WOCC(10)
#undef NRXX_WOCC
    default: return 0;
  }
  return per * ncu;
}

int wsweep_wavefronts_per_group(int M) { return M >= 7 ? 2 : 4; }

}  // namespace nrxx
