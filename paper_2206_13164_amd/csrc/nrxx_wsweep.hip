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
// of sweep s at row j, and columns i-2 .. i+2 at row j of sweep s-1.  Results
// are bit-identical to the cell-team kernels.
#include "nrxx_wave.hpp"

namespace nrxx {
namespace {

template <int M, int WPG>
struct WSweepLds {
  WTabs<M> tabs;
  LevelArgs args[WPG];
  double buf[WPG][WLay<M>::TOTAL];
};

// Wavefronts per SIMD the register allocation of the kernel must allow.
template <int M>
struct WOcc {
  static constexpr int W = M <= 6 ? 3 : 2;
};

template <int M, int ORDER, int WPG>
__global__ __launch_bounds__(WPG * WAVE) __attribute__((amdgpu_waves_per_eu(WOcc<M>::W)))
void k_wsweep(const BLevel *__restrict__ tab, const int *__restrict__ units, int U, int nsweep,
              unsigned dirs, int *queue, int cstride, const int *__restrict__ active, int *err,
              int *abort_flag, unsigned long long limit) {
  __shared__ WSweepLds<M, WPG> sh;
  load_tabs<M>(sh.tabs);
  __syncthreads();
  // from here on the wavefronts of the workgroup are independent: no
  // workgroup barrier follows
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  LevelArgs &A = sh.args[wv];
  double *lw = sh.buf[wv];
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
    double *const st = B.st;
    const double *const rhs = B.rhs;
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
    for (int b = 0; b < ny; ++b) {
      const int j = jrev ? ny - 1 - b : b;
      int ok = 1;
      if (lane == 0) {
        bool good = true;
        if (s > 0) {
          const int need = pjrev ? ny - (j - 2 > 0 ? j - 2 : 0) : (j + 2 < ny - 1 ? j + 2 : ny - 1) + 1;
          if (known < need) {
            int seen = need;
            good = wait_at_least(cp + i, need, abort_flag, limit, &seen);
            known = seen;
          }
          const int bp = pjrev ? ny - 1 - j : j;
          for (int d = -2; d <= 2 && good; ++d) {
            const int ii = i + d;
            if (d == 0 || ii < 0 || ii >= nx) continue;
            good = wait_at_least(cp + ii, bp + 1, abort_flag, limit);
          }
        }
        if (good && p > 0) good = wait_at_least(cs + prev, b + 1, abort_flag, limit);
        if (good) acquire_agent();
        ok = good ? 1 : 0;
      }
      ok = __shfl(ok, 0);
      if (!ok) {
        if (lane == 0) atomicOr(err, 4);
        return;  // uniform across the wavefront
      }
      wave_cell<double, M, ORDER>(A, lw, sh.tabs, S, lane, st, rhs, i, j, err);
      if (lane == 0) __hip_atomic_store(cs + i, b + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Wavefronts per workgroup of the kernel (each works alone; the workgroup
// only shares the layout maps).
constexpr int kWpg = 4;

template <int M, int ORDER>
int wsweep_occupancy() {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_wsweep<M, ORDER, kWpg>, kWpg * WAVE, 0) !=
      hipSuccess)
    return 0;
  return per;
}

}  // namespace

hipError_t launch_wsweep(int M, int order, int grid, const BLevel *tab, const int *units, int U,
                         int nsweep, unsigned dirs, int *queue, int cstride, const int *active,
                         int *err, int *abort_flag, unsigned long long limit, hipStream_t s) {
  if (grid < 1 || (order != 1 && order != 2)) return hipErrorInvalidValue;
  NRXX_DISPATCH_M(M, {
    if (order == 1)
      hipLaunchKernelGGL((k_wsweep<MM, 1, kWpg>), dim3(grid), dim3(kWpg * WAVE), 0, s, tab, units,
                         U, nsweep, dirs, queue, cstride, active, err, abort_flag, limit);
    else
      hipLaunchKernelGGL((k_wsweep<MM, 2, kWpg>), dim3(grid), dim3(kWpg * WAVE), 0, s, tab, units,
                         U, nsweep, dirs, queue, cstride, active, err, abort_flag, limit);
  });
  return hipGetLastError();
}

// Resident workgroups of the wavefront-per-cell sweep on the current device
// (kWpg wavefronts each), 0 if unknown.
int wsweep_resident(int M, int order) {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  int per = 0;
  switch (M) {
#define NRXX_WOCC(MM) \
    case MM: per = order == 1 ? wsweep_occupancy<MM, 1>() : wsweep_occupancy<MM, 2>(); break;
    NRXX_WOCC(3) NRXX_WOCC(4) NRXX_WOCC(5) NRXX_WOCC(6) NRXX_WOCC(7) NRXX_WOCC(8)
#undef NRXX_WOCC
    default: return 0;
  }
  return per * ncu;
}

int wsweep_wavefronts_per_group() { return kWpg; }

}  // namespace nrxx
