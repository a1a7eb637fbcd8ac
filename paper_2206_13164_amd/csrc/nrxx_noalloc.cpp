// nrxx_noalloc.cpp -- the context-free residual of include/nrxx.h
// (nrxx_residual_noalloc) for callers that cannot allocate device memory.
//
// It runs the kernels of nrxx_residual (k_residual, then the fixed-order
// reduction k_cell_sum) with their scratch -- the per-cell weighted squares of
// the defect and the reduced sum -- in a fixed, file-scope device array
// instead of context memory.  Host code never passes the array's name to a
// kernel: the name is a host-side stand-in, not a device address.  The
// device address is looked up once per device with hipGetSymbolAddress, with
// that device current, and only that address is used afterwards.
#include <math.h>
#include <mutex>

#include "nrxx_host.hpp"

using namespace nrxx;

namespace {

// Largest level (cells) the array serves, and the array: one weighted square
// per cell, then the reduced sum.  Each GPU holds its own copy (2 MiB) until
// the process ends.
constexpr int kMaxCells = NRXX_NOALLOC_MAX_CELLS;
static __device__ __align__(256) double scratch[kMaxCells + 64];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
double *g_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// Address of this device's copy of the array (nullptr and an error text on
// failure).  Looked up once per device, with the device current.
double *scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_context_free_error(NRXX_EHIP, "nrxx_residual_noalloc: no usable current device");
    return nullptr;
  }
  std::lock_guard<std::mutex> hold(g_lock);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_context_free_error(NRXX_EHIP, "nrxx_residual_noalloc: hipGetSymbolAddress: %s",
                             hipGetErrorString(e));
      return nullptr;
    }
    g_ptr[dev] = static_cast<double *>(p);
  }
  return g_ptr[dev];
}

__global__ void k_norm_from_sum(const double *__restrict__ sum, double *__restrict__ out) {
  if (threadIdx.x == 0) *out = sqrt(*sum);
}

int hipfail(hipError_t e, const char *what) {
  if (e == hipSuccess) return NRXX_OK;
  return set_context_free_error(NRXX_EHIP, "nrxx_residual_noalloc: %s: %s", what,
                                hipGetErrorString(e));
}

}  // namespace

extern "C" int nrxx_residual_noalloc(const nrxx_problem *p, int32_t level, const double *state,
                                     const double *rhs, double *R_out, double *norm_dev,
                                     double *norm_host, void *hip_stream) {
  if (!p) return set_context_free_error(NRXX_EINVAL, "nrxx_residual_noalloc: problem is NULL");
  char msg[256];
  if (!validate_problem(*p, msg, sizeof msg))
    return set_context_free_error(NRXX_EINVAL, "nrxx_residual_noalloc: %s", msg);
  if (level < 0 || level >= p->levels || !state)
    return set_context_free_error(NRXX_EINVAL, "nrxx_residual_noalloc: bad level or NULL state");
  const LevelArgs A = make_level(*p, level);
  const long long ncell = (long long)A.nx * A.ny;
  const bool want_norm = norm_dev || norm_host;
  if (want_norm && ncell > kMaxCells)
    return set_context_free_error(NRXX_EINVAL,
                                  "nrxx_residual_noalloc: level has %lld cells, the scratch array "
                                  "holds %d",
                                  ncell, kMaxCells);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  double *part = nullptr;
  if (want_norm) {
    part = scratch_ptr();
    if (!part) return NRXX_EHIP;
  }
  // every cell's weighted square is written by the residual kernel, and the
  // sum slot by the reduction: nothing in the array needs clearing
  int rc = hipfail(launch_residual(p->M, A, state, rhs, nullptr, R_out, part, 0, s), "k_residual");
  if (rc || !want_norm) return rc;
  double *sum = part + kMaxCells;
  rc = hipfail(launch_cell_sum(A, part, 1, 0, A.inv_area, sum, s), "k_cell_sum");
  if (rc) return rc;
  if (norm_dev) {
    hipLaunchKernelGGL(k_norm_from_sum, dim3(1), dim3(64), 0, s, sum, norm_dev);
    rc = hipfail(hipGetLastError(), "k_norm_from_sum");
    if (rc) return rc;
  }
  if (norm_host) {
    double v = 0.0;
    rc = hipfail(hipMemcpyAsync(&v, sum, sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    if (!rc) rc = hipfail(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (rc) return rc;
    *norm_host = sqrt(v);
    if (!isfinite(*norm_host))
      return set_context_free_error(NRXX_EDIVERGED, "nrxx_residual_noalloc: norm not finite");
  }
  return NRXX_OK;
}
