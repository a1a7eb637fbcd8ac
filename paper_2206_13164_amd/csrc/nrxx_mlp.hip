// nrxx_mlp.hip -- the warm-start network on gfx950: a stack of affine
// layers with SiLU activations between them, trained with Adam on a mean
// squared error, all in hand-written kernels.  Matrix products run on the
// matrix cores (gfx950's v_mfma_f32_16x16x32_bf16, and 16x16x16 for a last
// block of 16 in k: BF16 operands, FP32 accumulation);
// weights have an FP32 master copy and BF16 working copies (row-major and
// transposed); activations are kept in FP32 (pre-activations) and BF16
// (row-major and transposed, the MFMA operands).
//
// Every product is C[m][n] = sum_k A[m][k] B[n][k] with both operands
// row-major along k, so every MFMA operand fragment (8 consecutive k of one
// row, or 4 in a last block of 16) is one 16-byte (8-byte) load; lane l takes
// row l % 16 of A and of B and the same k of both, so the sum pairs equal k:
//   forward  layer l: A = a_l (rows x in), B = W_l (out x in)
//   backward dA:      A = dz_l (rows x out), B = W_l^T (in x out)
//   backward dW:      A = dz_l^T (out x rows), B = a_l^T (in x rows), the rows
//                     split into chunks whose partial products are summed in
//                     a fixed order (deterministic).
// Widths are padded to multiples of 16 (padding weights stay zero), rows to
// multiples of 64 (padding rows carry zero gradient).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/nrxx.h"

namespace {

typedef uint16_t bf16;
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;
constexpr int ROWPAD = 64;   // rows per GEMM workgroup (4 wavefronts x 16)
constexpr int CHUNK = 1024;  // rows per partial weight gradient

__device__ __forceinline__ bf16 to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (bf16)(u >> 16);
}
__device__ __forceinline__ float from_bf16(bf16 h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

enum { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_BWD = 2, EPI_PART = 3 };

struct Epi {
  const float *bias;  // EPI_HIDDEN, EPI_OUT
  float *z;           // HIDDEN: pre-activation; OUT: output; BWD: dz of the layer below; PART: partials
  bf16 *h;            // HIDDEN: next activation; BWD: dz (bf16)
  bf16 *ht;           // transposed copy of h (leading dimension = rows)
  const float *zp;    // BWD: pre-activation of the layer below
  int ldc, ldt;
};

// One workgroup = 4 wavefronts; wavefront w computes rows
// (blockIdx.x * 4 + w) * 16 .. + 15 and WN column tiles of 16 starting at
// blockIdx.y * 16 * WN; k runs over [kbeg, kbeg + klen), klen % 16 == 0,
// in blocks of 32 (16x16x32 MFMA) and a last block of 16 when klen % 32 = 16.
template <int WN, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const bf16 *__restrict__ A, int lda,
                                              const bf16 *__restrict__ B, int ldb, int Mrows,
                                              int Ncols, int kbeg, int klen, Epi e) {
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int m0 = (blockIdx.x * 4 + wv) * 16;
  if (m0 >= Mrows) return;
  const int n0 = blockIdx.y * 16 * WN;
  const int r = lane % 16, q = lane / 16;
  float4_t acc[WN];
#pragma unroll
  for (int t = 0; t < WN; ++t) acc[t] = float4_t{0.f, 0.f, 0.f, 0.f};
  const bf16 *ap = A + (size_t)(m0 + r) * lda + kbeg;
  const bf16 *bp[WN];
  bool ok[WN];
#pragma unroll
  for (int t = 0; t < WN; ++t) {
    ok[t] = n0 + 16 * t < Ncols;
    bp[t] = B + (size_t)(ok[t] ? n0 + 16 * t + r : 0) * ldb + kbeg;
  }
  const int k32 = klen - klen % 32;
  for (int k = 0; k < k32; k += 32) {
    const bf16x8_t a = *(const bf16x8_t *)(ap + k + 8 * q);
#pragma unroll
    for (int t = 0; t < WN; ++t)
      if (ok[t]) {
        const bf16x8_t b = *(const bf16x8_t *)(bp[t] + k + 8 * q);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
      }
  }
  if (k32 < klen) {
    const short4_t a = *(const short4_t *)(ap + k32 + 4 * q);
#pragma unroll
    for (int t = 0; t < WN; ++t)
      if (ok[t]) {
        const short4_t b = *(const short4_t *)(bp[t] + k32 + 4 * q);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
      }
  }
  // lane holds C[m0 + 4q + i][n0 + 16t + r], i = 0..3
#pragma unroll
  for (int t = 0; t < WN; ++t) {
    if (!ok[t]) continue;
    const int col = n0 + 16 * t + r;
    const int row0 = m0 + 4 * q;
    bf16 packed[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = row0 + i;
      const size_t o = (size_t)row * e.ldc + col;
      if (EPI == EPI_HIDDEN) {
        const float z = acc[t][i] + e.bias[col];
        e.z[o] = z;
        packed[i] = to_bf16(silu(z));
        e.h[o] = packed[i];
      } else if (EPI == EPI_OUT) {
        e.z[o] = acc[t][i] + e.bias[col];
      } else if (EPI == EPI_BWD) {
        const float g = acc[t][i] * silu_grad(e.zp[o]);
        e.z[o] = g;
        packed[i] = to_bf16(g);
        e.h[o] = packed[i];
      } else {
        e.z[(size_t)blockIdx.z * Mrows * Ncols + (size_t)row * Ncols + col] = acc[t][i];
      }
    }
    if (EPI == EPI_HIDDEN || EPI == EPI_BWD) {
      short4_t v{(short)packed[0], (short)packed[1], (short)packed[2], (short)packed[3]};
      *(short4_t *)(e.ht + (size_t)col * e.ldt + row0) = v;
    }
  }
}

// Standardised, padded input: a0[r][c] = (x[r][c] - mean[c]) / std[c] for
// c < din, 0 for padding columns and padding rows; also a0^T.
__global__ void k_std_in(const float *__restrict__ X, int rows, int rows_p, int din, int dp,
                         const float *__restrict__ mean, const float *__restrict__ sd,
                         bf16 *__restrict__ a0, bf16 *__restrict__ a0t) {
  const int tot = rows_p * dp;
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < tot; x += gridDim.x * blockDim.x) {
    const int rw = x / dp, c = x % dp;
    float v = 0.f;
    if (rw < rows && c < din) v = (X[(size_t)rw * din + c] - mean[c]) / sd[c];
    const bf16 h = to_bf16(v);
    a0[x] = h;
    a0t[(size_t)c * rows_p + rw] = h;
  }
}

// Output layer: d loss / d y for loss = mean over rows x dout of
// (y - (t - mean) / std)^2, in FP32 and BF16 (row-major and transposed);
// per-block partial sums of the squared error.
__global__ __launch_bounds__(256) void k_loss_grad(const float *__restrict__ Y, const float *__restrict__ T,
                                                   int rows, int rows_p, int dout, int np,
                                                   const float *__restrict__ mean,
                                                   const float *__restrict__ sd, float *__restrict__ dz,
                                                   bf16 *__restrict__ dzh, bf16 *__restrict__ dzt,
                                                   double *__restrict__ part) {
  __shared__ double sh[256];
  const int tot = rows_p * np;
  const float scale = 2.0f / ((float)rows * (float)dout);
  double s = 0.0;
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < tot; x += gridDim.x * blockDim.x) {
    const int rw = x / np, c = x % np;
    float g = 0.f;
    if (rw < rows && c < dout) {
      const float d = Y[x] - (T[(size_t)rw * dout + c] - mean[c]) / sd[c];
      s += (double)d * d;
      g = scale * d;
    }
    dz[x] = g;
    const bf16 h = to_bf16(g);
    dzh[x] = h;
    dzt[(size_t)c * rows_p + rw] = h;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out[i] = sum over chunks c (in order) of part[c * n + i]
__global__ void k_sum_chunks(const float *__restrict__ part, int chunks, int n, float *__restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(size_t)c * n + i];
    out[i] = s;
  }
}

// gb[c] = sum over rows of dz[r][c], one workgroup per column, fixed order.
__global__ __launch_bounds__(256) void k_col_sum(const float *__restrict__ dz, int rows_p, int np,
                                                 float *__restrict__ gb) {
  __shared__ float sh[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int r = threadIdx.x; r < rows_p; r += 256) s += dz[(size_t)r * np + c];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) gb[c] = sh[0];
}

__global__ void k_sum_doubles(const double *__restrict__ part, int n, double *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s;
  }
}

// Adam with bias correction on FP32 masters; refreshes the BF16 copies
// (row-major W[out][in] and transposed).  b1t = b1^t, b2t = b2^t.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, int in_p, float lr, float b1, float b2, float eps,
                       float b1t, float b2t, bf16 *__restrict__ h, bf16 *__restrict__ ht, int out_p) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - b1t), vh = vi / (1.0f - b2t);
    const float pi = p[i] - lr * mh / (sqrtf(vh) + eps);
    p[i] = pi;
    if (h) {
      const bf16 b = to_bf16(pi);
      h[i] = b;
      ht[(size_t)(i % in_p) * out_p + i / in_p] = b;
    }
  }
}

__global__ void k_refresh_bf16(const float *__restrict__ p, int n, int in_p, int out_p,
                               bf16 *__restrict__ h, bf16 *__restrict__ ht) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const bf16 b = to_bf16(p[i]);
    h[i] = b;
    ht[(size_t)(i % in_p) * out_p + i / in_p] = b;
  }
}

// y[r][c] = z[r][c] * std[c] + mean[c] for the first dout columns
__global__ void k_destd(const float *__restrict__ z, int rows, int np, int dout,
                        const float *__restrict__ mean, const float *__restrict__ sd,
                        float *__restrict__ y) {
  const int tot = rows * dout;
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < tot; x += gridDim.x * blockDim.x) {
    const int rw = x / dout, c = x % dout;
    y[x] = z[(size_t)rw * np + c] * sd[c] + mean[c];
  }
}

int grid_of(size_t n, int threads) {
  size_t b = (n + threads - 1) / threads;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

thread_local std::string g_mlp_error;

}  // namespace

struct nrxx_mlp {
  int L = 0, max_rows = 0, max_rows_p = 0;
  std::vector<int> dim, pd;  // widths and padded widths, L + 1 each
  hipStream_t s = nullptr;
  std::string err;
  std::vector<float *> W, b, mW, vW, mb, vb, gW, gb;
  std::vector<bf16 *> Wh, WhT;
  std::vector<bf16 *> a, at;  // a_k: rows x pd[k], k = 0..L-1
  std::vector<float *> z;     // z_k: rows x pd[k+1], k = 0..L-1 (last = output)
  float *dz[2] = {nullptr, nullptr};
  bf16 *dzh[2] = {nullptr, nullptr}, *dzt[2] = {nullptr, nullptr};
  float *part = nullptr;
  double *lpart = nullptr, *dloss = nullptr, *hloss = nullptr;
  float *in_mean = nullptr, *in_std = nullptr, *out_mean = nullptr, *out_std = nullptr;
  int t = 0;
  std::vector<void *> owned;
};

namespace {

int mfail(nrxx_mlp *m, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (m) m->err = buf;
  else g_mlp_error = buf;
  return code;
}

#define MCHK(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return mfail(m, NRXX_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int LOSS_BLOCKS = 256;

template <int EPI>
hipError_t gemm(const bf16 *A, int lda, const bf16 *B, int ldb, int Mrows, int Ncols, int kbeg,
                int klen, const Epi &e, int chunks, hipStream_t s) {
  const int gx = (Mrows + 63) / 64;
  if (Ncols >= 64) {
    dim3 grid(gx, (Ncols + 63) / 64, chunks);
    hipLaunchKernelGGL((k_gemm<4, EPI>), grid, dim3(256), 0, s, A, lda, B, ldb, Mrows, Ncols, kbeg, klen, e);
  } else {
    dim3 grid(gx, (Ncols + 15) / 16, chunks);
    hipLaunchKernelGGL((k_gemm<1, EPI>), grid, dim3(256), 0, s, A, lda, B, ldb, Mrows, Ncols, kbeg, klen, e);
  }
  return hipGetLastError();
}

// Forward pass on rows_p padded rows (input already standardised into a[0]).
int forward(nrxx_mlp *m, int rows_p) {
  for (int k = 0; k < m->L; ++k) {
    Epi e{};
    e.bias = m->b[k];
    e.z = m->z[k];
    e.ldc = m->pd[k + 1];
    e.ldt = rows_p;
    if (k < m->L - 1) {
      e.h = m->a[k + 1];
      e.ht = m->at[k + 1];
      MCHK(gemm<EPI_HIDDEN>(m->a[k], m->pd[k], m->Wh[k], m->pd[k], rows_p, m->pd[k + 1], 0, m->pd[k], e, 1, m->s));
    } else {
      MCHK(gemm<EPI_OUT>(m->a[k], m->pd[k], m->Wh[k], m->pd[k], rows_p, m->pd[k + 1], 0, m->pd[k], e, 1, m->s));
    }
  }
  return NRXX_OK;
}

int check_rows(nrxx_mlp *m, int rows) {
  if (rows < 1 || rows > m->max_rows) return mfail(m, NRXX_EINVAL, "rows = %d outside [1, %d]", rows, m->max_rows);
  return NRXX_OK;
}

int std_input(nrxx_mlp *m, const float *X, int rows, int rows_p) {
  const size_t n = (size_t)rows_p * m->pd[0];
  hipLaunchKernelGGL(k_std_in, dim3(grid_of(n, 256)), dim3(256), 0, m->s, X, rows, rows_p, m->dim[0],
                     m->pd[0], m->in_mean, m->in_std, m->a[0], m->at[0]);
  MCHK(hipGetLastError());
  return NRXX_OK;
}

// Gradients of the standardised MSE into gW / gb (and the loss into dloss).
int gradients(nrxx_mlp *m, const float *X, const float *T, int rows) {
  const int rows_p = (rows + ROWPAD - 1) / ROWPAD * ROWPAD;
  int rc = std_input(m, X, rows, rows_p);
  if (rc) return rc;
  rc = forward(m, rows_p);
  if (rc) return rc;
  const int L = m->L;
  int cur = 0;
  hipLaunchKernelGGL(k_loss_grad, dim3(LOSS_BLOCKS), dim3(256), 0, m->s, m->z[L - 1], T, rows, rows_p,
                     m->dim[L], m->pd[L], m->out_mean, m->out_std, m->dz[cur], m->dzh[cur], m->dzt[cur],
                     m->lpart);
  MCHK(hipGetLastError());
  hipLaunchKernelGGL(k_sum_doubles, dim3(1), dim3(64), 0, m->s, m->lpart, LOSS_BLOCKS, m->dloss);
  MCHK(hipGetLastError());
  const int chunks = (rows_p + CHUNK - 1) / CHUNK;
  for (int k = L - 1; k >= 0; --k) {
    const int out_p = m->pd[k + 1], in_p = m->pd[k];
    // dW_k = dz_k^T a_k, chunked over rows
    for (int c0 = 0; c0 < chunks; ++c0) {
      const int kb = c0 * CHUNK, kl = std::min(CHUNK, rows_p - kb);
      Epi e{};
      e.z = m->part + (size_t)c0 * out_p * in_p;
      MCHK(gemm<EPI_PART>(m->dzt[cur], rows_p, m->at[k], rows_p, out_p, in_p, kb, kl, e, 1, m->s));
    }
    hipLaunchKernelGGL(k_sum_chunks, dim3(grid_of((size_t)out_p * in_p, 256)), dim3(256), 0, m->s,
                       m->part, chunks, out_p * in_p, m->gW[k]);
    MCHK(hipGetLastError());
    hipLaunchKernelGGL(k_col_sum, dim3(out_p), dim3(256), 0, m->s, m->dz[cur], rows_p, out_p, m->gb[k]);
    MCHK(hipGetLastError());
    if (k > 0) {
      Epi e{};
      e.z = m->dz[1 - cur];
      e.h = m->dzh[1 - cur];
      e.ht = m->dzt[1 - cur];
      e.zp = m->z[k - 1];
      e.ldc = in_p;
      e.ldt = rows_p;
      MCHK(gemm<EPI_BWD>(m->dzh[cur], out_p, m->WhT[k], out_p, rows_p, in_p, 0, out_p, e, 1, m->s));
      cur = 1 - cur;
    }
  }
  return NRXX_OK;
}

int refresh(nrxx_mlp *m) {
  for (int k = 0; k < m->L; ++k) {
    const int n = m->pd[k + 1] * m->pd[k];
    hipLaunchKernelGGL(k_refresh_bf16, dim3(grid_of(n, 256)), dim3(256), 0, m->s, m->W[k], n, m->pd[k],
                       m->pd[k + 1], m->Wh[k], m->WhT[k]);
    MCHK(hipGetLastError());
  }
  return NRXX_OK;
}

}  // namespace

extern "C" {

int nrxx_mlp_create(const int32_t *widths, int32_t nlayers, int32_t max_rows, void *hip_stream,
                    nrxx_mlp **out) {
  if (!out) return mfail(nullptr, NRXX_EINVAL, "out is NULL");
  *out = nullptr;
  if (!widths || nlayers < 1 || nlayers > 16) return mfail(nullptr, NRXX_EINVAL, "bad layer count");
  for (int k = 0; k <= nlayers; ++k)
    if (widths[k] < 1 || widths[k] > 4096) return mfail(nullptr, NRXX_EINVAL, "width %d = %d", k, widths[k]);
  if (max_rows < 1 || max_rows > (1 << 22)) return mfail(nullptr, NRXX_EINVAL, "max_rows = %d", max_rows);
  nrxx_mlp *m = new nrxx_mlp();
  m->L = nlayers;
  m->s = (hipStream_t)hip_stream;
  m->max_rows = max_rows;
  m->max_rows_p = (max_rows + ROWPAD - 1) / ROWPAD * ROWPAD;
  for (int k = 0; k <= nlayers; ++k) {
    m->dim.push_back(widths[k]);
    m->pd.push_back((widths[k] + 15) / 16 * 16);
  }
  bool ok = true;
  auto al = [&](size_t bytes) -> void * {
    void *p = nullptr;
    if (!ok || hipMalloc(&p, bytes) != hipSuccess) {
      ok = false;
      return nullptr;
    }
    m->owned.push_back(p);
    if (hipMemset(p, 0, bytes) != hipSuccess) ok = false;
    return p;
  };
  const size_t R = m->max_rows_p;
  int maxw = 0;
  for (int k = 0; k <= nlayers; ++k) maxw = std::max(maxw, m->pd[k]);
  size_t maxwk = 0;
  for (int k = 0; k < nlayers; ++k) {
    const size_t n = (size_t)m->pd[k + 1] * m->pd[k];
    maxwk = std::max(maxwk, n);
    m->W.push_back((float *)al(n * 4));
    m->mW.push_back((float *)al(n * 4));
    m->vW.push_back((float *)al(n * 4));
    m->gW.push_back((float *)al(n * 4));
    m->Wh.push_back((bf16 *)al(n * 2));
    m->WhT.push_back((bf16 *)al(n * 2));
    m->b.push_back((float *)al(m->pd[k + 1] * 4));
    m->mb.push_back((float *)al(m->pd[k + 1] * 4));
    m->vb.push_back((float *)al(m->pd[k + 1] * 4));
    m->gb.push_back((float *)al(m->pd[k + 1] * 4));
    m->a.push_back((bf16 *)al(R * m->pd[k] * 2));
    m->at.push_back((bf16 *)al(R * m->pd[k] * 2));
    m->z.push_back((float *)al(R * m->pd[k + 1] * 4));
  }
  for (int i = 0; i < 2; ++i) {
    m->dz[i] = (float *)al(R * maxw * 4);
    m->dzh[i] = (bf16 *)al(R * maxw * 2);
    m->dzt[i] = (bf16 *)al(R * maxw * 2);
  }
  m->part = (float *)al(((R + CHUNK - 1) / CHUNK) * maxwk * 4);
  m->lpart = (double *)al(LOSS_BLOCKS * 8);
  m->dloss = (double *)al(8);
  m->in_mean = (float *)al(m->pd[0] * 4);
  m->in_std = (float *)al(m->pd[0] * 4);
  m->out_mean = (float *)al(m->pd[nlayers] * 4);
  m->out_std = (float *)al(m->pd[nlayers] * 4);
  if (ok) ok = hipHostMalloc((void **)&m->hloss, 8, hipHostMallocDefault) == hipSuccess;
  if (ok) {
    std::vector<float> one(std::max(m->pd[0], m->pd[nlayers]), 1.0f);
    ok = hipMemcpy(m->in_std, one.data(), m->pd[0] * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->out_std, one.data(), m->pd[nlayers] * 4, hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok) {
    nrxx_mlp_destroy(m);
    return mfail(nullptr, NRXX_ENOMEM, "device allocation failed");
  }
  *out = m;
  return NRXX_OK;
}

int nrxx_mlp_destroy(nrxx_mlp *m) {
  if (!m) return NRXX_OK;
  if (m->s) (void)hipStreamSynchronize(m->s);
  for (void *p : m->owned) (void)hipFree(p);
  if (m->hloss) (void)hipHostFree(m->hloss);
  delete m;
  return NRXX_OK;
}

const char *nrxx_mlp_last_error(const nrxx_mlp *m) { return m ? m->err.c_str() : g_mlp_error.c_str(); }

int64_t nrxx_mlp_param_count(const nrxx_mlp *m) {
  if (!m) return NRXX_EINVAL;
  int64_t n = 0;
  for (int k = 0; k < m->L; ++k) n += (int64_t)m->dim[k + 1] * m->dim[k] + m->dim[k + 1];
  return n;
}

int nrxx_mlp_set_params(nrxx_mlp *m, const float *p) {
  if (!m) return NRXX_EINVAL;
  if (!p) return mfail(m, NRXX_EINVAL, "params is NULL");
  MCHK(hipStreamSynchronize(m->s));
  size_t off = 0;
  for (int k = 0; k < m->L; ++k) {
    const int o = m->dim[k + 1], i = m->dim[k], op = m->pd[k + 1], ip = m->pd[k];
    std::vector<float> Wp((size_t)op * ip, 0.f), bp(op, 0.f);
    for (int r = 0; r < o; ++r)
      for (int c = 0; c < i; ++c) Wp[(size_t)r * ip + c] = p[off + (size_t)r * i + c];
    off += (size_t)o * i;
    for (int r = 0; r < o; ++r) bp[r] = p[off + r];
    off += o;
    MCHK(hipMemcpy(m->W[k], Wp.data(), Wp.size() * 4, hipMemcpyHostToDevice));
    MCHK(hipMemcpy(m->b[k], bp.data(), bp.size() * 4, hipMemcpyHostToDevice));
    MCHK(hipMemset(m->mW[k], 0, Wp.size() * 4));
    MCHK(hipMemset(m->vW[k], 0, Wp.size() * 4));
    MCHK(hipMemset(m->mb[k], 0, bp.size() * 4));
    MCHK(hipMemset(m->vb[k], 0, bp.size() * 4));
  }
  m->t = 0;
  int rc = refresh(m);
  if (rc) return rc;
  MCHK(hipStreamSynchronize(m->s));
  return NRXX_OK;
}

int nrxx_mlp_get_params(const nrxx_mlp *mc, float *p) {
  nrxx_mlp *m = const_cast<nrxx_mlp *>(mc);
  if (!m) return NRXX_EINVAL;
  if (!p) return mfail(m, NRXX_EINVAL, "params is NULL");
  MCHK(hipStreamSynchronize(m->s));
  size_t off = 0;
  for (int k = 0; k < m->L; ++k) {
    const int o = m->dim[k + 1], i = m->dim[k], op = m->pd[k + 1], ip = m->pd[k];
    std::vector<float> Wp((size_t)op * ip), bp(op);
    MCHK(hipMemcpy(Wp.data(), m->W[k], Wp.size() * 4, hipMemcpyDeviceToHost));
    MCHK(hipMemcpy(bp.data(), m->b[k], bp.size() * 4, hipMemcpyDeviceToHost));
    for (int r = 0; r < o; ++r)
      for (int c = 0; c < i; ++c) p[off + (size_t)r * i + c] = Wp[(size_t)r * ip + c];
    off += (size_t)o * i;
    for (int r = 0; r < o; ++r) p[off + r] = bp[r];
    off += o;
  }
  return NRXX_OK;
}

int nrxx_mlp_set_scaling(nrxx_mlp *m, const float *in_mean, const float *in_std,
                         const float *out_mean, const float *out_std) {
  if (!m) return NRXX_EINVAL;
  if (!in_mean || !in_std || !out_mean || !out_std) return mfail(m, NRXX_EINVAL, "NULL scaling");
  for (int c = 0; c < m->dim[0]; ++c)
    if (!(in_std[c] > 0)) return mfail(m, NRXX_EINVAL, "in_std[%d] <= 0", c);
  for (int c = 0; c < m->dim[m->L]; ++c)
    if (!(out_std[c] > 0)) return mfail(m, NRXX_EINVAL, "out_std[%d] <= 0", c);
  MCHK(hipStreamSynchronize(m->s));
  MCHK(hipMemcpy(m->in_mean, in_mean, m->dim[0] * 4, hipMemcpyHostToDevice));
  MCHK(hipMemcpy(m->in_std, in_std, m->dim[0] * 4, hipMemcpyHostToDevice));
  MCHK(hipMemcpy(m->out_mean, out_mean, m->dim[m->L] * 4, hipMemcpyHostToDevice));
  MCHK(hipMemcpy(m->out_std, out_std, m->dim[m->L] * 4, hipMemcpyHostToDevice));
  return NRXX_OK;
}

int nrxx_mlp_forward(nrxx_mlp *m, const float *X, int32_t rows, float *Y) {
  if (!m) return NRXX_EINVAL;
  if (!X || !Y) return mfail(m, NRXX_EINVAL, "NULL buffer");
  int rc = check_rows(m, rows);
  if (rc) return rc;
  const int rows_p = (rows + ROWPAD - 1) / ROWPAD * ROWPAD;
  rc = std_input(m, X, rows, rows_p);
  if (rc) return rc;
  rc = forward(m, rows_p);
  if (rc) return rc;
  const int L = m->L;
  hipLaunchKernelGGL(k_destd, dim3(grid_of((size_t)rows * m->dim[L], 256)), dim3(256), 0, m->s, m->z[L - 1],
                     rows, m->pd[L], m->dim[L], m->out_mean, m->out_std, Y);
  MCHK(hipGetLastError());
  return NRXX_OK;
}

int nrxx_mlp_gradients(nrxx_mlp *m, const float *X, const float *T, int32_t rows, float *g,
                       double *loss_out) {
  if (!m) return NRXX_EINVAL;
  if (!X || !T || !g) return mfail(m, NRXX_EINVAL, "NULL buffer");
  int rc = check_rows(m, rows);
  if (rc) return rc;
  rc = gradients(m, X, T, rows);
  if (rc) return rc;
  MCHK(hipMemcpyAsync(m->hloss, m->dloss, 8, hipMemcpyDeviceToHost, m->s));
  MCHK(hipStreamSynchronize(m->s));
  if (loss_out) *loss_out = m->hloss[0] / ((double)rows * m->dim[m->L]);
  size_t off = 0;
  for (int k = 0; k < m->L; ++k) {
    const int o = m->dim[k + 1], i = m->dim[k], op = m->pd[k + 1], ip = m->pd[k];
    std::vector<float> Wp((size_t)op * ip), bp(op);
    MCHK(hipMemcpy(Wp.data(), m->gW[k], Wp.size() * 4, hipMemcpyDeviceToHost));
    MCHK(hipMemcpy(bp.data(), m->gb[k], bp.size() * 4, hipMemcpyDeviceToHost));
    for (int r = 0; r < o; ++r)
      for (int c = 0; c < i; ++c) g[off + (size_t)r * i + c] = Wp[(size_t)r * ip + c];
    off += (size_t)o * i;
    for (int r = 0; r < o; ++r) g[off + r] = bp[r];
    off += o;
  }
  return NRXX_OK;
}

int nrxx_mlp_train_step(nrxx_mlp *m, const float *X, const float *T, int32_t rows, float lr,
                        double *loss_out) {
  if (!m) return NRXX_EINVAL;
  if (!X || !T || !(lr > 0)) return mfail(m, NRXX_EINVAL, "NULL buffer or lr <= 0");
  int rc = check_rows(m, rows);
  if (rc) return rc;
  rc = gradients(m, X, T, rows);
  if (rc) return rc;
  m->t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float b1t = powf(b1, (float)m->t), b2t = powf(b2, (float)m->t);
  for (int k = 0; k < m->L; ++k) {
    const int n = m->pd[k + 1] * m->pd[k];
    hipLaunchKernelGGL(k_adam, dim3(grid_of(n, 256)), dim3(256), 0, m->s, m->W[k], m->gW[k], m->mW[k],
                       m->vW[k], n, m->pd[k], lr, b1, b2, eps, b1t, b2t, m->Wh[k], m->WhT[k], m->pd[k + 1]);
    MCHK(hipGetLastError());
    hipLaunchKernelGGL(k_adam, dim3(1), dim3(256), 0, m->s, m->b[k], m->gb[k], m->mb[k], m->vb[k],
                       m->pd[k + 1], 1, lr, b1, b2, eps, b1t, b2t, (bf16 *)nullptr, (bf16 *)nullptr, 1);
    MCHK(hipGetLastError());
  }
  if (loss_out) {
    MCHK(hipMemcpyAsync(m->hloss, m->dloss, 8, hipMemcpyDeviceToHost, m->s));
    MCHK(hipStreamSynchronize(m->s));
    *loss_out = m->hloss[0] / ((double)rows * m->dim[m->L]);
  }
  return NRXX_OK;
}

}  // extern "C"
