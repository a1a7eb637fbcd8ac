// nrxx_device.hpp -- device-side building blocks of the gfx950 NRxx kernels
// (Hu & Li, arXiv 2206.13164), shared by the single-problem kernels and the
// batched kernels.
//
// Execution model.  A cell is evaluated by a workgroup of NW wavefronts (a
// "cell team").  The eight face-side items of the cell -- for each of the
// faces E, W, N, S the half-flux of the cell's own face state and of the
// neighbour's face state, each projected into the cell's basis (or, at a
// wall, the wall flux) -- are spread over the wavefronts and run in parallel;
// wavefront 0 then adds them up in a fixed order (independent of NW) with the
// regularisation and collision terms and, in a sweep, re-expands the updated
// cell in its new basis.
// Within a wavefront, lanes run over the expansion coefficients with even
// alpha_3 (the odd ones vanish identically for this xi_3-even, two-
// dimensional problem): 13 / 34 / 95 coefficients at M = 3 / 5 / 8 in 1 or 2
// registers per lane.  Coefficient vectors that lanes must read from each
// other live in LDS in a dense "cube" (alpha_1, alpha_2, alpha_3 / 2) of
// (M+1) x (M+1) x (M/2+1) doubles, so every shift alpha -/+ k e_d of the
// Hermite algebra is a compile-time LDS offset.
// Global memory holds cell records [u1, u2, theta, f_0 .. f_{N-1}] in the
// graded order of the C ABI, one record per cell, row-major.
#pragma once
#include <math.h>

#include "nrxx_internal.hpp"

namespace nrxx {
namespace {

constexpr int WAVE = 64;

__host__ __device__ constexpr int neven(int M) {
  int c = 0;
  for (int m = 0; 2 * m <= M; ++m) {
    int r = M - 2 * m;
    c += (r + 1) * (r + 2) / 2;
  }
  return c;
}
constexpr int NEMAX = neven(MMAX);
constexpr int NMAX = nalpha(MMAX);

// Coefficients with even alpha_3, in the graded order (a prefix of this list
// is the list for any smaller M).
struct EvenTab {
  uint8_t a1[NEMAX], a2[NEMAX], m[NEMAX];
  uint16_t ci[NEMAX];  // position in the full graded order
};
constexpr EvenTab make_even_tab() {
  EvenTab t{};
  int k = 0, ci = 0;
  for (int n = 0; n <= MMAX; ++n)
    for (int a1 = n; a1 >= 0; --a1)
      for (int a2 = n - a1; a2 >= 0; --a2, ++ci) {
        int a3 = n - a1 - a2;
        if (a3 & 1) continue;
        t.a1[k] = (uint8_t)a1;
        t.a2[k] = (uint8_t)a2;
        t.m[k] = (uint8_t)(a3 / 2);
        t.ci[k] = (uint16_t)ci;
        ++k;
      }
  return t;
}
// Full graded order: alpha of each position.
struct CanonTab {
  uint8_t a1[NMAX], a2[NMAX], a3[NMAX];
};
constexpr CanonTab make_canon_tab() {
  CanonTab t{};
  int k = 0;
  for (int n = 0; n <= MMAX; ++n)
    for (int a1 = n; a1 >= 0; --a1)
      for (int a2 = n - a1; a2 >= 0; --a2) {
        t.a1[k] = (uint8_t)a1;
        t.a2[k] = (uint8_t)a2;
        t.a3[k] = (uint8_t)(n - a1 - a2);
        ++k;
      }
  return t;
}
struct FactTab {
  double v[2 * MMAX + 4];
  double inv[2 * MMAX + 4];
};
constexpr FactTab make_fact_tab() {
  FactTab t{};
  double f = 1.0;
  t.v[0] = 1.0;
  t.inv[0] = 1.0;
  for (int n = 1; n < 2 * MMAX + 4; ++n) {
    f *= n;
    t.v[n] = f;
    t.inv[n] = 1.0 / f;
  }
  return t;
}

__constant__ EvenTab c_even = make_even_tab();
__constant__ CanonTab c_canon = make_canon_tab();
__constant__ FactTab c_fact = make_fact_tab();

template <int M>
struct G {
  static constexpr int N = nalpha(M);
  static constexpr int NR = N + 3;
  static constexpr int STRIDE = record_stride(M);
  static constexpr int D1 = M + 1;
  static constexpr int D2 = (M + 1) * (M + 1);
  static constexpr int MH = M / 2 + 1;
  static constexpr int CUBE = D2 * MH;
  static constexpr int NE = neven(M);
  static constexpr int SL = (NE + WAVE - 1) / WAVE;  // even-alpha slots per lane
  static constexpr int SR = (NR + WAVE - 1) / WAVE;  // record entries per lane
  static constexpr int SLOT = SL * WAVE;             // one per-slot buffer
  static constexpr int KOFF = 0;                     // K_n(a), n = 0 .. 2M+1
  static constexpr int JOFF = 2 * M + 2;             // J+_{kl}(a), (M+1)^2
  static constexpr int BOFF = JOFF + (M + 1) * (M + 1);  // broadcast slots
  static constexpr int MISC = BOFF + 16;
  // cube addresses of coefficients used by name
  static constexpr int E1 = 1, E2 = D1, XX = 2, YY = 2 * D1, ZZ = D2;
  static constexpr int X3 = 3, X1Y2 = 1 + 2 * D1, X1Z2 = 1 + D2;
  static constexpr int Y3 = 3 * D1, X2Y1 = 2 + D1, Y1Z2 = D1 + D2;
  static constexpr int XY = 1 + D1;
};

// LDS layout (in doubles) of a cell team of NW wavefronts (the last one also
// evaluates the cell-local terms).
template <int M, int NW>
struct Lay {
  using g = G<M>;
  static constexpr int C = 0;                      // cell coefficients (cube)
  static constexpr int F = C + g::CUBE;            // 8 face states (cubes), item q = f + 4 s
  static constexpr int WSZ = 3 * g::CUBE + g::MISC;
  static constexpr int W = F + 8 * g::CUBE;        // per-wavefront scratch, NW
  static constexpr int T = W + NW * WSZ;           // 12 partial results (per-slot layout)
  static constexpr int GR = T + 12 * g::SLOT;      // 4 face regularisation terms (per slot)
  static constexpr int S = GR + 4 * g::SLOT;       // scalars
  static constexpr int TOTAL = S + 64;
  // partial results: 0..7 face-side items, 8 right-hand side (or the
  // coarse-problem residual), 9 collision, 10/11 in-cell regularisation x/y
  static constexpr int T_RHS = 8, T_Q = 9, T_GX = 10;
  // scalar slots
  static constexpr int SP = 0;    // face-state parameters, 8 x 4
  static constexpr int SW = 32;   // weight of the regularisation jump per face, 4
  static constexpr int SC = 36;   // cell u1, u2, th
  static constexpr int SNU = 40;  // collision frequency of the cell
  static constexpr int SAB = 41;  // team flag: abort
};

// Order LDS traffic of one wavefront: a wavefront-scope fence is a compiler
// memory barrier; the LDS executes one wavefront's instructions in order.
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int M>
struct Slots {
  using g = G<M>;
  int ca[g::SL], ci[g::SL], a1[g::SL], a2[g::SL], m[g::SL], n[g::SL];
  bool ok[g::SL];
  __device__ __forceinline__ void init(int lane) {
#pragma unroll
    for (int r = 0; r < g::SL; ++r) {
      int e = lane + WAVE * r;
      ok[r] = e < g::NE;
      int ee = ok[r] ? e : 0;
      a1[r] = c_even.a1[ee];
      a2[r] = c_even.a2[ee];
      m[r] = c_even.m[ee];
      ci[r] = c_even.ci[ee];
      n[r] = a1[r] + a2[r] + 2 * m[r];
      ca[r] = a1[r] + g::D1 * a2[r] + g::D2 * m[r];
    }
  }
};

// Per-wavefront scratch and slot map.
template <typename Real, int M>
struct Wave {
  using g = G<M>;
  Real *bX, *bA, *bB, *misc;
  int lane;
  Slots<M> S;
  // pre: the lane's slot map built once by the caller (a kernel that loops
  // over cells passes it, so the table reads stay out of its loop), or null
  __device__ __forceinline__ void init(Real *base, int ln, const Slots<M> *pre = nullptr) {
    bX = base;
    bA = base + g::CUBE;
    bB = base + 2 * g::CUBE;
    misc = base + 3 * g::CUBE;
    lane = ln;
    if (pre) S = *pre;
    else S.init(ln);
  }
};

// Basis parameters (uniform) and the lane's coefficients of one record.
template <typename Real, int M>
struct Cell {
  Real u1, u2, th;
  Real f[G<M>::SL];
};

template <typename Real, int M>
__device__ __forceinline__ void load_cell(const Real *__restrict__ rec, const Slots<M> &S,
                                          Cell<Real, M> &c) {
  c.u1 = rec[0];
  c.u2 = rec[1];
  c.th = rec[2];
#pragma unroll
  for (int r = 0; r < G<M>::SL; ++r) c.f[r] = S.ok[r] ? rec[3 + S.ci[r]] : Real(0.0);
}

template <typename Real, int M>
__device__ __forceinline__ void put(Real *buf, const Slots<M> &S, const Real (&v)[G<M>::SL]) {
#pragma unroll
  for (int r = 0; r < G<M>::SL; ++r)
    if (S.ok[r]) buf[S.ca[r]] = v[r];
}

template <typename Real, int M>
__device__ __forceinline__ void put_slots(Real *buf, int lane, const Real (&v)[G<M>::SL]) {
#pragma unroll
  for (int r = 0; r < G<M>::SL; ++r) buf[lane + WAVE * r] = v[r];
}

template <typename Real, int M>
__device__ __forceinline__ void get_slots(const Real *buf, int lane, Real (&v)[G<M>::SL]) {
#pragma unroll
  for (int r = 0; r < G<M>::SL; ++r) v[r] = buf[lane + WAVE * r];
}

// Publishing a cell to the other workgroups of a sweep.  Each XCD has its
// own L2, so an agent-scope release fence writes back every dirty line of
// the XCD's L2 (buffer_wbl2) before the flag store; with thousands of
// wavefronts each releasing a cell every few microseconds that write-back
// dominated the sweep (2.6x slower at M = 5).  The records a sweep publishes
// are instead stored with agent-scope atomic stores, which are performed at
// the device's coherence point when they complete, so the flag store only has
// to follow the completion of this wavefront's stores: the release sequence
// without the write-back.  Readers keep the agent-scope acquire.
template <typename Real>
__device__ __forceinline__ void put_shared(Real *p, Real v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sets *flag = value once every store this wavefront issued before has
// completed (the cell's record was written with put_shared).  Called by the
// wavefront that stored the record.
__device__ __forceinline__ void publish(int *flag, int value) {
  __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
  __hip_atomic_store(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Coalesced write of a full record from (params, LDS cube); odd-alpha_3
// coefficients are written as zeros.
template <typename Real, int M, bool SHARED = false>
__device__ __forceinline__ void store_record(Real *__restrict__ rec, Real u1, Real u2,
                                             Real th, const Real *cube, int lane) {
  using g = G<M>;
#pragma unroll
  for (int t = 0; t < g::SR; ++t) {
    int v = lane + WAVE * t;
    if (v < g::NR) {
      Real x;
      if (v == 0) x = u1;
      else if (v == 1) x = u2;
      else if (v == 2) x = th;
      else {
        int al = v - 3;
        int a1 = c_canon.a1[al], a2 = c_canon.a2[al], a3 = c_canon.a3[al];
        x = (a3 & 1) ? Real(0.0) : cube[a1 + g::D1 * a2 + g::D2 * (a3 >> 1)];
      }
      if constexpr (SHARED) put_shared(rec + v, x);
      else rec[v] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// Hermite algebra on one wavefront
// ---------------------------------------------------------------------------

// Taylor coefficients of exp(-du t - dth t^2 / 2): the 1-D factors of the
// exact re-expansion F_M^[u,th] -> F_M^[u+du, th+dth] (Sec. 2.3).
template <typename Real, int M>
__device__ __forceinline__ void tcoef(Real du, Real dth, Real (&c)[M + 1]) {
  c[0] = Real(1.0);
  c[1] = -du;
#pragma unroll
  for (int k = 1; k < M; ++k) c[k + 1] = (-du * c[k] - dth * c[k - 1]) * (Real(1.0) / (k + 1));
}

// res = T(in) for the basis change by (du1, du2, dth): three 1-D lower-
// triangular convolutions along alpha_1, alpha_2, alpha_3.  in, t1, t2 are
// distinct LDS cubes; the result stays in registers.  Terms beyond alpha_d
// read a valid address with a zero coefficient, so every LDS read of a pass
// is issued at once (adding fma(0, x, acc) leaves acc unchanged).
template <typename Real, int M>
__device__ __forceinline__ void bchange(const Real *in, Real *t1, Real *t2, Real du1,
                                        Real du2, Real dth, const Slots<M> &S,
                                        Real (&res)[G<M>::SL]) {
  using g = G<M>;
  Real c[M + 1];
  tcoef<Real, M>(du1, dth, c);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    const Real *p = in + S.ca[r];
    Real x[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) x[k] = p[k <= S.a1[r] ? -k : 0];
    Real acc = x[0];
#pragma unroll
    for (int k = 1; k <= M; ++k) acc = fma(k <= S.a1[r] ? c[k] : Real(0.0), x[k], acc);
    if (S.ok[r]) t1[S.ca[r]] = acc;
  }
  wsync();
  tcoef<Real, M>(du2, dth, c);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    const Real *p = t1 + S.ca[r];
    Real x[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) x[k] = p[k <= S.a2[r] ? -k * g::D1 : 0];
    Real acc = x[0];
#pragma unroll
    for (int k = 1; k <= M; ++k) acc = fma(k <= S.a2[r] ? c[k] : Real(0.0), x[k], acc);
    if (S.ok[r]) t2[S.ca[r]] = acc;
  }
  wsync();
  tcoef<Real, M>(Real(0.0), dth, c);  // u_3 = 0 on both sides: only even powers survive
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    const Real *p = t2 + S.ca[r];
    Real x[M / 2 + 1];
#pragma unroll
    for (int k = 0; 2 * k <= M; ++k) x[k] = p[k <= S.m[r] ? -k * g::D2 : 0];
    Real acc = x[0];
#pragma unroll
    for (int k = 1; 2 * k <= M; ++k) acc = fma(k <= S.m[r] ? c[2 * k] : Real(0.0), x[k], acc);
    res[r] = S.ok[r] ? acc : Real(0.0);
  }
  wsync();
}

// (Pi_M xi_d f)_alpha = th f_{alpha-e_d} + u_d f_alpha + (alpha_d+1) f_{alpha+e_d}
template <typename Real, int M>
__device__ __forceinline__ Real ximul(int D, const Real *f, Real ud, Real th,
                                        const Slots<M> &S, int r) {
  const int st = D == 0 ? 1 : G<M>::D1;
  const Real *p = f + S.ca[r];
  const int ad = D == 0 ? S.a1[r] : S.a2[r];
  const Real x0 = p[0], xl = p[ad >= 1 ? -st : 0], xh = p[S.n[r] < M ? st : 0];
  Real v = ud * x0;
  if (ad >= 1) v += th * xl;
  if (S.n[r] < M) v += (ad + 1) * xh;
  return v;
}

// Regularisation term of direction D at |beta| = M (zero below):
// (beta_D + 1) [sum_k f_{b+e_D-e_k} du_k + 1/2 sum_k f_{b+e_D-2e_k} dth],
// du_3 = 0, taken of (fL + fR) / 2 (fR may equal fL for the in-cell term).
template <typename Real, int M>
__device__ __forceinline__ Real regul(int D, const Real *fL, const Real *fR, Real du1,
                                        Real du2, Real dth, const Slots<M> &S, int r) {
  using g = G<M>;
  if (!S.ok[r] || S.n[r] != M) return Real(0.0);
  const int base = S.ca[r] + (D == 0 ? 1 : g::D1);  // b + e_D
  const int b0 = S.a1[r] + (D == 0), b1 = S.a2[r] + (D == 1), b2 = 2 * S.m[r];
  Real acc = Real(0.0);
  if (b0 >= 1) acc += Real(0.5) * (fL[base - 1] + fR[base - 1]) * du1;
  if (b0 >= 2) acc += Real(0.5) * (Real(0.5) * (fL[base - 2] + fR[base - 2])) * dth;
  if (b1 >= 1) acc += Real(0.5) * (fL[base - g::D1] + fR[base - g::D1]) * du2;
  if (b1 >= 2) acc += Real(0.5) * (Real(0.5) * (fL[base - 2 * g::D1] + fR[base - 2 * g::D1])) * dth;
  // k = 3: du_3 = 0, and b - e_3 has odd alpha_3
  if (b2 >= 2) acc += Real(0.5) * (Real(0.5) * (fL[base - g::D2] + fR[base - g::D2])) * dth;
  const int bd = D == 0 ? S.a1[r] : S.a2[r];
  return (bd + 1) * acc;
}

// ES-BGK equilibrium of eq. (7) in the cell's own basis [u, th]: the
// Gaussian of covariance Lambda = th I + B, B = (1 - 1/Pr) sigma / rho, has
// the coefficients f^E_alpha = rho [t^alpha] exp(t^T B t / 2) (the generating
// function of the Hermite polynomials; the powers of th cancel).  In the
// plane flow sigma_13 = sigma_23 = 0, so the series factorises:
// [t1^a1 t2^a2] exp(B11 t1^2 / 2 + B12 t1 t2 + B22 t2^2 / 2) =
//   sum_k B12^k / k! (B11 / 2)^i1 / i1! (B22 / 2)^i2 / i2!, i_d = (a_d - k) / 2,
// times [t3^2m] exp(B33 t3^2 / 2) = (B33 / 2)^m / m!.
template <typename Real>
__device__ __forceinline__ Real esbgk_coef(int a1, int a2, int m, Real rho, Real b11, Real b12,
                                           Real b22, Real b33) {
  if ((a1 ^ a2) & 1) return Real(0.0);
  const Real h11 = Real(0.5) * b11, h22 = Real(0.5) * b22, h33 = Real(0.5) * b33;
  Real z = Real(1.0);
  for (int q = 1; q <= m; ++q) z = z * h33 / Real(q);
  const int kmax = a1 < a2 ? a1 : a2;
  Real acc = Real(0.0);
  for (int k = a1 & 1; k <= kmax; k += 2) {
    Real t = Real(1.0);
    for (int q = 1; q <= k; ++q) t = t * b12 / Real(q);
    for (int q = 1; q <= (a1 - k) / 2; ++q) t = t * h11 / Real(q);
    for (int q = 1; q <= (a2 - k) / 2; ++q) t = t * h22 / Real(q);
    acc += t;
  }
  return rho * acc * z;
}

template <typename Real>
__device__ __forceinline__ Real minmod(Real a, Real b) {
  if (a > Real(0.0) && b > Real(0.0)) return fmin(a, b);
  if (a < Real(0.0) && b < Real(0.0)) return fmax(a, b);
  return Real(0.0);
}

template <typename Real>
__device__ __forceinline__ Real limited(int limiter, Real hi, Real c, Real lo) {
  return limiter == 1 ? Real(0.5) * (hi - lo) : minmod<Real>(hi - c, c - lo);
}

// Probabilists' Hermite polynomial He_n(x), 0 <= n <= NMAX, by recurrence;
// the recurrence runs to NMAX for every n (unrolled, no lane-dependent trip
// count) and keeps step n.
template <typename Real, int NMAX>
__device__ __forceinline__ Real hermite(int n, Real x) {
  Real h0 = Real(1.0), h1 = x;
  Real hn = n == 0 ? Real(1.0) : x;
#pragma unroll
  for (int k = 1; k < NMAX; ++k) {
    const Real h2 = x * h1 - Real(k) * h0;
    h0 = h1;
    h1 = h2;
    if (k + 1 == n) hn = h1;
  }
  return hn;
}

// I_kl(a) = (2 pi)^-1/2 int_{-a}^inf He_k He_l e^{-w^2/2} dw from the
// half-range moments K_n (in LDS) and He_k He_l = sum_j k! l! / (j! (k-j)!
// (l-j)!) He_{k+l-2j}.  The integer coefficient is carried as a running
// product, c_j = c_{j-1} (k-j+1) (l-j+1) / j (every step divides exactly;
// in 64 bits, as the products pass 2^31 at M = 10; the c_j stay below 2^24,
// exact in FP32, for the M <= 8 of the FP32 kernels), so the loop reads no
// table from global memory, whose cached lines the acquires of the sweep
// kernels keep invalidating.  (Unrolling this loop spills registers in the
// sweep kernels.)
template <typename Real>
__device__ __forceinline__ Real halfI(const Real *K, int k, int l) {
  if (l < 0) return Real(0.0);
  const int jm = k < l ? k : l;
  Real acc = K[k + l];
  long long cf = 1;
  for (int j = 1; j <= jm; ++j) {
    cf = cf * (k - j + 1) * (l - j + 1) / j;
    acc += Real(cf) * K[k + l - 2 * j];
  }
  return acc;
}

// Half-range tables of a diffuse wall: K_n(a), n <= 2M+1, and J+_kl(a),
// k, l <= M, in the wavefront's misc scratch.  They depend on the cell only
// through a = sig u_d / sqrt(th), so a cell team can build them before it
// has the cell's coefficients in LDS; wall_flux then reads them.
template <typename Real, int M>
__device__ void wall_tables(int wall, Real u1, Real u2, Real th, Wave<Real, M> &W) {
  using g = G<M>;
  const int lane = W.lane;
  const int d = (wall == 0 || wall == 2) ? 1 : 0;
  const Real sig = (wall == 1 || wall == 2) ? Real(1.0) : -Real(1.0);
  const Real a = sig * (d == 0 ? u1 : u2) / sqrt(th);
  Real *K = W.misc + g::KOFF;
  Real *Jp = W.misc + g::JOFF;
  // K_n(a) = (2 pi)^-1/2 int_{-a}^inf He_n e^{-w^2/2}
  const Real ga = exp(-Real(0.5) * a * a) * (Real(0.5) * Real(M_2_SQRTPI) * Real(M_SQRT1_2));
  for (int n = lane; n <= 2 * M + 1; n += WAVE)
    K[n] = n == 0 ? Real(0.5) * erfc(-a * Real(M_SQRT1_2)) : hermite<Real, 2 * M>(n - 1, -a) * ga;
  wsync();
  // J+_kl(a) = a I_kl + I_{k,l+1} + l I_{k,l-1}
  for (int t = lane; t < (M + 1) * (M + 1); t += WAVE) {
    int k = t / (M + 1), l = t % (M + 1);
    Jp[t] = a * halfI<Real>(K, k, l) + halfI<Real>(K, k, l + 1) + l * halfI<Real>(K, k, l - 1);
  }
  wsync();
}

// Outward flux through a diffuse wall in the cell basis (reading of the
// Maxwell boundary condition of Sec. 2.3 / Sec. 4): the leaving half-range
// of the cell distribution plus the entering half of the wall Maxwellian,
// whose density makes the net mass flux zero.  fc: the cell's coefficients
// (LDS cube).  The same wavefront has built the wall's tables (wall_tables)
// for the same (wall, u1, u2, th).
template <typename Real, int M>
__device__ void wall_flux(const LevelArgs &A, int wall, Real u1, Real u2, Real th,
                          const Real *fc, Wave<Real, M> &W, Real (&phi)[G<M>::SL]) {
  using g = G<M>;
  const Slots<M> &S = W.S;
  const int lane = W.lane;
  const int d = (wall == 0 || wall == 2) ? 1 : 0;
  const Real sig = (wall == 1 || wall == 2) ? Real(1.0) : -Real(1.0);
  const Real sq = sqrt(th);
  const Real *Jp = W.misc + g::JOFF;
  Real *bc = W.misc + g::BOFF;
  // leaving half: sum_{beta_d} f_beta th^{(a_d-b_d)/2} sqrt(th) sig^{a_d+b_d} J+_{a_d b_d} / a_d!
  const Real isq = Real(1.0) / sq;
  const int dst = d == 0 ? 1 : g::D1;
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    Real acc = Real(0.0);
    if (S.ok[r]) {
      int ad = d == 0 ? S.a1[r] : S.a2[r];
      int at = (d == 0 ? S.a2[r] : S.a1[r]) + 2 * S.m[r];  // transverse degree
      int base = S.ca[r] - ad * dst;                      // alpha with alpha_d = 0
      Real pa = Real(1.0), fa = Real(1.0);
      for (int q = 0; q < ad; ++q) {
        pa *= sq;
        fa *= Real(q + 1);
      }
      const Real ifa = Real(1.0) / fa;  // 1 / a_d!, exact factorial, one rounding
      Real ib = Real(1.0);
#pragma unroll
      for (int bd = 0; bd <= M; ++bd) {
        if (bd + at <= M) {
          Real sgn = ((ad + bd) & 1) ? sig : Real(1.0);
          acc += fc[base + bd * dst] * (pa * ib) * sq * sgn * Jp[ad * (M + 1) + bd] * ifa;
        }
        ib *= isq;
      }
    }
    phi[r] = acc;
  }
  // wall density from zero net mass flux; phi_0 lives in lane 0, slot 0
  if (lane == 0) bc[0] = phi[0];
  wsync();
  const Real thw = Real(A.wall_th[wall]), sqw = sqrt(thw);
  const Real rhow = bc[0] * sqrt(Real(2.0) * Real(M_PI) / thw);
  // entering half in the wall basis: only alpha = k e_d is non-zero
#pragma unroll
  for (int r = 0; r < g::SL; ++r)
    if (S.ok[r]) W.bX[S.ca[r]] = Real(0.0);
  wsync();
  if (lane <= M) {
    int k = lane;
    Real pw = Real(1.0);
    for (int q = 0; q < k; ++q) pw *= sqw;
    Real sgn = (k & 1) ? sig : Real(1.0);
    W.bX[k * dst] = rhow * pw * sqw * sgn * Real(A.jminus[k]);
  }
  wsync();
  const Real uw1 = d == 1 ? Real(A.wall_u[wall]) : Real(0.0), uw2 = d == 0 ? Real(A.wall_u[wall]) : Real(0.0);
  Real t[g::SL];
  bchange<Real, M>(W.bX, W.bA, W.bB, u1 - uw1, u2 - uw2, th - thw, S, t);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) phi[r] += t[r];
}

// Face state of `c` on side `side` of a direction (eq. (15)): every variable
// v -> v + side/2 * limited slope; zero slope when `flat`.
template <typename Real, int M>
__device__ __forceinline__ void face_state(const Cell<Real, M> &c, const Cell<Real, M> &hi, const Cell<Real, M> &lo,
                                           int limiter, bool flat, Real side, Cell<Real, M> &out) {
  if (flat) {
    out = c;
    return;
  }
  out.u1 = c.u1 + Real(0.5) * side * limited<Real>(limiter, hi.u1, c.u1, lo.u1);
  out.u2 = c.u2 + Real(0.5) * side * limited<Real>(limiter, hi.u2, c.u2, lo.u2);
  out.th = c.th + Real(0.5) * side * limited<Real>(limiter, hi.th, c.th, lo.th);
#pragma unroll
  for (int r = 0; r < G<M>::SL; ++r)
    out.f[r] = c.f[r] + Real(0.5) * side * limited<Real>(limiter, hi.f[r], c.f[r], lo.f[r]);
}

// Local time step of eq. (18), capped so that nu dt <= nu_cap when nu_cap > Real(0.)
template <typename Real>
__device__ __forceinline__ Real local_dt(const LevelArgs &A, Real u1, Real u2, Real th,
                                           Real nu) {
  const Real sq = sqrt(th);
  Real dt = Real(A.cfl) / ((fabs(u1) + Real(A.C) * sq) * Real(A.idx) + (fabs(u2) + Real(A.C) * sq) * Real(A.idy));
  if (Real(A.nu_cap) > Real(0.0) && nu * dt > Real(A.nu_cap)) dt = Real(A.nu_cap) / nu;
  return dt;
}

// Two-step update of Sec. 2.4: new (u, th) from the coefficients fs given in
// the old basis (eq. (3)), re-expansion, and the exact constraints of
// eq. (10).  Result left in cube W.bA and in out; false for rho <= 0,
// th <= 0 or non-finite values.
template <typename Real, int M>
__device__ bool normalise(Real ou1, Real ou2, Real oth, const Real (&fs)[G<M>::SL],
                          Wave<Real, M> &W, Cell<Real, M> &out) {
  using g = G<M>;
  put<Real, M>(W.bX, W.S, fs);
  wsync();
  const Real rho = W.bX[0];
  const Real fe1 = W.bX[g::E1], fe2 = W.bX[g::E2];
  const Real tr = W.bX[g::XX] + W.bX[g::YY] + W.bX[g::ZZ];
  const Real irho = Real(1.0) / rho;
  const Real u1n = ou1 + fe1 * irho, u2n = ou2 + fe2 * irho;
  const Real thn = oth + (Real(2.0) * tr - (fe1 * fe1 + fe2 * fe2) * irho) * (irho * (Real(1.0) / Real(3.0)));
  bool okp = rho > Real(0.0) && thn > Real(0.0) && isfinite(rho) && isfinite(thn) && isfinite(u1n) &&
             isfinite(u2n);
  if (!okp) return false;  // uniform branch
  Real t[g::SL];
  bchange<Real, M>(W.bX, W.bA, W.bB, u1n - ou1, u2n - ou2, thn - oth, W.S, t);
  put<Real, M>(W.bA, W.S, t);
  wsync();
  const Real zz = -(W.bA[g::XX] + W.bA[g::YY]);
  bool fin = true;
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    const int ca = W.S.ca[r];
    if (ca == g::E1 || ca == g::E2) t[r] = Real(0.0);
    if (ca == g::ZZ) t[r] = zz;
    if (W.S.ok[r] && !isfinite(t[r])) fin = false;
  }
  wsync();
  if (W.lane < 2) W.bA[W.lane == 0 ? g::E1 : g::E2] = Real(0.0);
  if (W.lane == 0) W.bA[g::ZZ] = zz;
  wsync();
  out.u1 = u1n;
  out.u2 = u2n;
  out.th = thn;
#pragma unroll
  for (int r = 0; r < g::SL; ++r) out.f[r] = t[r];
  return __ballot(!fin) == 0;
}

template <typename Real, int M>
__device__ __forceinline__ const Real *recp(const LevelArgs &A, const Real *st, int i, int j) {
  return st + ((size_t)j * A.nx + i) * G<M>::STRIDE;
}

// ---------------------------------------------------------------------------
// The cell team: R_ij(f) of eq. (13) and what is done with it
// ---------------------------------------------------------------------------

enum { MODE_SWEEP = 0, MODE_DEFECT = 1, MODE_FAS = 2 };

// Faces: 0 = E (+x), 1 = W (-x), 2 = N (+y), 3 = S (-y).  Item q = f + 4 s:
// s = 0 the cell's own face state, s = 1 the neighbour's.
__device__ __forceinline__ int face_dir(int f) { return f >> 1; }
__device__ __forceinline__ int face_side(int f) { return (f & 1) ? -1 : 1; }
__device__ __forceinline__ int face_wall(int f) { return f == 0 ? 1 : f == 1 ? 3 : f == 2 ? 2 : 0; }

// Evaluate cell (i, j) with a team of NW wavefronts and
//  MODE_SWEEP : update the cell in place (Alg. 1): f <- normalise(f + dt (R - r)),
//  MODE_DEFECT: out = r - R(f) in the cell basis, norm_part[cell] = weighted norm^2 * ds,
//  MODE_FAS   : out = R(f) + Radd (coarse right-hand side of eq. (22)).
// Every wavefront returns; the team's LDS may be reused after a barrier.
// A non-physical update sets bit 0 of *err and leaves the cell unchanged.
// With SPLIT, the team first evaluates everything that reads only the
// cell's own grid column (the four y-direction face-side items, collision,
// y in-cell regularisation, right-hand side), then thread 0 calls wait()
// (which must make the neighbouring columns' data visible and return false
// to abort), and only then the four x-direction items and the x in-cell
// regularisation.  Each item's arithmetic and the order of assembly are the
// same in both forms, so the results are bitwise identical; returns false
// (uniformly) if wait() failed, leaving the cell untouched.
struct NoWait {
  __device__ bool operator()() const { return true; }
};

template <typename Real, int M, int ORDER, int NW, int MODE, bool SPLIT = false,
          typename Wait = NoWait>
__device__ bool cell_team(const LevelArgs &A, Real *lds, Real *__restrict__ st,
                          const Real *__restrict__ rhs, const Real *__restrict__ Radd,
                          Real *__restrict__ out, Real *__restrict__ norm_part, int i, int j,
                          int *err, Wait wait = Wait(), const Slots<M> *slots = nullptr) {
  using g = G<M>;
  using L = Lay<M, NW>;
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  Wave<Real, M> W;
  W.init(lds + L::W + wv * L::WSZ, lane, slots);
  const Slots<M> &S = W.S;
  Real *bC = lds + L::C;
  Real *sc = lds + L::S;
  const int nx = A.nx, ny = A.ny;
  const int cellidx = j * nx + i;

  // ---- phase 0: face states of this wavefront's items -------------------
  Cell<Real, M> c;
  load_cell<Real, M>(recp<Real, M>(A, st, i, j), S, c);
  if (wv == NW - 1) {
    put<Real, M>(bC, S, c.f);
    // collision frequency of eq. (29); rho = f_0 sits in lane 0, slot 0
    const Real rho = __shfl(c.f[0], 0);
    const Real nu = Real(A.beta) * sqrt(Real(M_PI) / Real(2.0)) * rho * pow(c.th, Real(1.0) - Real(A.omega)) / Real(A.Kn);
    if (lane == 0) {
      sc[L::SC] = c.u1;
      sc[L::SC + 1] = c.u2;
      sc[L::SC + 2] = c.th;
      sc[L::SNU] = nu;
    }
  }
  // item q = f + 4 s: face f (0 E, 1 W, 2 N, 3 S), s = 0 the cell's own face
  // state, s = 1 the neighbour's.  Items of a pass are spread over the
  // wavefronts: all eight in one pass, or y items (2, 3, 6, 7) then x items
  // (0, 1, 4, 5) when split.
  // Unsplit, wavefront wv takes items wv, wv + NW, ... in a run-time loop
  // (one copy of the item code keeps register use low for the many-cell
  // kernels).  Split, pass 0 spreads the y items 2, 3, 6, 7 over wavefronts
  // 0, 1, 2, 3 (mod NW) and pass 1 the x items 0, 1, 4, 5 over wavefronts
  // NW-1, NW-2, ... (mod NW), unrolled.  An own x item on a wall face (E of
  // the last column, W of the first) reads nothing but the cell itself, so it
  // moves to pass 0, on a wavefront that has no y item there when NW = 8:
  // the wall flux is the longest item, and in pass 1 it would sit on the
  // critical path of every wall cell -- and the wall column paces the whole
  // sweep.  Each item still runs the same code, so results do not change.
  // Only for M <= 5: at larger M the second inlined copy of the item code
  // spills registers.
  constexpr bool MOVE = SPLIT && M <= 5;
  constexpr int wE = NW >= 8 ? 4 : (NW >= 4 ? 2 : 0);  // wavefront of a moved E wall item
  constexpr int wW = NW >= 8 ? 5 : (NW >= 4 ? 3 : 0);  // and of a moved W wall item
  auto for_items = [&](int pass, auto &&body) {
    if constexpr (SPLIT) {
      const bool wallE = MOVE && i == nx - 1, wallW = MOVE && i == 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int w = pass == 0 ? t % NW : (NW - 1 - t % NW + NW) % NW;
        if (w != wv) continue;
        if (pass == 1 && ((t == 0 && wallE) || (t == 1 && wallW))) continue;
        body(pass == 0 ? (t < 2 ? 2 + t : 4 + t) : (t < 2 ? t : 2 + t));
      }
      if (MOVE && pass == 0) {
        if (wallE && wv == wE) body(0);
        if (wallW && wv == wW) body(1);
      }
    } else {
#pragma unroll 1
      for (int q = wv; q < 8; q += NW) body(q);
    }
  };

  // With NW >= 4 no wavefront holds two own items (the only ones that can
  // sit on a wall), so a wall's half-range tables are built here, in the
  // face-state stage, while the other wavefronts form their face states,
  // and stay in the wavefront's scratch until its flux stage.
  constexpr bool EARLY_TABLES = NW >= 4;
  auto face_states = [&](int pass) {
  for_items(pass, [&](const int q) {
    const int f = q & 3, s = q >> 2, D = face_dir(f);
    const Real side = (Real)face_side(f);
    const int k = D == 0 ? i : j, n = D == 0 ? nx : ny;
    const int sd = (int)side;
    const bool wall = (k + sd < 0) || (k + sd >= n);
    Cell<Real, M> X;
    if (s == 0) {
      const bool flat = ORDER == 1 || k == 0 || k == n - 1;
      if (EARLY_TABLES && wall) wall_tables<Real, M>(face_wall(f), c.u1, c.u2, c.th, W);
      if (flat) X = c;
      else {
        Cell<Real, M> hi, lo;
        load_cell<Real, M>(D == 0 ? recp<Real, M>(A, st, i + 1, j) : recp<Real, M>(A, st, i, j + 1), S, hi);
        load_cell<Real, M>(D == 0 ? recp<Real, M>(A, st, i - 1, j) : recp<Real, M>(A, st, i, j - 1), S, lo);
        face_state<Real, M>(c, hi, lo, A.limiter, false, side, X);
      }
    } else {
      if (wall) return;
      const int kn = k + sd;
      const bool nflat = ORDER == 1 || kn == 0 || kn == n - 1;
      Cell<Real, M> nb;
      load_cell<Real, M>(D == 0 ? recp<Real, M>(A, st, i + sd, j) : recp<Real, M>(A, st, i, j + sd), S, nb);
      if (nflat) X = nb;
      else {
        Cell<Real, M> far;
        load_cell<Real, M>(D == 0 ? recp<Real, M>(A, st, i + 2 * sd, j) : recp<Real, M>(A, st, i, j + 2 * sd), S, far);
        // neighbour's face on the cell's side: slope from (far, nb, c)
        if (sd > 0) face_state<Real, M>(nb, far, c, A.limiter, false, -side, X);
        else face_state<Real, M>(nb, c, far, A.limiter, false, -side, X);
      }
    }
    put<Real, M>(lds + L::F + q * g::CUBE, S, X.f);
    if (lane == 0) {
      sc[L::SP + 4 * q] = X.u1;
      sc[L::SP + 4 * q + 1] = X.u2;
      sc[L::SP + 4 * q + 2] = X.th;
    }
  });
  };

  // ---- phase 1: half-fluxes projected into the cell basis ---------------
  auto fluxes = [&](int pass) {
  for_items(pass, [&](const int q) {
    const int f = q & 3, s = q >> 2, D = face_dir(f);
    const Real side = (Real)face_side(f);
    const int k = D == 0 ? i : j, n = D == 0 ? nx : ny;
    const int sd = (int)side;
    const bool wall = (k + sd < 0) || (k + sd >= n);
    Real T[g::SL];
    if (wall) {
      if (s == 1) return;
      if (!EARLY_TABLES) wall_tables<Real, M>(face_wall(f), c.u1, c.u2, c.th, W);
      wall_flux<Real, M>(A, face_wall(f), c.u1, c.u2, c.th, bC, W, T);
      put_slots<Real, M>(lds + L::T + q * g::SLOT, lane, T);
      return;
    }
    // L / R face states: the cell is left of its E and N faces
    const int qo = f, qn = f + 4;
    const int qL = sd > 0 ? qo : qn, qR = sd > 0 ? qn : qo;
    const Real uL = sc[L::SP + 4 * qL + D], thL = sc[L::SP + 4 * qL + 2];
    const Real uR = sc[L::SP + 4 * qR + D], thR = sc[L::SP + 4 * qR + 2];
    const Real cL = Real(A.C) * sqrt(thL), cR = Real(A.C) * sqrt(thR);
    const Real lamL = fmin(uL - cL, uR - cR);
    const Real lamR = fmax(uL + cL, uR + cR);
    int kase;
    Real wm, wp;
    const Real iden = Real(1.0) / (lamR - lamL);
    if (lamL >= Real(0.0)) { kase = 0; wm = Real(0.0); wp = Real(1.0); }
    else if (lamR <= Real(0.0)) { kase = 1; wm = Real(1.0); wp = Real(0.0); }
    else { kase = 2; wm = -lamL * iden; wp = lamR * iden; }
    const bool isL = q == qL;
    const Real *fx = lds + L::F + q * g::CUBE;
    const Real ux = sc[L::SP + 4 * q + D], thx = sc[L::SP + 4 * q + 2];
    if ((isL && kase == 1) || (!isL && kase == 0)) {
#pragma unroll
      for (int r = 0; r < g::SL; ++r) T[r] = Real(0.0);
    } else {
      Real a[g::SL];
#pragma unroll
      for (int r = 0; r < g::SL; ++r) {
        const Real Fx = S.ok[r] ? ximul<Real, M>(D, fx, ux, thx, S, r) : Real(0.0);
        const Real fr = S.ok[r] ? fx[S.ca[r]] : Real(0.0);
        if (kase != 2) a[r] = Fx;
        else if (isL) a[r] = (lamR * Fx - lamL * lamR * fr) * iden;
        else a[r] = (-lamL * Fx + lamL * lamR * fr) * iden;
      }
      const Real xu1 = sc[L::SP + 4 * q], xu2 = sc[L::SP + 4 * q + 1];
      if (xu1 == c.u1 && xu2 == c.u2 && thx == c.th) {
#pragma unroll
        for (int r = 0; r < g::SL; ++r) T[r] = a[r];
      } else {
        put<Real, M>(W.bX, S, a);
        wsync();
        bchange<Real, M>(W.bX, W.bA, W.bB, c.u1 - xu1, c.u2 - xu2, c.th - thx, S, T);
      }
    }
    put_slots<Real, M>(lds + L::T + q * g::SLOT, lane, T);
    if (s == 0) {
      // regularisation jump of the face, straight path from L to R
      const Real *fL = lds + L::F + qL * g::CUBE, *fR = lds + L::F + qR * g::CUBE;
      const Real du1 = sc[L::SP + 4 * qR] - sc[L::SP + 4 * qL];
      const Real du2 = sc[L::SP + 4 * qR + 1] - sc[L::SP + 4 * qL + 1];
      const Real dth = thR - thL;
      Real gr[g::SL];
#pragma unroll
      for (int r = 0; r < g::SL; ++r) gr[r] = regul<Real, M>(D, fL, fR, du1, du2, dth, S, r);
      put_slots<Real, M>(lds + L::GR + f * g::SLOT, lane, gr);
      if (lane == 0) sc[L::SW + f] = sd > 0 ? wm : wp;
    }
  });
  };

  // in-cell regularisation of direction D: jump between the cell's own two
  // face states of that direction
  auto incell_reg = [&](int D) {
    const int fp = 2 * D, fm = 2 * D + 1;
    const Real j1 = sc[L::SP + 4 * fp] - sc[L::SP + 4 * fm];
    const Real j2 = sc[L::SP + 4 * fp + 1] - sc[L::SP + 4 * fm + 1];
    const Real j3 = sc[L::SP + 4 * fp + 2] - sc[L::SP + 4 * fm + 2];
    Real T[g::SL];
#pragma unroll
    for (int r = 0; r < g::SL; ++r) T[r] = regul<Real, M>(D, bC, bC, j1, j2, j3, S, r);
    put_slots<Real, M>(lds + L::T + (L::T_GX + D) * g::SLOT, lane, T);
  };

  // cell-local terms: collision, right-hand side (and, unsplit, both
  // in-cell regularisations; split, the y one)
  auto local_terms = [&]() {
    const Real rho = bC[0];
    const Real nu = sc[L::SNU];
    Real T[g::SL];
    // collision Q = nu (f^E - f), eq. (5), (29); Shakhov f^E from eq. (8),
    // ES-BGK f^E from eq. (7)
    Real c1 = Real(0.0), c2 = Real(0.0);
    if (A.collision == 1) {
      const Real q1 = Real(2.0) * bC[g::X3] + bC[g::X3] + bC[g::X1Y2] + bC[g::X1Z2];
      const Real q2 = Real(2.0) * bC[g::Y3] + bC[g::X2Y1] + bC[g::Y3] + bC[g::Y1Z2];
      c1 = (Real(1.0) - Real(A.Pr)) * q1 * Real(0.2);
      c2 = (Real(1.0) - Real(A.Pr)) * q2 * Real(0.2);
    }
    Real b11 = Real(0.0), b12 = Real(0.0), b22 = Real(0.0), b33 = Real(0.0);
    if (A.collision == 2) {
      // B = (1 - 1/Pr) sigma / rho, sigma_ij = (1 + delta_ij) f_{e_i+e_j}
      const Real kb = (Real(1.0) - Real(1.0) / Real(A.Pr)) / rho;
      b11 = kb * (Real(2.0) * bC[g::XX]);
      b12 = kb * bC[g::XY];
      b22 = kb * (Real(2.0) * bC[g::YY]);
      b33 = kb * (Real(2.0) * bC[g::ZZ]);
    }
#pragma unroll
    for (int r = 0; r < g::SL; ++r) {
      const int ca = S.ca[r];
      Real fE = ca == 0 ? rho : Real(0.0);
      if (ca == g::X3 || ca == g::X1Y2 || ca == g::X1Z2) fE += c1;
      if (ca == g::Y3 || ca == g::X2Y1 || ca == g::Y1Z2) fE += c2;
      if (A.collision == 2) fE = esbgk_coef<Real>(S.a1[r], S.a2[r], S.m[r], rho, b11, b12, b22, b33);
      T[r] = S.ok[r] ? nu * (fE - c.f[r]) : Real(0.0);
    }
    put_slots<Real, M>(lds + L::T + L::T_Q * g::SLOT, lane, T);
    if (ORDER == 2) {
      if (!SPLIT) incell_reg(0);
      incell_reg(1);
    }
    const Real *rr = MODE == MODE_FAS ? Radd : rhs;
    if (rr) {
      // right-hand side (Alg. 1) or the restricted residual (eq. (22)) in
      // the cell basis
      Cell<Real, M> r;
      load_cell<Real, M>(recp<Real, M>(A, rr, i, j), S, r);
      if ((r.u1 == c.u1 && r.u2 == c.u2 && r.th == c.th) || MODE == MODE_FAS) {
#pragma unroll
        for (int q = 0; q < g::SL; ++q) T[q] = r.f[q];
      } else {
        put<Real, M>(W.bX, S, r.f);
        wsync();
        bchange<Real, M>(W.bX, W.bA, W.bB, c.u1 - r.u1, c.u2 - r.u2, c.th - r.th, S, T);
      }
      put_slots<Real, M>(lds + L::T + L::T_RHS * g::SLOT, lane, T);
    }
  };

  if (!SPLIT) {
    face_states(0);
    __syncthreads();
    fluxes(0);
    if (wv == NW - 1) local_terms();
    __syncthreads();
  } else {
    face_states(0);
    __syncthreads();
    fluxes(0);
    if (wv == NW - 1) local_terms();
    if (threadIdx.x == 0) sc[L::SAB] = wait() ? Real(0.0) : Real(1.0);
    __syncthreads();
    if (sc[L::SAB] != Real(0.0)) return false;  // uniform across the team
    face_states(1);
    __syncthreads();
    fluxes(1);
    if (ORDER == 2 && wv == (NW >= 8 ? 3 : 0)) incell_reg(0);
    __syncthreads();
  }

  // ---- phase 2 (wavefront 0): assemble R_ij in a fixed order ------------
  if (wv == 0) {
    Real R[g::SL];
#pragma unroll
    for (int r = 0; r < g::SL; ++r) R[r] = Real(0.0);
#pragma unroll
    for (int D = 0; D < 2; ++D) {
      const int k = D == 0 ? i : j, n = D == 0 ? nx : ny;
      const Real ih = D == 0 ? Real(A.idx) : Real(A.idy);
#pragma unroll
      for (int sdi = 0; sdi < 2; ++sdi) {
        const int f = 2 * D + sdi;
        const int sd = sdi == 0 ? 1 : -1;
        Real TL[g::SL], TR[g::SL];
        if (k + sd < 0 || k + sd >= n) {
          get_slots<Real, M>(lds + L::T + f * g::SLOT, lane, TL);
#pragma unroll
          for (int r = 0; r < g::SL; ++r) R[r] -= TL[r] * ih;
          continue;
        }
        const int qL = sd > 0 ? f : f + 4, qR = sd > 0 ? f + 4 : f;
        Real gr[g::SL];
        get_slots<Real, M>(lds + L::T + qL * g::SLOT, lane, TL);
        get_slots<Real, M>(lds + L::T + qR * g::SLOT, lane, TR);
        get_slots<Real, M>(lds + L::GR + f * g::SLOT, lane, gr);
        const Real w = sc[L::SW + f];
        const Real sgnF = sd > 0 ? -Real(1.0) : Real(1.0);
#pragma unroll
        for (int r = 0; r < g::SL; ++r) R[r] += (sgnF * (TL[r] + TR[r]) + w * gr[r]) * ih;
      }
      if (ORDER == 2) {
        Real gc[g::SL];
        get_slots<Real, M>(lds + L::T + (L::T_GX + D) * g::SLOT, lane, gc);
#pragma unroll
        for (int r = 0; r < g::SL; ++r) R[r] += gc[r] * ih;
      }
    }
    {
      Real q[g::SL];
      get_slots<Real, M>(lds + L::T + L::T_Q * g::SLOT, lane, q);
#pragma unroll
      for (int r = 0; r < g::SL; ++r) R[r] += q[r];
    }
    const Real *rr = MODE == MODE_FAS ? Radd : rhs;
    Real rv[g::SL];
    if (rr) get_slots<Real, M>(lds + L::T + L::T_RHS * g::SLOT, lane, rv);
    if (MODE == MODE_SWEEP) {
      const Real dt = local_dt<Real>(A, c.u1, c.u2, c.th, sc[L::SNU]);
      Real fs[g::SL];
#pragma unroll
      for (int r = 0; r < g::SL; ++r) fs[r] = c.f[r] + dt * (rr ? R[r] - rv[r] : R[r]);
      Cell<Real, M> nc;
      if (normalise<Real, M>(c.u1, c.u2, c.th, fs, W, nc))
        store_record<Real, M, true>(const_cast<Real *>(recp<Real, M>(A, st, i, j)), nc.u1, nc.u2,
                                    nc.th, W.bA, lane);
      else if (lane == 0)
        atomicOr(err, 1);
    } else {
      Real o[g::SL];
#pragma unroll
      for (int r = 0; r < g::SL; ++r)
        o[r] = MODE == MODE_FAS ? R[r] + rv[r] : (rr ? rv[r] : Real(0.0)) - R[r];
      if (out) {
        put<Real, M>(W.bA, S, o);
        wsync();
        store_record<Real, M>(out + (size_t)cellidx * g::STRIDE, c.u1, c.u2, c.th, W.bA, lane);
      }
      if (MODE == MODE_DEFECT && norm_part) {
        Real s2 = Real(0.0);
#pragma unroll
        for (int q = 0; q < g::SL; ++q) {
          if (!S.ok[q]) continue;
          const Real w = Real(c_fact.v[S.a1[q]]) * Real(c_fact.v[S.a2[q]]) * Real(c_fact.v[2 * S.m[q]]);
          s2 += w * pow(c.th, -(Real)S.n[q]) * o[q] * o[q];
        }
#pragma unroll
        for (int off = WAVE / 2; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
        if (lane == 0) norm_part[cellidx] = s2 * Real(A.ds);
      }
    }
  }
  return true;
}

// Team width: 8 wavefronts (one face-side item each) while the LDS of a team
// fits comfortably, 4 at M >= 6 (two items each).  At most 8 wavefronts keeps
// the budget at 256 VGPRs per lane.
template <int M>
struct TeamWidth {
  static constexpr int NW = M <= 5 ? 8 : 4;
  static constexpr int THREADS = NW * WAVE;
};

// Wait until *flag >= target.  The polls are relaxed agent-scope loads: an
// acquire on every poll would invalidate the XCD's L2 each time, evicting the
// records every other team on the XCD is working on.  The caller issues one
// agent-scope acquire fence (acquire_agent) after all waits of a cell have
// succeeded.  Bounded: gives up after `limit` ticks of the 100 MHz wall clock
// or when another team has aborted; returns false then.  *seen (optional)
// receives the value that satisfied the wait: a fence after the wait makes
// the writes released up to that value visible, and no later ones.
__device__ __forceinline__ bool wait_at_least(const int *flag, int target, int *abort_flag,
                                              unsigned long long limit, int *seen = nullptr) {
  int v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (v >= target) {
    if (seen) *seen = v;
    return true;
  }
  const unsigned long long t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(2);
    v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v >= target) {
      if (seen) *seen = v;
      return true;
    }
    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (wall_clock64() - t0 > limit) {
      __hip_atomic_fetch_or(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
}

// Makes the stores published by the teams whose flags were observed visible
// to the loads that follow (agent-scope acquire: invalidates this XCD's
// caches of non-coherent lines).
__device__ __forceinline__ void acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }


// Table slot of a group's cell (entries sorted by their first cell).
__device__ __forceinline__ int find_slot(const BLevel *__restrict__ tab, int nslot, int cell) {
  int lo = 0, hi = nslot - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].cell0 <= cell) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Restriction (Sec. 3.2.2, eq. (24)-(25)): coarse cell (I, J) from fine cells
// (2I, 2J), (2I+1, 2J), (2I, 2J+1), (2I+1, 2J+1).
// One wavefront; lds holds RestrictLds<M>::N doubles; the coarse records
// are written at index cellC.
template <int M>
struct RestrictLds {
  static constexpr int N = 3 * G<M>::CUBE + G<M>::MISC;
};
template <int M>
__device__ void restrict_cell(const LevelArgs &Af, const double *__restrict__ fine,
                              const double *__restrict__ fineR, double *__restrict__ coarse,
                              double *__restrict__ coarseR, int I, int J, int cellC, double *lds,
                              int *err) {
  using g = G<M>;
  Wave<double, M> W;
  W.init(lds, threadIdx.x);
  Cell<double, M> ch[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    load_cell<double, M>(recp<double, M>(Af, fine, 2 * I + (q & 1), 2 * J + (q >> 1)), W.S, ch[q]);
  const double dsh = Af.ds, dsH = 4.0 * Af.ds;
  double mass = 0.0, m1 = 0.0, m2 = 0.0, en = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double rho = recp<double, M>(Af, fine, 2 * I + (q & 1), 2 * J + (q >> 1))[3];
    mass += rho * dsh;
    m1 += rho * ch[q].u1 * dsh;
    m2 += rho * ch[q].u2 * dsh;
    en += (rho * (ch[q].u1 * ch[q].u1 + ch[q].u2 * ch[q].u2) + 3.0 * rho * ch[q].th) * dsh;
  }
  const double rhoH = mass / dsH, u1 = m1 / (rhoH * dsH), u2 = m2 / (rhoH * dsH);
  const double th = (en / dsH - rhoH * (u1 * u1 + u2 * u2)) / (3.0 * rhoH);
  if (!(rhoH > 0.0) || !(th > 0.0)) {
    if (W.lane == 0) atomicOr(err, 1);
    return;
  }
  for (int pass = 0; pass < 2; ++pass) {
    const double *src = pass == 0 ? fine : fineR;
    double *dst = pass == 0 ? coarse : coarseR;
    if (!src || !dst) continue;
    double acc[g::SL];
#pragma unroll
    for (int r = 0; r < g::SL; ++r) acc[r] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Cell<double, M> x;
      if (pass == 0) x = ch[q];
      else load_cell<double, M>(recp<double, M>(Af, fineR, 2 * I + (q & 1), 2 * J + (q >> 1)), W.S, x);
      put<double, M>(W.bX, W.S, x.f);
      wsync();
      double t[g::SL];
      bchange<double, M>(W.bX, W.bA, W.bB, u1 - x.u1, u2 - x.u2, th - x.th, W.S, t);
#pragma unroll
      for (int r = 0; r < g::SL; ++r) acc[r] += t[r] * dsh / dsH;
    }
    put<double, M>(W.bA, W.S, acc);
    wsync();
    if (pass == 0) {  // state: exact constraints of eq. (10)
      const double zz = -(W.bA[g::XX] + W.bA[g::YY]);
      wsync();
      if (W.lane == 0) {
        W.bA[g::E1] = 0.0;
        W.bA[g::E2] = 0.0;
        W.bA[g::ZZ] = zz;
      }
      wsync();
    }
    store_record<double, M>(dst + (size_t)cellC * g::STRIDE, u1, u2, th, W.bA, W.lane);
    wsync();
  }
}

// Coarse-grid correction, eq. (26): delta = T(f~_H -> basis of f-bar_H) -
// f-bar_H, then each child f + T(delta) in its own basis, normalised.  A
// child that would become non-physical keeps its value.
// One wavefront; lds holds CorrectLds<M>::N doubles; the coarse records
// are read at index cellC.
template <int M>
struct CorrectLds {
  static constexpr int N = 4 * G<M>::CUBE + G<M>::MISC;
};
template <int M>
__device__ void correct_cell(const LevelArgs &Af, double *__restrict__ fine,
                             const double *__restrict__ cnew, const double *__restrict__ cold,
                             int I, int J, int cellC, double *lds, int *err) {
  using g = G<M>;
  Wave<double, M> W;
  W.init(lds + g::CUBE, threadIdx.x);
  double *bD = lds;
  Cell<double, M> fn, fo;
  load_cell<double, M>(cnew + (size_t)cellC * g::STRIDE, W.S, fn);
  load_cell<double, M>(cold + (size_t)cellC * g::STRIDE, W.S, fo);
  double delta[g::SL];
  put<double, M>(W.bX, W.S, fn.f);
  wsync();
  bchange<double, M>(W.bX, W.bA, W.bB, fo.u1 - fn.u1, fo.u2 - fn.u2, fo.th - fn.th, W.S, delta);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) delta[r] -= fo.f[r];
  put<double, M>(bD, W.S, delta);
  wsync();
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    double *rec = const_cast<double *>(recp<double, M>(Af, fine, 2 * I + (q & 1), 2 * J + (q >> 1)));
    Cell<double, M> x;
    load_cell<double, M>(rec, W.S, x);
    double t[g::SL];
    bchange<double, M>(bD, W.bA, W.bB, x.u1 - fo.u1, x.u2 - fo.u2, x.th - fo.th, W.S, t);
    double fs[g::SL];
#pragma unroll
    for (int r = 0; r < g::SL; ++r) fs[r] = x.f[r] + t[r];
    Cell<double, M> nc;
    if (normalise<double, M>(x.u1, x.u2, x.th, fs, W, nc)) store_record<double, M>(rec, nc.u1, nc.u2, nc.th, W.bA, W.lane);
    else if (W.lane == 0) atomicOr(err, 2);
    wsync();
  }
}

}  // namespace
}  // namespace nrxx

// Host-side dispatch of a runtime expansion order to the template argument
// MM: NRXX_DISPATCH_M for the kernels built up to MTEAM (cell teams, FP32
// blocks), NRXX_DISPATCH_MW for those built up to MMAX.
#define NRXX_DISPATCH_M(M, BODY)                  \
  switch (M) {                                    \
    case 3: { constexpr int MM = 3; BODY; } break; \
    case 4: { constexpr int MM = 4; BODY; } break; \
    case 5: { constexpr int MM = 5; BODY; } break; \
    case 6: { constexpr int MM = 6; BODY; } break; \
    case 7: { constexpr int MM = 7; BODY; } break; \
    case 8: { constexpr int MM = 8; BODY; } break; \
    default: return hipErrorInvalidValue;         \
  }
#define NRXX_DISPATCH_MW(M, BODY)                   \
  switch (M) {                                      \
    case 3: { constexpr int MM = 3; BODY; } break;   \
    case 4: { constexpr int MM = 4; BODY; } break;   \
    case 5: { constexpr int MM = 5; BODY; } break;   \
    case 6: { constexpr int MM = 6; BODY; } break;   \
    case 7: { constexpr int MM = 7; BODY; } break;   \
    case 8: { constexpr int MM = 8; BODY; } break;   \
    case 9: { constexpr int MM = 9; BODY; } break;   \
    case 10: { constexpr int MM = 10; BODY; } break; \
    default: return hipErrorInvalidValue;           \
  }
