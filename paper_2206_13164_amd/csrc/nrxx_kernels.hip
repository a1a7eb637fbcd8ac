// nrxx_kernels.hip -- gfx950 kernels of the NRxx steady-state solver
// (Hu & Li, arXiv 2206.13164): the finite-volume operator R_ij of eq. (13)
// evaluated per cell, the fast-sweeping cell update of Alg. 1, restriction
// (eq. (24)-(25)), coarse-grid correction (eq. (26)) and reductions.
//
// Execution model: one 64-lane wavefront ("team") owns one cell.  Lanes run
// over the expansion coefficients with even alpha_3 (the odd ones vanish
// identically for this xi_3-even, two-dimensional problem), so a team holds
// 13 / 34 / 95 coefficients at M = 3 / 5 / 8 in 1 or 2 registers per lane.
// Coefficient vectors that lanes must read from each other live in LDS in a
// dense "cube" (alpha_1, alpha_2, alpha_3 / 2) of (M+1) x (M+1) x (M/2+1)
// doubles: every shift alpha -/+ k e_d of the Hermite algebra is then a
// compile-time LDS offset folded into the ds_read instruction.
// Global memory holds cell records [u1, u2, theta, f_0 .. f_{N-1}] in the
// graded order of the C ABI, one record per cell, row-major.
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
};
constexpr FactTab make_fact_tab() {
  FactTab t{};
  double f = 1.0;
  t.v[0] = 1.0;
  for (int n = 1; n < 2 * MMAX + 4; ++n) {
    f *= n;
    t.v[n] = f;
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
  static constexpr int KOFF = 0;                     // K_n(a), n = 0 .. 2M+1
  static constexpr int JOFF = 2 * M + 2;             // J+_{kl}(a), (M+1)^2
  static constexpr int BOFF = JOFF + (M + 1) * (M + 1);  // broadcast slots
  static constexpr int MISC = BOFF + 16;
  static constexpr int TEAM_LDS = 6 * CUBE + MISC;  // doubles per team
  // cube addresses of coefficients used by name
  static constexpr int E1 = 1, E2 = D1, XX = 2, YY = 2 * D1, ZZ = D2;
  static constexpr int X3 = 3, X1Y2 = 1 + 2 * D1, X1Z2 = 1 + D2;
  static constexpr int Y3 = 3 * D1, X2Y1 = 2 + D1, Y1Z2 = D1 + D2;
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

template <int M>
struct Team {
  using g = G<M>;
  double *bC, *bL, *bR, *bX, *bA, *bB, *misc;
  int lane;
  Slots<M> S;
  __device__ __forceinline__ void init(double *base, int ln) {
    bC = base;
    bL = base + g::CUBE;
    bR = base + 2 * g::CUBE;
    bX = base + 3 * g::CUBE;
    bA = base + 4 * g::CUBE;
    bB = base + 5 * g::CUBE;
    misc = base + 6 * g::CUBE;
    lane = ln;
    S.init(ln);
  }
};

// Cell data held by a team: basis parameters (uniform) and the lane's
// coefficients.
template <int M>
struct Cell {
  double u1, u2, th;
  double f[G<M>::SL];
};

template <int M>
__device__ __forceinline__ void load_cell(const double *__restrict__ rec, const Slots<M> &S,
                                          Cell<M> &c) {
  c.u1 = rec[0];
  c.u2 = rec[1];
  c.th = rec[2];
#pragma unroll
  for (int r = 0; r < G<M>::SL; ++r) c.f[r] = S.ok[r] ? rec[3 + S.ci[r]] : 0.0;
}

template <int M>
__device__ __forceinline__ void put(double *buf, const Slots<M> &S, const double (&v)[G<M>::SL]) {
#pragma unroll
  for (int r = 0; r < G<M>::SL; ++r)
    if (S.ok[r]) buf[S.ca[r]] = v[r];
}

// Coalesced write of a full record from (params, LDS cube); odd-alpha_3
// coefficients are written as zeros.
template <int M>
__device__ __forceinline__ void store_record(double *__restrict__ rec, double u1, double u2,
                                             double th, const double *cube, int lane) {
  using g = G<M>;
#pragma unroll
  for (int t = 0; t < g::SR; ++t) {
    int v = lane + WAVE * t;
    if (v < g::NR) {
      double x;
      if (v == 0) x = u1;
      else if (v == 1) x = u2;
      else if (v == 2) x = th;
      else {
        int al = v - 3;
        int a1 = c_canon.a1[al], a2 = c_canon.a2[al], a3 = c_canon.a3[al];
        x = (a3 & 1) ? 0.0 : cube[a1 + g::D1 * a2 + g::D2 * (a3 >> 1)];
      }
      rec[v] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// Hermite algebra on one wavefront
// ---------------------------------------------------------------------------

// Taylor coefficients of exp(-du t - dth t^2 / 2): the 1-D factors of the
// exact re-expansion F_M^[u,th] -> F_M^[u+du, th+dth] (Sec. 2.3).
template <int M>
__device__ __forceinline__ void tcoef(double du, double dth, double (&c)[M + 1]) {
  c[0] = 1.0;
  c[1] = -du;
#pragma unroll
  for (int k = 1; k < M; ++k) c[k + 1] = (-du * c[k] - dth * c[k - 1]) / (double)(k + 1);
}

// res = T(in) for the basis change by (du1, du2, dth): three 1-D lower-
// triangular convolutions along alpha_1, alpha_2, alpha_3.  in, t1, t2 are
// distinct LDS cubes; the result stays in registers.
template <int M>
__device__ __forceinline__ void bchange(const double *in, double *t1, double *t2, double du1,
                                        double du2, double dth, const Slots<M> &S,
                                        double (&res)[G<M>::SL]) {
  using g = G<M>;
  double c[M + 1];
  tcoef<M>(du1, dth, c);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    if (!S.ok[r]) continue;
    const double *p = in + S.ca[r];
    double acc = p[0];
#pragma unroll
    for (int k = 1; k <= M; ++k)
      if (k <= S.a1[r]) acc = fma(c[k], p[-k], acc);
    t1[S.ca[r]] = acc;
  }
  wsync();
  tcoef<M>(du2, dth, c);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    if (!S.ok[r]) continue;
    const double *p = t1 + S.ca[r];
    double acc = p[0];
#pragma unroll
    for (int k = 1; k <= M; ++k)
      if (k <= S.a2[r]) acc = fma(c[k], p[-k * g::D1], acc);
    t2[S.ca[r]] = acc;
  }
  wsync();
  tcoef<M>(0.0, dth, c);  // u_3 = 0 on both sides: only even powers survive
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    const double *p = t2 + S.ca[r];
    double acc = S.ok[r] ? p[0] : 0.0;
#pragma unroll
    for (int k = 1; 2 * k <= M; ++k)
      if (S.ok[r] && k <= S.m[r]) acc = fma(c[2 * k], p[-k * g::D2], acc);
    res[r] = acc;
  }
  wsync();
}

// (Pi_M xi_d f)_alpha = th f_{alpha-e_d} + u_d f_alpha + (alpha_d+1) f_{alpha+e_d}
template <int M, int D>
__device__ __forceinline__ double ximul(const double *f, double ud, double th, const Slots<M> &S,
                                        int r) {
  constexpr int st = D == 0 ? 1 : G<M>::D1;
  const double *p = f + S.ca[r];
  int ad = D == 0 ? S.a1[r] : S.a2[r];
  double v = ud * p[0];
  if (ad >= 1) v += th * p[-st];
  if (S.n[r] < M) v += (ad + 1) * p[st];
  return v;
}

// Regularisation term of direction D at |beta| = M (zero below):
// (beta_D + 1) [sum_k f_{b+e_D-e_k} du_k + 1/2 sum_k f_{b+e_D-2e_k} dth],
// du_3 = 0.  avgL/avgR: the term is taken of (fL + fR)/2 (both cubes, fR may
// equal fL for the in-cell term).
template <int M, int D>
__device__ __forceinline__ double regul(const double *fL, const double *fR, double du1, double du2,
                                        double dth, const Slots<M> &S, int r) {
  using g = G<M>;
  if (!S.ok[r] || S.n[r] != M) return 0.0;
  const int base = S.ca[r] + (D == 0 ? 1 : g::D1);  // b + e_D
  int b[3] = {S.a1[r], S.a2[r], 2 * S.m[r]};
  b[D] += 1;
  auto av = [&](int off) { return 0.5 * (fL[base + off] + fR[base + off]); };
  double acc = 0.0;
  // k = 1 (x)
  if (b[0] >= 1) acc += av(-1) * du1;
  if (b[0] >= 2) acc += 0.5 * av(-2) * dth;
  // k = 2 (y)
  if (b[1] >= 1) acc += av(-g::D1) * du2;
  if (b[1] >= 2) acc += 0.5 * av(-2 * g::D1) * dth;
  // k = 3 (z): du_3 = 0 and b - e_3 has odd alpha_3
  if (b[2] >= 2) acc += 0.5 * av(-g::D2) * dth;
  int bd = D == 0 ? S.a1[r] : S.a2[r];
  return (bd + 1) * acc;
}

__device__ __forceinline__ double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return fmin(a, b);
  if (a < 0.0 && b < 0.0) return fmax(a, b);
  return 0.0;
}

__device__ __forceinline__ double limited(int limiter, double hi, double c, double lo) {
  return limiter == 1 ? 0.5 * (hi - lo) : minmod(hi - c, c - lo);
}

// Probabilists' Hermite polynomial by recurrence.
__device__ __forceinline__ double hermite(int n, double x) {
  double h0 = 1.0, h1 = x;
  if (n == 0) return 1.0;
  for (int k = 1; k < n; ++k) {
    double h2 = x * h1 - k * h0;
    h0 = h1;
    h1 = h2;
  }
  return h1;
}

// I_kl(a) = (2 pi)^-1/2 int_{-a}^inf He_k He_l e^{-w^2/2} dw from the
// half-range moments K_n (in LDS) and He_k He_l = sum_j k! l! / (j! (k-j)!
// (l-j)!) He_{k+l-2j}.
__device__ __forceinline__ double halfI(const double *K, int k, int l) {
  if (l < 0) return 0.0;
  double acc = 0.0;
  int jm = k < l ? k : l;
  for (int j = 0; j <= jm; ++j)
    acc += c_fact.v[k] * c_fact.v[l] / (c_fact.v[j] * c_fact.v[k - j] * c_fact.v[l - j]) *
           K[k + l - 2 * j];
  return acc;
}

// Outward flux through a diffuse wall in the cell basis (reading of the
// Maxwell boundary condition of Sec. 2.3 / Sec. 4): the leaving half-range
// of the cell distribution plus the entering half of the wall Maxwellian,
// whose density makes the net mass flux zero.  The cell's coefficients are
// in the team's bC cube.
template <int M>
__device__ void wall_flux(const LevelArgs &A, int wall, const Cell<M> &c, Team<M> &T,
                          double (&phi)[G<M>::SL]) {
  using g = G<M>;
  const Slots<M> &S = T.S;
  const int lane = T.lane;
  const int d = (wall == 0 || wall == 2) ? 1 : 0;
  const double sig = (wall == 1 || wall == 2) ? 1.0 : -1.0;
  const double sq = sqrt(c.th);
  const double a = sig * (d == 0 ? c.u1 : c.u2) / sq;
  double *K = T.misc + g::KOFF;
  double *Jp = T.misc + g::JOFF;
  double *bc = T.misc + g::BOFF;
  // K_n(a) = (2 pi)^-1/2 int_{-a}^inf He_n e^{-w^2/2}
  for (int n = lane; n <= 2 * M + 1; n += WAVE)
    K[n] = n == 0 ? 0.5 * erfc(-a / sqrt(2.0))
                  : hermite(n - 1, -a) * exp(-0.5 * a * a) / sqrt(2.0 * M_PI);
  wsync();
  // J+_kl(a) = a I_kl + I_{k,l+1} + l I_{k,l-1}
  for (int t = lane; t < (M + 1) * (M + 1); t += WAVE) {
    int k = t / (M + 1), l = t % (M + 1);
    Jp[t] = a * halfI(K, k, l) + halfI(K, k, l + 1) + l * halfI(K, k, l - 1);
  }
  wsync();
  // leaving half: sum_{beta_d} f_beta th^{(a_d-b_d)/2} sqrt(th) sig^{a_d+b_d} J+_{a_d b_d} / a_d!
  const double isq = 1.0 / sq;
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    double acc = 0.0;
    if (S.ok[r]) {
      int ad = d == 0 ? S.a1[r] : S.a2[r];
      int at = (d == 0 ? S.a2[r] : S.a1[r]) + 2 * S.m[r];  // transverse degree
      int base = S.ca[r] - ad * (d == 0 ? 1 : g::D1);    // alpha with alpha_d = 0
      double pa = 1.0;
      for (int q = 0; q < ad; ++q) pa *= sq;
      double ib = 1.0;
#pragma unroll
      for (int bd = 0; bd <= M; ++bd) {
        if (bd + at <= M) {
          double sgn = ((ad + bd) & 1) ? sig : 1.0;
          double fb = T.bC[base + bd * (d == 0 ? 1 : g::D1)];
          acc += fb * (pa * ib) * sq * sgn * Jp[ad * (M + 1) + bd] / c_fact.v[ad];
        }
        ib *= isq;
      }
    }
    phi[r] = acc;
  }
  // wall density from zero net mass flux; phi_0 lives in lane 0, slot 0
  if (lane == 0) bc[0] = phi[0];
  wsync();
  const double thw = A.wall_th[wall], sqw = sqrt(thw);
  const double rhow = bc[0] * sqrt(2.0 * M_PI / thw);
  // entering half in the wall basis: only alpha = k e_d is non-zero
#pragma unroll
  for (int r = 0; r < g::SL; ++r)
    if (S.ok[r]) T.bX[S.ca[r]] = 0.0;
  wsync();
  if (lane <= M) {
    int k = lane;
    double pw = 1.0;
    for (int q = 0; q < k; ++q) pw *= sqw;
    double sgn = (k & 1) ? sig : 1.0;
    T.bX[k * (d == 0 ? 1 : g::D1)] = rhow * pw * sqw * sgn * A.jminus[k];
  }
  wsync();
  double uw1 = d == 1 ? A.wall_u[wall] : 0.0, uw2 = d == 0 ? A.wall_u[wall] : 0.0;
  double t[g::SL];
  bchange<M>(T.bX, T.bA, T.bB, c.u1 - uw1, c.u2 - uw2, c.th - thw, S, t);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) phi[r] += t[r];
}

// Interior face with normal e_D between face states L and R (reading of the
// numerical flux of Sec. 2.3: HLL with signal speeds u_D -/+ C_{M+1} sqrt(th),
// the speeds of the CFL condition eq. (18)).  Both halves are projected into
// the cell basis; the regularisation jump g is split w- (left cell) / w+
// (right cell).  Adds (sgnF * F + w * g) / h to acc, w = w- if the cell is
// the left one (cellIsLeft) else w+.
template <int M, int D>
__device__ void face(const LevelArgs &A, const Cell<M> &L, const Cell<M> &R, const Cell<M> &c,
                     bool cellIsLeft, double h, Team<M> &T, double (&acc)[G<M>::SL]) {
  using g = G<M>;
  const Slots<M> &S = T.S;
  put<M>(T.bL, S, L.f);
  put<M>(T.bR, S, R.f);
  wsync();
  const double C = A.C;
  const double uL = D == 0 ? L.u1 : L.u2, uR = D == 0 ? R.u1 : R.u2;
  const double cL = C * sqrt(L.th), cR = C * sqrt(R.th);
  const double lamL = fmin(uL - cL, uR - cR);
  const double lamR = fmax(uL + cL, uR + cR);
  int kase;
  double wm, wp, den = lamR - lamL;
  if (lamL >= 0.0) { kase = 0; wm = 0.0; wp = 1.0; }
  else if (lamR <= 0.0) { kase = 1; wm = 1.0; wp = 0.0; }
  else { kase = 2; wm = -lamL / den; wp = lamR / den; }
  double F[g::SL];
#pragma unroll
  for (int r = 0; r < g::SL; ++r) F[r] = 0.0;
  // left half A^L, in L's basis
  if (kase != 1) {
    double a[g::SL];
#pragma unroll
    for (int r = 0; r < g::SL; ++r) {
      double Fx = S.ok[r] ? ximul<M, D>(T.bL, uL, L.th, S, r) : 0.0;
      a[r] = kase == 0 ? Fx : (lamR * Fx - lamL * lamR * L.f[r]) / den;
    }
    if (L.u1 == c.u1 && L.u2 == c.u2 && L.th == c.th) {
#pragma unroll
      for (int r = 0; r < g::SL; ++r) F[r] += a[r];
    } else {
      put<M>(T.bX, S, a);
      wsync();
      double t[g::SL];
      bchange<M>(T.bX, T.bA, T.bB, c.u1 - L.u1, c.u2 - L.u2, c.th - L.th, S, t);
#pragma unroll
      for (int r = 0; r < g::SL; ++r) F[r] += t[r];
    }
  }
  if (kase != 0) {
    double a[g::SL];
#pragma unroll
    for (int r = 0; r < g::SL; ++r) {
      double Fx = S.ok[r] ? ximul<M, D>(T.bR, uR, R.th, S, r) : 0.0;
      a[r] = kase == 1 ? Fx : (-lamL * Fx + lamL * lamR * R.f[r]) / den;
    }
    if (R.u1 == c.u1 && R.u2 == c.u2 && R.th == c.th) {
#pragma unroll
      for (int r = 0; r < g::SL; ++r) F[r] += a[r];
    } else {
      put<M>(T.bX, S, a);
      wsync();
      double t[g::SL];
      bchange<M>(T.bX, T.bA, T.bB, c.u1 - R.u1, c.u2 - R.u2, c.th - R.th, S, t);
#pragma unroll
      for (int r = 0; r < g::SL; ++r) F[r] += t[r];
    }
  }
  const double w = cellIsLeft ? wm : wp;
  const double sgnF = cellIsLeft ? -1.0 : 1.0;
  const double du1 = R.u1 - L.u1, du2 = R.u2 - L.u2, dth = R.th - L.th;
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    double gr = regul<M, D>(T.bL, T.bR, du1, du2, dth, S, r);
    acc[r] += (sgnF * F[r] + w * gr) / h;
  }
  wsync();
}

// Face state of `c` on side `side` of direction D (eq. (15)): every variable
// v -> v + side/2 * limited slope; zero slope when `flat`.
template <int M>
__device__ __forceinline__ void face_state(const Cell<M> &c, const Cell<M> &hi, const Cell<M> &lo,
                                           int limiter, bool flat, double side, Cell<M> &out) {
  if (flat) {
    out = c;
    return;
  }
  out.u1 = c.u1 + 0.5 * side * limited(limiter, hi.u1, c.u1, lo.u1);
  out.u2 = c.u2 + 0.5 * side * limited(limiter, hi.u2, c.u2, lo.u2);
  out.th = c.th + 0.5 * side * limited(limiter, hi.th, c.th, lo.th);
#pragma unroll
  for (int r = 0; r < G<M>::SL; ++r) out.f[r] = c.f[r] + 0.5 * side * limited(limiter, hi.f[r], c.f[r], lo.f[r]);
}

// Contribution of direction D to R_ij: both faces (interior or wall) and, at
// second order, the in-cell regularisation term.
template <int M, int ORDER, int D>
__device__ void direction(const LevelArgs &A, int k, int n, const Cell<M> &c, const Cell<M> &lo,
                          const Cell<M> &hi, const Cell<M> &lolo, const Cell<M> &hihi, Team<M> &T,
                          double (&acc)[G<M>::SL]) {
  using g = G<M>;
  const double h = D == 0 ? A.dx : A.dy;
  const bool cflat = ORDER == 1 || k == 0 || k == n - 1;
  double jump[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int si = 0; si < 2; ++si) {
    const double side = si == 0 ? 1.0 : -1.0;
    Cell<M> own;
    face_state<M>(c, hi, lo, A.limiter, cflat, side, own);
    if (si == 0) { jump[0] = own.u1; jump[1] = own.u2; jump[2] = own.th; }
    else { jump[0] -= own.u1; jump[1] -= own.u2; jump[2] -= own.th; }
    const int kn = k + (si == 0 ? 1 : -1);
    if (kn < 0 || kn >= n) {
      const int wall = D == 0 ? (si == 0 ? 1 : 3) : (si == 0 ? 2 : 0);
      double phi[g::SL];
      wall_flux<M>(A, wall, c, T, phi);
#pragma unroll
      for (int r = 0; r < g::SL; ++r) acc[r] -= phi[r] / h;
      continue;
    }
    const bool nflat = ORDER == 1 || kn == 0 || kn == n - 1;
    Cell<M> nb;
    if (si == 0) face_state<M>(hi, hihi, c, A.limiter, nflat, -1.0, nb);
    else face_state<M>(lo, c, lolo, A.limiter, nflat, 1.0, nb);
    if (si == 0) face<M, D>(A, own, nb, c, true, h, T, acc);
    else face<M, D>(A, nb, own, c, false, h, T, acc);
  }
  if (ORDER == 2) {
#pragma unroll
    for (int r = 0; r < g::SL; ++r)
      acc[r] += regul<M, D>(T.bC, T.bC, jump[0], jump[1], jump[2], T.S, r) / h;
  }
}

// Collision term Q = nu (f^E - f), eq. (5) and (29); BGK f^E = rho e_0
// (eq. (6)); Shakhov adds (1-Pr) q_i / 5 at 3e_i and e_i + 2e_d (eq. (8)),
// q_i from eq. (10).
template <int M>
__device__ __forceinline__ void collision(const LevelArgs &A, const Cell<M> &c, Team<M> &T,
                                          double (&acc)[G<M>::SL]) {
  using g = G<M>;
  const double *f = T.bC;
  const double rho = f[0];
  const double nu = A.beta * sqrt(M_PI / 2.0) * rho * pow(c.th, 1.0 - A.omega) / A.Kn;
  double c1 = 0.0, c2 = 0.0;
  if (A.collision == 1) {
    const double q1 = 2.0 * f[g::X3] + f[g::X3] + f[g::X1Y2] + f[g::X1Z2];
    const double q2 = 2.0 * f[g::Y3] + f[g::X2Y1] + f[g::Y3] + f[g::Y1Z2];
    c1 = (1.0 - A.Pr) * q1 / 5.0;
    c2 = (1.0 - A.Pr) * q2 / 5.0;
  }
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    if (!T.S.ok[r]) continue;
    const int ca = T.S.ca[r];
    double fE = ca == 0 ? rho : 0.0;
    if (ca == g::X3 || ca == g::X1Y2 || ca == g::X1Z2) fE += c1;
    if (ca == g::Y3 || ca == g::X2Y1 || ca == g::Y1Z2) fE += c2;
    acc[r] += nu * (fE - c.f[r]);
  }
}

template <int M>
__device__ __forceinline__ const double *recp(const LevelArgs &A, const double *st, int i, int j) {
  return st + ((size_t)j * A.nx + i) * G<M>::STRIDE;
}

// R_ij(f) of eq. (13) for cell (i, j): team-wide, result in acc; c receives
// the cell (its coefficients are also left in bC).
template <int M, int ORDER>
__device__ void cell_R(const LevelArgs &A, const double *__restrict__ st, int i, int j, Team<M> &T,
                       Cell<M> &c, double (&acc)[G<M>::SL]) {
  using g = G<M>;
  Cell<M> W, E, Sx, Nx, WW, EE, SS, NN;
  load_cell<M>(recp<M>(A, st, i, j), T.S, c);
  const bool hasW = i > 0, hasE = i < A.nx - 1, hasS = j > 0, hasN = j < A.ny - 1;
  if (hasW) load_cell<M>(recp<M>(A, st, i - 1, j), T.S, W); else W = c;
  if (hasE) load_cell<M>(recp<M>(A, st, i + 1, j), T.S, E); else E = c;
  if (hasS) load_cell<M>(recp<M>(A, st, i, j - 1), T.S, Sx); else Sx = c;
  if (hasN) load_cell<M>(recp<M>(A, st, i, j + 1), T.S, Nx); else Nx = c;
  if (ORDER == 2) {
    if (i > 1) load_cell<M>(recp<M>(A, st, i - 2, j), T.S, WW); else WW = W;
    if (i < A.nx - 2) load_cell<M>(recp<M>(A, st, i + 2, j), T.S, EE); else EE = E;
    if (j > 1) load_cell<M>(recp<M>(A, st, i, j - 2), T.S, SS); else SS = Sx;
    if (j < A.ny - 2) load_cell<M>(recp<M>(A, st, i, j + 2), T.S, NN); else NN = Nx;
  } else {
    WW = W; EE = E; SS = Sx; NN = Nx;
  }
  put<M>(T.bC, T.S, c.f);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) acc[r] = 0.0;
  wsync();
  direction<M, ORDER, 0>(A, i, A.nx, c, W, E, WW, EE, T, acc);
  direction<M, ORDER, 1>(A, j, A.ny, c, Sx, Nx, SS, NN, T, acc);
  collision<M>(A, c, T, acc);
}

// Local time step of eq. (18), capped so that nu dt <= nu_cap when nu_cap > 0.
__device__ __forceinline__ double local_dt(const LevelArgs &A, double u1, double u2, double th,
                                           double rho) {
  const double sq = sqrt(th);
  double dt = A.cfl / ((fabs(u1) + A.C * sq) / A.dx + (fabs(u2) + A.C * sq) / A.dy);
  if (A.nu_cap > 0.0) {
    const double nu = A.beta * sqrt(M_PI / 2.0) * rho * pow(th, 1.0 - A.omega) / A.Kn;
    if (nu * dt > A.nu_cap) dt = A.nu_cap / nu;
  }
  return dt;
}

// Load a right-hand-side record and project it into the basis (u1, u2, th).
template <int M>
__device__ __forceinline__ void rhs_in_basis(const double *__restrict__ rrec, double u1, double u2,
                                             double th, Team<M> &T, double (&out)[G<M>::SL]) {
  Cell<M> r;
  load_cell<M>(rrec, T.S, r);
  if (r.u1 == u1 && r.u2 == u2 && r.th == th) {
#pragma unroll
    for (int q = 0; q < G<M>::SL; ++q) out[q] = r.f[q];
    return;
  }
  put<M>(T.bX, T.S, r.f);
  wsync();
  bchange<M>(T.bX, T.bA, T.bB, u1 - r.u1, u2 - r.u2, th - r.th, T.S, out);
}

// Two-step update of Sec. 2.4: new (u, th) from the coefficients f* given in
// the old basis (eq. (3)), re-expansion, and the exact constraints of
// eq. (10).  Result in cube bA and in out; returns false for rho <= 0,
// th <= 0 or non-finite values.
template <int M>
__device__ bool normalise(const Cell<M> &old, const double (&fs)[G<M>::SL], Team<M> &T,
                          Cell<M> &out) {
  using g = G<M>;
  put<M>(T.bX, T.S, fs);
  wsync();
  const double rho = T.bX[0];
  const double fe1 = T.bX[g::E1], fe2 = T.bX[g::E2];
  const double tr = T.bX[g::XX] + T.bX[g::YY] + T.bX[g::ZZ];
  const double u1n = old.u1 + fe1 / rho, u2n = old.u2 + fe2 / rho;
  const double thn = old.th + (2.0 * tr - (fe1 * fe1 + fe2 * fe2) / rho) / (3.0 * rho);
  bool okp = rho > 0.0 && thn > 0.0 && isfinite(rho) && isfinite(thn) && isfinite(u1n) &&
             isfinite(u2n);
  if (!okp) return false;  // uniform branch
  double t[g::SL];
  bchange<M>(T.bX, T.bA, T.bB, u1n - old.u1, u2n - old.u2, thn - old.th, T.S, t);
  put<M>(T.bA, T.S, t);
  wsync();
  const double zz = -(T.bA[g::XX] + T.bA[g::YY]);
  bool fin = true;
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    const int ca = T.S.ca[r];
    if (ca == g::E1 || ca == g::E2) t[r] = 0.0;
    if (ca == g::ZZ) t[r] = zz;
    if (T.S.ok[r] && !isfinite(t[r])) fin = false;
  }
  wsync();
  if (T.lane < 2) T.bA[T.lane == 0 ? g::E1 : g::E2] = 0.0;
  if (T.lane == 0) T.bA[g::ZZ] = zz;
  wsync();
  out.u1 = u1n;
  out.u2 = u2n;
  out.th = thn;
#pragma unroll
  for (int r = 0; r < g::SL; ++r) out.f[r] = t[r];
  // all lanes agree (ballot over the finiteness of every coefficient)
  return __ballot(!fin) == 0;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// One anti-diagonal t of sweep direction `dir` (0..3 = D1..D4 of Sec. 3.1):
// cell a of the diagonal is (a0 + blockIdx.x, t - a) in the direction's
// coordinates.  Cells of one diagonal never read each other (cross-shaped
// stencil of radius <= 2), earlier diagonals are already updated and later
// ones are not: the serial Gauss-Seidel order of Alg. 1 exactly.
template <int M, int ORDER>
__global__ __launch_bounds__(WAVE) void k_sweep_diag(LevelArgs A, double *__restrict__ st,
                                                     const double *__restrict__ rhs, int dir, int t,
                                                     int a0, int *err) {
  using g = G<M>;
  __shared__ double lds[g::TEAM_LDS];
  Team<M> T;
  T.init(lds, threadIdx.x);
  const int a = a0 + blockIdx.x, b = t - a;
  const bool irev = dir == 1 || dir == 2, jrev = dir == 2 || dir == 3;
  const int i = irev ? A.nx - 1 - a : a, j = jrev ? A.ny - 1 - b : b;
  Cell<M> c;
  double R[g::SL];
  cell_R<M, ORDER>(A, st, i, j, T, c, R);
  const double dt = local_dt(A, c.u1, c.u2, c.th, T.bC[0]);
  if (rhs) {
    double r[g::SL];
    rhs_in_basis<M>(recp<M>(A, rhs, i, j), c.u1, c.u2, c.th, T, r);
#pragma unroll
    for (int q = 0; q < g::SL; ++q) R[q] -= r[q];
  }
  double fs[g::SL];
#pragma unroll
  for (int q = 0; q < g::SL; ++q) fs[q] = c.f[q] + dt * R[q];
  Cell<M> nc;
  if (normalise<M>(c, fs, T, nc)) {
    store_record<M>(const_cast<double *>(recp<M>(A, st, i, j)), nc.u1, nc.u2, nc.th, T.bA, T.lane);
  } else if (T.lane == 0) {
    atomicOr(err, 1);
  }
}

// Residual over all cells.  mode 0: out = r - R(f) in the cell basis (rhs
// may be NULL), norm_part[cell] = ds * sum_alpha alpha! th^-|alpha| out^2.
// mode 1: out = R(f) + Radd (coarse right-hand side of eq. (22); Radd is in
// the basis of f).
template <int M, int ORDER>
__global__ __launch_bounds__(WAVE) void k_residual(LevelArgs A, const double *__restrict__ st,
                                                   const double *__restrict__ rhs,
                                                   const double *__restrict__ Radd,
                                                   double *__restrict__ out,
                                                   double *__restrict__ norm_part, int mode) {
  using g = G<M>;
  __shared__ double lds[g::TEAM_LDS];
  Team<M> T;
  T.init(lds, threadIdx.x);
  const int cell = blockIdx.x;
  const int i = cell % A.nx, j = cell / A.nx;
  Cell<M> c;
  double R[g::SL], o[g::SL];
  cell_R<M, ORDER>(A, st, i, j, T, c, R);
  if (mode == 1) {
    Cell<M> ra;
    load_cell<M>(recp<M>(A, Radd, i, j), T.S, ra);
#pragma unroll
    for (int q = 0; q < g::SL; ++q) o[q] = R[q] + ra.f[q];
  } else {
    double r[g::SL];
    if (rhs) rhs_in_basis<M>(recp<M>(A, rhs, i, j), c.u1, c.u2, c.th, T, r);
#pragma unroll
    for (int q = 0; q < g::SL; ++q) o[q] = (rhs ? r[q] : 0.0) - R[q];
  }
  if (out) {
    put<M>(T.bA, T.S, o);
    wsync();
    store_record<M>(out + (size_t)cell * g::STRIDE, c.u1, c.u2, c.th, T.bA, T.lane);
  }
  if (norm_part && mode == 0) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < g::SL; ++q) {
      if (!T.S.ok[q]) continue;
      const double w = c_fact.v[T.S.a1[q]] * c_fact.v[T.S.a2[q]] * c_fact.v[2 * T.S.m[q]];
      s += w * pow(c.th, -(double)T.S.n[q]) * o[q] * o[q];
    }
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (T.lane == 0) norm_part[cell] = s * A.ds;
  }
}

// Restriction (Sec. 3.2.2, eq. (24)-(25)): coarse cell (I, J) from fine cells
// (2I, 2J), (2I+1, 2J), (2I, 2J+1), (2I+1, 2J+1).
template <int M>
__global__ __launch_bounds__(WAVE) void k_restrict(LevelArgs Af, const double *__restrict__ fine,
                                                   const double *__restrict__ fineR,
                                                   double *__restrict__ coarse,
                                                   double *__restrict__ coarseR, int *err) {
  using g = G<M>;
  __shared__ double lds[g::TEAM_LDS];
  Team<M> T;
  T.init(lds, threadIdx.x);
  const int cnx = Af.nx / 2;
  const int I = blockIdx.x % cnx, J = blockIdx.x / cnx;
  Cell<M> ch[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) load_cell<M>(recp<M>(Af, fine, 2 * I + (q & 1), 2 * J + (q >> 1)), T.S, ch[q]);
  const double dsh = Af.ds, dsH = 4.0 * Af.ds;
  double mass = 0.0, m1 = 0.0, m2 = 0.0, en = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double rho = recp<M>(Af, fine, 2 * I + (q & 1), 2 * J + (q >> 1))[3];
    mass += rho * dsh;
    m1 += rho * ch[q].u1 * dsh;
    m2 += rho * ch[q].u2 * dsh;
    en += (rho * (ch[q].u1 * ch[q].u1 + ch[q].u2 * ch[q].u2) + 3.0 * rho * ch[q].th) * dsh;
  }
  const double rhoH = mass / dsH, u1 = m1 / (rhoH * dsH), u2 = m2 / (rhoH * dsH);
  const double th = (en / dsH - rhoH * (u1 * u1 + u2 * u2)) / (3.0 * rhoH);
  if (!(rhoH > 0.0) || !(th > 0.0)) {
    if (T.lane == 0) atomicOr(err, 1);
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
      Cell<M> x;
      if (pass == 0) x = ch[q];
      else load_cell<M>(recp<M>(Af, fineR, 2 * I + (q & 1), 2 * J + (q >> 1)), T.S, x);
      put<M>(T.bX, T.S, x.f);
      wsync();
      double t[g::SL];
      bchange<M>(T.bX, T.bA, T.bB, u1 - x.u1, u2 - x.u2, th - x.th, T.S, t);
#pragma unroll
      for (int r = 0; r < g::SL; ++r) acc[r] += t[r] * dsh / dsH;
    }
    put<M>(T.bA, T.S, acc);
    wsync();
    if (pass == 0) {  // state: exact constraints of eq. (10)
      const double zz = -(T.bA[g::XX] + T.bA[g::YY]);
      wsync();
      if (T.lane == 0) {
        T.bA[g::E1] = 0.0;
        T.bA[g::E2] = 0.0;
        T.bA[g::ZZ] = zz;
      }
      wsync();
    }
    store_record<M>(dst + (size_t)blockIdx.x * g::STRIDE, u1, u2, th, T.bA, T.lane);
    wsync();
  }
}

// Coarse-grid correction, eq. (26): delta = T(f~_H -> basis of f-bar_H) -
// f-bar_H, then each child f + T(delta) in its own basis, normalised.  A
// child that would become non-physical keeps its value.
template <int M>
__global__ __launch_bounds__(WAVE) void k_correct(LevelArgs Af, double *__restrict__ fine,
                                                  const double *__restrict__ cnew,
                                                  const double *__restrict__ cold, int *err) {
  using g = G<M>;
  __shared__ double lds[g::TEAM_LDS];
  Team<M> T;
  T.init(lds, threadIdx.x);
  const int cnx = Af.nx / 2;
  const int I = blockIdx.x % cnx, J = blockIdx.x / cnx;
  Cell<M> fn, fo;
  load_cell<M>(cnew + (size_t)blockIdx.x * g::STRIDE, T.S, fn);
  load_cell<M>(cold + (size_t)blockIdx.x * g::STRIDE, T.S, fo);
  double delta[g::SL];
  put<M>(T.bX, T.S, fn.f);
  wsync();
  bchange<M>(T.bX, T.bA, T.bB, fo.u1 - fn.u1, fo.u2 - fn.u2, fo.th - fn.th, T.S, delta);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) delta[r] -= fo.f[r];
  put<M>(T.bC, T.S, delta);  // bC is free in this kernel
  wsync();
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    double *rec = const_cast<double *>(recp<M>(Af, fine, 2 * I + (q & 1), 2 * J + (q >> 1)));
    Cell<M> x;
    load_cell<M>(rec, T.S, x);
    double t[g::SL];
    bchange<M>(T.bC, T.bA, T.bB, x.u1 - fo.u1, x.u2 - fo.u2, x.th - fo.th, T.S, t);
    double fs[g::SL];
#pragma unroll
    for (int r = 0; r < g::SL; ++r) fs[r] = x.f[r] + t[r];
    Cell<M> nc;
    if (normalise<M>(x, fs, T, nc)) store_record<M>(rec, nc.u1, nc.u2, nc.th, T.bA, T.lane);
    else if (T.lane == 0) atomicOr(err, 2);
    wsync();
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

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

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

hipError_t launch_sweep_diag(int M, const LevelArgs &A, double *st, const double *rhs, int dir,
                             int t, int *err, hipStream_t s) {
  const int a0 = t - (A.ny - 1) > 0 ? t - (A.ny - 1) : 0;
  const int a1 = t < A.nx - 1 ? t : A.nx - 1;
  const int ncell = a1 - a0 + 1;
  if (ncell <= 0) return hipSuccess;
  NRXX_DISPATCH_M(M, {
    if (A.order == 1)
      hipLaunchKernelGGL((k_sweep_diag<MM, 1>), dim3(ncell), dim3(WAVE), 0, s, A, st, rhs, dir, t, a0, err);
    else
      hipLaunchKernelGGL((k_sweep_diag<MM, 2>), dim3(ncell), dim3(WAVE), 0, s, A, st, rhs, dir, t, a0, err);
  });
  return hipGetLastError();
}

hipError_t launch_residual(int M, const LevelArgs &A, const double *st, const double *rhs,
                           const double *Radd, double *out, double *norm_part, int mode,
                           hipStream_t s) {
  const int ncell = A.nx * A.ny;
  NRXX_DISPATCH_M(M, {
    if (A.order == 1)
      hipLaunchKernelGGL((k_residual<MM, 1>), dim3(ncell), dim3(WAVE), 0, s, A, st, rhs, Radd, out, norm_part, mode);
    else
      hipLaunchKernelGGL((k_residual<MM, 2>), dim3(ncell), dim3(WAVE), 0, s, A, st, rhs, Radd, out, norm_part, mode);
  });
  return hipGetLastError();
}

hipError_t launch_restrict(int M, const LevelArgs &Af, const double *fine, const double *fineR,
                           double *coarse, double *coarseR, int *err, hipStream_t s) {
  const int nc = (Af.nx / 2) * (Af.ny / 2);
  NRXX_DISPATCH_M(M, {
    hipLaunchKernelGGL((k_restrict<MM>), dim3(nc), dim3(WAVE), 0, s, Af, fine, fineR, coarse, coarseR, err);
  });
  return hipGetLastError();
}

hipError_t launch_correct(int M, const LevelArgs &Af, double *fine, const double *cnew,
                          const double *cold, int *err, hipStream_t s) {
  const int nc = (Af.nx / 2) * (Af.ny / 2);
  NRXX_DISPATCH_M(M, {
    hipLaunchKernelGGL((k_correct<MM>), dim3(nc), dim3(WAVE), 0, s, Af, fine, cnew, cold, err);
  });
  return hipGetLastError();
}

hipError_t launch_init_maxwellian(int M, const LevelArgs &A, double *st, double rho, double u1,
                                  double u2, double th, hipStream_t s) {
  const int ncell = A.nx * A.ny;
  NRXX_DISPATCH_M(M, {
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

hipError_t launch_mass_scale(int M, const LevelArgs &A, double *st, const double *mass,
                             double mass0, hipStream_t s) {
  const int ncell = A.nx * A.ny;
  NRXX_DISPATCH_M(M, {
    const size_t tot = (size_t)ncell * G<MM>::STRIDE;
    int blocks = (int)((tot + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_mass_scale<MM>), dim3(blocks), dim3(256), 0, s, ncell, st, mass, mass0);
  });
  return hipGetLastError();
}

}  // namespace nrxx
