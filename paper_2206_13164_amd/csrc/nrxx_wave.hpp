// nrxx_wave.hpp -- one wavefront per cell: the Gauss-Seidel cell update of
// Alg. 1 (R_ij of eq. (13), local step of eq. (18), update and re-expansion
// of Sec. 2.4) evaluated by a single wavefront with a small LDS footprint,
// for sweeps with many independent cells in flight (batches of cavities).
//
// The cell-team form (nrxx_device.hpp) spreads a cell's eight face-side items
// over up to eight wavefronts and keeps all of them in LDS at once; it has
// the shortest latency per cell but fits one or two cells per CU.  Here one
// wavefront walks the faces E, W, N, S in turn and adds each face's terms to
// registers as soon as they are known, so it needs only four coefficient
// vectors of LDS and far fewer registers, and a CU holds tens of cells.  The
// arithmetic of every term and the order in which the terms are added are
// those of the cell team (same expressions, same fused multiply-adds), so
// both forms give bit-identical results.
//
// Packed LDS layouts.  A coefficient vector holds only the even-alpha_3
// coefficients E_M = {(a1, a2, m) : a1 + a2 + 2m <= M} (NE of them), stored
// in one of three orders: L1 with alpha_1 fastest, L2 with alpha_2 fastest,
// L3 with m = alpha_3 / 2 fastest.  Along the fastest index the Hermite
// shifts alpha -/+ k e_d are the constant offsets -/+ k, so the three passes
// of a basis change read L1, L2, L3 in turn and each writes the next layout;
// the flux xi_d f reads L1 (d = 1) or L2 (d = 2) at +-1.  Mixed shifts (the
// regularisation term) go through LDS maps from the dense (a1, a2, m) cube
// address to the packed position.  The packed vectors are 3-4x smaller than
// the dense cube the cell team uses (95 against 405 doubles at M = 8).
#pragma once

#include "nrxx_device.hpp"

namespace nrxx {
namespace {

// A wavefront-uniform value moved to scalar registers: vector registers are
// what limits the number of cells in flight, and a uniform double held in a
// vector register takes two of them.
__device__ __forceinline__ double uni(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __builtin_bit_cast(double, (unsigned long long)hi << 32 | lo);
}

// Packed layouts of order M.  Every line along the fastest index is
// preceded by a run of zeros as long as the basis change reaches back (M in
// L1 and L2, M / 2 in L3), so a basis-change pass reads alpha - k e_d for
// every k with no select: below the line's start it reads a zero.
template <int M>
constexpr int pad_size(int lay) {
  int s = 0;
  if (lay == 3) {
    for (int a1 = 0; a1 <= M; ++a1)
      for (int a2 = 0; a1 + a2 <= M; ++a2) s += M / 2 + (M - a1 - a2) / 2 + 1;
  } else {
    for (int m = 0; 2 * m <= M; ++m)
      for (int b = 0; b + 2 * m <= M; ++b) s += M + (M - 2 * m - b + 1);
  }
  return s;
}

template <int M>
struct Pack {
  static constexpr int NE = neven(M);
  static constexpr int D1 = M + 1, D2 = (M + 1) * (M + 1);
  static constexpr int CUBE = D2 * (M / 2 + 1);
  static constexpr int N = nalpha(M);
  static constexpr int P12 = pad_size<M>(1), P3 = pad_size<M>(3);
  static constexpr int PV = P12 > P3 ? P12 : P3;  // one padded vector
  // per slot e (the even-alpha_3 coefficients in graded order, as in the
  // cell team): alpha, position in the graded record order, cube address,
  // positions in L1, L2, L3
  int16_t a1[NE], a2[NE], m[NE], ci[NE], ca[NE], p1[NE], p2[NE], p3[NE];
  int16_t map1[CUBE], map2[CUBE];  // cube address -> L1 / L2 position (0 outside E_M)
  int16_t canon1[N];               // graded index -> L1 position (-1 for odd alpha_3)
};

template <int M>
constexpr Pack<M> make_pack() {
  Pack<M> t{};
  using P = Pack<M>;
  int16_t l1[P::CUBE] = {}, l2[P::CUBE] = {}, l3[P::CUBE] = {};
  int k = 0;
  for (int m = 0; 2 * m <= M; ++m)
    for (int a2 = 0; a2 + 2 * m <= M; ++a2) {
      k += M;  // zeros ahead of the line
      for (int a1 = 0; a1 + a2 + 2 * m <= M; ++a1) l1[a1 + P::D1 * a2 + P::D2 * m] = (int16_t)k++;
    }
  k = 0;
  for (int m = 0; 2 * m <= M; ++m)
    for (int a1 = 0; a1 + 2 * m <= M; ++a1) {
      k += M;
      for (int a2 = 0; a1 + a2 + 2 * m <= M; ++a2) l2[a1 + P::D1 * a2 + P::D2 * m] = (int16_t)k++;
    }
  k = 0;
  for (int a1 = 0; a1 <= M; ++a1)
    for (int a2 = 0; a1 + a2 <= M; ++a2) {
      k += M / 2;
      for (int m = 0; a1 + a2 + 2 * m <= M; ++m) l3[a1 + P::D1 * a2 + P::D2 * m] = (int16_t)k++;
    }
  for (int c = 0; c < P::CUBE; ++c) {
    t.map1[c] = l1[c];
    t.map2[c] = l2[c];
  }
  int e = 0, g = 0;
  for (int n = 0; n <= M; ++n)
    for (int a1 = n; a1 >= 0; --a1)
      for (int a2 = n - a1; a2 >= 0; --a2, ++g) {
        const int a3 = n - a1 - a2;
        if (a3 & 1) {
          t.canon1[g] = -1;
          continue;
        }
        const int c = a1 + P::D1 * a2 + P::D2 * (a3 / 2);
        t.canon1[g] = l1[c];
        t.a1[e] = (int16_t)a1;
        t.a2[e] = (int16_t)a2;
        t.m[e] = (int16_t)(a3 / 2);
        t.ci[e] = (int16_t)g;
        t.ca[e] = (int16_t)c;
        t.p1[e] = l1[c];
        t.p2[e] = l2[c];
        t.p3[e] = l3[c];
        ++e;
      }
  return t;
}

__constant__ Pack<3> c_pack3 = make_pack<3>();
__constant__ Pack<4> c_pack4 = make_pack<4>();
__constant__ Pack<5> c_pack5 = make_pack<5>();
__constant__ Pack<6> c_pack6 = make_pack<6>();
__constant__ Pack<7> c_pack7 = make_pack<7>();
__constant__ Pack<8> c_pack8 = make_pack<8>();
__constant__ Pack<9> c_pack9 = make_pack<9>();
__constant__ Pack<10> c_pack10 = make_pack<10>();

template <int M>
__device__ __forceinline__ const Pack<M> &pack_of() {
  if constexpr (M == 3) return c_pack3;
  else if constexpr (M == 4) return c_pack4;
  else if constexpr (M == 5) return c_pack5;
  else if constexpr (M == 6) return c_pack6;
  else if constexpr (M == 7) return c_pack7;
  else if constexpr (M == 8) return c_pack8;
  else if constexpr (M == 9) return c_pack9;
  else return c_pack10;
}

// L1 position of alpha = (a1, a2, 2m), for coefficients used by name.
template <int M>
constexpr int l1pos(int a1, int a2, int m) {
  return make_pack<M>().map1[a1 + (M + 1) * a2 + (M + 1) * (M + 1) * m];
}
template <int M>
struct Named {
  static constexpr int R0 = l1pos<M>(0, 0, 0);
  static constexpr int E1 = l1pos<M>(1, 0, 0), E2 = l1pos<M>(0, 1, 0);
  static constexpr int XX = l1pos<M>(2, 0, 0), YY = l1pos<M>(0, 2, 0), ZZ = l1pos<M>(0, 0, 1);
  static constexpr int X3 = l1pos<M>(3, 0, 0), X1Y2 = l1pos<M>(1, 2, 0), X1Z2 = l1pos<M>(1, 0, 1);
  static constexpr int Y3 = l1pos<M>(0, 3, 0), X2Y1 = l1pos<M>(2, 1, 0), Y1Z2 = l1pos<M>(0, 1, 1);
  static constexpr int XY = l1pos<M>(1, 1, 0);
};

// LDS of the workgroup shared by its wavefronts: the cube -> position maps.
template <int M>
struct WTabs {
  int16_t map1[Pack<M>::CUBE], map2[Pack<M>::CUBE], canon1[Pack<M>::N];
};

template <int M>
__device__ __forceinline__ void load_tabs(WTabs<M> &t) {
  const Pack<M> &P = pack_of<M>();
#pragma unroll 1
  for (int x = threadIdx.x; x < Pack<M>::CUBE; x += blockDim.x) {
    t.map1[x] = P.map1[x];
    t.map2[x] = P.map2[x];
  }
#pragma unroll 1
  for (int x = threadIdx.x; x < Pack<M>::N; x += blockDim.x) t.canon1[x] = P.canon1[x];
}

// Per-wavefront LDS (in Reals): the cell (L1); the own and neighbour face
// states of a face (L1 for x faces, L2 for y faces); the basis-change input X
// (L1) and its temporaries Y (L2) and Z (L3), whose zero runs must stay zero;
// the wall tables; and (M <= 6) the records of the cell's stencil.
template <int M>
struct WLay {
  static constexpr int NE = neven(M);
  static constexpr int V = Pack<M>::PV;              // one padded vector
  static constexpr int C = 0, FO = V, FN = 2 * V, X = 3 * V, Y = 4 * V, Z = 5 * V;
  static constexpr int KOFF = 6 * V;                 // K_n(a), n <= 2M+1
  static constexpr int JOFF = KOFF + 2 * M + 2;      // J+_{kl}(a), (M+1)^2
  static constexpr int BC = JOFF + (M + 1) * (M + 1);  // broadcast slot
  static constexpr int OP = BC + 2;                  // own face-state parameters, 4 x 3
  // the records of the cell's stencil and its right-hand side, gathered
  // from memory in one batch: [u1, u2, th, f_e (slot order)] each; at
  // M >= 7 the LDS is better spent on cells in flight and records are read
  // from memory where used
  static constexpr bool GATHER = M <= 6;
  static constexpr int GREC = (NE + 3 + 1) / 2 * 2;
  static constexpr int GOFF = OP + 12;
  static constexpr int TOTAL = GOFF + (GATHER ? 10 * GREC : 0);
};

// Zero the basis-change buffers once per kernel (their zero runs are never
// written afterwards).
template <typename Real, int M>
__device__ __forceinline__ void wzero(Real *lw, int lane) {
  using L = WLay<M>;
  for (int x = L::X + lane; x < L::X + 3 * L::V; x += WAVE) lw[x] = Real(0.0);
  wsync();
}

// Stencil records of a cell in the gather area: the cell, its x and y
// neighbours at distance 1 and 2, and the right-hand side record.
enum { Q_C = 0, Q_XP1, Q_XM1, Q_XP2, Q_XM2, Q_YP1, Q_YM1, Q_YP2, Q_YM2, Q_RHS, NQ };
__device__ __forceinline__ int q_of(int D, int off) {
  const int base = D == 0 ? Q_XP1 : Q_YP1;
  return base + (off > 0 ? 0 : 1) + (off == 2 || off == -2 ? 2 : 0);
}

// The lane's slots: which coefficients it holds and where they live.
template <int M>
struct WSlot {
  static constexpr int SL = G<M>::SL;
  int a1[SL], a2[SL], m[SL], n[SL], ci[SL], ca[SL], p1[SL], p2[SL], p3[SL];
  bool ok[SL];
  __device__ __forceinline__ void init(int lane) {
    const Pack<M> &P = pack_of<M>();
#pragma unroll
    for (int r = 0; r < SL; ++r) {
      const int e = lane + WAVE * r;
      ok[r] = e < Pack<M>::NE;
      const int ee = ok[r] ? e : 0;
      a1[r] = P.a1[ee];
      a2[r] = P.a2[ee];
      m[r] = P.m[ee];
      n[r] = a1[r] + a2[r] + 2 * m[r];
      ci[r] = P.ci[ee];
      ca[r] = P.ca[ee];
      p1[r] = P.p1[ee];
      p2[r] = P.p2[ee];
      p3[r] = P.p3[ee];
    }
  }
};

template <typename Real, int M>
__device__ __forceinline__ void wload_cell(const Real *__restrict__ rec, const WSlot<M> &S,
                                           Cell<Real, M> &c) {
  c.u1 = uni(rec[0]);
  c.u2 = uni(rec[1]);
  c.th = uni(rec[2]);
#pragma unroll
  for (int r = 0; r < G<M>::SL; ++r) c.f[r] = S.ok[r] ? rec[3 + S.ci[r]] : Real(0.0);
}

// Loads every record the update of cell (i, j) reads -- the cell, its
// neighbours at distance 1 (and 2 at second order) inside the grid, and the
// right-hand side `rr` (if any) -- with all loads in flight at once, and
// stores them in the gather area (lane e holds slot e).
template <typename Real, int M, int ORDER, int Q0, int Q1>
__device__ __forceinline__ void wgather_part(const LevelArgs &A, const Real *__restrict__ st,
                                             const Real *__restrict__ rr, int i, int j, Real *G0,
                                             const WSlot<M> &S, int lane) {
  using g = G<M>;
  using L = WLay<M>;
  constexpr int NP = Q1 - Q0;
  Real v[NP][g::SL], pv[NP];
  bool have[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    const int q = Q0 + t;
    int ii = i, jj = j;
    if (q >= Q_XP1 && q <= Q_XM2) ii += (q == Q_XP1 ? 1 : q == Q_XM1 ? -1 : q == Q_XP2 ? 2 : -2);
    if (q >= Q_YP1 && q <= Q_YM2) jj += (q == Q_YP1 ? 1 : q == Q_YM1 ? -1 : q == Q_YP2 ? 2 : -2);
    const bool far = q == Q_XP2 || q == Q_XM2 || q == Q_YP2 || q == Q_YM2;
    have[t] = ii >= 0 && ii < A.nx && jj >= 0 && jj < A.ny && !(far && ORDER == 1) &&
              (q != Q_RHS || rr != nullptr);
    if (have[t]) {
      const Real *rec = recp<Real, M>(A, q == Q_RHS ? rr : st, ii, jj);
#pragma unroll
      for (int r = 0; r < g::SL; ++r) v[t][r] = S.ok[r] ? rec[3 + S.ci[r]] : Real(0.0);
      pv[t] = rec[lane < 3 ? lane : 0];
    }
  }
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    if (!have[t]) continue;
    Real *Gq = G0 + (Q0 + t) * L::GREC;
#pragma unroll
    for (int r = 0; r < g::SL; ++r)
      if (S.ok[r]) Gq[3 + lane + WAVE * r] = v[t][r];
    if (lane < 3) Gq[lane] = pv[t];
  }
}

// Loads every record the update of cell (i, j) reads -- the cell, its
// neighbours at distance 1 (and 2 at second order) inside the grid, and the
// right-hand side `rr` (if any) -- in two batches of loads in flight at
// once, into the gather area (lane e holds slot e).
template <typename Real, int M, int ORDER>
__device__ __forceinline__ void wgather(const LevelArgs &A, const Real *__restrict__ st,
                                        const Real *__restrict__ rr, int i, int j, Real *lw,
                                        const WSlot<M> &S, int lane) {
  if constexpr (WLay<M>::GATHER) {
    Real *G0 = lw + WLay<M>::GOFF;
    wgather_part<Real, M, ORDER, 0, 5>(A, st, rr, i, j, G0, S, lane);
    wgather_part<Real, M, ORDER, 5, NQ>(A, st, rr, i, j, G0, S, lane);
    wsync();
  }
}

// Record q of the cell's stencil as a Cell: from the gather area, or (no
// gather) from memory.
template <typename Real, int M>
__device__ __forceinline__ void cell_q(const LevelArgs &A, const Real *__restrict__ st,
                                       const Real *__restrict__ rr, int i, int j, const Real *lw,
                                       int q, const WSlot<M> &S, int lane, Cell<Real, M> &c) {
  using L = WLay<M>;
  if constexpr (L::GATHER) {
    const Real *Gq = lw + L::GOFF + q * L::GREC;
    c.u1 = uni(Gq[0]);
    c.u2 = uni(Gq[1]);
    c.th = uni(Gq[2]);
#pragma unroll
    for (int r = 0; r < G<M>::SL; ++r) c.f[r] = S.ok[r] ? Gq[3 + lane + WAVE * r] : Real(0.0);
  } else {
    int ii = i, jj = j;
    if (q >= Q_XP1 && q <= Q_XM2) ii += (q == Q_XP1 ? 1 : q == Q_XM1 ? -1 : q == Q_XP2 ? 2 : -2);
    if (q >= Q_YP1 && q <= Q_YM2) jj += (q == Q_YP1 ? 1 : q == Q_YM1 ? -1 : q == Q_YP2 ? 2 : -2);
    wload_cell<Real, M>(recp<Real, M>(A, q == Q_RHS ? rr : st, ii, jj), S, c);
  }
}

// v -> packed vector `buf` in layout L1 (lay = 1) or L2 (lay = 2)
template <typename Real, int M>
__device__ __forceinline__ void wput(Real *buf, int lay, const WSlot<M> &S,
                                     const Real (&v)[G<M>::SL]) {
#pragma unroll
  for (int r = 0; r < G<M>::SL; ++r)
    if (S.ok[r]) buf[lay == 1 ? S.p1[r] : S.p2[r]] = v[r];
}

// Basis change by (du1, du2, dth) of the vector X (layout L1) through Y (L2)
// and Z (L3); the result stays in registers.  The terms are those of
// bchange, added in the same order; a term beyond alpha_d reads a zero of the
// layout's zero run instead of being selected away.
template <typename Real, int M>
__device__ __forceinline__ void wbchange(const Real *X, Real *Y, Real *Z, Real du1, Real du2,
                                         Real dth, const WSlot<M> &S, Real (&res)[G<M>::SL]) {
  using g = G<M>;
  Real c[M + 1];
  tcoef<Real, M>(du1, dth, c);
#pragma unroll
  for (int k = 0; k <= M; ++k) c[k] = uni(c[k]);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    const Real *p = X + S.p1[r];
    Real x[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) x[k] = p[-k];
    Real acc = x[0];
#pragma unroll
    for (int k = 1; k <= M; ++k) acc = fma(c[k], x[k], acc);
    if (S.ok[r]) Y[S.p2[r]] = acc;
  }
  wsync();
  tcoef<Real, M>(du2, dth, c);
#pragma unroll
  for (int k = 0; k <= M; ++k) c[k] = uni(c[k]);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    const Real *p = Y + S.p2[r];
    Real x[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) x[k] = p[-k];
    Real acc = x[0];
#pragma unroll
    for (int k = 1; k <= M; ++k) acc = fma(c[k], x[k], acc);
    if (S.ok[r]) Z[S.p3[r]] = acc;
  }
  wsync();
  tcoef<Real, M>(Real(0.0), dth, c);
#pragma unroll
  for (int k = 0; k <= M; k += 2) c[k] = uni(c[k]);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    const Real *p = Z + S.p3[r];
    Real x[M / 2 + 1];
#pragma unroll
    for (int k = 0; 2 * k <= M; ++k) x[k] = p[-k];
    Real acc = x[0];
#pragma unroll
    for (int k = 1; 2 * k <= M; ++k) acc = fma(c[2 * k], x[k], acc);
    res[r] = S.ok[r] ? acc : Real(0.0);
  }
  wsync();
}

// (Pi_M xi_D f)_alpha of the vector F stored in L1 (D = 0) or L2 (D = 1).
template <typename Real, int M>
__device__ __forceinline__ Real wximul(int D, const Real *F, Real ud, Real th, const WSlot<M> &S,
                                       int r) {
  const int p = D == 0 ? S.p1[r] : S.p2[r];
  const int ad = D == 0 ? S.a1[r] : S.a2[r];
  const Real x0 = F[p], xl = F[ad >= 1 ? p - 1 : p], xh = F[S.n[r] < M ? p + 1 : p];
  Real v = ud * x0;
  if (ad >= 1) v += th * xl;
  if (S.n[r] < M) v += (ad + 1) * xh;
  return v;
}

// Regularisation term of direction D at |beta| = M (zero below) of
// (fL + fR) / 2, the vectors read through `map` (cube address -> position).
// Same arithmetic as regul.
template <typename Real, int M>
__device__ __forceinline__ Real wregul(int D, const Real *fL, const Real *fR, const int16_t *map,
                                       Real du1, Real du2, Real dth, const WSlot<M> &S, int r) {
  using g = G<M>;
  if (!S.ok[r] || S.n[r] != M) return Real(0.0);
  const int base = S.ca[r] + (D == 0 ? 1 : g::D1);  // b + e_D (cube address)
  const int b0 = S.a1[r] + (D == 0), b1 = S.a2[r] + (D == 1), b2 = 2 * S.m[r];
  Real acc = Real(0.0);
  if (b0 >= 1) {
    const int q = map[base - 1];
    acc += Real(0.5) * (fL[q] + fR[q]) * du1;
  }
  if (b0 >= 2) {
    const int q = map[base - 2];
    acc += Real(0.5) * (Real(0.5) * (fL[q] + fR[q])) * dth;
  }
  if (b1 >= 1) {
    const int q = map[base - g::D1];
    acc += Real(0.5) * (fL[q] + fR[q]) * du2;
  }
  if (b1 >= 2) {
    const int q = map[base - 2 * g::D1];
    acc += Real(0.5) * (Real(0.5) * (fL[q] + fR[q])) * dth;
  }
  if (b2 >= 2) {
    const int q = map[base - g::D2];
    acc += Real(0.5) * (Real(0.5) * (fL[q] + fR[q])) * dth;
  }
  const int bd = D == 0 ? S.a1[r] : S.a2[r];
  return (bd + 1) * acc;
}

// Half-range tables of a diffuse wall in the wavefront's scratch (same
// arithmetic as wall_tables).
template <typename Real, int M>
__device__ void wwall_tables(int wall, Real u1, Real u2, Real th, Real *lw, int lane) {
  using L = WLay<M>;
  const int d = (wall == 0 || wall == 2) ? 1 : 0;
  const Real sig = (wall == 1 || wall == 2) ? Real(1.0) : -Real(1.0);
  const Real a = sig * (d == 0 ? u1 : u2) / sqrt(th);
  Real *K = lw + L::KOFF;
  Real *Jp = lw + L::JOFF;
  const Real ga = exp(-Real(0.5) * a * a) * (Real(0.5) * Real(M_2_SQRTPI) * Real(M_SQRT1_2));
  for (int n = lane; n <= 2 * M + 1; n += WAVE)
    K[n] = n == 0 ? Real(0.5) * erfc(-a * Real(M_SQRT1_2)) : hermite<Real, 2 * M>(n - 1, -a) * ga;
  wsync();
  for (int t = lane; t < (M + 1) * (M + 1); t += WAVE) {
    int k = t / (M + 1), l = t % (M + 1);
    Jp[t] = a * halfI<Real>(K, k, l) + halfI<Real>(K, k, l + 1) + l * halfI<Real>(K, k, l - 1);
  }
  wsync();
}

// Outward flux through a diffuse wall in the cell basis (same arithmetic as
// wall_flux).  fc: the cell's coefficients in L1 (x walls) or L2 (y walls).
template <typename Real, int M>
__device__ void wwall_flux(const LevelArgs &A, int wall, Real u1, Real u2, Real th, const Real *fc,
                           Real *lw, const WTabs<M> &T, const WSlot<M> &S, int lane,
                           Real (&phi)[G<M>::SL]) {
  using g = G<M>;
  using L = WLay<M>;
  const int d = (wall == 0 || wall == 2) ? 1 : 0;
  const Real sig = (wall == 1 || wall == 2) ? Real(1.0) : -Real(1.0);
  const Real sq = sqrt(th);
  const Real *Jp = lw + L::JOFF;
  const Real isq = Real(1.0) / sq;
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    Real acc = Real(0.0);
    if (S.ok[r]) {
      int ad = d == 0 ? S.a1[r] : S.a2[r];
      int at = (d == 0 ? S.a2[r] : S.a1[r]) + 2 * S.m[r];  // transverse degree
      int base = (d == 0 ? S.p1[r] : S.p2[r]) - ad;        // alpha with alpha_d = 0
      Real pa = Real(1.0), fa = Real(1.0);
      for (int q = 0; q < ad; ++q) {
        pa *= sq;
        fa *= Real(q + 1);
      }
      const Real ifa = Real(1.0) / fa;
      Real ib = Real(1.0);
#pragma unroll
      for (int bd = 0; bd <= M; ++bd) {
        if (bd + at <= M) {
          Real sgn = ((ad + bd) & 1) ? sig : Real(1.0);
          acc += fc[base + bd] * (pa * ib) * sq * sgn * Jp[ad * (M + 1) + bd] * ifa;
        }
        ib *= isq;
      }
    }
    phi[r] = acc;
  }
  Real *bc = lw + L::BC;
  if (lane == 0) bc[0] = phi[0];
  wsync();
  const Real thw = Real(A.wall_th[wall]), sqw = sqrt(thw);
  const Real rhow = bc[0] * sqrt(Real(2.0) * Real(M_PI) / thw);
  Real *X = lw + L::X;
#pragma unroll
  for (int r = 0; r < g::SL; ++r)
    if (S.ok[r]) X[S.p1[r]] = Real(0.0);
  wsync();
  if (lane <= M) {
    int k = lane;
    Real pw = Real(1.0);
    for (int q = 0; q < k; ++q) pw *= sqw;
    Real sgn = (k & 1) ? sig : Real(1.0);
    X[T.map1[d == 0 ? k : k * g::D1]] = rhow * pw * sqw * sgn * Real(A.jminus[k]);
  }
  wsync();
  const Real uw1 = d == 1 ? Real(A.wall_u[wall]) : Real(0.0), uw2 = d == 0 ? Real(A.wall_u[wall]) : Real(0.0);
  Real t[g::SL];
  wbchange<Real, M>(X, lw + L::Y, lw + L::Z, u1 - uw1, u2 - uw2, th - thw, S, t);
#pragma unroll
  for (int r = 0; r < g::SL; ++r) phi[r] += t[r];
}

// Update of sweeps (Sec. 2.4) with the result in X (L1) and `out`; same
// arithmetic as normalise.  false for rho <= 0, th <= 0 or non-finite values.
template <typename Real, int M>
__device__ bool wnormalise(Real ou1, Real ou2, Real oth, const Real (&fs)[G<M>::SL], Real *lw,
                           const WSlot<M> &S, int lane, Cell<Real, M> &out) {
  using g = G<M>;
  using L = WLay<M>;
  using NM = Named<M>;
  Real *X = lw + L::X;
  wput<Real, M>(X, 1, S, fs);
  wsync();
  const Real rho = X[NM::R0];
  const Real fe1 = X[NM::E1], fe2 = X[NM::E2];
  const Real tr = X[NM::XX] + X[NM::YY] + X[NM::ZZ];
  const Real irho = Real(1.0) / rho;
  const Real u1n = ou1 + fe1 * irho, u2n = ou2 + fe2 * irho;
  const Real thn = oth + (Real(2.0) * tr - (fe1 * fe1 + fe2 * fe2) * irho) * (irho * (Real(1.0) / Real(3.0)));
  bool okp = rho > Real(0.0) && thn > Real(0.0) && isfinite(rho) && isfinite(thn) && isfinite(u1n) &&
             isfinite(u2n);
  if (!okp) return false;  // uniform branch
  Real t[g::SL];
  wbchange<Real, M>(X, lw + L::Y, lw + L::Z, u1n - ou1, u2n - ou2, thn - oth, S, t);
  wput<Real, M>(X, 1, S, t);
  wsync();
  const Real zz = -(X[NM::XX] + X[NM::YY]);
  bool fin = true;
#pragma unroll
  for (int r = 0; r < g::SL; ++r) {
    const int p = S.p1[r];
    if (p == NM::E1 || p == NM::E2) t[r] = Real(0.0);
    if (p == NM::ZZ) t[r] = zz;
    if (S.ok[r] && !isfinite(t[r])) fin = false;
  }
  wsync();
  if (lane < 2) X[lane == 0 ? NM::E1 : NM::E2] = Real(0.0);
  if (lane == 0) X[NM::ZZ] = zz;
  wsync();
  out.u1 = u1n;
  out.u2 = u2n;
  out.th = thn;
#pragma unroll
  for (int r = 0; r < g::SL; ++r) out.f[r] = t[r];
  return __ballot(!fin) == 0;
}

// Coalesced write of a full record from (params, X in L1); odd-alpha_3
// coefficients as zeros.
template <typename Real, int M, bool SHARED = false>
__device__ __forceinline__ void wstore_record(Real *__restrict__ rec, Real u1, Real u2, Real th,
                                              const Real *X, const WTabs<M> &T, int lane) {
  using g = G<M>;
#pragma unroll
  for (int t = 0; t < g::SR; ++t) {
    const int v = lane + WAVE * t;
    if (v < g::NR) {
      Real x;
      if (v == 0) x = u1;
      else if (v == 1) x = u2;
      else if (v == 2) x = th;
      else {
        const int q = T.canon1[v - 3];
        x = q < 0 ? Real(0.0) : X[q];
      }
      if constexpr (SHARED) put_shared(rec + v, x);
      else rec[v] = x;
    }
  }
}

// Cell (i, j) by one wavefront, in the modes of cell_team:
//  MODE_SWEEP : one Gauss-Seidel update, f <- normalise(f + dt (R_ij(f) - r))
//               (Alg. 1); a non-physical update sets bit 0 of *err and leaves
//               the cell unchanged;
//  MODE_DEFECT: out = r - R(f) in the cell basis, norm_part[cell] = weighted
//               norm^2 * ds (eq. (28));
//  MODE_FAS   : out = R(f) + Radd (coarse right-hand side of eq. (22)).
// R is assembled in the cell team's order with the same arithmetic.
template <typename Real, int M, int ORDER, int MODE = MODE_SWEEP>
__device__ void wave_cell(const LevelArgs &A, Real *lw, const WTabs<M> &T, const WSlot<M> &S,
                          int lane, Real *__restrict__ st, const Real *__restrict__ rhs, int i,
                          int j, int *err, const Real *__restrict__ Radd = nullptr,
                          Real *__restrict__ out = nullptr, Real *__restrict__ norm_part = nullptr) {
  using g = G<M>;
  using L = WLay<M>;
  using NM = Named<M>;
  Real *bC = lw + L::C, *bA = lw + L::FO, *bB = lw + L::FN, *bX = lw + L::X;
  Real *bY = lw + L::Y, *bZ = lw + L::Z;
  const int nx = A.nx, ny = A.ny;
  const Real *rr = MODE == MODE_FAS ? Radd : rhs;
  wgather<Real, M, ORDER>(A, st, rr, i, j, lw, S, lane);
  Cell<Real, M> c;
  cell_q<Real, M>(A, st, rr, i, j, lw, Q_C, S, lane, c);
  wput<Real, M>(bC, 1, S, c.f);
  const Real rho = uni(c.f[0]);  // f_0 sits in lane 0, slot 0
  const Real nu = uni(Real(A.beta) * sqrt(Real(M_PI) / Real(2.0)) * rho * pow(c.th, Real(1.0) - Real(A.omega)) / Real(A.Kn));
  wsync();
  Real R[g::SL];
#pragma unroll
  for (int r = 0; r < g::SL; ++r) R[r] = Real(0.0);
  // parameters of the cell's own face states (E, W, N, S), kept for the
  // in-cell regularisation
  Real *op = lw + L::OP;
  // the stencil records of the face direction at hand (+1, -1, +2, -2
  // along it), read together at the direction's first face: one memory
  // round trip per direction when they are not gathered
  Cell<Real, M> P1, M1, P2, M2;
  // faces E, W, N, S in turn (a run-time loop: one copy of the face code)
#pragma unroll 1
  for (int f = 0; f < 4; ++f) {
    const int D = f >> 1;
    const int k = D == 0 ? i : j, n = D == 0 ? nx : ny;
    const Real ih = D == 0 ? Real(A.idx) : Real(A.idy);
    const int lay = D == 0 ? 1 : 2;
    const int sd = (f & 1) ? -1 : 1;
    const Real side = (Real)sd;
    const bool flat = ORDER == 1 || k == 0 || k == n - 1;
    // (gathered records are read from LDS where used instead)
    if (!L::GATHER && (f & 1) == 0) {
      // only records inside the grid (the uses below stay within them)
      if (k + 1 < n) cell_q<Real, M>(A, st, rr, i, j, lw, q_of(D, 1), S, lane, P1);
      if (k >= 1) cell_q<Real, M>(A, st, rr, i, j, lw, q_of(D, -1), S, lane, M1);
      if (ORDER == 2 && k + 2 < n) cell_q<Real, M>(A, st, rr, i, j, lw, q_of(D, 2), S, lane, P2);
      if (ORDER == 2 && k >= 2) cell_q<Real, M>(A, st, rr, i, j, lw, q_of(D, -2), S, lane, M2);
    }

    // own face state (not flat: 1 <= k <= n - 2, so P1 and M1 are inside)
    Cell<Real, M> Xo;
    if (flat) Xo = c;
    else {
      if constexpr (L::GATHER) {
        Cell<Real, M> hi, lo;
        cell_q<Real, M>(A, st, rr, i, j, lw, q_of(D, 1), S, lane, hi);
        cell_q<Real, M>(A, st, rr, i, j, lw, q_of(D, -1), S, lane, lo);
        face_state<Real, M>(c, hi, lo, A.limiter, false, side, Xo);
      } else {
        face_state<Real, M>(c, P1, M1, A.limiter, false, side, Xo);
      }
      Xo.u1 = uni(Xo.u1);
      Xo.u2 = uni(Xo.u2);
      Xo.th = uni(Xo.th);
    }
    if (lane == 0) {
      op[3 * f] = Xo.u1;
      op[3 * f + 1] = Xo.u2;
      op[3 * f + 2] = Xo.th;
    }
    if (k + sd < 0 || k + sd >= n) {
      // wall: the cell's coefficients along the normal, in L1 / L2
      const Real *fc = bC;
      if (D == 1) {
        wput<Real, M>(bA, 2, S, c.f);
        fc = bA;
      }
      wwall_tables<Real, M>(face_wall(f), c.u1, c.u2, c.th, lw, lane);
      Real Tw[g::SL];
      wwall_flux<Real, M>(A, face_wall(f), c.u1, c.u2, c.th, fc, lw, T, S, lane, Tw);
#pragma unroll
      for (int r = 0; r < g::SL; ++r) R[r] -= Tw[r] * ih;
    } else {
      // the neighbour's face state on the cell's side
      const int kn = k + sd;
      const bool nflat = ORDER == 1 || kn == 0 || kn == n - 1;
      Cell<Real, M> Xn;
      {
        // the neighbour (inside the grid) and, not flat (1 <= kn <= n - 2),
        // the one beyond it
        Cell<Real, M> nb, far;
        if constexpr (L::GATHER) cell_q<Real, M>(A, st, rr, i, j, lw, q_of(D, sd), S, lane, nb);
        else nb = sd > 0 ? P1 : M1;
        if (nflat) Xn = nb;
        else {
          if constexpr (L::GATHER) cell_q<Real, M>(A, st, rr, i, j, lw, q_of(D, 2 * sd), S, lane, far);
          else far = sd > 0 ? P2 : M2;
          if (sd > 0) face_state<Real, M>(nb, far, c, A.limiter, false, -side, Xn);
          else face_state<Real, M>(nb, c, far, A.limiter, false, -side, Xn);
          Xn.u1 = uni(Xn.u1);
          Xn.u2 = uni(Xn.u2);
          Xn.th = uni(Xn.th);
        }
      }
      wput<Real, M>(bA, lay, S, Xo.f);
      wput<Real, M>(bB, lay, S, Xn.f);
      wsync();
      // L / R: the cell is left of its E and N faces
      const Real uL = sd > 0 ? (D == 0 ? Xo.u1 : Xo.u2) : (D == 0 ? Xn.u1 : Xn.u2);
      const Real uR = sd > 0 ? (D == 0 ? Xn.u1 : Xn.u2) : (D == 0 ? Xo.u1 : Xo.u2);
      const Real thL = sd > 0 ? Xo.th : Xn.th, thR = sd > 0 ? Xn.th : Xo.th;
      const Real cL = uni(Real(A.C) * sqrt(thL)), cR = uni(Real(A.C) * sqrt(thR));
      const Real lamL = uni(fmin(uL - cL, uR - cR));
      const Real lamR = uni(fmax(uL + cL, uR + cR));
      int kase;
      Real wm, wp;
      const Real iden = uni(Real(1.0) / (lamR - lamL));
      if (lamL >= Real(0.0)) { kase = 0; wm = Real(0.0); wp = Real(1.0); }
      else if (lamR <= Real(0.0)) { kase = 1; wm = Real(1.0); wp = Real(0.0); }
      else { kase = 2; wm = -lamL * iden; wp = lamR * iden; }
      // regularisation jump of the face, straight path from L to R
      Real gr[g::SL];
      {
        const Real du1 = sd > 0 ? Xn.u1 - Xo.u1 : Xo.u1 - Xn.u1;
        const Real du2 = sd > 0 ? Xn.u2 - Xo.u2 : Xo.u2 - Xn.u2;
        const Real dth = thR - thL;
        const Real *fL = sd > 0 ? bA : bB, *fR = sd > 0 ? bB : bA;
        const int16_t *map = D == 0 ? T.map1 : T.map2;
#pragma unroll
        for (int r = 0; r < g::SL; ++r) gr[r] = wregul<Real, M>(D, fL, fR, map, du1, du2, dth, S, r);
      }
      // half fluxes of both face states (item s = 0 own, s = 1 neighbour)
      Real ah[2][g::SL];
      bool zero[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const Real *fx = s == 0 ? bA : bB;
        const bool isL = (s == 0) == (sd > 0);
        zero[s] = (isL && kase == 1) || (!isL && kase == 0);
        const Real ux = s == 0 ? (D == 0 ? Xo.u1 : Xo.u2) : (D == 0 ? Xn.u1 : Xn.u2);
        const Real thx = s == 0 ? Xo.th : Xn.th;
#pragma unroll
        for (int r = 0; r < g::SL; ++r) {
          const Real Fx = S.ok[r] ? wximul<Real, M>(D, fx, ux, thx, S, r) : Real(0.0);
          const Real fr = S.ok[r] ? fx[lay == 1 ? S.p1[r] : S.p2[r]] : Real(0.0);
          Real a;
          if (kase != 2) a = Fx;
          else if (isL) a = (lamR * Fx - lamL * lamR * fr) * iden;
          else a = (-lamL * Fx + lamL * lamR * fr) * iden;
          ah[s][r] = a;
        }
      }
      wsync();
      Real Th[2][g::SL];
#pragma unroll 1
      for (int s = 0; s < 2; ++s) {
        const Real xu1 = s == 0 ? Xo.u1 : Xn.u1, xu2 = s == 0 ? Xo.u2 : Xn.u2;
        const Real xth = s == 0 ? Xo.th : Xn.th;
        Real t[g::SL];
        if (zero[s]) {
#pragma unroll
          for (int r = 0; r < g::SL; ++r) t[r] = Real(0.0);
        } else if (xu1 == c.u1 && xu2 == c.u2 && xth == c.th) {
#pragma unroll
          for (int r = 0; r < g::SL; ++r) t[r] = s == 0 ? ah[0][r] : ah[1][r];
        } else {
          Real a[g::SL];
#pragma unroll
          for (int r = 0; r < g::SL; ++r) a[r] = s == 0 ? ah[0][r] : ah[1][r];
          wput<Real, M>(bX, 1, S, a);
          wsync();
          wbchange<Real, M>(bX, bY, bZ, c.u1 - xu1, c.u2 - xu2, c.th - xth, S, t);
        }
#pragma unroll
        for (int r = 0; r < g::SL; ++r) {
          if (s == 0) Th[0][r] = t[r];
          else Th[1][r] = t[r];
        }
      }
      const Real w = sd > 0 ? wm : wp;
      const Real sgnF = sd > 0 ? -Real(1.0) : Real(1.0);
#pragma unroll
      for (int r = 0; r < g::SL; ++r) {
        const Real TL = sd > 0 ? Th[0][r] : Th[1][r], TR = sd > 0 ? Th[1][r] : Th[0][r];
        R[r] += (sgnF * (TL + TR) + w * gr[r]) * ih;
      }
    }
    if (ORDER == 2 && (f & 1)) {
      // in-cell regularisation of direction D: jump between the cell's own
      // two face states of that direction
      wsync();
      const int fp = 2 * D, fm = 2 * D + 1;
      const Real j1 = op[3 * fp] - op[3 * fm], j2 = op[3 * fp + 1] - op[3 * fm + 1];
      const Real j3 = op[3 * fp + 2] - op[3 * fm + 2];
#pragma unroll
      for (int r = 0; r < g::SL; ++r) {
        const Real gc = wregul<Real, M>(D, bC, bC, T.map1, j1, j2, j3, S, r);
        R[r] += gc * ih;
      }
    }
  }
  {
    // collision Q = nu (f^E - f), eq. (5), (29); Shakhov f^E from eq. (8),
    // ES-BGK f^E from eq. (7)
    Real c1 = Real(0.0), c2 = Real(0.0);
    if (A.collision == 1) {
      const Real q1 = Real(2.0) * bC[NM::X3] + bC[NM::X3] + bC[NM::X1Y2] + bC[NM::X1Z2];
      const Real q2 = Real(2.0) * bC[NM::Y3] + bC[NM::X2Y1] + bC[NM::Y3] + bC[NM::Y1Z2];
      c1 = (Real(1.0) - Real(A.Pr)) * q1 * Real(0.2);
      c2 = (Real(1.0) - Real(A.Pr)) * q2 * Real(0.2);
    }
    Real b11 = Real(0.0), b12 = Real(0.0), b22 = Real(0.0), b33 = Real(0.0);
    if (A.collision == 2) {
      const Real kb = (Real(1.0) - Real(1.0) / Real(A.Pr)) / rho;
      b11 = kb * (Real(2.0) * bC[NM::XX]);
      b12 = kb * bC[NM::XY];
      b22 = kb * (Real(2.0) * bC[NM::YY]);
      b33 = kb * (Real(2.0) * bC[NM::ZZ]);
    }
#pragma unroll
    for (int r = 0; r < g::SL; ++r) {
      const int p = S.p1[r];
      Real fE = p == NM::R0 ? rho : Real(0.0);
      if (p == NM::X3 || p == NM::X1Y2 || p == NM::X1Z2) fE += c1;
      if (p == NM::Y3 || p == NM::X2Y1 || p == NM::Y1Z2) fE += c2;
      if (A.collision == 2) fE = esbgk_coef<Real>(S.a1[r], S.a2[r], S.m[r], rho, b11, b12, b22, b33);
      const Real q = S.ok[r] ? nu * (fE - c.f[r]) : Real(0.0);
      R[r] += q;
    }
  }
  Real rv[g::SL];
  if (rr) {
    // right-hand side (Alg. 1) or the restricted residual (eq. (22)) in the
    // cell basis
    Cell<Real, M> r0;
    cell_q<Real, M>(A, st, rr, i, j, lw, Q_RHS, S, lane, r0);
    if ((r0.u1 == c.u1 && r0.u2 == c.u2 && r0.th == c.th) || MODE == MODE_FAS) {
#pragma unroll
      for (int r = 0; r < g::SL; ++r) rv[r] = r0.f[r];
    } else {
      wput<Real, M>(bX, 1, S, r0.f);
      wsync();
      wbchange<Real, M>(bX, bY, bZ, c.u1 - r0.u1, c.u2 - r0.u2, c.th - r0.th, S, rv);
    }
  }
  if constexpr (MODE == MODE_SWEEP) {
    const Real dt = uni(local_dt<Real>(A, c.u1, c.u2, c.th, nu));
    Real fs[g::SL];
#pragma unroll
    for (int r = 0; r < g::SL; ++r) fs[r] = c.f[r] + dt * (rr ? R[r] - rv[r] : R[r]);
    Cell<Real, M> nc;
    if (wnormalise<Real, M>(c.u1, c.u2, c.th, fs, lw, S, lane, nc))
      wstore_record<Real, M, true>(const_cast<Real *>(recp<Real, M>(A, st, i, j)), nc.u1, nc.u2,
                                   nc.th, lw + L::X, T, lane);
    else if (lane == 0)
      atomicOr(err, 1);
  } else {
    Real o[g::SL];
#pragma unroll
    for (int r = 0; r < g::SL; ++r)
      o[r] = MODE == MODE_FAS ? R[r] + rv[r] : (rr ? rv[r] : Real(0.0)) - R[r];
    const int cellidx = j * nx + i;
    if (out) {
      wput<Real, M>(bX, 1, S, o);
      wsync();
      wstore_record<Real, M>(out + (size_t)cellidx * g::STRIDE, c.u1, c.u2, c.th, bX, T, lane);
    }
    if (MODE == MODE_DEFECT && norm_part) {
      // per-cell weight alpha! th^-|alpha| of eq. (28), reduced in the cell
      // team's order
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

}  // namespace
}  // namespace nrxx
