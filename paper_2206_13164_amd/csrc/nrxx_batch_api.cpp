// nrxx_batch_api.cpp -- host side of the batch C ABI (include/nrxx.h):
// groups of problems sharing (M, order), their level tables, the batched
// V-cycle of Alg. 2 with per-problem convergence masks, HIP-graph replay of a
// group's cycle, and the autotuner of the sweep schedule.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "nrxx_host.hpp"

using namespace nrxx;

struct nrxx_batch {
  struct Group {
    int M = 0, order = 0, stride = 0;
    std::vector<int> inst;                 // batch indices in slot order
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<std::vector<BLevel>> htab;  // [level][slot]
    std::vector<BLevel *> dtab;             // device copies
    std::vector<int> ncell;                 // cells of the group per level
    std::vector<int *> cnt;                 // [queue | per sweep: counters of every slot]
    std::vector<int> cntsize, cols;         // cols = columns of the group per level
    // unit lists per unit order, per level, for the problems that continue
    // to a coarser level (c = 0) and for those whose coarsest level it is (1)
    std::vector<int *> units[2][2];
    std::vector<int> U[2];                  // units per sweep per level
    double *partial = nullptr;              // level-0 per-cell scalars
    std::vector<void *> owned;
    int nw = 0, grid = 0, major = 0, split = 1;
    int kernel = 0;  // 0: cell-team sweep kernel, 1: wavefront-per-cell sweep kernel
    int rows = 1;    // wavefront-per-cell kernel: rows per wait/acquire/release
    double tuned_ms = 0.0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // sweep-kernel timing (nrxx_batch_set_timing): an event pair around each
    // eagerly enqueued sweep launch, with the level and the problems it served
    struct Timed {
      hipEvent_t a = nullptr, b = nullptr;
      int k = 0, which = 0, nsw = 0;
    };
    std::vector<Timed> tl;
    size_t tl_used = 0;
    bool ran = false;       // work of this group was enqueued since the last harvest
    double k_ms = 0.0, k_launches = 0.0, k_cells_fine = 0.0, k_cells_coarse = 0.0;
  };
  int n = 0, L = 0, s1 = 0, s2 = 0, s3 = 0, gamma = 1;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<nrxx_problem> P;
  std::vector<Group> g;
  int *active = nullptr, *cycles = nullptr, *derr = nullptr, *dabort = nullptr;
  double *norms = nullptr, *ref = nullptr, *mass = nullptr, *tol = nullptr;
  int *h_int = nullptr;         // pinned: active[n], cycles[n], err
  double *h_dbl = nullptr;      // pinned: norms[n], ref[n], tol
  std::vector<double *> cur;    // level-0 state pointers in the tables
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double ms = 0.0, cells = 0.0;
  int timing = 0;               // 1: time every sweep launch (nrxx_batch_kernel_stats)
  std::vector<int> hact;        // active flags of the work being enqueued or replayed
  unsigned long long wait_ticks = 200000000ULL;  // bound of one cross-column wait: 2 s at 100 MHz
};

namespace {

thread_local std::string g_batch_create_error;

int bfail(nrxx_batch *b, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b) b->err = buf;
  else g_batch_create_error = buf;
  return code;
}

int bhip(nrxx_batch *b, hipError_t e, const char *what) {
  if (e == hipSuccess) return NRXX_OK;
  return bfail(b, NRXX_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define BCHK(expr)                                  \
  do {                                              \
    int rc_ = bhip(b, (expr), #expr);               \
    if (rc_) return rc_;                            \
  } while (0)

using Group = nrxx_batch::Group;


double cycle_cells(const nrxx_batch *b, int inst) {
  const nrxx_problem &P = b->P[inst];
  double c = 0.0;
  for (int k = 0; k < P.levels; ++k) {
    const int steps = k == P.levels - 1 ? b->s3 : b->s1 + b->s2;
    c += 4.0 * steps * (double)(P.nx >> k) * (P.ny >> k);
  }
  return c;
}

// Unit list of one sweep on level k over the slots whose `cont` flag equals
// cont (and that have cells there): (slot << 16 | position), ordered by
// position then slot (major 0) or by slot, largest grid first, then position.
std::vector<int> make_units(const Group &G, int k, int major, int cont) {
  const auto &T = G.htab[k];
  auto use = [&](int s) { return T[s].ncell > 0 && T[s].cont == cont; };
  std::vector<int> u;
  if (major == 0) {
    int maxnx = 0;
    for (const auto &e : T) maxnx = std::max(maxnx, e.A.nx);
    for (int p = 0; p < maxnx; ++p)
      for (int s = 0; s < (int)T.size(); ++s)
        if (use(s) && p < T[s].A.nx) u.push_back(s << 16 | p);
  } else {
    std::vector<int> order;
    for (int s = 0; s < (int)T.size(); ++s)
      if (use(s)) order.push_back(s);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return T[a].ncell > T[c].ncell; });
    for (int s : order)
      for (int p = 0; p < T[s].A.nx; ++p) u.push_back(s << 16 | p);
  }
  return u;
}

int upload_states(nrxx_batch *b, double *const *states) {
  if (!states) return bfail(b, NRXX_EINVAL, "states is NULL");
  for (int i = 0; i < b->n; ++i)
    if (!states[i]) return bfail(b, NRXX_EINVAL, "state %d is NULL", i);
  bool changed = false;
  for (int i = 0; i < b->n; ++i)
    if (b->cur[i] != states[i]) changed = true;
  if (!changed) return NRXX_OK;
  for (auto &G : b->g) {
    for (size_t s = 0; s < G.inst.size(); ++s) G.htab[0][s].st = states[G.inst[s]];
    BCHK(hipMemcpyAsync(G.dtab[0], G.htab[0].data(), sizeof(BLevel) * G.htab[0].size(),
                        hipMemcpyHostToDevice, b->stream));
  }
  for (int i = 0; i < b->n; ++i) b->cur[i] = states[i];
  BCHK(hipStreamSynchronize(b->stream));
  return NRXX_OK;
}

// ---- enqueue helpers (group stream) -------------------------------------

// nsteps fast-sweeping steps on level k for the problems that continue to
// a coarser level (which = 0) or whose coarsest level k is (which = 1).
int smooth(nrxx_batch *b, Group &G, int k, int nsteps, int which) {
  const int U = G.U[which][k];
  if (U == 0) return NRXX_OK;
  const int total = 4 * nsteps;
  for (int s0 = 0; s0 < total; s0 += kMaxSweepsPerLaunch) {
    const int nsw = std::min(kMaxSweepsPerLaunch, total - s0);
    unsigned dirs = 0;
    for (int q = 0; q < nsw; ++q) dirs |= (unsigned)((s0 + q) & 3) << (2 * q);
    BCHK(launch_bfill(G.cnt[k], G.cntsize[k], 0, G.stream));
    const int grid = std::max(1, std::min(G.grid, nsw * U));
    Group::Timed *t = nullptr;
    if (b->timing) {
      if (G.tl_used == G.tl.size()) {
        G.tl.emplace_back();
        BCHK(hipEventCreate(&G.tl.back().a));
        BCHK(hipEventCreate(&G.tl.back().b));
      }
      t = &G.tl[G.tl_used++];
      G.ran = true;
      t->k = k;
      t->which = which;
      t->nsw = nsw;
      BCHK(hipEventRecord(t->a, G.stream));
    }
    if (G.kernel == 1)
      BCHK(launch_wsweep(G.M, G.order, grid, G.dtab[k], G.units[G.major][which][k], U, nsw, dirs,
                         G.cnt[k], G.cols[k], b->active, b->derr, b->dabort, b->wait_ticks, G.rows,
                         G.stream));
    else
      BCHK(launch_bsweep(G.M, G.order, G.nw, G.split, grid, G.dtab[k], G.units[G.major][which][k], U,
                         nsw, dirs, G.cnt[k], G.cols[k], b->active, b->derr, b->dabort,
                         b->wait_ticks, G.stream));
    if (t) BCHK(hipEventRecord(t->b, G.stream));
  }
  return NRXX_OK;
}

// Adds the recorded sweep launches of every group (work finished: called
// after a synchronisation) to the kernel statistics; cell updates count the
// problems active in that work (b->hact); the lists are then emptied.
int harvest_timing(nrxx_batch *b) {
  if (!b->timing) return NRXX_OK;
  for (auto &G : b->g) {
    if (!G.ran) continue;
    G.ran = false;
    for (size_t q = 0; q < G.tl_used; ++q) {
      const Group::Timed &t = G.tl[q];
      float ms = 0.f;
      BCHK(hipEventElapsedTime(&ms, t.a, t.b));
      double cells = 0.0;
      for (size_t s = 0; s < G.inst.size(); ++s) {
        const BLevel &e = G.htab[t.k][s];
        if (e.ncell > 0 && e.cont == (t.which == 0 ? 1 : 0) && b->hact[e.inst]) cells += e.ncell;
      }
      if (cells == 0.0) continue;  // every problem of the launch was masked off
      G.k_ms += ms;
      G.k_launches += 1.0;
      (t.k == 0 ? G.k_cells_fine : G.k_cells_coarse) += cells * t.nsw;
    }
    G.tl_used = 0;
  }
  return NRXX_OK;
}

// Alg. 2 on level k for every problem of the group that has level k: the
// problems whose coarsest level this is take s3 steps; the others recurse.
int vcycle(nrxx_batch *b, Group &G, int k) {
  const int nslot = (int)G.inst.size();
  int rc = smooth(b, G, k, b->s3, 1);
  if (rc) return rc;
  if (G.U[0][k] == 0) return NRXX_OK;
  rc = smooth(b, G, k, b->s1, 0);
  if (rc) return rc;
  BCHK(launch_wresidual(G.M, G.order, G.ncell[k], G.dtab[k], nslot, b->active, 0, nullptr, G.stream));
  BCHK(launch_brestrict(G.M, G.ncell[k + 1], G.dtab[k], G.dtab[k + 1], nslot, b->active, b->derr,
                        G.stream));
  BCHK(launch_wresidual(G.M, G.order, G.ncell[k + 1], G.dtab[k + 1], nslot, b->active, 1, nullptr,
                         G.stream));
  BCHK(launch_bcopy(G.M, G.ncell[k + 1], G.dtab[k + 1], nslot, b->active, G.stream));
  for (int r = 0; r < b->gamma; ++r) {
    rc = vcycle(b, G, k + 1);
    if (rc) return rc;
  }
  BCHK(launch_bcorrect(G.M, G.ncell[k + 1], G.dtab[k], G.dtab[k + 1], nslot, b->active, b->derr,
                       G.stream));
  return smooth(b, G, k, b->s2, 0);
}

int norms_enqueue(nrxx_batch *b, Group &G) {
  const int nslot = (int)G.inst.size();
  BCHK(launch_wresidual(G.M, G.order, G.ncell[0], G.dtab[0], nslot, b->active, 2, G.partial, G.stream));
  BCHK(launch_bsum(G.dtab[0], nslot, G.stride, b->active, G.partial, 0, b->norms, G.stream));
  return NRXX_OK;
}

// A whole NMG iteration of a group: V-cycle, mass fix, norm, status.
int cycle_enqueue(nrxx_batch *b, Group &G, bool status) {
  const int nslot = (int)G.inst.size();
  int rc = vcycle(b, G, 0);
  if (rc) return rc;
  BCHK(launch_bsum(G.dtab[0], nslot, G.stride, b->active, nullptr, 1, b->mass, G.stream));
  BCHK(launch_bmass_scale(G.M, G.ncell[0], G.dtab[0], nslot, b->active, b->mass, G.stream));
  rc = norms_enqueue(b, G);
  if (rc) return rc;
  if (status)
    BCHK(launch_bstatus(G.dtab[0], nslot, b->norms, b->ref, b->tol, b->active, b->cycles, b->derr,
                        G.stream));
  return NRXX_OK;
}

void drop_graph(Group &G) {
  if (G.exec) (void)hipGraphExecDestroy(G.exec);
  if (G.graph) (void)hipGraphDestroy(G.graph);
  G.exec = nullptr;
  G.graph = nullptr;
}

int capture(nrxx_batch *b, Group &G) {
  drop_graph(G);
  G.tl_used = 0;
  // HIP reports no elapsed time between events recorded by graph nodes, so
  // captured cycles carry no timing events (timing covers eager work only)
  const int timing = b->timing;
  b->timing = 0;
  BCHK(hipStreamBeginCapture(G.stream, hipStreamCaptureModeThreadLocal));
  int rc = cycle_enqueue(b, G, true);
  b->timing = timing;
  G.ran = false;  // captured, not run
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(G.stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  BCHK(e);
  G.graph = graph;
  BCHK(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
  return NRXX_OK;
}

// Run `fn` on every group's stream after the work already on b->stream, and
// make b->stream wait for all of them.
template <typename F>
int on_groups(nrxx_batch *b, F fn) {
  BCHK(hipEventRecord(b->ev0, b->stream));
  for (auto &G : b->g) {
    BCHK(hipStreamWaitEvent(G.stream, b->ev0, 0));
    int rc = fn(G);
    if (rc) return rc;
    BCHK(hipEventRecord(G.done, G.stream));
    BCHK(hipStreamWaitEvent(b->stream, G.done, 0));
  }
  return NRXX_OK;
}

// Read active flags, cycles, norms and the error word; map errors.
int fetch(nrxx_batch *b) {
  BCHK(hipMemcpyAsync(b->h_int, b->active, sizeof(int) * b->n, hipMemcpyDeviceToHost, b->stream));
  BCHK(hipMemcpyAsync(b->h_int + b->n, b->cycles, sizeof(int) * b->n, hipMemcpyDeviceToHost,
                      b->stream));
  BCHK(hipMemcpyAsync(b->h_int + 2 * b->n, b->derr, sizeof(int), hipMemcpyDeviceToHost, b->stream));
  BCHK(hipMemcpyAsync(b->h_dbl, b->norms, sizeof(double) * b->n, hipMemcpyDeviceToHost, b->stream));
  BCHK(hipStreamSynchronize(b->stream));
  const int e = b->h_int[2 * b->n];
  if (e) {
    BCHK(hipMemsetAsync(b->derr, 0, sizeof(int), b->stream));
    BCHK(hipMemsetAsync(b->dabort, 0, sizeof(int), b->stream));
    BCHK(hipStreamSynchronize(b->stream));
    if (e & 4) return bfail(b, NRXX_EHIP, "sweep kernel wait timed out");
    if (e & 3) return bfail(b, NRXX_ENONPHYS, "non-physical state (rho <= 0 or theta <= 0)");
    if (e & 8) return bfail(b, NRXX_EDIVERGED, "residual norm not finite");
  }
  return NRXX_OK;
}

int set_all_active(nrxx_batch *b, int v) {
  BCHK(launch_bfill(b->active, b->n, v, b->stream));
  return NRXX_OK;
}

// Joint step of the autotuner.  The groups' persistent sweeps run at once
// and share the CUs, so the grid each group chose alone can crowd the other
// groups' sweeps and light kernels out, and the best shares depend on each
// other (one group's smaller grid pays off only with another's).  Every
// combination of per-group grids of 1, 3/4, 1/2 and 1/4 times the group's
// own choice (at most SHARE_MAX_COMBOS combinations, else each group in
// turn) is timed as one whole NMG iteration (V-cycle, mass fix, norms) of
// all groups at once from the same states; the SHARE_FINALISTS fastest are
// timed SHARE_REPS times more, interleaved with the groups' own grids (one
// iteration varies by a few per cent), and the lowest median is kept only
// when it beats the own grids' median by at least SHARE_GAIN.  Every
// problem's finest-level state is restored afterwards (coarse levels are
// rebuilt by restriction in every cycle).
constexpr double SHARE_GAIN = 0.015;
constexpr int SHARE_MAX_COMBOS = 64;
constexpr int SHARE_FINALISTS = 4;
constexpr int SHARE_REPS = 3;

int tune_shares(nrxx_batch *b, double *const *states, hipEvent_t t0, hipEvent_t t1) {
  std::vector<double *> bak(b->n, nullptr);
  std::vector<size_t> nbytes(b->n, 0);
  bool ok = true;
  for (auto &G : b->g)
    for (size_t s = 0; s < G.inst.size() && ok; ++s) {
      const int i = G.inst[s];
      nbytes[i] = (size_t)G.htab[0][s].ncell * G.stride * sizeof(double);
      ok = hipMalloc((void **)&bak[i], nbytes[i]) == hipSuccess &&
           hipMemcpyAsync(bak[i], states[i], nbytes[i], hipMemcpyDeviceToDevice, b->stream) == hipSuccess;
    }
  auto release = [&]() {
    for (double *p : bak)
      if (p) (void)hipFree(p);
  };
  auto restore = [&]() {
    for (int i = 0; i < b->n; ++i)
      if (hipMemcpyAsync(states[i], bak[i], nbytes[i], hipMemcpyDeviceToDevice, b->stream) != hipSuccess)
        return false;
    return hipStreamSynchronize(b->stream) == hipSuccess;
  };
  // one concurrent NMG iteration from the backed-up states, in ms
  auto cycle_ms = [&](float *ms) -> int {
    if (!restore()) return bfail(b, NRXX_EHIP, "autotune: copy failed");
    BCHK(hipEventRecord(t0, b->stream));
    int rc = on_groups(b, [&](Group &G) { return cycle_enqueue(b, G, false); });
    if (rc) return rc;
    BCHK(hipEventRecord(t1, b->stream));
    BCHK(hipEventSynchronize(t1));
    BCHK(hipEventElapsedTime(ms, t0, t1));
    return fetch(b);
  };
  if (!ok) {
    release();
    return bfail(b, NRXX_EHIP, "autotune: copy or allocation failed");
  }
  const int ng = (int)b->g.size();
  const int eighths[4] = {8, 6, 4, 2};
  std::vector<int> own;
  for (auto &G : b->g) own.push_back(G.grid);
  auto set_grids = [&](const std::vector<int> &pick) {
    for (int gi = 0; gi < ng; ++gi) b->g[gi].grid = std::max(1, own[gi] * eighths[pick[gi]] / 8);
  };
  // candidate combinations (indices into eighths), the own grids first
  std::vector<std::vector<int>> combos;
  int ncombo = 1;
  for (int gi = 0; gi < ng && ncombo <= SHARE_MAX_COMBOS; ++gi) ncombo *= 4;
  if (ncombo <= SHARE_MAX_COMBOS) {
    for (int c = 0; c < ncombo; ++c) {
      std::vector<int> pick(ng);
      for (int gi = 0, x = c; gi < ng; ++gi, x /= 4) pick[gi] = x % 4;
      combos.push_back(pick);
    }
  } else {
    combos.push_back(std::vector<int>(ng, 0));
    for (int gi = 0; gi < ng; ++gi)
      for (int e = 1; e < 4; ++e) {
        std::vector<int> pick(ng, 0);
        pick[gi] = e;
        combos.push_back(pick);
      }
  }
  // stage 1: one iteration per combination; stage 2: the SHARE_FINALISTS
  // fastest and the own grids, SHARE_REPS iterations each, interleaved; the
  // lowest median wins if it beats the own grids' median by SHARE_GAIN
  float ms = 0.f;
  int rc = cycle_ms(&ms);  // loads the light kernels' code objects
  std::vector<std::pair<float, size_t>> first;
  for (size_t c = 0; c < combos.size() && !rc; ++c) {
    set_grids(combos[c]);
    rc = cycle_ms(&ms);
    first.push_back({ms, c});
  }
  size_t bi = 0;
  if (!rc) {
    std::sort(first.begin(), first.end());
    std::vector<size_t> fin{0};
    for (const auto &f : first)
      if (f.second != 0 && (int)fin.size() <= SHARE_FINALISTS) fin.push_back(f.second);
    std::vector<std::vector<float>> t(fin.size());
    for (int r = 0; r < SHARE_REPS && !rc; ++r)
      for (size_t k = 0; k < fin.size() && !rc; ++k) {
        set_grids(combos[fin[k]]);
        rc = cycle_ms(&ms);
        t[k].push_back(ms);
      }
    if (!rc) {
      auto median = [](std::vector<float> v) {
        std::sort(v.begin(), v.end());
        return v[v.size() / 2];
      };
      const float own_ms = median(t[0]);
      float best = own_ms;
      for (size_t k = 1; k < fin.size(); ++k) {
        const float m = median(t[k]);
        if (m < best && m < own_ms * (1.0 - SHARE_GAIN)) {
          best = m;
          bi = fin[k];
        }
      }
    }
  }
  set_grids(combos[rc ? 0 : bi]);
  if (!restore() && !rc) rc = bfail(b, NRXX_EHIP, "autotune: copy failed");
  release();
  for (auto &G : b->g) drop_graph(G);
  return rc;
}

}  // namespace

extern "C" {

int nrxx_batch_create(const nrxx_problem *probs, int32_t n, void *hip_stream, nrxx_batch **out) {
  if (!out) return bfail(nullptr, NRXX_EINVAL, "out is NULL");
  *out = nullptr;
  if (!probs || n < 1 || n > 32767) return bfail(nullptr, NRXX_EINVAL, "need 1..32767 problems");
  for (int i = 0; i < n; ++i) {
    std::string msg;
    if (!validate_problem(probs[i], msg))
      return bfail(nullptr, NRXX_EINVAL, "problem %d: %s", i, msg.c_str());
    if (probs[i].precision != 0) return bfail(nullptr, NRXX_EINVAL, "problem %d: batches are FP64", i);
    if (probs[i].nx > 65535) return bfail(nullptr, NRXX_EINVAL, "problem %d: nx > 65535", i);
    const nrxx_problem &a = probs[0], &c = probs[i];
    if (c.s1 != a.s1 || c.s2 != a.s2 || c.s3 != a.s3 || c.gamma != a.gamma)
      return bfail(nullptr, NRXX_EINVAL, "problem %d: s1, s2, s3 and gamma must be shared", i);
  }
  nrxx_batch *b = new nrxx_batch();
  b->n = n;
  b->P.assign(probs, probs + n);
  b->L = 0;
  for (int i = 0; i < n; ++i) b->L = std::max(b->L, (int)probs[i].levels);
  b->s1 = probs[0].s1;
  b->s2 = probs[0].s2;
  b->s3 = probs[0].s3;
  b->gamma = probs[0].gamma;
  b->stream = (hipStream_t)hip_stream;
  b->cur.assign(n, nullptr);
  std::map<std::pair<int, int>, int> gid;
  for (int i = 0; i < n; ++i) {
    auto key = std::make_pair(probs[i].M, probs[i].order);
    if (!gid.count(key)) {
      gid[key] = (int)b->g.size();
      b->g.emplace_back();
      b->g.back().M = probs[i].M;
      b->g.back().order = probs[i].order;
      b->g.back().stride = record_stride(probs[i].M);
    }
    b->g[gid[key]].inst.push_back(i);
  }
  bool ok = true;
  auto dalloc = [&](Group &G, size_t bytes) -> void * {
    void *p = nullptr;
    if (!ok || hipMalloc(&p, bytes) != hipSuccess) {
      ok = false;
      return nullptr;
    }
    G.owned.push_back(p);
    return p;
  };
  for (auto &G : b->g) {
    const int L = b->L, nslot = (int)G.inst.size();
    G.htab.assign(L, std::vector<BLevel>(nslot));
    G.dtab.assign(L, nullptr);
    G.ncell.assign(L, 0);
    G.cnt.assign(L, nullptr);
    G.cntsize.assign(L, 0);
    G.cols.assign(L, 0);
    for (int m = 0; m < 2; ++m)
      for (int c = 0; c < 2; ++c) G.units[m][c].assign(L, nullptr);
    G.U[0].assign(L, 0);
    G.U[1].assign(L, 0);
    for (int k = 0; k < L && ok; ++k) {
      int cell0 = 0, cols = 0;
      for (int s = 0; s < nslot; ++s) {
        const nrxx_problem &Pi = probs[G.inst[s]];
        BLevel &e = G.htab[k][s];
        e = BLevel{};
        e.A = make_level(Pi, std::min(k, Pi.levels - 1));
        if (k >= Pi.levels) e.A.nx = e.A.ny = 0;  // the problem has no level k
        e.cell0 = cell0;
        e.ncell = e.A.nx * e.A.ny;
        e.inst = G.inst[s];
        e.cont = k < Pi.levels - 1 ? 1 : 0;
        e.mass0 = Pi.mass0;
        cell0 += e.ncell;
        cols += e.A.nx;
      }
      G.ncell[k] = cell0;
      G.cols[k] = cols;
      G.cntsize[k] = 1 + kMaxSweepsPerLaunch * cols;
      G.cnt[k] = (int *)dalloc(G, sizeof(int) * G.cntsize[k]);
      int off = 1;
      for (int s = 0; s < nslot && ok; ++s) {
        BLevel &e = G.htab[k][s];
        const size_t nd = (size_t)e.ncell * G.stride * sizeof(double);
        if (e.ncell == 0) continue;
        if (e.cont) e.Rbar = (double *)dalloc(G, nd);
        if (k >= 1) {
          e.st = (double *)dalloc(G, nd);
          e.rhs = (double *)dalloc(G, nd);
          e.fbar = (double *)dalloc(G, nd);
          e.RH = (double *)dalloc(G, nd);
        }
        e.cnt = G.cnt[k] ? G.cnt[k] + off : nullptr;
        off += e.A.nx;
      }
      G.dtab[k] = (BLevel *)dalloc(G, sizeof(BLevel) * nslot);
      for (int m = 0; m < 2 && ok; ++m)
        for (int c = 0; c < 2 && ok; ++c) {
          std::vector<int> u = make_units(G, k, m, c == 0 ? 1 : 0);
          G.U[c][k] = (int)u.size();
          if (u.empty()) continue;
          G.units[m][c][k] = (int *)dalloc(G, sizeof(int) * u.size());
          if (ok)
            ok = hipMemcpy(G.units[m][c][k], u.data(), sizeof(int) * u.size(),
                           hipMemcpyHostToDevice) == hipSuccess;
        }
      if (ok)
        ok = hipMemcpy(G.dtab[k], G.htab[k].data(), sizeof(BLevel) * nslot, hipMemcpyHostToDevice) ==
             hipSuccess;
    }
    G.partial = (double *)dalloc(G, sizeof(double) * std::max(G.ncell[0], 1));
    if (ok) ok = hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking) == hipSuccess;
    if (ok) ok = hipEventCreateWithFlags(&G.done, hipEventDisableTiming) == hipSuccess;
    G.nw = batch_default_width(G.M);
    if (G.M > MTEAM) {  // past the cell team's largest M: one wavefront per cell
      G.kernel = 1;
      G.rows = 1;
      G.grid = wsweep_resident(G.M, G.order);
    } else {
      G.grid = bsweep_resident(G.M, G.order, G.nw, 1);
    }
    if (G.grid < 1) ok = false;
    G.major = 0;
  }
  auto balloc = [&](void **p, size_t bytes) {
    if (ok) ok = hipMalloc(p, bytes) == hipSuccess;
  };
  balloc((void **)&b->active, sizeof(int) * n);
  balloc((void **)&b->cycles, sizeof(int) * n);
  balloc((void **)&b->derr, sizeof(int));
  balloc((void **)&b->dabort, sizeof(int));
  balloc((void **)&b->norms, sizeof(double) * n);
  balloc((void **)&b->ref, sizeof(double) * n);
  balloc((void **)&b->mass, sizeof(double) * n);
  balloc((void **)&b->tol, sizeof(double));
  if (ok) ok = hipHostMalloc((void **)&b->h_int, sizeof(int) * (2 * n + 1), hipHostMallocDefault) == hipSuccess;
  if (ok) ok = hipHostMalloc((void **)&b->h_dbl, sizeof(double) * (2 * n + 1), hipHostMallocDefault) == hipSuccess;
  if (ok) ok = hipEventCreate(&b->ev0) == hipSuccess && hipEventCreate(&b->ev1) == hipSuccess;
  if (ok)
    ok = hipMemset(b->derr, 0, sizeof(int)) == hipSuccess &&
         hipMemset(b->dabort, 0, sizeof(int)) == hipSuccess &&
         hipMemset(b->cycles, 0, sizeof(int) * n) == hipSuccess &&
         hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    nrxx_batch_destroy(b);
    return bfail(nullptr, NRXX_ENOMEM, "device allocation or stream creation failed");
  }
  *out = b;
  return NRXX_OK;
}

int nrxx_batch_destroy(nrxx_batch *b) {
  if (!b) return NRXX_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (auto &G : b->g) {
    if (G.stream) (void)hipStreamSynchronize(G.stream);
    drop_graph(G);
    for (auto &t : G.tl) {
      if (t.a) (void)hipEventDestroy(t.a);
      if (t.b) (void)hipEventDestroy(t.b);
    }
    for (void *p : G.owned) (void)hipFree(p);
    if (G.done) (void)hipEventDestroy(G.done);
    if (G.stream) (void)hipStreamDestroy(G.stream);
  }
  for (void *p : {(void *)b->active, (void *)b->cycles, (void *)b->derr, (void *)b->dabort,
                  (void *)b->norms, (void *)b->ref, (void *)b->mass, (void *)b->tol})
    if (p) (void)hipFree(p);
  if (b->h_int) (void)hipHostFree(b->h_int);
  if (b->h_dbl) (void)hipHostFree(b->h_dbl);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  delete b;
  return NRXX_OK;
}

const char *nrxx_batch_last_error(const nrxx_batch *b) {
  return b ? b->err.c_str() : g_batch_create_error.c_str();
}

int nrxx_batch_groups(const nrxx_batch *b) { return b ? (int)b->g.size() : NRXX_EINVAL; }

int nrxx_batch_get_tuning(const nrxx_batch *b, int group, nrxx_batch_tuning *t) {
  if (!b || !t || group < 0 || group >= (int)b->g.size()) return NRXX_EINVAL;
  const Group &G = b->g[group];
  t->M = G.M;
  t->order = G.order;
  t->problems = (int)G.inst.size();
  t->team_width = G.nw;
  t->grid = G.grid;
  t->unit_order = G.major;
  t->split = G.split;
  t->block_ms = G.tuned_ms;
  t->kernel = G.kernel;
  t->rows_per_sync = G.rows;
  return NRXX_OK;
}

int nrxx_batch_set_tuning(nrxx_batch *b, int group, const nrxx_batch_tuning *t) {
  if (!b) return NRXX_EINVAL;
  if (!t || group < 0 || group >= (int)b->g.size()) return bfail(b, NRXX_EINVAL, "bad group");
  Group &G = b->g[group];
  if (t->kernel != 0 && t->kernel != 1) return bfail(b, NRXX_EINVAL, "kernel %d", t->kernel);
  if (t->kernel == 0 && G.M > MTEAM)
    return bfail(b, NRXX_EINVAL, "M = %d > %d needs the wavefront-per-cell kernel", G.M, MTEAM);
  if (t->kernel == 1 && (t->rows_per_sync < 1 || t->rows_per_sync > 65535))
    return bfail(b, NRXX_EINVAL, "rows_per_sync %d", t->rows_per_sync);
  if (t->kernel == 0 && !batch_width_ok(G.M, t->team_width))
    return bfail(b, NRXX_EINVAL, "team width %d", t->team_width);
  if (t->grid < 1 || (t->unit_order != 0 && t->unit_order != 1) || (t->split != 0 && t->split != 1))
    return bfail(b, NRXX_EINVAL, "bad grid, unit order or split");
  if (G.kernel != t->kernel || G.nw != t->team_width || G.grid != t->grid ||
      G.major != t->unit_order || G.split != t->split || (t->kernel == 1 && G.rows != t->rows_per_sync))
    drop_graph(G);
  G.kernel = t->kernel;
  if (t->kernel == 1) G.rows = t->rows_per_sync;
  if (t->kernel == 0) G.nw = t->team_width;
  G.grid = t->grid;
  G.major = t->unit_order;
  G.split = t->split;
  return NRXX_OK;
}

int nrxx_batch_init_maxwellian(nrxx_batch *b, double *const *states, double rho, double u1,
                               double u2, double theta) {
  if (!b) return NRXX_EINVAL;
  if (!(rho > 0) || !(theta > 0)) return bfail(b, NRXX_EINVAL, "rho and theta must be positive");
  int rc = upload_states(b, states);
  if (rc) return rc;
  for (int i = 0; i < b->n; ++i) {
    LevelArgs A = make_level(b->P[i], 0);
    BCHK(launch_init_maxwellian(b->P[i].M, A, states[i], rho, u1, u2, theta, b->stream));
  }
  BCHK(hipStreamSynchronize(b->stream));
  return NRXX_OK;
}

int nrxx_batch_residual_norms(nrxx_batch *b, double *const *states, double *norms_out) {
  if (!b) return NRXX_EINVAL;
  if (!norms_out) return bfail(b, NRXX_EINVAL, "norms_out is NULL");
  int rc = upload_states(b, states);
  if (rc) return rc;
  rc = set_all_active(b, 1);
  if (rc) return rc;
  rc = on_groups(b, [&](Group &G) { return norms_enqueue(b, G); });
  if (rc) return rc;
  rc = fetch(b);
  if (rc) return rc;
  memcpy(norms_out, b->h_dbl, sizeof(double) * b->n);
  return NRXX_OK;
}

int nrxx_batch_sweep(nrxx_batch *b, double *const *states, int nsteps) {
  if (!b) return NRXX_EINVAL;
  if (nsteps < 0) return bfail(b, NRXX_EINVAL, "nsteps < 0");
  int rc = upload_states(b, states);
  if (rc) return rc;
  rc = set_all_active(b, 1);
  if (rc) return rc;
  b->hact.assign(b->n, 1);
  rc = on_groups(b, [&](Group &G) {
    int r = smooth(b, G, 0, nsteps, 0);
    return r ? r : smooth(b, G, 0, nsteps, 1);
  });
  if (rc) return rc;
  rc = fetch(b);
  return rc ? rc : harvest_timing(b);
}

int nrxx_batch_vcycle(nrxx_batch *b, double *const *states, double *norms_out) {
  if (!b) return NRXX_EINVAL;
  int rc = upload_states(b, states);
  if (rc) return rc;
  rc = set_all_active(b, 1);
  if (rc) return rc;
  b->hact.assign(b->n, 1);
  rc = on_groups(b, [&](Group &G) { return cycle_enqueue(b, G, false); });
  if (rc) return rc;
  rc = fetch(b);
  if (rc) return rc;
  rc = harvest_timing(b);
  if (rc) return rc;
  if (norms_out) memcpy(norms_out, b->h_dbl, sizeof(double) * b->n);
  return NRXX_OK;
}

int nrxx_batch_solve(nrxx_batch *b, double *const *states, double tol, int32_t max_cycles,
                     int32_t use_graph, int32_t *cycles_out, double *norms_out, double *ref_out) {
  if (!b) return NRXX_EINVAL;
  if (max_cycles < 0 || !(tol >= 0)) return bfail(b, NRXX_EINVAL, "bad tol or max_cycles");
  int rc = upload_states(b, states);
  if (rc) return rc;
  // initial norms: every problem active, reference = its own initial norm
  rc = set_all_active(b, 1);
  if (rc) return rc;
  rc = on_groups(b, [&](Group &G) { return norms_enqueue(b, G); });
  if (rc) return rc;
  BCHK(hipMemcpyAsync(b->ref, b->norms, sizeof(double) * b->n, hipMemcpyDeviceToDevice, b->stream));
  b->h_dbl[2 * b->n] = tol;
  BCHK(hipMemcpyAsync(b->tol, b->h_dbl + 2 * b->n, sizeof(double), hipMemcpyHostToDevice, b->stream));
  BCHK(hipMemsetAsync(b->cycles, 0, sizeof(int) * b->n, b->stream));
  rc = fetch(b);
  if (rc) return rc;
  std::vector<double> ref(b->h_dbl, b->h_dbl + b->n);
  for (int i = 0; i < b->n; ++i) b->h_int[i] = ref[i] > tol * ref[i] ? 1 : 0;
  BCHK(hipMemcpyAsync(b->active, b->h_int, sizeof(int) * b->n, hipMemcpyHostToDevice, b->stream));
  BCHK(hipStreamSynchronize(b->stream));
  std::vector<int> act(b->h_int, b->h_int + b->n);
  if (use_graph)
    for (auto &G : b->g)
      if (!G.exec) {
        rc = capture(b, G);
        if (rc) return rc;
      }
  for (int c = 0; c < max_cycles; ++c) {
    int nact = 0;
    for (int i = 0; i < b->n; ++i) nact += act[i];
    if (!nact) break;
    for (int i = 0; i < b->n; ++i)
      if (act[i]) b->cells += cycle_cells(b, i);
    b->hact = act;
    BCHK(hipEventRecord(b->ev1, b->stream));
    rc = on_groups(b, [&](Group &G) {
      bool any = false;
      for (int i : G.inst) any = any || act[i];
      if (!any) return (int)NRXX_OK;
      if (use_graph) return bhip(b, hipGraphLaunch(G.exec, G.stream), "hipGraphLaunch");
      return cycle_enqueue(b, G, true);
    });
    if (rc) return rc;
    BCHK(hipEventRecord(b->ev0, b->stream));
    rc = fetch(b);
    if (rc) return rc;
    rc = harvest_timing(b);
    if (rc) return rc;
    float ms = 0.f;
    BCHK(hipEventElapsedTime(&ms, b->ev1, b->ev0));
    b->ms += ms;
    act.assign(b->h_int, b->h_int + b->n);
  }
  bool all = true;
  for (int i = 0; i < b->n; ++i) {
    if (act[i]) all = false;
    if (cycles_out) cycles_out[i] = b->h_int[b->n + i];
    if (norms_out) norms_out[i] = b->h_dbl[i];
    if (ref_out) ref_out[i] = ref[i];
  }
  return all ? NRXX_OK : NRXX_EMAXIT;
}

int nrxx_batch_autotune(nrxx_batch *b, double *const *states) {
  if (!b) return NRXX_EINVAL;
  int rc = upload_states(b, states);
  if (rc) return rc;
  rc = set_all_active(b, 1);
  if (rc) return rc;
  hipEvent_t t0, t1;
  BCHK(hipEventCreate(&t0));
  BCHK(hipEventCreate(&t1));
  // the candidates' sweeps are not part of the kernel statistics
  struct Untimed {
    nrxx_batch *b;
    int was;
    ~Untimed() { b->timing = was; }
  } untimed{b, b->timing};
  b->timing = 0;
  for (auto &G : b->g) {
    // back up the group's finest-level states
    std::vector<double *> bak(G.inst.size(), nullptr);
    bool ok = true;
    for (size_t s = 0; s < G.inst.size() && ok; ++s) {
      const size_t nd = (size_t)G.htab[0][s].ncell * G.stride * sizeof(double);
      ok = hipMalloc((void **)&bak[s], nd) == hipSuccess &&
           hipMemcpyAsync(bak[s], states[G.inst[s]], nd, hipMemcpyDeviceToDevice, b->stream) == hipSuccess;
    }
    auto restore = [&]() {
      for (size_t s = 0; s < G.inst.size(); ++s) {
        const size_t nd = (size_t)G.htab[0][s].ncell * G.stride * sizeof(double);
        if (hipMemcpyAsync(states[G.inst[s]], bak[s], nd, hipMemcpyDeviceToDevice, b->stream) != hipSuccess)
          return false;
      }
      return hipStreamSynchronize(b->stream) == hipSuccess;
    };
    // candidates: (kernel, team width, split, grid, unit order)
    struct Cand {
      int kernel, nw, split, grid, major, rows;
    };
    std::vector<Cand> cands;
    const int widths[4] = {8, 4, 2, 1};
    for (int sp = 1; sp >= 0; --sp)
      for (int wi = 0; wi < 4; ++wi) {
        if (!batch_width_ok(G.M, widths[wi])) continue;
        const int res = bsweep_resident(G.M, G.order, widths[wi], sp);
        if (res < 1) continue;
        for (int gr : {res, std::max(1, res / 2)})
          for (int m = 0; m < 2; ++m) cands.push_back({0, widths[wi], sp, gr, m, G.rows});
      }
    {
      const int res = wsweep_resident(G.M, G.order);
      if (res >= 1)
        for (int gr : {res, std::max(1, res / 2)})
          for (int m = 0; m < 2; ++m) cands.push_back({1, G.nw, G.split, gr, m, 1});
    }
    double best = 1e300;
    Cand keep{G.kernel, G.nw, G.split, G.grid, G.major, G.rows};
    for (const Cand &cd : cands) {
      if (!ok) break;
      G.kernel = cd.kernel;
      G.nw = cd.nw;
      G.split = cd.split;
      G.grid = cd.grid;
      G.major = cd.major;
      G.rows = cd.rows;
      float ms = 0.f;
      for (int rep = 0; rep < 2 && ok; ++rep) {  // the first run loads the code object
        ok = restore();
        if (!ok) break;
        BCHK(hipEventRecord(t0, G.stream));
        rc = smooth(b, G, 0, std::max(1, b->s1), 0);
        if (rc) return rc;
        rc = smooth(b, G, 0, std::max(1, b->s1), 1);
        if (rc) return rc;
        BCHK(hipEventRecord(t1, G.stream));
        BCHK(hipEventSynchronize(t1));
        BCHK(hipEventElapsedTime(&ms, t0, t1));
      }
      rc = fetch(b);
      if (rc) return rc;
      if (ms < best) {
        best = ms;
        keep = cd;
      }
    }
    if (ok) ok = restore();
    for (double *p : bak)
      if (p) (void)hipFree(p);
    if (!ok) return bfail(b, NRXX_EHIP, "autotune: copy or allocation failed");
    G.kernel = keep.kernel;
    G.nw = keep.nw;
    G.split = keep.split;
    G.grid = keep.grid;
    G.major = keep.major;
    G.rows = keep.rows;
    G.tuned_ms = best;
    drop_graph(G);
  }
  if (b->g.size() >= 2) {
    rc = tune_shares(b, states, t0, t1);
    if (rc) return rc;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  return NRXX_OK;
}

int nrxx_batch_set_wait_limit(nrxx_batch *b, double seconds) {
  if (!b) return NRXX_EINVAL;
  if (!(seconds >= 1e-8) || seconds > 3600.0) return bfail(b, NRXX_EINVAL, "wait limit %g s", seconds);
  b->wait_ticks = (unsigned long long)(seconds * 1e8);
  for (auto &G : b->g) drop_graph(G);  // captured cycles hold the old limit
  return NRXX_OK;
}

int nrxx_batch_set_timing(nrxx_batch *b, int32_t on) {
  if (!b) return NRXX_EINVAL;
  if (on != 0 && on != 1) return bfail(b, NRXX_EINVAL, "timing must be 0 or 1");
  if (b->timing != on)
    for (auto &G : b->g) {
      drop_graph(G);  // re-captured with (or without) the event pairs
      G.tl_used = 0;
    }
  b->timing = on;
  return NRXX_OK;
}

int nrxx_batch_kernel_stats(nrxx_batch *b, int32_t group, double *ms_out, double *launches_out,
                            double *cells_fine_out, double *cells_coarse_out, int32_t reset) {
  if (!b) return NRXX_EINVAL;
  if (group < 0 || group >= (int)b->g.size()) return bfail(b, NRXX_EINVAL, "bad group");
  Group &G = b->g[group];
  if (ms_out) *ms_out = G.k_ms;
  if (launches_out) *launches_out = G.k_launches;
  if (cells_fine_out) *cells_fine_out = G.k_cells_fine;
  if (cells_coarse_out) *cells_coarse_out = G.k_cells_coarse;
  if (reset) G.k_ms = G.k_launches = G.k_cells_fine = G.k_cells_coarse = 0.0;
  return NRXX_OK;
}

int nrxx_batch_stats(nrxx_batch *b, double *ms_out, double *cells_out, int reset) {
  if (!b) return NRXX_EINVAL;
  if (ms_out) *ms_out = b->ms;
  if (cells_out) *cells_out = b->cells;
  if (reset) b->ms = b->cells = 0.0;
  return NRXX_OK;
}

}  // extern "C"
