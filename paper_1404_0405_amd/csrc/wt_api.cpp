// C ABI of libwt (declared in include/wt.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/wt.h"
#include "wt_grid.hpp"
#include "wt_internal.hpp"
#include "wt_alloc.hpp"
#include "wt_batch.hpp"
#include "wt_compact.hpp"
#include "wt_lattice_dev.hpp"
#include "wt_learn.hpp"
#include "wt_ml.hpp"
#include "wt_pair.hpp"

using namespace wt;

static thread_local std::string g_err;

static int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}

namespace wt {
int api_fail(int code, const std::string& m) { return fail(code, m); }
}  // namespace wt

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)

struct LevelState {
  Level geo;         // host geometry (cell areas replaced by effective areas below jmax)
  DevTables tab;     // device tables
  DevWork work;      // device buffers
  uint8_t *na = nullptr, *ea = nullptr;  // active nodes / edges
  uint8_t *nn = nullptr, *ne = nullptr;  // masks under construction (adapt)
  uint8_t *sn = nullptr, *se = nullptr;  // significant points (adapt)
  DevLattice lat;                        // fused lattice form (uniform grids, n >= 64)
  // learned adjacent zone
  float *rn = nullptr, *re = nullptr;    // detail size of every point (details of the pair below)
  int64_t npatch = 0;                    // patches with a learned gate of the children rule
  float *stats = nullptr, *X = nullptr, *Pr = nullptr;
  uint8_t *allow = nullptr, *dropped = nullptr, *viol = nullptr;
  double *snap_dh = nullptr, *snap_u = nullptr;   // state and masks before a gated adapt
  uint8_t *snap_na = nullptr, *snap_ea = nullptr;
  // work lists of the adaptive stage: support rings of the active points (3 rings: where the
  // stage intermediates are computed; 5 rings: where inactive points are prolonged)
  uint8_t *s3n = nullptr, *s3e = nullptr, *s5n = nullptr, *s5e = nullptr, *rn_ = nullptr, *re_ = nullptr;
  uint8_t *pred_t = nullptr, *pred_e = nullptr, *pred_a = nullptr;   // triangles, support / active elements
  uint8_t* pf = nullptr;        // 8 x 8 patch flags of the ring dilation
  int32_t* plist = nullptr;     // patches the ring dilation visits (count after the list)
  WorkList l_tri, l_elem, l_edge, l_node, l_tend;
  // finest level, masked lattice form: tiles of each lozenge holding support points
  uint8_t* tflag = nullptr;
  int32_t* tcount = nullptr;
  bool tflag_ok = false;   // the flags match the current work lists
};

struct PairState {
  WorkList l_cn, l_ce, l_ct;   // coarse nodes / edges / triangles with a fine point in the 5-ring support
  double* ph_det = nullptr;    // partial height transform: odd-node details of every coarse edge
  uint8_t* ph_act = nullptr;   // and their stencil activity
  uint8_t* pred = nullptr;     // their predicates (Nc + Ec + Tc bytes)
  PairTables host;
  DevPair dev{};
  double *d_h = nullptr, *d_p = nullptr, *d_i = nullptr, *d_k = nullptr;  // details
  double *r_h = nullptr, *r_p = nullptr, *r_i = nullptr;  // details of a reconstruction (read-out)
};

struct wt_mlp;
namespace wt {
void mlp_predict(wt_mlp* m, const float* X, int64_t n, float* P, hipStream_t s);
}

struct wt_grid {
  int jmin = 0, jmax = 0, patch = 8;
  // learned adjacent zone
  wt_mlp* predictor = nullptr;
  double pred_thr = 0.5;
  std::vector<std::pair<int, int64_t>> force_drop;   // (level, patch) withheld at the next gated adapt
  bool gated = false;         // the last adapt used the learned gate; the next step is judged
  double last_eps = 0, last_eh = 0, last_eu = 0;
  int64_t redo = 0;
  // Version of the state and masks (bumped by everything that changes them) and the version the
  // last passing threshold test saw: the adapt that follows such a test on the same state with
  // the same eps takes its details, thresholds and significant points instead of recomputing them.
  uint64_t state_ver = 0, judge_ver = ~uint64_t(0);
  bool use_lists = true;      // adaptive stage over work lists (false: whole levels)
  // The finest level runs whole through the masked lattice kernel when its listed support holds
  // at least this fraction of its elements (above 1: never; built by wt_set_dense_levels).
  double dense_min = 2.0;
  int dense2_min_tiles = -1;   // tile positions the level below the finest needs to run dense (-1: cus)
  int cus = 0;                 // compute units of the grid's device
  bool splan_dense = false;   // the merged-phase plan was built with the finest level dense
  bool splan_dense2 = false;  // ... and with the level below it running the intermediates-only form
  bool lists_ok = false;      // the lists match the current masks
  bool details_partial = false;   // the stored details cover only the work-list support
  uint64_t epoch = 0;         // bumped whenever the launches of a step change (see touch_epoch)
  std::vector<int64_t> step_sig;   // what the launches of a step depend on, as of the last bump
  // the listed step as one launch per phase (all levels of a phase together), from a plan built
  // for the step signature and dt it was made for
  bool step_phases = true;
  BatchPlan splan;
  std::vector<PhaseArgs> sphase;
  std::vector<int64_t> splan_sig;
  double splan_dt = 0.0;
  CompactScratch csc;
  CompactBatch cb;
  // batched read-backs of per-level maxima (pinned)
  static constexpr int kSlots = 256;
  static constexpr int kThr = 254;   // slots of the adapt's thresholds (eh, eu)
  double* host_val = nullptr;
  wt_params prm{};
  std::vector<std::unique_ptr<LevelState>> lev;    // index j - jmin
  std::vector<std::unique_ptr<PairState>> pairs;   // pair (j, j+1) at index j - jmin
  hipStream_t own = nullptr, stream = nullptr;
  AllocHook hook;             // device allocator of the grid's buffers (none: hipMalloc)
  bool have_state = false;
  Timer timer;
  LevelState& L(int j) { return *lev[j - jmin]; }
  PairState& P(int j) { return *pairs[j - jmin]; }
  bool multi() const { return jmax > jmin; }
};

// The grid's device buffers come from its allocator while one of its calls runs.
struct GridScope : AllocScope {
  explicit GridScope(wt_grid* g) : AllocScope(g ? &g->hook : nullptr, g, g ? g->stream : nullptr) {}
};

static void alloc_work(LevelState& ls) {
  const int64_t N = ls.tab.N, E = ls.tab.E, T = ls.tab.T;
  DevWork& w = ls.work;
  auto A = [](double** p, int64_t n) { HIPCHK(wt::dmalloc(p, n * sizeof(double))); HIPCHK(hipMemset(*p, 0, n * sizeof(double))); };
  A(&w.dh, N); A(&w.u, E);
  A(&w.dh_acc, N); A(&w.u_acc, E);
  A(&w.dh_s[0], N); A(&w.u_s[0], E);
  A(&w.dh_s[1], N); A(&w.u_s[1], E);
  A(&w.ddh, N); A(&w.du, E);
  double* p;
  A(&p, T); w.qv = p;
  A(&p, N); w.B = p;
  A(&p, E); w.F = p;
  A(&p, E); w.qe = p;
  A(&p, E); w.Q = p;
  A(&w.c, N);
  A(&w.red, MAX_JOBS * MAX_BLOCKS + MAX_JOBS + 8);   // batched maxima: partials, results, thresholds
  auto M = [](uint8_t** q, int64_t n) { HIPCHK(wt::dmalloc(q, n)); HIPCHK(hipMemset(*q, 0, n)); };
  M(&ls.na, N); M(&ls.ea, E); M(&ls.nn, N); M(&ls.ne, E); M(&ls.sn, N); M(&ls.se, E);
}

static void free_work(LevelState& ls) {
  DevWork& w = ls.work;
  void* ps[] = {w.dh, w.u, w.dh_acc, w.u_acc, w.dh_s[0], w.u_s[0], w.dh_s[1], w.u_s[1],
                w.ddh, w.du, w.qv, w.B, w.F, w.qe, w.Q, w.c, w.red, w.G,
                ls.na, ls.ea, ls.nn, ls.ne, ls.sn, ls.se,
                ls.rn, ls.re, ls.stats, ls.X, ls.Pr, ls.allow, ls.dropped, ls.viol,
                ls.snap_dh, ls.snap_u, ls.snap_na, ls.snap_ea, ls.s3n, ls.s3e, ls.s5n, ls.s5e, ls.rn_, ls.re_, ls.pred_t,
                ls.pred_e, ls.pred_a, ls.pf, ls.plist, ls.tflag, ls.tcount};
  for (void* p : ps)
    if (p) (void)wt::dfree(p);
  w = DevWork{};
  free_list(ls.l_tri);
  free_list(ls.l_elem);
  free_list(ls.l_edge);
  free_list(ls.l_node);
  free_list(ls.l_tend);
}

static PhysParams phys(const wt_grid* g) {
  return PhysParams{g->prm.gravity, g->prm.mean_depth, g->prm.viscosity, g->prm.equations == WT_ADVECTION ? 1 : 0};
}
static bool fp32_of(const wt_grid* g) { return g->prm.precision == WT_FP32_TENDENCY; }

// ---------------------------------------------------------------- Runge-Kutta stages
// Stage s of a step: input x, and the epilogue o1/o2 = a*y + b*acc + c*x + d*k (see
// StageOut).  Classical RK4 in three registers (y, acc, two stage buffers); the SSP scheme in
// Shu-Osher form.
struct StageSpec {
  const double *xdh, *xu;
  StagePtrs pdh, pu;
  StageOut c;
};

static StageSpec rk_stage(int rk, int s, DevWork& w, double dt) {
  StageSpec r{};
  StageOut c{};
  const double *xdh, *xu;
  double *o1dh = nullptr, *o1u = nullptr, *o2dh = nullptr, *o2u = nullptr;
  if (rk == WT_RK4) {
    const double bk[4] = {dt / 6, dt / 3, dt / 3, dt / 6};
    const double ck[4] = {dt / 2, dt / 2, dt, 0};
    const double* X[4] = {w.dh, w.dh_s[0], w.dh_s[1], w.dh_s[0]};
    const double* XU[4] = {w.u, w.u_s[0], w.u_s[1], w.u_s[0]};
    double* O2[4] = {w.dh_s[0], w.dh_s[1], w.dh_s[0], nullptr};
    double* O2U[4] = {w.u_s[0], w.u_s[1], w.u_s[0], nullptr};
    xdh = X[s]; xu = XU[s];
    c.d1 = bk[s];
    if (s == 0) c.a1 = 1.0; else c.b1 = 1.0;
    o1dh = s == 3 ? w.dh : w.dh_acc;
    o1u = s == 3 ? w.u : w.u_acc;
    if (s < 3) { c.a2 = 1.0; c.d2 = ck[s]; o2dh = O2[s]; o2u = O2U[s]; }
  } else {
    const double* X[4] = {w.dh, w.dh_s[0], w.dh_s[1], w.dh_s[0]};
    const double* XU[4] = {w.u, w.u_s[0], w.u_s[1], w.u_s[0]};
    double* O1[4] = {w.dh_s[0], w.dh_s[1], w.dh_s[0], w.dh};
    double* O1U[4] = {w.u_s[0], w.u_s[1], w.u_s[0], w.u};
    xdh = X[s]; xu = XU[s]; o1dh = O1[s]; o1u = O1U[s];
    if (s == 0) { c.a1 = 1.0; c.d1 = dt / 2; }
    else if (s == 1) { c.c1 = 1.0; c.d1 = dt / 2; }
    else if (s == 2) { c.a1 = 2.0 / 3.0; c.c1 = 1.0 / 3.0; c.d1 = dt / 6; }
    else { c.c1 = 1.0; c.d1 = dt / 2; }
  }
  r.xdh = xdh; r.xu = xu; r.c = c;
  r.pdh = StagePtrs{w.dh, w.dh_acc, xdh, o1dh, o2dh};
  r.pu = StagePtrs{w.u, w.u_acc, xu, o1u, o2u};
  return r;
}

static void uniform_step(wt_grid* g, LevelState& ls, double dt) {
  ++g->state_ver;
  const bool fp32 = g->prm.precision == WT_FP32_TENDENCY;
  for (int s = 0; s < 4; ++s) {
    StageSpec sp = rk_stage(g->prm.rk, s, ls.work, dt);
    launch_stage(ls.tab, ls.work, phys(g), fp32, sp.pdh, sp.pu, sp.c, g->stream, &g->timer, &ls.lat);
  }
}

// ---------------------------------------------------------------- multilevel operations
// Fill inactive points of every level above jmin from the level below (top-down).
// launches over a work list cover its padded bound (padding entries are -1)
static Span span(const WorkList& L) { return Span{L.idx, L.bound}; }

// listed: only the work-list support of the current masks (the rest keeps stale values)
static void prolong_all(wt_grid* g, const std::vector<double*>& dh, const std::vector<double*>& u,
                        bool listed = false) {
  const bool L = listed && g->lists_ok;
  for (int j = g->jmin; j < g->jmax; ++j) {
    LevelState& F = g->L(j + 1);
    PairState& P = g->P(j);
    ml_prolong(P.dev, g->L(j).tab, F.na, F.ea, dh[j - g->jmin], u[j - g->jmin], dh[j + 1 - g->jmin],
               u[j + 1 - g->jmin], fp32_of(g), g->stream, L ? span(P.l_cn) : Span{}, L ? span(P.l_ce) : Span{},
               L ? span(P.l_ct) : Span{});
  }
}

static void details_all(wt_grid* g, const std::vector<double*>& dh, const std::vector<double*>& u,
                        bool listed = false) {
  const bool L = listed && g->lists_ok;
  std::vector<MaskJob> jobs;   // pairs are independent: one launch
  for (int j = g->jmin; j < g->jmax; ++j) {
    PairState& P = g->P(j);
    ml_details_jobs(jobs, P.dev, g->L(j).tab, dh[j + 1 - g->jmin], u[j + 1 - g->jmin], u[j - g->jmin], P.d_h,
                    P.d_p, P.d_i, fp32_of(g), L ? span(P.l_ce) : Span{}, L ? span(P.l_ct) : Span{});
  }
  ml_mask_ops(jobs.data(), int(jobs.size()), g->stream);
  g->details_partial = L;
}

// Inverse transform top-down with the details kept where (old & new) activity holds.

// swapped: the new masks are already in na/ea and the old ones in nn/ne (adapt); listed: only
// the fine points of the current work-list support are rewritten (the others are inactive, and
// every stage prolongs the inactive points of the support before reading them)
static void inverse_all(wt_grid* g, const std::vector<double*>& dh, const std::vector<double*>& u,
                        bool use_new, bool swapped = false, bool listed = false) {
  auto masks = [&](int j, const uint8_t*& na_old, const uint8_t*& na_new, const uint8_t*& ea_old,
                   const uint8_t*& ea_new) {
    LevelState& F = g->L(j + 1);
    na_old = na_new = F.na;
    ea_old = ea_new = F.ea;
    if (use_new && !swapped) { na_new = F.nn; ea_new = F.ne; }
    if (use_new && swapped) { na_old = F.nn; ea_old = F.ne; }
  };
  std::vector<KeepJob> keep;
  for (int j = g->jmin; j < g->jmax; ++j) {
    PairState& P = g->P(j);
    const uint8_t *na_old, *na_new, *ea_old, *ea_new;
    masks(j, na_old, na_new, ea_old, ea_new);
    keep.push_back(KeepJob{P.dev.mid, P.dev.Ec, na_old, na_new, P.d_h, P.d_k});
  }
  ml_inverse_keep_batch(keep.data(), int(keep.size()), g->stream);
  const bool L = listed && g->lists_ok;
  for (int j = g->jmin; j < g->jmax; ++j) {
    PairState& P = g->P(j);
    const uint8_t *na_old, *na_new, *ea_old, *ea_new;
    masks(j, na_old, na_new, ea_old, ea_new);
    ml_inverse_pair(P.dev, g->L(j).tab, ea_old, ea_new, P.d_p, P.d_i, P.d_k, dh[j - g->jmin], u[j - g->jmin],
                    dh[j + 1 - g->jmin], u[j + 1 - g->jmin], fp32_of(g), g->stream, L ? span(P.l_cn) : Span{},
                    L ? span(P.l_ce) : Span{}, L ? span(P.l_ct) : Span{});
  }
}

static std::vector<double*> state_dh(wt_grid* g) {
  std::vector<double*> v;
  for (auto& l : g->lev) v.push_back(l->work.dh);
  return v;
}
static std::vector<double*> state_u(wt_grid* g) {
  std::vector<double*> v;
  for (auto& l : g->lev) v.push_back(l->work.u);
  return v;
}

// Reconstruction of every level into the first stage buffers (the state is not changed, nor
// are the details kept from the last forward transform / adapt: the reconstruction computes its
// own details in separate buffers).
static void reconstruct(wt_grid* g, std::vector<double*>& rdh, std::vector<double*>& ru) {
  rdh.clear();
  ru.clear();
  for (auto& l : g->lev) {
    HIPCHK(hipMemcpyAsync(l->work.dh_s[0], l->work.dh, l->tab.N * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
    HIPCHK(hipMemcpyAsync(l->work.u_s[0], l->work.u, l->tab.E * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
    rdh.push_back(l->work.dh_s[0]);
    ru.push_back(l->work.u_s[0]);
  }
  auto swap_details = [&]() {
    for (auto& ps : g->pairs) {
      std::swap(ps->d_h, ps->r_h);
      std::swap(ps->d_p, ps->r_p);
      std::swap(ps->d_i, ps->r_i);
    }
  };
  const bool partial = g->details_partial;   // describes the stored (swapped-out) details
  swap_details();
  try {
    prolong_all(g, rdh, ru);
    details_all(g, rdh, ru);
    inverse_all(g, rdh, ru, false);
  } catch (...) {
    swap_details();
    g->details_partial = partial;
    throw;
  }
  swap_details();
  g->details_partial = partial;
}

// ---------------------------------------------------------------- work lists

// Whether the finest level of a multilevel grid runs through the masked lattice kernel this step:
// the level has a lattice form, the stage is the inviscid shallow-water one, and the level is
// dense (its 3-ring support holds at least dense_min of its elements; always when the stage runs
// over whole levels).  Deterministic in the masks, so every path of a step takes the same choice.
static bool dense_finest(const wt_grid* g) {
  if (!g->multi() || !(g->dense_min <= 1.0)) return false;
  const LevelState& l = *g->lev.back();
  if (!l.lat.ok || g->prm.viscosity != 0.0 || g->prm.equations == WT_ADVECTION) return false;
  if (!(g->use_lists && g->lists_ok)) return true;
  return double(l.l_elem.n) >= g->dense_min * double(l.tab.N);
}

// Whether the level below the finest computes its intermediates (F, Q, B) through the masked
// lattice kernel's intermediates-only form: the finest level is dense, the level has a lattice
// form and is as dense by the same measure.  Its tendencies stay listed: they follow the
// restriction from the finest level, which replaces F, Q and B at its non-leaf points.
static bool dense_second(const wt_grid* g) {
  if (!dense_finest(g)) return false;
  const LevelState& l = *g->lev[g->lev.size() - 2];
  if (!l.lat.ok) return false;
  // one workgroup per tile position: with fewer positions than compute units the launch leaves
  // part of the device idle and the listed kernels are faster (the spun-up jet's level 8: 124
  // positions, its step 1.61 -> 1.69 ms)
  if (l.lat.args.ntile < (g->dense2_min_tiles >= 0 ? g->dense2_min_tiles : g->cus)) return false;
  if (!(g->use_lists && g->lists_ok)) return true;
  return double(l.l_elem.n) >= g->dense_min * double(l.tab.N);
}

// The launches of a multilevel step depend on whether the work lists are used, on the lists'
// addresses and padded bounds, and on the mask addresses; a captured step stays valid while
// none of these change.
static void touch_epoch(wt_grid* g) {
  std::vector<int64_t> sig;
  sig.push_back(g->use_lists && g->lists_ok);
  // the physical constants and scheme are kernel arguments too
  int64_t bits[2];
  std::memcpy(&bits[0], &g->prm.gravity, 8);
  std::memcpy(&bits[1], &g->prm.mean_depth, 8);
  sig.push_back(bits[0]);
  sig.push_back(bits[1]);
  sig.push_back(g->prm.rk);
  sig.push_back(g->prm.precision);
  int64_t nub = 0;
  std::memcpy(&nub, &g->prm.viscosity, 8);
  sig.push_back(nub);
  sig.push_back(g->prm.equations);
  sig.push_back(dense_finest(g));
  sig.push_back(g->lev.back()->tflag_ok);
  sig.push_back(g->multi() && dense_second(g));
  if (g->multi()) sig.push_back(g->lev[g->lev.size() - 2]->tflag_ok);
  auto add = [&](const WorkList& L) {
    sig.push_back(reinterpret_cast<int64_t>(L.idx));
    sig.push_back(L.bound);
  };
  for (auto& l : g->lev) {
    sig.push_back(reinterpret_cast<int64_t>(l->na));
    sig.push_back(reinterpret_cast<int64_t>(l->ea));
    add(l->l_tri);
    add(l->l_elem);
    add(l->l_edge);
    add(l->l_node);
    add(l->l_tend);
  }
  for (auto& p : g->pairs) {
    add(p->l_cn);
    add(p->l_ce);
    add(p->l_ct);
  }
  if (sig != g->step_sig) {
    g->step_sig.swap(sig);
    ++g->epoch;
  }
}

// Support rings of the active points of every level and the index lists of the adaptive stage
// (ballot / prefix-scan compaction).  Called whenever the masks change.
// Tile flags of the masked lattice forms of the two finest levels from the 5-ring support of the
// work lists just built (without lists the masked form runs every tile).
static void update_tile_flags(wt_grid* g) {
  for (auto& lp : g->lev) lp->tflag_ok = false;
  if (!g->multi() || !(g->dense_min <= 1.0) || !(g->use_lists && g->lists_ok)) return;
  for (size_t q = g->lev.size() - 2; q < g->lev.size(); ++q) {
    LevelState& l = *g->lev[q];
    if (!l.lat.ok) continue;
    if (!l.tflag) {
      HIPCHK(wt::dmalloc(&l.tflag, size_t(l.lat.args.ntile) * 10));
      HIPCHK(wt::dmalloc(&l.tcount, sizeof(int32_t)));
    }
    lattice_tile_flags(l.lat, l.s5n, l.s5e, l.tflag, l.tcount, g->stream);
    l.tflag_ok = true;
  }
}

static void build_work_lists(wt_grid* g, bool touch = true) {
  g->lists_ok = false;
  for (auto& lp : g->lev) lp->tflag_ok = false;
  if (!g->multi() || !g->use_lists) {
    if (touch) touch_epoch(g);
    return;
  }
  hipStream_t s = g->stream;
  CompactBatch& cb = g->cb;
  // every level's rings, patch lists and predicates in batched launches (levels are independent)
  std::vector<PatchJob> pj;
  std::vector<ByteJob> clr;
  for (auto& lp : g->lev) {
    LevelState& l = *lp;
    const int64_t N = l.tab.N, E = l.tab.E, T = l.tab.T;
    if (!l.s3n) {
      HIPCHK(wt::dmalloc(&l.s3n, N));
      HIPCHK(wt::dmalloc(&l.s3e, E));
      HIPCHK(wt::dmalloc(&l.s5n, N));
      HIPCHK(wt::dmalloc(&l.s5e, E));
      HIPCHK(wt::dmalloc(&l.rn_, N));
      HIPCHK(wt::dmalloc(&l.re_, E));
      HIPCHK(wt::dmalloc(&l.pred_t, T));
      HIPCHK(wt::dmalloc(&l.pred_e, N));
      HIPCHK(wt::dmalloc(&l.pred_a, N));
    }
    // rings of same-level neighbours: 1, 2 (scratch), 3 (kept), 4, 5 (kept); patches far from
    // every active point skip the gathers (their points are cleared here)
    const int nl = 1 << l.geo.J;
    if (nl >= 8) {
      const int64_t np = 10 * int64_t(nl / 8) * (nl / 8);
      if (!l.pf) {
        HIPCHK(wt::dmalloc(&l.pf, np));
        HIPCHK(wt::dmalloc(&l.plist, (np + 1) * sizeof(int32_t)));
      }
      pj.push_back(PatchJob{l.geo.J, l.na, l.ea, l.pf, l.plist, l.plist + np});
      const ByteJob c[] = {{l.rn_, nullptr, N, 0}, {l.re_, nullptr, E, 0}, {l.s5n, nullptr, N, 0},
                           {l.s5e, nullptr, E, 0}, {l.s3n, nullptr, N, 0}, {l.s3e, nullptr, E, 0}};
      clr.insert(clr.end(), c, c + 6);
    }
  }
  if (!clr.empty()) ml_bytes_batch(clr.data(), int(clr.size()), s);
  if (!pj.empty()) ml_patch_list_batch(pj.data(), int(pj.size()), s);
  for (int r = 0; r < 5; ++r) {
    std::vector<RingJob> rj;
    for (auto& lp : g->lev) {
      LevelState& l = *lp;
      const int nl = 1 << l.geo.J;
      const uint8_t* an[5] = {l.na, l.rn_, l.s5n, l.s3n, l.rn_};
      const uint8_t* ae[5] = {l.ea, l.re_, l.s5e, l.s3e, l.re_};
      uint8_t* bn[5] = {l.rn_, l.s5n, l.s3n, l.rn_, l.s5n};
      uint8_t* be[5] = {l.re_, l.s5e, l.s3e, l.re_, l.s5e};
      if (nl >= 8) rj.push_back(ring_job(l.tab, nl, an[r], ae[r], bn[r], be[r], l.plist));
      else ml_ring(l.tab, nl, an[r], ae[r], bn[r], be[r], s);
    }
    if (!rj.empty()) ml_ring_batch(rj.data(), int(rj.size()), s);
  }
  std::vector<PredJob> pr;
  for (auto& lp : g->lev) {
    LevelState& l = *lp;
    const int64_t N = l.tab.N, E = l.tab.E, T = l.tab.T;
    pr.push_back(pred_tri_job(T, l.geo.J, l.tab.t_e, l.s3e, l.pred_t));
    pr.push_back(pred_elem_job(N, l.tab.n_elem, l.s3n, l.s3e, l.pred_e));
    pr.push_back(pred_elem_job(N, l.tab.n_elem, l.na, l.ea, l.pred_a));
    cb.add(l.pred_t, T, l.l_tri);
    cb.add(l.pred_e, N, l.l_elem);
    cb.add(l.s3e, E, l.l_edge);
    cb.add(l.s3n, N, l.l_node);
    cb.add(l.pred_a, N, l.l_tend);
  }
  for (int j = g->jmin; j < g->jmax; ++j) {
    PairState& P = g->P(j);
    LevelState& F = g->L(j + 1);
    const int64_t Nc = P.dev.Nc, Ec = P.dev.Ec, Tc = P.dev.Tc;
    if (!P.pred) HIPCHK(wt::dmalloc(&P.pred, Nc + Ec + Tc));
    uint8_t *pn = P.pred, *pe = P.pred + Nc, *pt = P.pred + Nc + Ec;
    pr.push_back(pred_pair_job(P.dev, j, F.s5n, F.s5e, pn, pe, pt));
    cb.add(pn, Nc, P.l_cn);
    cb.add(pe, Ec, P.l_ce);
    cb.add(pt, Tc, P.l_ct);
  }
  pred_batch(pr.data(), int(pr.size()), s);
  cb.run(s);
  g->lists_ok = true;
  update_tile_flags(g);
  if (touch) touch_epoch(g);
}

// A level's stage through the masked lattice kernel (flagged tiles only when the flags are
// current; their count is read back only for the byte count of a timed launch): the finest
// level whole, or (inter) the intermediates of the level below it.
static void dense_stage(wt_grid* g, LevelState& l, const StageSpec& sp, const PhysParams& p, bool fp32,
                        bool inter = false) {
  const uint8_t* tf = l.tflag_ok ? l.tflag : nullptr;
  int64_t flagged = 0;
  if (tf && g->timer.enabled) {
    int32_t c = 0;
    HIPCHK(hipMemcpyAsync(&c, l.tcount, sizeof(c), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    flagged = c;
  }
  launch_lattice_masked(l.lat, l.work, l.na, l.ea, tf, flagged, p, fp32, sp.pdh, sp.pu, sp.c, g->stream, &g->timer,
                        inter);
}

static void ml_step(wt_grid* g, double dt) {
  ++g->state_ver;
  const bool fp32 = g->prm.precision == WT_FP32_TENDENCY;
  const int nl = g->jmax - g->jmin + 1;
  PhysParams p = phys(g);
  const bool wl = g->use_lists && g->lists_ok;
  auto LS = [&](const WorkList& L) { return wl ? span(L) : Span{}; };
  const bool dense = dense_finest(g), dense2 = dense_second(g);
  const DevLattice& lat = g->lev.back()->lat;
  for (int s = 0; s < 4; ++s) {
    std::vector<StageSpec> sp(nl);
    std::vector<double*> xdh(nl), xu(nl);
    for (int q = 0; q < nl; ++q) {
      sp[q] = rk_stage(g->prm.rk, s, g->lev[q]->work, dt);
      xdh[q] = const_cast<double*>(sp[q].xdh);
      xu[q] = const_cast<double*>(sp[q].xu);
    }
    // prolongation of the inactive points of the support (every inactive point without lists)
    for (int j = g->jmin; j < g->jmax; ++j) {
      LevelState& F = g->L(j + 1);
      PairState& P = g->P(j);
      ml_prolong(P.dev, g->L(j).tab, F.na, F.ea, xdh[j - g->jmin], xu[j - g->jmin], xdh[j + 1 - g->jmin],
                 xu[j + 1 - g->jmin], fp32, g->stream, LS(P.l_cn), LS(P.l_ce), LS(P.l_ct));
    }
    for (int q = 0; q < nl; ++q) {
      LevelState& l = *g->lev[q];
      if ((dense && q == nl - 1) || (dense2 && q == nl - 2)) {
        // the tile elements through the lattice kernel (the finest level whole, the level below
        // it its intermediates only), then the rim's intermediates from the tables
        const DevLattice& lt = l.lat;
        dense_stage(g, l, sp[q], p, fp32, q == nl - 2);
        ml_level_intermediates(l.tab, l.work, p, fp32, xdh[q], xu[q], g->stream, Span{lt.sup_tris, lt.n_sup_tris},
                               Span{lt.sup_elems, lt.n_sup_elems}, Span{lt.rim_edges, lt.n_rim_edges});
        continue;
      }
      ml_level_intermediates(l.tab, l.work, p, fp32, xdh[q], xu[q], g->stream, LS(l.l_tri), LS(l.l_elem),
                             LS(l.l_edge));
    }
    for (int j = g->jmax - 1; j >= g->jmin; --j) {
      LevelState &C = g->L(j), &F = g->L(j + 1);
      PairState& P = g->P(j);
      // a dense finest level's tile nodes have their divergence from the lattice kernel: the rim's
      const Span lfn = dense && j + 1 == g->jmax ? Span{lat.rim, lat.n_rim} : LS(F.l_node);
      ml_restrict(P.dev, C.tab, F.tab, C.work, F.work, F.na, F.ea, p, fp32, g->stream, lfn, LS(P.l_ce),
                  LS(P.l_cn));
    }
    for (int q = 0; q < nl; ++q) {
      LevelState& l = *g->lev[q];
      const Span lt = dense && q == nl - 1 ? Span{lat.rim, lat.n_rim} : LS(l.l_tend);
      ml_tend(l.tab, l.work, l.na, l.ea, p, fp32, sp[q].pdh, sp[q].pu, sp[q].c, g->stream, lt);
    }
  }
  // partial height transform at complete nodes, bottom-up
  for (int j = g->jmax - 1; j >= g->jmin; --j) {
    LevelState &C = g->L(j), &F = g->L(j + 1);
    PairState& P = g->P(j);
    ml_partial_h(P.dev, C.tab, C.na, F.na, F.ea, F.work.dh, C.work.dh, P.ph_det, P.ph_act, g->stream, LS(P.l_cn));
  }
}

// max |dh| over the active nodes and max |u| over the active edges of all levels: one batched
// reduction and one read-back
static void masked_max_all(wt_grid* g, double* mh, double* mu) {
  if (!g->host_val) HIPCHK(hipHostMalloc(&g->host_val, wt_grid::kSlots * sizeof(double), hipHostMallocDefault));
  MaxJobs jobs{};
  int k = 0;
  for (auto& l : g->lev) jobs.j[k++] = MaxJob{l->work.dh, l->na, l->tab.N};
  for (auto& l : g->lev) jobs.j[k++] = MaxJob{l->work.u, l->ea, l->tab.E};
  double* red = g->lev.front()->work.red;   // MAX_JOBS * MAX_BLOCKS partials, then the results
  ml_masked_max_batch(jobs, k, red, red + MAX_JOBS * MAX_BLOCKS, g->stream);
  HIPCHK(hipMemcpyAsync(g->host_val, red + MAX_JOBS * MAX_BLOCKS, k * sizeof(double), hipMemcpyDeviceToHost,
                        g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  const int nl = k / 2;
  double bh = 0.0, bu = 0.0;
  for (int q = 0; q < nl; ++q) {
    bh = std::fmax(bh, g->host_val[q]);
    bu = std::fmax(bu, g->host_val[nl + q]);
  }
  *mh = bh;
  *mu = bu;
}

// Regime thresholds of Sec. 3.1 (the reading stated with WT_THR_QG / WT_THR_IG in wt.h): the
// velocity threshold in m/s and the height threshold in metres.
static void regime_thresholds(const wt_params& p, double eps, double* eh, double* eu) {
  const double e32 = eps * std::sqrt(eps);
  if (p.threshold == WT_THR_QG) {
    const double Ro = p.scale_u / (p.scale_f * p.scale_l);
    *eu = p.scale_u * Ro * e32;
    *eh = p.scale_f * p.scale_u * p.scale_l * Ro * e32 / p.gravity;
  } else {
    const double c = std::sqrt(p.gravity * p.mean_depth);
    *eu = p.scale_u * e32;
    *eh = c * p.scale_u * e32 / p.gravity;
  }
}

// The same maxima turned into the thresholds eps * max on the device (no read-back); the host
// copy (host_val[kThr], [kThr + 1]) is valid once the stream has been synchronised.  Returns the
// device thresholds.  With the regime thresholds the device values are the host's formulas.
static const double* thresholds_async(wt_grid* g, double eps) {
  if (!g->host_val) HIPCHK(hipHostMalloc(&g->host_val, wt_grid::kSlots * sizeof(double), hipHostMallocDefault));
  MaxJobs jobs{};
  int k = 0;
  for (auto& l : g->lev) jobs.j[k++] = MaxJob{l->work.dh, l->na, l->tab.N};
  for (auto& l : g->lev) jobs.j[k++] = MaxJob{l->work.u, l->ea, l->tab.E};
  double* red = g->lev.front()->work.red;
  double* out = red + MAX_JOBS * MAX_BLOCKS;
  double* thr = out + MAX_JOBS;
  ml_masked_max_batch(jobs, k, red, out, g->stream);
  ml_thresholds(out, k / 2, eps, thr, g->stream);
  if (g->prm.threshold != WT_THR_RELATIVE) {
    double* up = g->host_val + wt_grid::kThr - 2;   // pinned staging of the upload
    regime_thresholds(g->prm, eps, &up[0], &up[1]);
    HIPCHK(hipMemcpyAsync(thr, up, 2 * sizeof(double), hipMemcpyHostToDevice, g->stream));
  }
  HIPCHK(hipMemcpyAsync(g->host_val + wt_grid::kThr, thr, 2 * sizeof(double), hipMemcpyDeviceToHost, g->stream));
  return thr;
}

// ---------------------------------------------------------------- learned adjacent zone
// Levels whose children rule can be gated: jmin < j < jmax (level jmin has no significant
// points of its own) with at least one 8 x 8 patch per lozenge side.
static bool learnable(const wt_grid* g, int j) { return j > g->jmin && j < g->jmax && j >= 3; }

static void ensure_learn_buffers(wt_grid* g) {
  for (int j = g->jmin + 1; j <= g->jmax; ++j) {
    LevelState& l = g->L(j);
    if (!l.rn) {
      HIPCHK(wt::dmalloc(&l.rn, l.tab.N * sizeof(float)));
      HIPCHK(wt::dmalloc(&l.re, l.tab.E * sizeof(float)));
    }
    if (learnable(g, j) && !l.stats) {
      const int64_t n = int64_t(1) << j, m = n / 8;
      l.npatch = 10 * m * m;
      HIPCHK(wt::dmalloc(&l.stats, l.npatch * LEARN_STATS * sizeof(float)));
      HIPCHK(wt::dmalloc(&l.X, l.npatch * 64 * sizeof(float)));
      HIPCHK(wt::dmalloc(&l.Pr, l.npatch * 4 * sizeof(float)));
      HIPCHK(wt::dmalloc(&l.allow, l.npatch * 4));
      HIPCHK(wt::dmalloc(&l.dropped, l.npatch * 4));
      HIPCHK(wt::dmalloc(&l.viol, l.npatch * 4));
    }
  }
}

// Patch statistics of every learnable level from the current details (thresholds eh, eu) and
// the current significant points.
static void learn_stats_all(wt_grid* g, double eh, double eu) {
  ensure_learn_buffers(g);
  const bool L = g->details_partial;   // then only the work lists' details are current
  std::vector<PointRJob> pr;
  for (int j = g->jmin + 1; j <= g->jmax; ++j) {
    PairState& P = g->P(j - 1);
    LevelState& l = g->L(j);
    pr.push_back(point_r_job(P.dev, P.d_h, P.d_p, P.d_i, eh, eu, l.rn, l.re, L ? span(P.l_ce) : Span{},
                             L ? span(P.l_ct) : Span{}));
  }
  learn_point_r_batch(pr.data(), int(pr.size()), g->stream);
  for (int j = g->jmin + 1; j < g->jmax; ++j) {
    if (!learnable(g, j)) continue;
    LevelState &l = g->L(j), &F = g->L(j + 1);
    learn_patch_stats(l.npatch, 1 << j, l.rn, l.re, F.rn, F.re, l.na, F.na, l.sn, l.se, l.stats, g->stream);
  }
}

static float level_pos(const wt_grid* g, int j) { return float(j - g->jmin) / float(g->jmax - g->jmin); }

static void snapshot(wt_grid* g, bool restore) {
  // the work lists describe the masks being discarded; the adapt that follows a restore builds
  // them again (and bumps the epoch if the launches change)
  if (restore) {
    g->lists_ok = false;
    touch_epoch(g);
    ++g->state_ver;
  }
  for (auto& lp : g->lev) {
    LevelState& l = *lp;
    const int64_t N = l.tab.N, E = l.tab.E;
    if (!l.snap_dh) {
      HIPCHK(wt::dmalloc(&l.snap_dh, N * sizeof(double)));
      HIPCHK(wt::dmalloc(&l.snap_u, E * sizeof(double)));
      HIPCHK(wt::dmalloc(&l.snap_na, N));
      HIPCHK(wt::dmalloc(&l.snap_ea, E));
    }
    auto cp = [&](void* dst, const void* src, size_t b) {
      HIPCHK(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToDevice, g->stream));
    };
    if (restore) {
      cp(l.work.dh, l.snap_dh, N * sizeof(double));
      cp(l.work.u, l.snap_u, E * sizeof(double));
      cp(l.na, l.snap_na, N);
      cp(l.ea, l.snap_ea, E);
    } else {
      cp(l.snap_dh, l.work.dh, N * sizeof(double));
      cp(l.snap_u, l.work.u, E * sizeof(double));
      cp(l.snap_na, l.na, N);
      cp(l.snap_ea, l.ea, E);
    }
  }
}

static void clear_significant(wt_grid* g) {
  std::vector<ByteJob> clr;
  for (auto& l : g->lev) {
    clr.push_back({l->sn, nullptr, l->tab.N, 0});
    clr.push_back({l->se, nullptr, l->tab.E, 0});
  }
  ml_bytes_batch(clr.data(), int(clr.size()), g->stream);
}

static void adapt_impl(wt_grid* g, double eps, double* eh_out, double* eu_out, bool gate = false) {
  // The threshold test reads the details of active points only, whose prolongation and
  // prediction stencils lie in the work-list support; the learned gate's patch features read
  // every point's detail, but outside the support the points are inactive with prolonged values
  // and their details vanish, so the transform runs over the work lists in both cases.
  std::vector<double*> dh = state_dh(g), u = state_u(g);
  // thresholds: reused from the passing test, or computed on the device (their host copy is read
  // once the stream has been synchronised, by the gate below or by the work-list build)
  double eh = 0.0, eu = 0.0;
  bool thr_pending = false;
  if (g->judge_ver == g->state_ver && eps == g->last_eps && g->lists_ok) {
    // the passing threshold test after the last step computed exactly this (details, maxima,
    // R1) on this state
    eh = g->last_eh;
    eu = g->last_eu;
  } else {
    prolong_all(g, dh, u, true);
    details_all(g, dh, u, true);
    const double* thr = thresholds_async(g, eps);
    thr_pending = true;
    clear_significant(g);
    // R1: significant points
    const bool listed = g->lists_ok;
    std::vector<MaskJob> jobs;
    for (int j = g->jmin; j < g->jmax; ++j) {
      PairState& P = g->P(j);
      LevelState& F = g->L(j + 1);
      ml_significant_jobs(jobs, P.dev, F.na, F.ea, P.d_h, P.d_p, P.d_i, 0.0, 0.0, F.sn, F.se,
                          listed ? span(P.l_ce) : Span{}, listed ? span(P.l_ct) : Span{});
      jobs[jobs.size() - 1].thr = thr;
      jobs[jobs.size() - 2].thr = thr;
    }
    ml_mask_ops(jobs.data(), int(jobs.size()), g->stream);
  }
  auto read_thresholds = [&]() {
    if (!thr_pending) return;
    HIPCHK(hipStreamSynchronize(g->stream));
    eh = g->host_val[wt_grid::kThr];
    eu = g->host_val[wt_grid::kThr + 1];
    thr_pending = false;
  };
  {
    std::vector<ByteJob> cp;
    for (auto& l : g->lev) {
      cp.push_back({l->nn, l->sn, l->tab.N, 0});
      cp.push_back({l->ne, l->se, l->tab.E, 0});
    }
    ml_bytes_batch(cp.data(), int(cp.size()), g->stream);
  }
  // learned zone: the predictor proposes, per patch quadrant, whether the children rule applies
  if (gate) {
    read_thresholds();
    learn_stats_all(g, eh, eu);
    for (int j = g->jmin + 1; j < g->jmax; ++j) {
      if (!learnable(g, j)) continue;
      LevelState& l = g->L(j);
      learn_features(l.npatch, 1 << j, level_pos(g, j), l.stats, l.X, g->stream);
      mlp_predict(g->predictor, l.X, l.npatch, l.Pr, g->stream);
      learn_gate(l.npatch, l.Pr, g->pred_thr, l.stats, l.allow, l.dropped, g->stream);
      for (const auto& fd : g->force_drop)
        if (fd.first == j) learn_force_drop(l.npatch, fd.second, l.stats, l.allow, l.dropped, g->stream);
    }
    g->force_drop.clear();
  }
  // R2: same-level neighbours; R3: children on the next level (all levels in one batch: the rules
  // only set mask bytes)
  {
    std::vector<MaskJob> jobs;
    for (int j = g->jmin; j <= g->jmax; ++j) {
      LevelState& l = g->L(j);
      ml_r2_jobs(jobs, l.tab, l.sn, l.se, l.nn, l.ne);
      if (j < g->jmax) {
        LevelState& F = g->L(j + 1);
        const bool gj = gate && learnable(g, j);
        ml_r3_jobs(jobs, g->P(j).dev, F.tab, l.sn, l.se, F.nn, F.ne, gj ? l.allow : nullptr, gj ? (1 << j) : 0);
      }
    }
    ml_mask_ops(jobs.data(), int(jobs.size()), g->stream);
  }
  LevelState& L0 = g->L(g->jmin);
  const ByteJob all0[] = {{L0.nn, nullptr, L0.tab.N, 1}, {L0.ne, nullptr, L0.tab.E, 1}};
  ml_bytes_batch(all0, 2, g->stream);
  // R4 consistency and R5 prediction stencils, top-down
  for (int j = g->jmax; j >= g->jmin; --j) {
    LevelState& l = g->L(j);
    ml_r4(l.tab, l.nn, l.ne, g->stream);
    if (j > g->jmin) {
      LevelState& C = g->L(j - 1);
      ml_r5(g->P(j - 1).dev, C.tab, l.nn, l.ne, C.nn, C.ne, g->stream);
    }
  }
  for (auto& l : g->lev) {
    std::swap(l->na, l->nn);
    std::swap(l->ea, l->ne);
  }
  // the new masks' work lists first: the inverse then rewrites only the support (the old masks
  // stay in nn/ne for it)
  build_work_lists(g, false);
  if (thr_pending && g->lists_ok) {
    // the list build's compaction synchronised the stream after the thresholds' copy
    eh = g->host_val[wt_grid::kThr];
    eu = g->host_val[wt_grid::kThr + 1];
    thr_pending = false;
  }
  read_thresholds();
  g->last_eh = eh;
  g->last_eu = eu;
  inverse_all(g, dh, u, true, true, true);
  // the new masks go back into the buffers that held the old ones, so the mask addresses a
  // recorded step uses stay the same from one adapt to the next
  {
    std::vector<ByteJob> cp;
    for (auto& l : g->lev) {
      cp.push_back({l->nn, l->na, l->tab.N, 0});
      cp.push_back({l->ne, l->ea, l->tab.E, 0});
    }
    ml_bytes_batch(cp.data(), int(cp.size()), g->stream);
    for (auto& l : g->lev) {
      std::swap(l->na, l->nn);
      std::swap(l->ea, l->ne);
    }
  }
  touch_epoch(g);
  ++g->state_ver;
  if (eh_out) *eh_out = eh;
  if (eu_out) *eu_out = eu;
}

// Threshold test after a gated step: the significant points of the new state (thresholds from
// eps and the new maxima) must not fall in a quadrant whose children the gate dropped.  Returns
// the number of such quadrants.
static int64_t judge_gated_step(wt_grid* g) {
  // only the significance of active points matters here: prolongation, details and the test
  // run over the work lists
  std::vector<double*> dh = state_dh(g), u = state_u(g);
  prolong_all(g, dh, u, true);
  details_all(g, dh, u, true);
  double mh, mu;
  masked_max_all(g, &mh, &mu);
  double eh = g->last_eps * mh, eu = g->last_eps * mu;
  if (g->prm.threshold != WT_THR_RELATIVE) regime_thresholds(g->prm, g->last_eps, &eh, &eu);
  clear_significant(g);
  const bool L = g->lists_ok;
  std::vector<MaskJob> jobs;
  for (int j = g->jmin; j < g->jmax; ++j) {
    PairState& P = g->P(j);
    LevelState& F = g->L(j + 1);
    ml_significant_jobs(jobs, P.dev, F.na, F.ea, P.d_h, P.d_p, P.d_i, eh, eu, F.sn, F.se,
                        L ? span(P.l_ce) : Span{}, L ? span(P.l_ct) : Span{});
  }
  ml_mask_ops(jobs.data(), int(jobs.size()), g->stream);
  g->last_eh = eh;
  g->last_eu = eu;
  learn_stats_all(g, eh, eu);
  int k = 0;
  for (int j = g->jmin + 1; j < g->jmax; ++j) {
    if (!learnable(g, j)) continue;
    LevelState& l = g->L(j);
    learn_violations(l.npatch, l.stats, l.dropped, l.viol, g->stream);
    ml_count(4 * l.npatch, l.viol, l.work.red, l.work.red + 4096, g->stream);
    HIPCHK(hipMemcpyAsync(g->host_val + k++, l.work.red + 4096, sizeof(double), hipMemcpyDeviceToHost, g->stream));
  }
  HIPCHK(hipStreamSynchronize(g->stream));
  int64_t total = 0;
  for (int q = 0; q < k; ++q) total += int64_t(g->host_val[q]);
  g->judge_ver = total == 0 ? g->state_ver : ~uint64_t(0);
  return total;
}

// Host threads of an ensemble: created once with the ensemble and kept until it is destroyed
// (a thread per call would create and tear down threads, and their HIP thread state, every
// step).  run(n, fn) calls fn(k) for every member k: thread t takes k = t, t + nt, ... and the
// calling thread is thread 0, so a member is always served by the same thread.  Four threads: a
// process gets four hardware queues by default, and more threads only contend for them (32-member
// ensemble: batched step 16.1 ms with 4 or 8 threads, 17.2 with 16, 17.7 with 32).
class MemberPool {
 public:
  MemberPool() {
    const size_t hw = std::max<size_t>(1, std::thread::hardware_concurrency());
    nt_ = std::min<size_t>(hw, 4);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    for (size_t t = 1; t < nt_; ++t) {
      try {
        th_.emplace_back([this, t, dev]() { loop(t, dev); });
      } catch (const std::exception&) {
        break;   // fewer threads: the caller covers the shares of the missing ones
      }
    }
  }
  ~MemberPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& x : th_) x.join();
  }
  // fn(k) for k in [0, n); the first failure (in member order) is returned with its message.  fn
  // returns WT_OK or an error code and leaves its message in the calling thread's g_err.
  int run(size_t n, const std::function<int(size_t)>& fn) {
    std::vector<int> rc(n, WT_OK);
    std::vector<std::string> msg(n);
    const std::function<void(size_t)> share = [&](size_t t) {
      for (size_t k = t; k < n; k += nt_) {
        try {
          rc[k] = fn(k);
        } catch (const std::exception& x) {
          rc[k] = fail(WT_EDEVICE, x.what());
        }
        if (rc[k] != WT_OK) msg[k] = g_err;
      }
    };
    {
      std::unique_lock<std::mutex> lk(mu_);
      job_ = &share;
      pending_ = th_.size();
      ++gen_;
    }
    cv_.notify_all();
    share(0);
    for (size_t t = th_.size() + 1; t < nt_; ++t) share(t);   // shares of threads that failed to start
    {
      std::unique_lock<std::mutex> lk(mu_);
      done_cv_.wait(lk, [&] { return pending_ == 0; });
      job_ = nullptr;
    }
    for (size_t k = 0; k < n; ++k)
      if (rc[k] != WT_OK) return fail(rc[k], msg[k]);
    return WT_OK;
  }

 private:
  void loop(size_t t, int dev) {
    (void)hipSetDevice(dev);
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(size_t)>* job = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        job = job_;
      }
      (*job)(t);
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (--pending_ == 0) done_cv_.notify_all();
      }
    }
  }
  size_t nt_ = 1;
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(size_t)>* job_ = nullptr;
  size_t pending_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

// Host tables are expensive to build (seconds at level 9) and depend only on the level (pairs:
// on the coarse level) and the sphere's radius and rotation rate: grids built in one process share
// the geometry-only parts through this cache; effective areas are applied per grid.
namespace {
std::mutex g_cache_mu;
std::map<std::tuple<int, double, double>, std::shared_ptr<const Level>> g_level_cache;
std::map<std::tuple<int, double, double>, std::shared_ptr<const PairTables>> g_pair_cache;
}  // namespace

static std::shared_ptr<const Level> cached_level(int j, double radius, double omega) {
  const auto key = std::make_tuple(j, radius, omega);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_level_cache.find(key);
    if (it != g_level_cache.end()) return it->second;
  }
  auto L = std::make_shared<Level>();
  build_level(j, radius, omega, *L);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  return g_level_cache.emplace(key, std::move(L)).first->second;
}

static std::shared_ptr<const PairTables> cached_pair(const Level& C, const Level& F) {
  const auto key = std::make_tuple(C.J, C.radius, C.omega);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_pair_cache.find(key);
    if (it != g_pair_cache.end()) return it->second;
  }
  auto P = std::make_shared<PairTables>();
  build_pair(C, F, *P);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  return g_pair_cache.emplace(key, std::move(P)).first->second;
}

extern "C" {

const char* wt_last_error(void) { return g_err.c_str(); }

void wt_table_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_level_cache.clear();
  g_pair_cache.clear();
}

const char* wt_kernel_names(void) {
  return "trisk_vertex,trisk_edge_cell,trisk_tend,trisk_lattice,trisk_lattice_masked,trisk_lattice_inter";
}

wt_grid* wt_grid_create(int jmin, int jmax, int patch) {
  if (jmin < 0 || jmax < jmin || jmax > 12) {
    fail(WT_EINVAL, "wt_grid_create: need 0 <= jmin <= jmax <= 12");
    return nullptr;
  }
  if (patch != 4 && patch != 8 && patch != 16) {
    fail(WT_EINVAL, "wt_grid_create: patch must be 4, 8 or 16");
    return nullptr;
  }
  if (jmax > 11) {
    fail(WT_EINVAL, "wt_grid_create: levels above 11 exceed the 32-bit tables");
    return nullptr;
  }
  try {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
      fail(WT_EDEVICE, "wt_grid_create: no HIP device");
      return nullptr;
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
      fail(WT_EDEVICE, std::string("wt_grid_create: device is ") + prop.gcnArchName + ", need gfx950");
      return nullptr;
    }
    auto g = std::make_unique<wt_grid>();
    g->jmin = jmin; g->jmax = jmax; g->patch = patch;
    g->cus = prop.multiProcessorCount;
    g->prm.radius = 6.371e6;
    g->prm.omega = 7.292e-5;
    g->prm.gravity = 9.80616;
    g->prm.mean_depth = 2.94e4 / 9.80616;
    g->prm.rk = WT_RK4;
    g->prm.precision = WT_FP64;
    g->prm.viscosity = 0.0;
    g->prm.equations = WT_SWE;
    g->prm.threshold = WT_THR_RELATIVE;
    HIPCHK(hipStreamCreate(&g->own));
    g->stream = g->own;
    g->hook = default_hook();
    GridScope scope(g.get());
    std::vector<std::shared_ptr<const Level>> raw;
    for (int j = jmin; j <= jmax; ++j) raw.push_back(cached_level(j, g->prm.radius, g->prm.omega));
    for (int j = jmin; j < jmax; ++j) {
      auto ps = std::make_unique<PairState>();
      ps->host = *cached_pair(*raw[j - jmin], *raw[j + 1 - jmin]);
      g->pairs.push_back(std::move(ps));
    }
    // effective areas, bottom-up from the geometric areas of jmax (area conditions, Sec. 4.1)
    const int nl = jmax - jmin + 1;
    std::vector<std::vector<double>> Aeff(nl);
    Aeff[nl - 1] = raw[nl - 1]->A_i;
    for (int j = jmax - 1; j >= jmin; --j)
      finish_pair(*raw[j - jmin], *raw[j + 1 - jmin], Aeff[j + 1 - jmin], g->P(j).host, Aeff[j - jmin]);
    for (int q = 0; q < nl; ++q) {
      const Level& R = *raw[q];
      auto ls = std::make_unique<LevelState>();
      upload_tables(R, Aeff[q], ls->tab);
      // the host keeps what coordinates, counts and diagnostics read
      Level& L = ls->geo;
      L.J = R.J;
      L.n = R.n; L.N = R.N; L.E = R.E; L.T = R.T;
      L.radius = R.radius; L.omega = R.omega;
      L.pos = R.pos;
      L.e_c = R.e_c;
      L.A_i = std::move(Aeff[q]);
      g->lev.push_back(std::move(ls));
      alloc_work(*g->lev.back());
    }
    if (!g->multi()) {
      LatticeHost lh;
      if (build_lattice(*raw[nl - 1], lh)) upload_lattice(lh, g->L(jmax).lat);
    }
    raw.clear();
    for (auto& ps : g->pairs) {
      upload_pair(ps->host, ps->dev);
      auto A2 = [](double** q, int64_t n) { HIPCHK(wt::dmalloc(q, n * sizeof(double))); HIPCHK(hipMemset(*q, 0, n * sizeof(double))); };
      A2(&ps->d_h, ps->host.Ec); A2(&ps->d_p, ps->host.Ec); A2(&ps->d_k, ps->host.Ec); A2(&ps->d_i, 3 * ps->host.Tc);
      A2(&ps->ph_det, ps->host.Ec);
      HIPCHK(wt::dmalloc(&ps->ph_act, ps->host.Ec));
      HIPCHK(hipMemset(ps->ph_act, 0, ps->host.Ec));
      A2(&ps->r_h, ps->host.Ec); A2(&ps->r_p, ps->host.Ec); A2(&ps->r_i, 3 * ps->host.Tc);
      // keep only what the device path needs on the host
      ps->host = PairTables{};
    }
    g_err.clear();
    return g.release();
  } catch (const std::bad_alloc&) {
    fail(WT_ENOMEM, "wt_grid_create: out of memory");
  } catch (const std::exception& e) {
    fail(WT_EDEVICE, std::string("wt_grid_create: ") + e.what());
  }
  return nullptr;
}

void wt_grid_destroy(wt_grid* g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  for (auto& r : g->timer.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto& ls : g->lev) {
    free_tables(ls->tab);
    free_work(*ls);
    free_lattice(ls->lat);
  }
  for (auto& ps : g->pairs) {
    free_pair(ps->dev);
    free_list(ps->l_cn);
    free_list(ps->l_ce);
    free_list(ps->l_ct);
    if (ps->pred) (void)wt::dfree(ps->pred);
    void* q[] = {ps->d_h, ps->d_p, ps->d_i, ps->d_k, ps->r_h, ps->r_p, ps->r_i, ps->ph_det, ps->ph_act};
    for (void* x : q)
      if (x) (void)wt::dfree(x);
  }
  free_scratch(g->csc);
  g->cb.release();
  g->splan.release();
  if (g->host_val) (void)hipHostFree(g->host_val);
  if (g->own) (void)hipStreamDestroy(g->own);
  delete g;
}

int wt_set_params(wt_grid* g, const wt_params* p) {
  GridScope scope_(g);
  if (!g || !p) return fail(WT_EINVAL, "wt_set_params: null argument");
  if (p->radius != g->prm.radius || p->omega != g->prm.omega)
    return fail(WT_EINVAL, "wt_set_params: radius and omega are fixed at grid creation");
  if (p->equations != WT_SWE && p->equations != WT_ADVECTION) return fail(WT_EINVAL, "wt_set_params: bad equations");
  const bool adv = p->equations == WT_ADVECTION;
  if (!(p->gravity > 0) || !(adv ? p->mean_depth >= 0 : p->mean_depth > 0) || !std::isfinite(p->mean_depth))
    return fail(WT_EINVAL, "wt_set_params: gravity and mean_depth must be positive (mean_depth >= 0 for advection)");
  if (p->rk != WT_RK4 && p->rk != WT_SSPRK43) return fail(WT_EINVAL, "wt_set_params: bad rk");
  if (p->precision != WT_FP64 && p->precision != WT_FP32_TENDENCY)
    return fail(WT_EINVAL, "wt_set_params: bad precision");
  if (!(p->viscosity >= 0) || !std::isfinite(p->viscosity))
    return fail(WT_EINVAL, "wt_set_params: viscosity must be >= 0");
  if (adv && p->viscosity != 0) return fail(WT_EINVAL, "wt_set_params: the advection form has no viscosity");
  if (p->threshold != WT_THR_RELATIVE && p->threshold != WT_THR_QG && p->threshold != WT_THR_IG)
    return fail(WT_EINVAL, "wt_set_params: bad threshold");
  if (p->threshold != WT_THR_RELATIVE && !(p->scale_u > 0))
    return fail(WT_EINVAL, "wt_set_params: the regime thresholds need scale_u > 0");
  if (p->threshold == WT_THR_QG && !(p->scale_l > 0 && p->scale_f > 0))
    return fail(WT_EINVAL, "wt_set_params: the quasi-geostrophic thresholds need scale_l, scale_f > 0");
  if (p->threshold == WT_THR_IG && !(p->mean_depth > 0))
    return fail(WT_EINVAL, "wt_set_params: the inertia-gravity thresholds need mean_depth > 0");
  try {
    // the viscous form's total mass flux G: one more edge array per level
    if (p->viscosity != 0)
      for (auto& l : g->lev)
        if (!l->work.G) {
          HIPCHK(wt::dmalloc(&l->work.G, l->tab.E * sizeof(double)));
          HIPCHK(hipMemsetAsync(l->work.G, 0, l->tab.E * sizeof(double), g->stream));
        }
  } catch (const std::exception& e) {
    return fail(WT_ENOMEM, std::string("wt_set_params: ") + e.what());
  }
  g->prm = *p;
  ++g->state_ver;
  touch_epoch(g);
  return WT_OK;
}

int wt_get_params(const wt_grid* g, wt_params* p) {
  if (!g || !p) return fail(WT_EINVAL, "wt_get_params: null argument");
  *p = g->prm;
  return WT_OK;
}

static bool bad_level(const wt_grid* g, int level) { return !g || level < g->jmin || level > g->jmax; }

int wt_grid_info(const wt_grid* g, int level, int64_t* nn, int64_t* ne, int64_t* nt) {
  if (bad_level(g, level)) return fail(WT_EINVAL, "wt_grid_info: bad level");
  const Level& L = g->lev[level - g->jmin]->geo;
  if (nn) *nn = L.N;
  if (ne) *ne = L.E;
  if (nt) *nt = L.T;
  return WT_OK;
}

int wt_grid_coords(const wt_grid* g, int level, double* nx, double* em, double* et) {
  if (bad_level(g, level)) return fail(WT_EINVAL, "wt_grid_coords: bad level");
  const Level& L = g->lev[level - g->jmin]->geo;
  if (nx)
    for (int64_t i = 0; i < L.N; ++i) {
      nx[3 * i] = L.pos[i].x; nx[3 * i + 1] = L.pos[i].y; nx[3 * i + 2] = L.pos[i].z;
    }
  for (int64_t e = 0; e < L.E; ++e) {
    V3 a = L.pos[L.e_c[2 * e]], b = L.pos[L.e_c[2 * e + 1]];
    if (em) {
      V3 m = unit(a + b);
      em[3 * e] = m.x; em[3 * e + 1] = m.y; em[3 * e + 2] = m.z;
    }
    if (et) {
      V3 t = unit(b - a);
      et[3 * e] = t.x; et[3 * e + 1] = t.y; et[3 * e + 2] = t.z;
    }
  }
  return WT_OK;
}

static int set_state_impl(wt_grid* g, int level, const void* dh, const void* u, hipMemcpyKind k) {
  if (bad_level(g, level)) return fail(WT_EINVAL, "wt_set_state: bad level");
  ++g->state_ver;
  if (!dh || !u) return fail(WT_EINVAL, "wt_set_state: null array");
  try {
    LevelState& ls = g->L(level);
    HIPCHK(hipMemcpyAsync(ls.work.dh, dh, ls.tab.N * sizeof(double), k, g->stream));
    HIPCHK(hipMemcpyAsync(ls.work.u, u, ls.tab.E * sizeof(double), k, g->stream));
    for (int j = g->jmin; j <= g->jmax; ++j) {
      LevelState& l = g->L(j);
      HIPCHK(hipMemsetAsync(l.na, j <= level ? 1 : 0, l.tab.N, g->stream));
      HIPCHK(hipMemsetAsync(l.ea, j <= level ? 1 : 0, l.tab.E, g->stream));
    }
    for (int j = level - 1; j >= g->jmin; --j)
      ml_restrict_state(g->P(j).dev, g->L(j + 1).work.dh, g->L(j + 1).work.u, g->L(j).work.dh,
                        g->L(j).work.u, g->stream);
    build_work_lists(g);
    HIPCHK(hipStreamSynchronize(g->stream));
    g->have_state = true;
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_set_state: ") + e.what());
  }
  return WT_OK;
}

int wt_set_state(wt_grid* g, int level, const double* dh, const double* u) {
  GridScope scope_(g);
  return set_state_impl(g, level, dh, u, hipMemcpyHostToDevice);
}

int wt_set_state_device(wt_grid* g, int level, const void* dh, const void* u) {
  GridScope scope_(g);
  return set_state_impl(g, level, dh, u, hipMemcpyDeviceToDevice);
}

// Checkpoint file: magic, the grid's shape and parameters, the learned-zone thresholds and redo
// count, then per level the raw device state (every point, active or not) and the masks.
static const char kCkptMagic[8] = {'W', 'T', 'C', 'K', 'P', 'T', '0', '1'};
static const char kCkptEnd[8] = {'W', 'T', 'C', 'K', 'P', 'E', 'N', 'D'};

int wt_save(wt_grid* g, const char* path) {
  GridScope scope_(g);
  if (!g || !path) return fail(WT_EINVAL, "wt_save: null argument");
  if (!g->have_state) return fail(WT_ESTATE, "wt_save: no state loaded");
  std::FILE* f = std::fopen(path, "wb");
  if (!f) return fail(WT_EINVAL, std::string("wt_save: cannot open ") + path);
  bool ok = true;
  auto put = [&](const void* p, size_t n) { ok = ok && std::fwrite(p, 1, n, f) == n; };
  try {
    const int32_t head[4] = {g->jmin, g->jmax, g->patch, int32_t(sizeof(wt_params))};
    const double lasts[3] = {g->last_eps, g->last_eh, g->last_eu};
    put(kCkptMagic, 8);
    put(head, sizeof(head));
    put(&g->prm, sizeof(wt_params));
    put(lasts, sizeof(lasts));
    put(&g->redo, sizeof(int64_t));
    std::vector<double> hv;
    std::vector<uint8_t> hm;
    for (auto& lp : g->lev) {
      LevelState& l = *lp;
      const int64_t ne[2] = {l.tab.N, l.tab.E};
      put(ne, sizeof(ne));
      hv.resize(size_t(l.tab.N + l.tab.E));
      hm.resize(size_t(l.tab.N + l.tab.E));
      HIPCHK(hipMemcpyAsync(hv.data(), l.work.dh, l.tab.N * sizeof(double), hipMemcpyDeviceToHost, g->stream));
      HIPCHK(hipMemcpyAsync(hv.data() + l.tab.N, l.work.u, l.tab.E * sizeof(double), hipMemcpyDeviceToHost,
                            g->stream));
      HIPCHK(hipMemcpyAsync(hm.data(), l.na, l.tab.N, hipMemcpyDeviceToHost, g->stream));
      HIPCHK(hipMemcpyAsync(hm.data() + l.tab.N, l.ea, l.tab.E, hipMemcpyDeviceToHost, g->stream));
      HIPCHK(hipStreamSynchronize(g->stream));
      put(hv.data(), hv.size() * sizeof(double));
      put(hm.data(), hm.size());
    }
    put(kCkptEnd, 8);
  } catch (const std::exception& e) {
    std::fclose(f);
    return fail(WT_EDEVICE, std::string("wt_save: ") + e.what());
  }
  if (std::fclose(f) != 0) ok = false;
  if (!ok) return fail(WT_EINVAL, std::string("wt_save: write failed: ") + path);
  return WT_OK;
}

int wt_load(wt_grid* g, const char* path) {
  GridScope scope_(g);
  if (!g || !path) return fail(WT_EINVAL, "wt_load: null argument");
  std::FILE* f = std::fopen(path, "rb");
  if (!f) return fail(WT_EINVAL, std::string("wt_load: cannot open ") + path);
  bool ok = true;
  auto get = [&](void* p, size_t n) { ok = ok && std::fread(p, 1, n, f) == n; };
  auto bad = [&](const std::string& why) {
    std::fclose(f);
    return fail(WT_EINVAL, "wt_load: " + why + ": " + path);
  };
  char magic[8];
  int32_t head[4];
  wt_params prm{};
  double lasts[3];
  int64_t redo = 0;
  get(magic, 8);
  if (!ok || std::memcmp(magic, kCkptMagic, 8) != 0) return bad("not a checkpoint");
  get(head, sizeof(head));
  if (!ok || head[0] != g->jmin || head[1] != g->jmax || head[2] != g->patch || head[3] != int32_t(sizeof(wt_params)))
    return bad("levels, patch size or format differ from the grid's");
  get(&prm, sizeof(prm));
  get(lasts, sizeof(lasts));
  get(&redo, sizeof(redo));
  if (!ok) return bad("truncated header");
  if (prm.radius != g->prm.radius || prm.omega != g->prm.omega) return bad("radius or omega differ from the grid's");
  std::vector<std::vector<double>> hv(g->lev.size());
  std::vector<std::vector<uint8_t>> hm(g->lev.size());
  for (size_t q = 0; q < g->lev.size(); ++q) {
    const LevelState& l = *g->lev[q];
    int64_t ne[2];
    get(ne, sizeof(ne));
    if (!ok || ne[0] != l.tab.N || ne[1] != l.tab.E) return bad("level sizes differ");
    hv[q].resize(size_t(ne[0] + ne[1]));
    hm[q].resize(size_t(ne[0] + ne[1]));
    get(hv[q].data(), hv[q].size() * sizeof(double));
    get(hm[q].data(), hm[q].size());
    if (!ok) return bad("truncated level data");
  }
  get(magic, 8);
  if (!ok || std::memcmp(magic, kCkptEnd, 8) != 0) return bad("missing end marker");
  std::fclose(f);
  ++g->state_ver;
  try {
    for (size_t q = 0; q < g->lev.size(); ++q) {
      LevelState& l = *g->lev[q];
      HIPCHK(hipMemcpyAsync(l.work.dh, hv[q].data(), l.tab.N * sizeof(double), hipMemcpyHostToDevice, g->stream));
      HIPCHK(hipMemcpyAsync(l.work.u, hv[q].data() + l.tab.N, l.tab.E * sizeof(double), hipMemcpyHostToDevice,
                            g->stream));
      HIPCHK(hipMemcpyAsync(l.na, hm[q].data(), l.tab.N, hipMemcpyHostToDevice, g->stream));
      HIPCHK(hipMemcpyAsync(l.ea, hm[q].data() + l.tab.N, l.tab.E, hipMemcpyHostToDevice, g->stream));
    }
    HIPCHK(hipStreamSynchronize(g->stream));   // the host vectors are released at return
    g->prm = prm;
    g->last_eps = lasts[0];
    g->last_eh = lasts[1];
    g->last_eu = lasts[2];
    g->redo = redo;
    g->gated = false;
    g->details_partial = true;   // the stored details are recomputed when read
    g->have_state = true;
    build_work_lists(g);
    HIPCHK(hipStreamSynchronize(g->stream));
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_load: ") + e.what());
  }
  return WT_OK;
}

int wt_get_state(wt_grid* g, int level, double* dh, double* u, uint8_t* na, uint8_t* ea) {
  GridScope scope_(g);
  if (bad_level(g, level)) return fail(WT_EINVAL, "wt_get_state: bad level");
  if (!g->have_state) return fail(WT_ESTATE, "wt_get_state: no state loaded");
  try {
    LevelState& ls = g->L(level);
    const double *sdh = ls.work.dh, *su = ls.work.u;
    if (g->multi()) {
      std::vector<double*> rdh, ru;
      reconstruct(g, rdh, ru);
      sdh = rdh[level - g->jmin];
      su = ru[level - g->jmin];
    }
    if (dh) HIPCHK(hipMemcpyAsync(dh, sdh, ls.tab.N * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    if (u) HIPCHK(hipMemcpyAsync(u, su, ls.tab.E * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    if (na) HIPCHK(hipMemcpyAsync(na, ls.na, ls.tab.N, hipMemcpyDeviceToHost, g->stream));
    if (ea) HIPCHK(hipMemcpyAsync(ea, ls.ea, ls.tab.E, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_get_state: ") + e.what());
  }
  return WT_OK;
}

static void build_batch_plan(const std::vector<wt_grid*>& members, const double* dt, BatchPlan& pl,
                             bool allow_dense = false);

// The listed multilevel step with the launches of independent work merged: per stage, the even
// prolongation of a pair, then its odd and interior prolongation together, the three
// intermediate kernels each over all levels, per pair the fine divergence, then the edge and B
// restriction together, the tendencies of all levels; then the partial transform pair by pair
// (88 launches for five levels instead of ~185).  Every entry runs the same per-point body as
// ml_step, so the results are bitwise equal.
// Whether the merged form applies, with its plan brought up to date (this synchronises when the
// plan is rebuilt, so it is called before a capture, not inside one).
static bool phase_plan_ready(wt_grid* g, double dt) {
  if (!g->step_phases || !(g->use_lists && g->lists_ok)) return false;
  touch_epoch(g);
  if (g->sphase.empty() || g->splan_sig != g->step_sig || g->splan_dt != dt) {
    build_batch_plan({g}, &dt, g->splan, true);
    g->splan_dense = dense_finest(g);
    g->splan_dense2 = dense_second(g);
    g->splan.upload(g->stream);
    phase_prepare(g->splan, g->sphase);
    g->splan_sig = g->step_sig;
    g->splan_dt = dt;
  }
  return !g->sphase.empty();
}

// A plan fixes each member's precision, physical constants and state buffers when it is built;
// one launched after a parameter change that did not rebuild it would step with the old values, so
// every launch checks the plan against the members' current parameters and fails loudly instead.
static void check_plan(const BatchPlan& pl, const std::vector<wt_grid*>& members) {
  size_t q = 0;
  for (wt_grid* g : members) {
    const int32_t fp = g->prm.precision == WT_FP32_TENDENCY ? 1 : 0;
    for (auto& lp : g->lev) {
      if (q >= pl.levels.size()) throw std::runtime_error("step plan does not cover every level");
      const BatchLevel& b = pl.levels[q++];
      const PhysParams p = phys(g);
      if (b.fp32 != fp || b.ph.g != p.g || b.ph.H != p.H || b.ph.nu != p.nu || b.ph.adv != p.adv ||
          b.dh != lp->work.dh || b.G != total_flux(lp->work, p))
        throw std::runtime_error("step plan built for other parameters than the grid's current ones");
    }
  }
  if (q != pl.levels.size()) throw std::runtime_error("step plan holds other levels than the members'");
  for (const BatchJob& jb : pl.jobs) {
    const bool on_level = jb.kind == BK_VERTEX || jb.kind == BK_EDGE_CELL || jb.kind == BK_Q || jb.kind == BK_DIV ||
                          jb.kind == BK_TEND;
    const int lev = on_level ? jb.a : pl.pairs.at(size_t(jb.a)).c;
    if (jb.fp32 != pl.levels.at(size_t(lev)).fp32)
      throw std::runtime_error("step plan job precision differs from its level's");
  }
}

// the step with a ready plan: launches only (capturable)
static void ml_step_phases(wt_grid* g) {
  check_plan(g->splan, {g});
  if (g->splan_dense != dense_finest(g) || g->splan_dense2 != dense_second(g))
    throw std::runtime_error("step plan built for another choice of the finest levels' kernels");
  ++g->state_ver;
  LevelState& fl = *g->lev.back();
  LevelState& sl = *g->lev[g->lev.size() - 2];
  const PhysParams p = phys(g);
  for (const PhaseArgs& a : g->sphase) {
    if (a.j0 < 0 && a.j0 >= -4) {
      // marker of the finest level's masked lattice launch of stage -1 - j0
      dense_stage(g, fl, rk_stage(g->prm.rk, -1 - a.j0, fl.work, g->splan_dt), p, fp32_of(g));
    } else if (a.j0 < 0) {
      // marker of the intermediates-only launch of the level below, stage -5 - j0
      dense_stage(g, sl, rk_stage(g->prm.rk, -5 - a.j0, sl.work, g->splan_dt), p, fp32_of(g), true);
    } else {
      phase_launch(g->splan, a, g->stream);
    }
  }
}

static void ml_step_run(wt_grid* g, double dt) {
  if (phase_plan_ready(g, dt)) ml_step_phases(g);
  else ml_step(g, dt);
}

int wt_step(wt_grid* g, double dt) {
  GridScope scope_(g);
  if (!g) return fail(WT_EINVAL, "wt_step: null grid");
  if (!g->have_state) return fail(WT_ESTATE, "wt_step: call wt_set_state first");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(WT_EINVAL, "wt_step: dt must be positive");
  try {
    if (g->multi()) {
      ml_step_run(g, dt);
      if (g->gated) {
        // the exact threshold test judges the learned zone; a miss redoes the step from the
        // state before the gated adapt with the blanket zone
        g->gated = false;
        if (judge_gated_step(g) > 0) {
          snapshot(g, true);
          adapt_impl(g, g->last_eps, nullptr, nullptr, false);
          ml_step_run(g, dt);
          ++g->redo;
        }
      }
    } else {
      uniform_step(g, g->L(g->jmax), dt);
    }
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_step: ") + e.what());
  }
  return WT_OK;
}

int wt_adapt(wt_grid* g, double eps) {
  GridScope scope_(g);
  if (!g) return fail(WT_EINVAL, "wt_adapt: null grid");
  if (!g->have_state) return fail(WT_ESTATE, "wt_adapt: call wt_set_state first");
  if (!(eps >= 0) || !std::isfinite(eps)) return fail(WT_EINVAL, "wt_adapt: eps must be >= 0");
  if (!g->multi()) return WT_OK;
  try {
    const bool gate = g->predictor != nullptr;
    if (gate) snapshot(g, false);
    adapt_impl(g, eps, nullptr, nullptr, gate);
    g->gated = gate;
    g->last_eps = eps;
    HIPCHK(hipStreamSynchronize(g->stream));
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_adapt: ") + e.what());
  }
  return WT_OK;
}

int wt_set_predictor(wt_grid* g, wt_mlp* m, double threshold) {
  GridScope scope_(g);
  if (!g) return fail(WT_EINVAL, "wt_set_predictor: null grid");
  if (m && !(threshold >= 0.0 && threshold <= 1.5)) return fail(WT_EINVAL, "wt_set_predictor: threshold out of range");
  g->predictor = m;
  g->pred_thr = threshold;
  g->gated = false;
  return WT_OK;
}

int wt_debug_force_drop(wt_grid* g, int level, int64_t patch) {
  if (!g) return fail(WT_EINVAL, "wt_debug_force_drop: null grid");
  if (!g->predictor) return fail(WT_ESTATE, "wt_debug_force_drop: no predictor set");
  if (level < g->jmin || level > g->jmax || !learnable(g, level))
    return fail(WT_EINVAL, "wt_debug_force_drop: level has no patches");
  const int64_t m = (int64_t(1) << level) / 8;
  if (patch < 0 || patch >= 10 * m * m) return fail(WT_EINVAL, "wt_debug_force_drop: patch out of range");
  g->force_drop.emplace_back(level, patch);
  return WT_OK;
}

int wt_set_step_phases(wt_grid* g, int enable) {
  GridScope scope_(g);
  if (!g) return fail(WT_EINVAL, "wt_set_step_phases: null grid");
  try {
    HIPCHK(hipStreamSynchronize(g->stream));
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_set_step_phases: ") + e.what());
  }
  g->step_phases = enable != 0;
  return WT_OK;
}

int wt_set_work_lists(wt_grid* g, int enable) {
  GridScope scope_(g);
  if (!g) return fail(WT_EINVAL, "wt_set_work_lists: null grid");
  ++g->state_ver;
  try {
    g->use_lists = enable != 0;
    build_work_lists(g);
    HIPCHK(hipStreamSynchronize(g->stream));
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_set_work_lists: ") + e.what());
  }
  return WT_OK;
}

int wt_set_dense_levels(wt_grid* g, double min_fraction) {
  GridScope scope_(g);
  if (!g) return fail(WT_EINVAL, "wt_set_dense_levels: null grid");
  if (!(min_fraction >= 0.0) || !std::isfinite(min_fraction))
    return fail(WT_EINVAL, "wt_set_dense_levels: min_fraction must be finite and >= 0 (above 1: off)");
  try {
    if (min_fraction <= 1.0 && g->multi()) {
      LevelState& l = g->L(g->jmax);
      if (!l.lat.ok) {
        if (g->jmax < 6)
          return fail(WT_EINVAL, "wt_set_dense_levels: the finest level has no lattice form below level 6");
        auto lv = cached_level(g->jmax, g->prm.radius, g->prm.omega);
        LatticeHost lh;
        if (!build_lattice(*lv, lh)) return fail(WT_EINVAL, "wt_set_dense_levels: no regular tiles");
        upload_lattice(lh, l.lat);
      }
      // the level below it, when it has a lattice form (level 6 and up)
      LevelState& l2 = g->L(g->jmax - 1);
      if (!l2.lat.ok && g->jmax - 1 >= 6) {
        auto lv = cached_level(g->jmax - 1, g->prm.radius, g->prm.omega);
        LatticeHost lh;
        if (build_lattice(*lv, lh)) upload_lattice(lh, l2.lat);
      }
    }
    g->dense_min = min_fraction;
    update_tile_flags(g);
    touch_epoch(g);
  } catch (const std::bad_alloc&) {
    return fail(WT_ENOMEM, "wt_set_dense_levels: out of memory");
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_set_dense_levels: ") + e.what());
  }
  return WT_OK;
}

int wt_set_dense_min_tiles(wt_grid* g, int min_tiles) {
  GridScope scope_(g);
  if (!g) return fail(WT_EINVAL, "wt_set_dense_min_tiles: null grid");
  if (min_tiles < -1) return fail(WT_EINVAL, "wt_set_dense_min_tiles: min_tiles must be >= -1");
  try {
    g->dense2_min_tiles = min_tiles;
    touch_epoch(g);
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_set_dense_min_tiles: ") + e.what());
  }
  return WT_OK;
}

int wt_redo_count(const wt_grid* g, int64_t* redo) {
  if (!g || !redo) return fail(WT_EINVAL, "wt_redo_count: null argument");
  *redo = g->redo;
  return WT_OK;
}

int64_t wt_patch_count(const wt_grid* g, int level) {
  if (!g) return fail(WT_EINVAL, "wt_patch_count: null grid");
  if (level < g->jmin || level > g->jmax) return fail(WT_EINVAL, "wt_patch_count: level out of range");
  if (!learnable(g, level)) return 0;
  const int64_t m = (int64_t(1) << level) / 8;
  return 10 * m * m;
}

// Details of every point of the current state (after a listed pass only the support was fresh).
static void dense_details(wt_grid* g) {
  if (!g->details_partial) return;
  std::vector<double*> dh = state_dh(g), u = state_u(g);
  prolong_all(g, dh, u);
  details_all(g, dh, u);
}

static int patch_data(wt_grid* g, int level, float* out, bool labels, const char* who) {
  if (!g || !out) return fail(WT_EINVAL, std::string(who) + ": null argument");
  if (!g->have_state) return fail(WT_ESTATE, std::string(who) + ": call wt_set_state first");
  if (level < g->jmin || level > g->jmax || !learnable(g, level))
    return fail(WT_EINVAL, std::string(who) + ": level has no patches (needs jmin < level < jmax, level >= 3)");
  try {
    dense_details(g);
    learn_stats_all(g, g->last_eh, g->last_eu);
    LevelState& l = g->L(level);
    if (labels) learn_labels(l.npatch, l.stats, out, g->stream);
    else learn_features(l.npatch, 1 << level, level_pos(g, level), l.stats, out, g->stream);
    HIPCHK(hipStreamSynchronize(g->stream));
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string(who) + ": " + e.what());
  }
  return WT_OK;
}

int wt_patch_features(wt_grid* g, int level, float* x_device) {
  GridScope scope_(g);
  return patch_data(g, level, x_device, false, "wt_patch_features");
}

int wt_patch_labels(wt_grid* g, int level, float* y_device) {
  GridScope scope_(g);
  return patch_data(g, level, y_device, true, "wt_patch_labels");
}

int wt_forward(wt_grid* g) {
  GridScope scope_(g);
  if (!g) return fail(WT_EINVAL, "wt_forward: null grid");
  ++g->state_ver;
  if (!g->have_state) return fail(WT_ESTATE, "wt_forward: call wt_set_state first");
  if (!g->multi()) return WT_OK;
  try {
    std::vector<double*> dh = state_dh(g), u = state_u(g);
    prolong_all(g, dh, u);
    details_all(g, dh, u);
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_forward: ") + e.what());
  }
  return WT_OK;
}

int wt_inverse(wt_grid* g) {
  GridScope scope_(g);
  if (!g) return fail(WT_EINVAL, "wt_inverse: null grid");
  ++g->state_ver;
  if (!g->have_state) return fail(WT_ESTATE, "wt_inverse: call wt_set_state first");
  if (!g->multi()) return WT_OK;
  try {
    std::vector<double*> dh = state_dh(g), u = state_u(g);
    prolong_all(g, dh, u);
    details_all(g, dh, u);
    inverse_all(g, dh, u, false);
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_inverse: ") + e.what());
  }
  return WT_OK;
}

int wt_get_details(wt_grid* g, int level, double* dh, double* dpair, double* dint) {
  GridScope scope_(g);
  if (!g || level <= g->jmin || level > g->jmax) return fail(WT_EINVAL, "wt_get_details: bad level");
  try {
    if (g->have_state) dense_details(g);
    PairState& P = g->P(level - 1);
    const LevelState& C = g->L(level - 1);
    if (dh) HIPCHK(hipMemcpyAsync(dh, P.d_h, C.tab.E * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    if (dpair) HIPCHK(hipMemcpyAsync(dpair, P.d_p, C.tab.E * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    if (dint) HIPCHK(hipMemcpyAsync(dint, P.d_i, 3 * C.tab.T * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_get_details: ") + e.what());
  }
  return WT_OK;
}

int wt_set_mask(wt_grid* g, int level, const uint8_t* na, const uint8_t* ea) {
  GridScope scope_(g);
  if (bad_level(g, level) || !na || !ea) return fail(WT_EINVAL, "wt_set_mask: bad argument");
  ++g->state_ver;
  try {
    LevelState& l = g->L(level);
    HIPCHK(hipMemcpyAsync(l.na, na, l.tab.N, hipMemcpyHostToDevice, g->stream));
    HIPCHK(hipMemcpyAsync(l.ea, ea, l.tab.E, hipMemcpyHostToDevice, g->stream));
    build_work_lists(g);
    HIPCHK(hipStreamSynchronize(g->stream));
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_set_mask: ") + e.what());
  }
  return WT_OK;
}

int wt_tendency(wt_grid* g, int level, double* ddh, double* du) {
  GridScope scope_(g);
  if (bad_level(g, level)) return fail(WT_EINVAL, "wt_tendency: bad level");
  if (!g->have_state) return fail(WT_ESTATE, "wt_tendency: no state loaded");
  try {
    LevelState& ls = g->L(level);
    DevWork& w = ls.work;
    StageOut c{};
    c.d1 = 1.0;
    launch_stage(ls.tab, w, phys(g), g->prm.precision == WT_FP32_TENDENCY,
                 StagePtrs{w.dh, nullptr, w.dh, w.ddh, nullptr},
                 StagePtrs{w.u, nullptr, w.u, w.du, nullptr}, c, g->stream, nullptr, &ls.lat);
    if (ddh) HIPCHK(hipMemcpyAsync(ddh, w.ddh, ls.tab.N * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    if (du) HIPCHK(hipMemcpyAsync(du, w.du, ls.tab.E * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_tendency: ") + e.what());
  }
  return WT_OK;
}

// raw reductions of the finest level's reconstruction (multilevel) or state (uniform)
static void diag_fine(wt_grid* g, double* r) {
  LevelState& ls = g->L(g->jmax);
  if (g->multi()) {
    std::vector<double*> rdh, ru;
    reconstruct(g, rdh, ru);
    launch_diagnostics(ls.tab, ls.work, phys(g), g->stream, r, rdh.back(), ru.back());
  } else {
    launch_diagnostics(ls.tab, ls.work, phys(g), g->stream, r);
  }
}

int wt_diagnostics(wt_grid* g, wt_diag* d) {
  GridScope scope_(g);
  if (!g || !d) return fail(WT_EINVAL, "wt_diagnostics: null argument");
  if (!g->have_state) return fail(WT_ESTATE, "wt_diagnostics: no state loaded");
  try {
    std::memset(d, 0, sizeof(*d));
    double r[8], r0[8];
    diag_fine(g, r);
    const Level& L = g->L(g->jmax).geo;
    double A_S = 0;
    for (double a : L.A_i) A_S += a;
    double c2 = g->prm.gravity * r[0] / A_S;
    d->mass_reconstructed = r[0];
    d->energy = r[1] - 0.5 * c2 * c2 * A_S;
    double nonfinite = r[4];
    if (g->multi()) {
      LevelState& l0 = g->L(g->jmin);
      launch_diagnostics(l0.tab, l0.work, phys(g), g->stream, r0);
      d->mass = r0[0];
      nonfinite += r0[4];
      masked_max_all(g, &d->max_abs_dh, &d->max_abs_u);
    } else {
      d->mass = r[0];
      d->max_abs_dh = r[2];
      d->max_abs_u = r[3];
    }
    for (int j = g->jmin; j <= g->jmax && j < 16; ++j) {
      LevelState& l = g->L(j);
      double cn, ce;
      ml_count(l.tab.N, l.na, l.work.red, l.work.red + 4096, g->stream);
      HIPCHK(hipMemcpyAsync(&cn, l.work.red + 4096, sizeof(double), hipMemcpyDeviceToHost, g->stream));
      HIPCHK(hipStreamSynchronize(g->stream));
      ml_count(l.tab.E, l.ea, l.work.red, l.work.red + 4096, g->stream);
      HIPCHK(hipMemcpyAsync(&ce, l.work.red + 4096, sizeof(double), hipMemcpyDeviceToHost, g->stream));
      HIPCHK(hipStreamSynchronize(g->stream));
      d->active_nodes[j] = int64_t(cn);
      d->active_edges[j] = int64_t(ce);
      if (cn > 0 || ce > 0) d->finest_level = j;
    }
    if (nonfinite > 0) return fail(WT_ENUMERIC, "wt_diagnostics: non-finite values in the state");
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_diagnostics: ") + e.what());
  }
  return WT_OK;
}

double wt_suggest_dt(wt_grid* g, double cfl) {
  GridScope scope_(g);
  if (!g || !(cfl > 0)) { fail(WT_EINVAL, "wt_suggest_dt: bad argument"); return -1.0; }
  if (!g->have_state) { fail(WT_ESTATE, "wt_suggest_dt: no state loaded"); return -1.0; }
  try {
    double r[8];
    diag_fine(g, r);
    // the advection form has no gravity waves: the advective limit alone
    if (g->prm.equations == WT_ADVECTION) return cfl * r[6];
    return cfl * std::fmin(1.0 / r[5], r[6]);
  } catch (const std::exception& e) {
    fail(WT_EDEVICE, std::string("wt_suggest_dt: ") + e.what());
    return -1.0;
  }
}

int wt_set_allocator(wt_grid* g, void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx) {
  if ((alloc == nullptr) != (free_ == nullptr))
    return fail(WT_EINVAL, "wt_set_allocator: give both functions or neither");
  // the hook's own signature has no stream; the trampolines keep the caller's pair in ctx
  struct Pair {
    void* (*a)(size_t, void*);
    void (*f)(void*, void*);
    void* ctx;
  };
  AllocHook h;
  if (alloc) {
    // one record per distinct (alloc, free, ctx); records live as long as the process
    static std::mutex mu;
    static std::vector<std::unique_ptr<Pair>>* keep = new std::vector<std::unique_ptr<Pair>>();
    Pair* pr = nullptr;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (auto& x : *keep)
        if (x->a == alloc && x->f == free_ && x->ctx == ctx) pr = x.get();
      if (!pr) {
        keep->push_back(std::make_unique<Pair>(Pair{alloc, free_, ctx}));
        pr = keep->back().get();
      }
    }
    h.alloc = [](size_t bytes, void*, void* c) { auto* q = static_cast<Pair*>(c); return q->a(bytes, q->ctx); };
    h.free_ = [](void* p, void* c) {
      auto* q = static_cast<Pair*>(c);
      // the memory may be handed to other work as soon as it is returned: wait for all queued
      // device work first (hipFree does the same)
      (void)hipDeviceSynchronize();
      q->f(p, q->ctx);
    };
    h.ctx = pr;
  }
  if (g) g->hook = h;
  else set_default_hook(h);
  return WT_OK;
}

int wt_alloc_stats(const wt_grid* g, int64_t* n_hook, int64_t* bytes_hook, int64_t* n_direct,
                   int64_t* bytes_direct) {
  if (!g) return fail(WT_EINVAL, "wt_alloc_stats: null grid");
  alloc_stats(g, n_hook, bytes_hook, n_direct, bytes_direct);
  return WT_OK;
}

int wt_set_stream(wt_grid* g, void* s) {
  if (!g) return fail(WT_EINVAL, "wt_set_stream: null grid");
  g->stream = s ? static_cast<hipStream_t>(s) : g->own;
  return WT_OK;
}

int wt_timing_enable(wt_grid* g, int enable) {
  if (!g) return fail(WT_EINVAL, "wt_timing_enable: null grid");
  g->timer.enabled = enable != 0;
  return WT_OK;
}

int wt_timing_reset(wt_grid* g) {
  if (!g) return fail(WT_EINVAL, "wt_timing_reset: null grid");
  (void)hipStreamSynchronize(g->stream);
  for (auto& r : g->timer.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g->timer.recs.clear();
  return WT_OK;
}

int wt_kernel_units(wt_grid* g, const char* name, int64_t* units) {
  if (!g || !name || !units) return fail(WT_EINVAL, "wt_kernel_units: null argument");
  int k = -1;
  for (int q = 0; q < K_COUNT; ++q)
    if (std::strcmp(name, kKernelNames[q]) == 0) k = q;
  if (k < 0) return fail(WT_EINVAL, std::string("wt_kernel_units: unknown kernel ") + name);
  *units = 0;
  for (auto& r : g->timer.recs)
    if (r.k == k) *units = r.units;
  return WT_OK;
}

int wt_kernel_time(wt_grid* g, const char* name, double* total_ms, int64_t* launches, double* total_bytes) {
  if (!g || !name || !total_ms || !launches) return fail(WT_EINVAL, "wt_kernel_time: null argument");
  int k = -1;
  for (int q = 0; q < K_COUNT; ++q)
    if (std::strcmp(name, kKernelNames[q]) == 0) k = q;
  if (k < 0) return fail(WT_EINVAL, std::string("wt_kernel_time: unknown kernel ") + name);
  double tot = 0, by = 0;
  int64_t cnt = 0;
  for (auto& r : g->timer.recs) {
    if (r.k != k) continue;
    by += r.bytes;
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(WT_EDEVICE, "wt_kernel_time: event");
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(WT_EDEVICE, "wt_kernel_time: elapsed");
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  if (total_bytes) *total_bytes = by;
  return WT_OK;
}

int wt_host_level_tables(int level, double radius, double omega, double* A_i, double* A_v,
                         double* d_e, double* l_e, int32_t* e_nodes, int32_t* ecp, double* w) {
  if (level < 0 || level > 9) return fail(WT_EINVAL, "wt_host_level_tables: level must be 0..9");
  if (!(radius > 0)) return fail(WT_EINVAL, "wt_host_level_tables: radius must be positive");
  try {
    Level L;
    build_level(level, radius, omega, L);
    if (A_i) std::memcpy(A_i, L.A_i.data(), L.N * sizeof(double));
    if (A_v) std::memcpy(A_v, L.A_v.data(), L.T * sizeof(double));
    if (d_e) std::memcpy(d_e, L.d_e.data(), L.E * sizeof(double));
    if (l_e) std::memcpy(l_e, L.l_e.data(), L.E * sizeof(double));
    if (e_nodes) std::memcpy(e_nodes, L.e_c.data(), 2 * L.E * sizeof(int32_t));
    if (ecp) std::memcpy(ecp, L.ecp.data(), 10 * L.E * sizeof(int32_t));
    if (w) std::memcpy(w, L.w.data(), 10 * L.E * sizeof(double));
  } catch (const std::bad_alloc&) {
    return fail(WT_ENOMEM, "wt_host_level_tables: out of memory");
  }
  return WT_OK;
}

int wt_host_pair_tables(int jc, int jmax, double radius, double omega, int32_t* cells, double* st,
                        double* s_upd, double* A_c, int32_t* v_sten, double* w_int, double* w_pl,
                        double* w_pr, int32_t* rf_f, double* rf_fw, int32_t* rf_c, double* rf_cw) {
  if (jc < 0 || jmax <= jc || jmax > 8) return fail(WT_EINVAL, "wt_host_pair_tables: need 0 <= jc < jmax <= 8");
  try {
    std::vector<Level> L(jmax - jc + 1);
    for (int j = jc; j <= jmax; ++j) build_level(j, radius, omega, L[j - jc]);
    std::vector<double> A = L.back().A_i, Ac;
    PairTables P;
    for (int j = jmax - 1; j >= jc; --j) {
      P = PairTables{};
      build_pair(L[j - jc], L[j + 1 - jc], P);
      finish_pair(L[j - jc], L[j + 1 - jc], A, P, Ac);
      A.swap(Ac);
    }
    auto cp = [](auto* dst, const auto& v) {
      if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    };
    cp(cells, P.cells); cp(st, P.st); cp(s_upd, P.s_upd); cp(A_c, A); cp(v_sten, P.v_sten);
    cp(w_int, P.w_int); cp(w_pl, P.w_pl); cp(w_pr, P.w_pr); cp(rf_f, P.rf_f); cp(rf_fw, P.rf_fw);
    cp(rf_c, P.rf_c); cp(rf_cw, P.rf_cw);
  } catch (const std::bad_alloc&) {
    return fail(WT_ENOMEM, "wt_host_pair_tables: out of memory");
  }
  return WT_OK;
}

int wt_host_lattice_check(int level, int64_t* n_tiles, int64_t* n_rim, double* max_rel_err) {
  if (level < 6 || level > 9) return fail(WT_EINVAL, "wt_host_lattice_check: level must be 6..9");
  try {
    Level L;
    build_level(level, 6.371e6, 7.292e-5, L);
    LatticeHost h;
    if (!build_lattice(L, h)) return fail(WT_EINVAL, "wt_host_lattice_check: no regular tiles");
    const int64_t n = L.n, W = h.W, W2 = h.W2;
    double err = 0;
    auto rel = [&](double a, double b) { err = std::fmax(err, std::fabs(a / b - 1.0)); };
    for (int Lz = 0; Lz < 10; ++Lz)
      for (int64_t i = 1; i < n - 1; ++i)
        for (int64_t j = 1; j < n - 1; ++j) {
          if ((i < 4 && j < 4) || (i > n - 5 && j > n - 5) || (i < 4 && j > n - 5) || (i > n - 5 && j < 4)) continue;
          int64_t id = (int64_t(Lz) * n + i) * n + j, p = (i + LT_G) * W + (j + LT_G);
          rel(1.0 / L.A_i[id], h.tab[LQ_INVA * W2 + p]);
          for (int d = 0; d < 3; ++d) {
            int64_t e = 3 * id + d;
            rel(L.l_e[e], h.tab[(LQ_LEN + d) * W2 + p]);
            rel(1.0 / L.d_e[e], h.tab[(LQ_INVD + d) * W2 + p]);
            double a[10], b[10];
            for (int k = 0; k < 10; ++k) {
              a[k] = L.w[10 * e + k] * L.l_e[L.ecp[10 * e + k]] / L.d_e[e];
              b[k] = h.tab[(LQ_WL + 10 * d + k) * W2 + p];
            }
            std::sort(a, a + 10);
            std::sort(b, b + 10);
            double scale = std::fmax(std::fabs(a[0]), std::fabs(a[9]));
            for (int k = 0; k < 10; ++k) err = std::fmax(err, std::fabs(a[k] - b[k]) / scale);
          }
        }
    if (n_tiles) *n_tiles = int64_t(h.tiles.size() / 2);
    if (n_rim) *n_rim = int64_t(h.rim_elems.size());
    if (max_rel_err) *max_rel_err = err;
  } catch (const std::bad_alloc&) {
    return fail(WT_ENOMEM, "wt_host_lattice_check: out of memory");
  }
  return WT_OK;
}

// ---------------------------------------------------------------- ensemble
struct wt_ensemble {
  std::vector<wt_grid*> m;
  std::unique_ptr<MemberPool> pool;   // host threads of the members' adapts and threshold tests
  hipStream_t s0 = nullptr;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uint64_t> epochs;   // member epochs the graph (or the batch plan) was built with
  std::vector<char> phased;       // members captured in the merged-phase form
  // merged phases across members: one launch per phase over every member's jobs (graph form)
  bool merged = false;            // the current graph holds this form
  wt::BatchPlan mplan;
  std::vector<wt::PhaseDev> mphase;
  std::vector<double> dts;
  int64_t captures = 0, launches = 0;
  // batched persistent step
  bool batched = false;
  bool plan_ok = false;
  wt::BatchPlan plan;
  std::vector<int64_t> plan_sig;   // what the plan was built from
  hipEvent_t t0 = nullptr, t1 = nullptr;
  // launch-shape tuning: each candidate (workgroups per CU, chunk entries, work queue or
  // round-robin deal) runs one step, the fastest is kept
  struct Shape {
    int bpc, chunk;
    bool queue;
  };
  std::vector<Shape> cand;
  std::vector<float> cand_ms;
  int bpc = 0, chunk = 0;
  bool queue = false;
  bool tuned = false;
  float last_ms = 0.f;   // device time of the last batched launch
};

// The batched step replays the phases of ml_step for every member at once (same per-point code
// and the same dependencies: prolongation pair by pair upwards, intermediates, restriction pair
// by pair downwards, tendencies, per stage; then the partial height transform downwards).
// allow_dense (a single grid's merged-phase step): a member whose finest level is dense runs
// that level's tile elements through the masked lattice kernel, marked in the phase list by a
// phase with j0 = j1 = -1 - stage after the stage's prolongation, and only its rim through jobs.
static void build_batch_plan(const std::vector<wt_grid*>& members, const double* dt, BatchPlan& pl,
                             bool allow_dense) {
  pl.levels.clear();
  pl.pairs.clear();
  pl.jobs.clear();
  pl.phases.clear();
  struct MInfo {
    int lev0, pair0, jmin, jmax;
    bool wl, fp32, dense, dense2;
  };
  std::vector<MInfo> mi;
  int J0 = 1 << 30, J1 = -1;
  for (size_t k = 0; k < members.size(); ++k) {
    wt_grid* g = members[k];
    if (!g->multi()) throw std::runtime_error("the batched step needs multilevel members");
    MInfo x{int(pl.levels.size()), int(pl.pairs.size()), g->jmin, g->jmax, g->use_lists && g->lists_ok,
            g->prm.precision == WT_FP32_TENDENCY, allow_dense && dense_finest(g), allow_dense && dense_second(g)};
    if (x.dense && members.size() != 1) throw std::runtime_error("batched step: dense finest level of a member");
    const PhysParams p = phys(g);
    for (auto& lp : g->lev) {
      LevelState& l = *lp;
      BatchLevel bl{};
      bl.t = l.tab;
      bl.na = l.na;
      bl.ea = l.ea;
      bl.qv = l.work.qv;
      bl.B = l.work.B;
      bl.F = l.work.F;
      bl.qe = l.work.qe;
      bl.Q = l.work.Q;
      bl.c = l.work.c;
      bl.dh = l.work.dh;
      bl.ph = p;
      bl.G = total_flux(l.work, p);
      bl.fp32 = x.fp32;
      for (int st = 0; st < 4; ++st) {
        const StageSpec sp = rk_stage(g->prm.rk, st, l.work, dt[k]);
        bl.pdh[st] = sp.pdh;
        bl.pu[st] = sp.pu;
        bl.so[st] = sp.c;
      }
      pl.levels.push_back(bl);
    }
    for (int j = g->jmin; j < g->jmax; ++j)
      pl.pairs.push_back(BatchPair{g->P(j).dev, x.lev0 + (j - g->jmin), x.lev0 + (j + 1 - g->jmin), g->P(j).ph_det,
                                   g->P(j).ph_act});
    J0 = std::min(J0, g->jmin);
    J1 = std::max(J1, g->jmax);
    mi.push_back(x);
  }
  // jobs are appended phase by phase; a listed job reads its length on the device
  int32_t j0 = 0;
  auto job = [&](int kind, int a, int st, const MInfo& x, const WorkList& L, int64_t dense) {
    if (x.wl) {
      if (!L.idx || !L.dn) throw std::runtime_error("batched step: a member's work lists are not built");
      pl.jobs.push_back(BatchJob{kind, a, st, x.fp32 ? 1 : 0, L.idx, L.dn, L.bound});
    } else if (dense > 0) {
      pl.jobs.push_back(BatchJob{kind, a, st, x.fp32 ? 1 : 0, nullptr, nullptr, dense});
    }
  };
  // a fixed index list (the lattice rim of a dense finest level)
  auto fixed = [&](int kind, int a, int st, const MInfo& x, const int32_t* lst, int64_t n) {
    if (n > 0) pl.jobs.push_back(BatchJob{kind, a, st, x.fp32 ? 1 : 0, lst, nullptr, n});
  };
  auto flush = [&]() {
    const int32_t j1 = int32_t(pl.jobs.size());
    if (j1 > j0) pl.phases.push_back(BatchPhase{j0, j1});
    j0 = j1;
  };
  for (int st = 0; st < 4; ++st) {
    for (int j = J0; j < J1; ++j) {
      for (size_t k = 0; k < mi.size(); ++k)
        if (mi[k].jmin <= j && j < mi[k].jmax) {
          const PairState& P = members[k]->P(j);
          job(BK_PRO_EVEN, mi[k].pair0 + j - mi[k].jmin, st, mi[k], P.l_cn, P.dev.Nc);
        }
      flush();
      for (size_t k = 0; k < mi.size(); ++k)
        if (mi[k].jmin <= j && j < mi[k].jmax) {
          const PairState& P = members[k]->P(j);
          job(BK_PRO_ODD, mi[k].pair0 + j - mi[k].jmin, st, mi[k], P.l_ce, P.dev.Ec);
          job(BK_PRO_INT, mi[k].pair0 + j - mi[k].jmin, st, mi[k], P.l_ct, P.dev.Tc);
        }
      flush();
    }
    for (size_t k = 0; k < mi.size(); ++k) {
      if (mi[k].dense) pl.phases.push_back(BatchPhase{-1 - st, -1 - st});
      if (mi[k].dense2) pl.phases.push_back(BatchPhase{-5 - st, -5 - st});
    }
    const int kinds[3] = {BK_VERTEX, BK_EDGE_CELL, BK_Q};
    for (int kind : kinds) {
      for (size_t k = 0; k < mi.size(); ++k) {
        wt_grid* g = members[k];
        for (int q = 0; q < int(g->lev.size()); ++q) {
          const LevelState& l = *g->lev[q];
          if ((mi[k].dense && q + 1 == int(g->lev.size())) || (mi[k].dense2 && q + 2 == int(g->lev.size()))) {
            const DevLattice& lt = l.lat;
            if (kind == BK_VERTEX) fixed(kind, mi[k].lev0 + q, st, mi[k], lt.sup_tris, lt.n_sup_tris);
            else if (kind == BK_EDGE_CELL) fixed(kind, mi[k].lev0 + q, st, mi[k], lt.sup_elems, lt.n_sup_elems);
            else fixed(kind, mi[k].lev0 + q, st, mi[k], lt.rim_edges, lt.n_rim_edges);
            continue;
          }
          if (kind == BK_VERTEX) job(kind, mi[k].lev0 + q, st, mi[k], l.l_tri, l.tab.T);
          else if (kind == BK_EDGE_CELL) job(kind, mi[k].lev0 + q, st, mi[k], l.l_elem, l.tab.N);
          else job(kind, mi[k].lev0 + q, st, mi[k], l.l_edge, l.tab.E);
        }
      }
      flush();
    }
    for (int j = J1 - 1; j >= J0; --j) {
      for (size_t k = 0; k < mi.size(); ++k)
        if (mi[k].jmin <= j && j < mi[k].jmax) {
          const LevelState& F = members[k]->L(j + 1);
          if (mi[k].dense && j + 1 == mi[k].jmax)   // the tile nodes' divergence comes from the lattice
            fixed(BK_DIV, mi[k].lev0 + (j + 1 - mi[k].jmin), st, mi[k], F.lat.rim, F.lat.n_rim);
          else
            job(BK_DIV, mi[k].lev0 + (j + 1 - mi[k].jmin), st, mi[k], F.l_node, F.tab.N);
        }
      flush();
      for (size_t k = 0; k < mi.size(); ++k)
        if (mi[k].jmin <= j && j < mi[k].jmax) {
          const PairState& P = members[k]->P(j);
          job(BK_RES_E, mi[k].pair0 + j - mi[k].jmin, st, mi[k], P.l_ce, P.dev.Ec);
          job(BK_RES_B, mi[k].pair0 + j - mi[k].jmin, st, mi[k], P.l_cn, P.dev.Nc);
        }
      flush();
    }
    for (size_t k = 0; k < mi.size(); ++k) {
      wt_grid* g = members[k];
      for (int q = 0; q < int(g->lev.size()); ++q) {
        if (mi[k].dense && q + 1 == int(g->lev.size()))
          fixed(BK_TEND, mi[k].lev0 + q, st, mi[k], g->lev[q]->lat.rim, g->lev[q]->lat.n_rim);
        else
          job(BK_TEND, mi[k].lev0 + q, st, mi[k], g->lev[q]->l_tend, g->lev[q]->tab.N);
      }
    }
    flush();
  }
  // the partial transform pair by pair downwards, each in two passes: the details and stencil
  // activity of every coarse edge (whole pair, so none is stale), then the listed coarse nodes
  for (int j = J1 - 1; j >= J0; --j) {
    for (size_t k = 0; k < mi.size(); ++k)
      if (mi[k].jmin <= j && j < mi[k].jmax) {
        const PairState& P = members[k]->P(j);
        if (mi[k].wl ? P.l_cn.bound > 0 : P.dev.Nc > 0)
          fixed(BK_PARTIAL_D, mi[k].pair0 + j - mi[k].jmin, 0, mi[k], nullptr, P.dev.Ec);
      }
    flush();
    for (size_t k = 0; k < mi.size(); ++k)
      if (mi[k].jmin <= j && j < mi[k].jmax) {
        const PairState& P = members[k]->P(j);
        job(BK_PARTIAL_H, mi[k].pair0 + j - mi[k].jmin, 0, mi[k], P.l_cn, P.dev.Nc);
      }
    flush();
  }
}

static void batched_step(wt_ensemble* e, const double* dt) {
  const size_t n = e->m.size();
  if (e->cand.empty()) {
    const int maxb = batch_max_blocks_per_cu();
    if (maxb < 1) throw std::runtime_error("the batch kernel does not fit on a CU");
    for (int b : {1, 2})
      if (b <= maxb)
        for (int c : {256, 1024})
          for (bool q : {false, true}) e->cand.push_back({b, c, q});
    e->bpc = e->cand[0].bpc;
    e->chunk = e->cand[0].chunk;
    e->queue = e->cand[0].queue;
  }
  // launch shape of this step: the next untried candidate while tuning
  int bpc = e->bpc, chunk = e->chunk;
  bool queue = e->queue;
  const size_t tried = e->cand_ms.size();
  if (!e->tuned) {
    bpc = e->cand[tried].bpc;
    chunk = e->cand[tried].chunk;
    queue = e->cand[tried].queue;
  }
  // what the plan depends on: list use, list and mask addresses, levels, parameters, time steps
  // (not the list lengths, which the kernel reads on the device)
  std::vector<int64_t> sig;
  for (size_t k = 0; k < n; ++k) {
    wt_grid* g = e->m[k];
    sig.push_back(g->use_lists && g->lists_ok);
    sig.push_back(g->jmin);
    sig.push_back(g->jmax);
    sig.push_back(g->prm.rk);
    sig.push_back(g->prm.precision);
    int64_t bits = 0;
    std::memcpy(&bits, &dt[k], sizeof(bits));
    sig.push_back(bits);
    std::memcpy(&bits, &g->prm.gravity, sizeof(bits));
    sig.push_back(bits);
    std::memcpy(&bits, &g->prm.mean_depth, sizeof(bits));
    sig.push_back(bits);
    std::memcpy(&bits, &g->prm.viscosity, sizeof(bits));
    sig.push_back(bits);
    sig.push_back(g->prm.equations);
    for (auto& l : g->lev) {
      for (const WorkList* L : {&l->l_tri, &l->l_elem, &l->l_edge, &l->l_node, &l->l_tend}) {
        sig.push_back(reinterpret_cast<int64_t>(L->idx));
        sig.push_back(reinterpret_cast<int64_t>(L->dn));
      }
      sig.push_back(reinterpret_cast<int64_t>(l->na));
      sig.push_back(reinterpret_cast<int64_t>(l->ea));
    }
    for (auto& p : g->pairs)
      for (const WorkList* L : {&p->l_cn, &p->l_ce, &p->l_ct}) {
        sig.push_back(reinterpret_cast<int64_t>(L->idx));
        sig.push_back(reinterpret_cast<int64_t>(L->dn));
      }
  }
  if (!e->plan_ok || sig != e->plan_sig) {
    build_batch_plan(e->m, dt, e->plan);
    e->plan.upload(e->s0);
    e->plan_ok = true;
    e->plan_sig.swap(sig);
    ++e->captures;
  }
  // members' own streams are idle here (their adapts synchronise)
  if (!e->t0) {
    HIPCHK(hipEventCreate(&e->t0));
    HIPCHK(hipEventCreate(&e->t1));
  }
  HIPCHK(hipEventRecord(e->t0, e->s0));
  check_plan(e->plan, e->m);
  batch_launch(e->plan, bpc, chunk, queue, e->s0);
  HIPCHK(hipEventRecord(e->t1, e->s0));
  batch_check(e->plan, e->s0);
  ++e->launches;
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, e->t0, e->t1));
  e->last_ms = ms;
  if (!e->tuned) {
    e->cand_ms.push_back(ms);
    if (e->cand_ms.size() == e->cand.size()) {
      const size_t best = size_t(std::min_element(e->cand_ms.begin(), e->cand_ms.end()) - e->cand_ms.begin());
      e->bpc = e->cand[best].bpc;
      e->chunk = e->cand[best].chunk;
      e->queue = e->cand[best].queue;
      e->tuned = true;
    }
  }
}

wt_ensemble* wt_ensemble_create(wt_grid* const* members, int n) {
  if (!members || n < 1) {
    fail(WT_EINVAL, "wt_ensemble_create: need at least one member");
    return nullptr;
  }
  for (int k = 0; k < n; ++k)
    for (int q = 0; q < k; ++q)
      if (!members[k] || members[k] == members[q] || members[k]->stream == members[q]->stream) {
        fail(WT_EINVAL, "wt_ensemble_create: members must be distinct grids on distinct streams");
        return nullptr;
      }
  if (!members[0]) {
    fail(WT_EINVAL, "wt_ensemble_create: null member");
    return nullptr;
  }
  auto* e = new wt_ensemble;
  try {
    e->m.assign(members, members + n);
    e->pool = std::make_unique<MemberPool>();
    HIPCHK(hipStreamCreateWithFlags(&e->s0, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&e->fork, hipEventDisableTiming));
    e->join.resize(n);
    for (auto& j : e->join) HIPCHK(hipEventCreateWithFlags(&j, hipEventDisableTiming));
  } catch (const std::exception& x) {
    fail(WT_EDEVICE, std::string("wt_ensemble_create: ") + x.what());
    delete e;
    return nullptr;
  }
  return e;
}

void wt_ensemble_destroy(wt_ensemble* e) {
  if (!e) return;
  if (e->s0) (void)hipStreamSynchronize(e->s0);
  e->plan.release();
  e->mplan.release();
  if (e->t0) (void)hipEventDestroy(e->t0);
  if (e->t1) (void)hipEventDestroy(e->t1);
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  if (e->graph) (void)hipGraphDestroy(e->graph);
  for (auto& j : e->join)
    if (j) (void)hipEventDestroy(j);
  if (e->fork) (void)hipEventDestroy(e->fork);
  if (e->s0) (void)hipStreamDestroy(e->s0);
  delete e;
}

int wt_ensemble_adapt(wt_ensemble* e, const double* eps) {
  if (!e || !eps) return fail(WT_EINVAL, "wt_ensemble_adapt: null argument");
  return e->pool->run(e->m.size(), [&](size_t k) { return wt_adapt(e->m[k], eps[k]); });
}

int wt_ensemble_step(wt_ensemble* e, const double* dt) {
  if (!e || !dt) return fail(WT_EINVAL, "wt_ensemble_step: null argument");
  const size_t n = e->m.size();
  for (size_t k = 0; k < n; ++k) {
    if (!e->m[k]->have_state) return fail(WT_ESTATE, "wt_ensemble_step: a member has no state");
    if (!(dt[k] > 0) || !std::isfinite(dt[k])) return fail(WT_EINVAL, "wt_ensemble_step: dt must be positive");
  }
  try {
    for (auto* m : e->m)
      if (m->multi()) touch_epoch(m);   // the signatures below see every change of the launches
    bool stale = !e->exec || e->dts.size() != n;
    for (size_t k = 0; k < n && !stale; ++k) stale = e->epochs[k] != e->m[k]->epoch || e->dts[k] != dt[k];
    bool merged = false;
    if (e->batched) {
      batched_step(e, dt);
    } else {
      // every member listed and multilevel: one launch per phase over all members' jobs
      merged = true;
      for (auto* m : e->m) merged = merged && m->multi() && m->step_phases && m->use_lists && m->lists_ok;
      if (merged) {
        if (stale || !e->merged) {
          build_batch_plan(e->m, dt, e->mplan);
          e->mplan.upload(e->s0);
          phase_prepare_dev(e->mplan, e->mphase, e->s0);
          stale = true;
        }
      } else {
        // members whose merged-phase plan had to be rebuilt change their launches
        std::vector<char> phased(n);
        for (size_t k = 0; k < n; ++k) {
          wt_grid* m = e->m[k];
          const bool had = !m->sphase.empty() && m->splan_sig == m->step_sig && m->splan_dt == dt[k];
          GridScope scope(m);
          phased[k] = m->multi() && phase_plan_ready(m, dt[k]);
          if (phased[k] && !had) stale = true;
        }
        if (phased != e->phased || e->merged) stale = true;
        e->phased.swap(phased);
      }
    }
    if (!e->batched && stale) {
      // capture the merged phases on s0, or every member's step on its own stream, forked from
      // and joined into s0
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(e->s0, hipStreamCaptureModeRelaxed));
      try {
        if (merged) {
          check_plan(e->mplan, e->m);
          for (const auto& ph : e->mphase) phase_launch_dev(e->mplan, ph, e->s0);
        } else {
          HIPCHK(hipEventRecord(e->fork, e->s0));
          for (size_t k = 0; k < n; ++k) {
            wt_grid* m = e->m[k];
            HIPCHK(hipStreamWaitEvent(m->stream, e->fork, 0));
            if (e->phased[k]) ml_step_phases(m);
            else if (m->multi()) ml_step(m, dt[k]);
            else uniform_step(m, m->L(m->jmax), dt[k]);
            HIPCHK(hipEventRecord(e->join[k], m->stream));
            HIPCHK(hipStreamWaitEvent(e->s0, e->join[k], 0));
          }
        }
      } catch (...) {
        hipGraph_t dropped = nullptr;
        (void)hipStreamEndCapture(e->s0, &dropped);
        if (dropped) (void)hipGraphDestroy(dropped);
        throw;
      }
      HIPCHK(hipStreamEndCapture(e->s0, &g));
      bool updated = false;
      if (e->exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        updated = hipGraphExecUpdate(e->exec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
        if (!updated) {
          (void)hipGetLastError();
          HIPCHK(hipGraphExecDestroy(e->exec));
          e->exec = nullptr;
        }
      }
      if (!updated) HIPCHK(hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0));
      if (e->graph) HIPCHK(hipGraphDestroy(e->graph));
      e->graph = g;
      e->epochs.resize(n);
      for (size_t k = 0; k < n; ++k) e->epochs[k] = e->m[k]->epoch;
      e->dts.assign(dt, dt + n);
      e->merged = merged;
      ++e->captures;
    }
    if (!e->batched) {
      HIPCHK(hipGraphLaunch(e->exec, e->s0));
      HIPCHK(hipStreamSynchronize(e->s0));
      ++e->launches;
    }
    for (auto* m : e->m) ++m->state_ver;   // the launch stepped every member
  } catch (const std::exception& x) {
    return fail(WT_EDEVICE, std::string("wt_ensemble_step: ") + x.what());
  }
  // the threshold test of the learned zone needs the host: each member judged (and redone if
  // needed) on its own stream, members spread over host threads
  return e->pool->run(n, [&](size_t k) {
    wt_grid* m = e->m[k];
    if (!m->multi() || !m->gated) return int(WT_OK);
    GridScope scope(m);
    try {
      m->gated = false;
      if (judge_gated_step(m) > 0) {
        snapshot(m, true);
        adapt_impl(m, m->last_eps, nullptr, nullptr, false);
        ml_step_run(m, dt[k]);
        ++m->redo;
      }
      HIPCHK(hipStreamSynchronize(m->stream));
    } catch (const std::exception& x) {
      return fail(WT_EDEVICE, std::string("wt_ensemble_step: ") + x.what());
    }
    return int(WT_OK);
  });
}

int wt_ensemble_set_batched(wt_ensemble* e, int on) {
  if (!e) return fail(WT_EINVAL, "wt_ensemble_set_batched: null ensemble");
  if (on) {
    for (auto* g : e->m)
      if (!g->multi()) return fail(WT_EINVAL, "wt_ensemble_set_batched: every member must have jmin < jmax");
  }
  try {
    HIPCHK(hipStreamSynchronize(e->s0));
  } catch (const std::exception& x) {
    return fail(WT_EDEVICE, std::string("wt_ensemble_set_batched: ") + x.what());
  }
  e->batched = on != 0;
  // the next step rebuilds what the mode launches
  e->plan_ok = false;
  if (e->exec) {
    (void)hipGraphExecDestroy(e->exec);
    e->exec = nullptr;
  }
  return WT_OK;
}

int wt_ensemble_tuning(const wt_ensemble* e, int* blocks_per_cu, int* chunk, int* queue, int* tuned,
                       float* last_ms) {
  if (!e) return fail(WT_EINVAL, "wt_ensemble_tuning: null ensemble");
  if (blocks_per_cu) *blocks_per_cu = e->bpc;
  if (chunk) *chunk = e->chunk;
  if (queue) *queue = e->queue ? 1 : 0;
  if (tuned) *tuned = e->tuned ? 1 : 0;
  if (last_ms) *last_ms = e->last_ms;
  return WT_OK;
}

int wt_ensemble_stats(const wt_ensemble* e, int64_t* captures, int64_t* launches) {
  if (!e) return fail(WT_EINVAL, "wt_ensemble_stats: null ensemble");
  if (captures) *captures = e->captures;
  if (launches) *launches = e->launches;
  return WT_OK;
}

}  // extern "C"
