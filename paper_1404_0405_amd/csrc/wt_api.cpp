// C ABI of libwt (declared in include/wt.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/wt.h"
#include "wt_grid.hpp"
#include "wt_internal.hpp"

using namespace wt;

static thread_local std::string g_err;

static int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)

struct LevelState {
  Level geo;         // host geometry
  DevTables tab;     // device tables
  DevWork work;      // device buffers
  bool full = false;  // state loaded on every point of the level
};

struct wt_grid {
  int jmin = 0, jmax = 0, patch = 8;
  wt_params prm{};
  std::vector<std::unique_ptr<LevelState>> lev;  // index j - jmin
  hipStream_t own = nullptr, stream = nullptr;
  bool have_state = false;
  Timer timer;
  LevelState& L(int j) { return *lev[j - jmin]; }
};

static void alloc_work(LevelState& ls) {
  const int64_t N = ls.tab.N, E = ls.tab.E, T = ls.tab.T;
  DevWork& w = ls.work;
  auto A = [](double** p, int64_t n) { HIPCHK(hipMalloc(p, n * sizeof(double))); HIPCHK(hipMemset(*p, 0, n * sizeof(double))); };
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
  A(&w.red, 8 * 1024 + 16);
}

static void free_work(DevWork& w) {
  void* ps[] = {w.dh, w.u, w.dh_acc, w.u_acc, w.dh_s[0], w.u_s[0], w.dh_s[1], w.u_s[1],
                w.ddh, w.du, w.qv, w.B, w.F, w.qe, w.red};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  w = DevWork{};
}

static PhysParams phys(const wt_grid* g) { return PhysParams{g->prm.gravity, g->prm.mean_depth}; }

extern "C" {

const char* wt_last_error(void) { return g_err.c_str(); }

const char* wt_kernel_names(void) { return "trisk_vertex,trisk_edge_cell,trisk_tend"; }

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
    g->prm.radius = 6.371e6;
    g->prm.omega = 7.292e-5;
    g->prm.gravity = 9.80616;
    g->prm.mean_depth = 2.94e4 / 9.80616;
    g->prm.rk = WT_RK4;
    g->prm.precision = WT_FP64;
    HIPCHK(hipStreamCreate(&g->own));
    g->stream = g->own;
    for (int j = jmin; j <= jmax; ++j) {
      auto ls = std::make_unique<LevelState>();
      build_level(j, g->prm.radius, g->prm.omega, ls->geo);
      upload_tables(ls->geo, ls->tab);
      alloc_work(*ls);
      g->lev.push_back(std::move(ls));
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
    free_work(ls->work);
  }
  if (g->own) (void)hipStreamDestroy(g->own);
  delete g;
}

int wt_set_params(wt_grid* g, const wt_params* p) {
  if (!g || !p) return fail(WT_EINVAL, "wt_set_params: null argument");
  if (p->radius != g->prm.radius || p->omega != g->prm.omega)
    return fail(WT_EINVAL, "wt_set_params: radius and omega are fixed at grid creation");
  if (!(p->gravity > 0) || !(p->mean_depth > 0))
    return fail(WT_EINVAL, "wt_set_params: gravity and mean_depth must be positive");
  if (p->rk != WT_RK4 && p->rk != WT_SSPRK43) return fail(WT_EINVAL, "wt_set_params: bad rk");
  if (p->precision != WT_FP64 && p->precision != WT_FP32_TENDENCY)
    return fail(WT_EINVAL, "wt_set_params: bad precision");
  g->prm = *p;
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
  if (!dh || !u) return fail(WT_EINVAL, "wt_set_state: null array");
  if (g->jmin != g->jmax) return fail(WT_EINVAL, "wt_set_state: adaptive grids not supported yet");
  try {
    LevelState& ls = g->L(level);
    HIPCHK(hipMemcpyAsync(ls.work.dh, dh, ls.tab.N * sizeof(double), k, g->stream));
    HIPCHK(hipMemcpyAsync(ls.work.u, u, ls.tab.E * sizeof(double), k, g->stream));
    if (k == hipMemcpyHostToDevice) HIPCHK(hipStreamSynchronize(g->stream));
    ls.full = true;
    g->have_state = true;
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_set_state: ") + e.what());
  }
  return WT_OK;
}

int wt_set_state(wt_grid* g, int level, const double* dh, const double* u) {
  return set_state_impl(g, level, dh, u, hipMemcpyHostToDevice);
}

int wt_set_state_device(wt_grid* g, int level, const void* dh, const void* u) {
  return set_state_impl(g, level, dh, u, hipMemcpyDeviceToDevice);
}

int wt_get_state(wt_grid* g, int level, double* dh, double* u, uint8_t* na, uint8_t* ea) {
  if (bad_level(g, level)) return fail(WT_EINVAL, "wt_get_state: bad level");
  if (!g->have_state) return fail(WT_ESTATE, "wt_get_state: no state loaded");
  try {
    LevelState& ls = g->L(level);
    if (dh) HIPCHK(hipMemcpyAsync(dh, ls.work.dh, ls.tab.N * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    if (u) HIPCHK(hipMemcpyAsync(u, ls.work.u, ls.tab.E * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    if (na) std::memset(na, ls.full ? 1 : 0, ls.tab.N);
    if (ea) std::memset(ea, ls.full ? 1 : 0, ls.tab.E);
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_get_state: ") + e.what());
  }
  return WT_OK;
}

// One Runge-Kutta step on a uniform level.
static void uniform_step(wt_grid* g, LevelState& ls, double dt) {
  DevWork& w = ls.work;
  const bool fp32 = g->prm.precision == WT_FP32_TENDENCY;
  PhysParams p = phys(g);
  auto P = [](const double* y, const double* acc, const double* x, double* o1, double* o2) {
    return StagePtrs{y, acc, x, o1, o2};
  };
  if (g->prm.rk == WT_RK4) {
    // acc = y + dt/6 k1 ; s0 = y + dt/2 k1 ; acc += dt/3 k2 ; s1 = y + dt/2 k2 ;
    // acc += dt/3 k3 ; s0 = y + dt k3 ; y = acc + dt/6 k4
    const double* X[4] = {w.dh, w.dh_s[0], w.dh_s[1], w.dh_s[0]};
    const double* XU[4] = {w.u, w.u_s[0], w.u_s[1], w.u_s[0]};
    double* O2[4] = {w.dh_s[0], w.dh_s[1], w.dh_s[0], nullptr};
    double* O2U[4] = {w.u_s[0], w.u_s[1], w.u_s[0], nullptr};
    const double bk[4] = {dt / 6, dt / 3, dt / 3, dt / 6};
    const double ck[4] = {dt / 2, dt / 2, dt, 0};
    for (int s = 0; s < 4; ++s) {
      StageOut c{};
      c.d1 = bk[s];
      if (s == 0) c.a1 = 1.0; else c.b1 = 1.0;
      c.a2 = 1.0; c.d2 = ck[s];
      double* o1 = s == 3 ? w.dh : w.dh_acc;
      double* o1u = s == 3 ? w.u : w.u_acc;
      launch_stage(ls.tab, w, p, fp32, P(w.dh, w.dh_acc, X[s], o1, O2[s]),
                   P(w.u, w.u_acc, XU[s], o1u, O2U[s]), c, g->stream, &g->timer);
    }
  } else {
    // y1 = y + dt/2 L(y); y2 = y1 + dt/2 L(y1); y3 = 2/3 y + 1/3 y2 + dt/6 L(y2);
    // y = y3 + dt/2 L(y3)
    StageOut c{};
    c.a1 = 1.0; c.d1 = dt / 2;
    launch_stage(ls.tab, w, p, fp32, P(w.dh, nullptr, w.dh, w.dh_s[0], nullptr),
                 P(w.u, nullptr, w.u, w.u_s[0], nullptr), c, g->stream, &g->timer);
    c = StageOut{}; c.c1 = 1.0; c.d1 = dt / 2;
    launch_stage(ls.tab, w, p, fp32, P(w.dh, nullptr, w.dh_s[0], w.dh_s[1], nullptr),
                 P(w.u, nullptr, w.u_s[0], w.u_s[1], nullptr), c, g->stream, &g->timer);
    c = StageOut{}; c.a1 = 2.0 / 3.0; c.c1 = 1.0 / 3.0; c.d1 = dt / 6;
    launch_stage(ls.tab, w, p, fp32, P(w.dh, nullptr, w.dh_s[1], w.dh_s[0], nullptr),
                 P(w.u, nullptr, w.u_s[1], w.u_s[0], nullptr), c, g->stream, &g->timer);
    c = StageOut{}; c.c1 = 1.0; c.d1 = dt / 2;
    launch_stage(ls.tab, w, p, fp32, P(w.dh, nullptr, w.dh_s[0], w.dh, nullptr),
                 P(w.u, nullptr, w.u_s[0], w.u, nullptr), c, g->stream, &g->timer);
  }
}

int wt_step(wt_grid* g, double dt) {
  if (!g) return fail(WT_EINVAL, "wt_step: null grid");
  if (!g->have_state) return fail(WT_ESTATE, "wt_step: call wt_set_state first");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(WT_EINVAL, "wt_step: dt must be positive");
  try {
    if (g->jmin == g->jmax) {
      uniform_step(g, g->L(g->jmax), dt);
    } else {
      return fail(WT_EINVAL, "wt_step: adaptive grids not supported yet");
    }
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_step: ") + e.what());
  }
  return WT_OK;
}

int wt_tendency(wt_grid* g, int level, double* ddh, double* du) {
  if (bad_level(g, level)) return fail(WT_EINVAL, "wt_tendency: bad level");
  if (!g->have_state) return fail(WT_ESTATE, "wt_tendency: no state loaded");
  try {
    LevelState& ls = g->L(level);
    DevWork& w = ls.work;
    StageOut c{};
    c.d1 = 1.0;
    launch_stage(ls.tab, w, phys(g), g->prm.precision == WT_FP32_TENDENCY,
                 StagePtrs{w.dh, nullptr, w.dh, w.ddh, nullptr},
                 StagePtrs{w.u, nullptr, w.u, w.du, nullptr}, c, g->stream, nullptr);
    if (ddh) HIPCHK(hipMemcpyAsync(ddh, w.ddh, ls.tab.N * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    if (du) HIPCHK(hipMemcpyAsync(du, w.du, ls.tab.E * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_tendency: ") + e.what());
  }
  return WT_OK;
}

static int diag_raw(wt_grid* g, double* r) {
  LevelState& ls = g->L(g->jmax);
  launch_diagnostics(ls.tab, ls.work, phys(g), g->stream, r);
  return WT_OK;
}

int wt_diagnostics(wt_grid* g, wt_diag* d) {
  if (!g || !d) return fail(WT_EINVAL, "wt_diagnostics: null argument");
  if (!g->have_state) return fail(WT_ESTATE, "wt_diagnostics: no state loaded");
  try {
    double r[8];
    diag_raw(g, r);
    std::memset(d, 0, sizeof(*d));
    const Level& L = g->L(g->jmax).geo;
    double A_S = 0;
    for (double a : L.A_i) A_S += a;
    double c2 = g->prm.gravity * r[0] / A_S;
    d->mass = r[0];
    d->energy = r[1] - 0.5 * c2 * c2 * A_S;
    d->max_abs_dh = r[2];
    d->max_abs_u = r[3];
    for (int j = g->jmin; j <= g->jmax; ++j) {
      if (j < 16) {
        d->active_nodes[j] = g->L(j).full ? g->L(j).tab.N : 0;
        d->active_edges[j] = g->L(j).full ? g->L(j).tab.E : 0;
      }
    }
    if (r[4] > 0) return fail(WT_ENUMERIC, "wt_diagnostics: non-finite values in the state");
  } catch (const std::exception& e) {
    return fail(WT_EDEVICE, std::string("wt_diagnostics: ") + e.what());
  }
  return WT_OK;
}

double wt_suggest_dt(wt_grid* g, double cfl) {
  if (!g || !(cfl > 0)) { fail(WT_EINVAL, "wt_suggest_dt: bad argument"); return -1.0; }
  if (!g->have_state) { fail(WT_ESTATE, "wt_suggest_dt: no state loaded"); return -1.0; }
  try {
    double r[8];
    diag_raw(g, r);
    return cfl * std::fmin(1.0 / r[5], r[6]);
  } catch (const std::exception& e) {
    fail(WT_EDEVICE, std::string("wt_suggest_dt: ") + e.what());
    return -1.0;
  }
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

int wt_kernel_time(wt_grid* g, const char* name, double* total_ms, int64_t* launches) {
  if (!g || !name || !total_ms || !launches) return fail(WT_EINVAL, "wt_kernel_time: null argument");
  int k = -1;
  for (int q = 0; q < K_COUNT; ++q)
    if (std::strcmp(name, kKernelNames[q]) == 0) k = q;
  if (k < 0) return fail(WT_EINVAL, std::string("wt_kernel_time: unknown kernel ") + name);
  double tot = 0;
  int64_t cnt = 0;
  for (auto& r : g->timer.recs) {
    if (r.k != k) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(WT_EDEVICE, "wt_kernel_time: event");
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(WT_EDEVICE, "wt_kernel_time: elapsed");
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
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

}  // extern "C"
