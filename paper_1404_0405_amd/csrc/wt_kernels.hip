// TRiSK stage kernels for gfx950 (table-driven form, one thread per element).
//
// One tendency evaluation of eqs. (height) and (velo) (Sec. 3.1) in three launches:
//   k_vertex     q_v = (zeta_v + f_v) / h_v at both triangles of the element
//   k_edge_cell  B_i = g dh_i + K_i at the node;  F_e = h_e u_e, q_e at its three edges
//   k_tend       d(dh)/dt = -div F at the node, du/dt = -Q_e - grad B at the edges, fused
//                with the Runge-Kutta stage combination (always in double)
// The viscous form (Sec. 3.1) adds -nu div u to B, -nu grad dh to the flux whose divergence is
// taken (G) and nu grad^perp curl u to Q; the advection form (Sec. 6.1) keeps u fixed.
// The compute type T is double, or float for the single-precision tendency mode; the
// divergence sum, the state and the stage combination are double in both.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <stdexcept>

#include "wt_alloc.hpp"
#include "wt_body.hpp"
#include "wt_internal.hpp"
#include "wt_lattice_dev.hpp"

#include <type_traits>

namespace wt {

const char* const kKernelNames[K_COUNT] = {"trisk_vertex", "trisk_edge_cell", "trisk_tend", "trisk_lattice",
                                             "trisk_lattice_masked", "trisk_lattice_inter"};

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)

constexpr int BS = 256;

template <typename T>
__global__ __launch_bounds__(BS) void k_vertex(int64_t n_tri, const int32_t* __restrict__ list, DevTables tb,
                                               const double* __restrict__ dh, const double* __restrict__ u,
                                               double H, T* __restrict__ qv) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  if (list) {
    t = list[t];
    if (t < 0) return;   // padding of a work list
  }
  body_vertex<T>(t, tb, dh, u, H, qv);
}

template <typename T>
__global__ __launch_bounds__(BS) void k_edge_cell(int64_t N, const int32_t* __restrict__ list, DevTables tb,
                                                  const double* __restrict__ dh, const double* __restrict__ u,
                                                  const T* __restrict__ qv, PhysParams ph, T* __restrict__ B,
                                                  double* __restrict__ F, double* __restrict__ G,
                                                  T* __restrict__ qe) {
  int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= N) return;
  if (list) {
    id = list[id];
    if (id < 0) return;   // padding of a work list
  }
  body_edge_cell<T>(id, tb, dh, u, qv, ph, B, F, G, qe);
}

__device__ __forceinline__ void rk_epilogue(int64_t i, double k, const StagePtrs& p,
                                            const StageOut& c) {
  if (p.o1) {
    double v = c.d1 * k;
    if (c.a1 != 0.0) v += c.a1 * p.y[i];
    if (c.b1 != 0.0) v += c.b1 * p.acc[i];
    if (c.c1 != 0.0) v += c.c1 * p.x[i];
    p.o1[i] = v;
  }
  if (p.o2) {
    double v = c.d2 * k;
    if (c.a2 != 0.0) v += c.a2 * p.y[i];
    if (c.b2 != 0.0) v += c.b2 * p.acc[i];
    if (c.c2 != 0.0) v += c.c2 * p.x[i];
    p.o2[i] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_tend(int64_t N, int64_t n_elem,
                                             const int32_t* __restrict__ list,
                                             const int32_t* __restrict__ c_e,
                                             const double* __restrict__ c_div,
                                             const int32_t* __restrict__ e_c,
                                             const double* __restrict__ inv_d,
                                             const int32_t* __restrict__ ecp,
                                             const double* __restrict__ wl,
                                             const T* __restrict__ B, const double* __restrict__ F,
                                             const double* __restrict__ G,
                                             const T* __restrict__ qe, StagePtrs pdh, StagePtrs pu,
                                             StageOut c, DevTables tb, double nu, int32_t adv) {
  int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= N) return;
  if (list) {
    id = list[id];
    if (id < 0) return;   // padding of a work list
  }
  double div = 0.0;  // divergence sums stay in double in both precisions
#pragma unroll
  for (int k = 0; k < 6; ++k) div += c_div[6 * id + k] * G[c_e[6 * id + k]];
  rk_epilogue(id, -div, pdh, c);
  if (id >= n_elem) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int64_t e = 3 * id + d;
    if (adv) {
      rk_epilogue(e, 0.0, pu, c);
      continue;
    }
    T q0 = qe[e];
    T Q = T(0);
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      int32_t ep = ecp[10 * e + k];
      Q += tv<T>(wl, tb.wl_f, 10 * e + k) * T(F[ep]) * (T(0.5) * (q0 + qe[ep]));
    }
    if (nu != 0.0)
      Q += T(nu) * (tri_curl<T>(tb.e_v[2 * e], tb, pu.x) - tri_curl<T>(tb.e_v[2 * e + 1], tb, pu.x)) / tv<T>(tb.l_e, tb.l_e_f, e);
    T gradB = (B[e_c[2 * e + 1]] - B[e_c[2 * e]]) * tv<T>(inv_d, tb.inv_d_f, e);
    rk_epilogue(e, double(-Q - gradB), pu, c);
  }
}

// ------------------------------------------------------------------ launch helpers
static inline unsigned nblk(int64_t n) { return unsigned((n + BS - 1) / BS); }

struct TimedLaunch {
  Timer* tm;
  int k;
  hipStream_t s;
  double bytes;
  hipEvent_t a = nullptr, b = nullptr;
  int64_t units;
  TimedLaunch(Timer* tm_, int k_, hipStream_t s_, double bytes_, int64_t units_)
      : tm(tm_), k(k_), s(s_), bytes(bytes_), units(units_) {
    if (tm && tm->enabled) {
      HIPCHK(hipEventCreate(&a));
      HIPCHK(hipEventCreate(&b));
      HIPCHK(hipEventRecord(a, s));
    }
  }
  ~TimedLaunch() {
    if (a) {
      hipEventRecord(b, s);
      tm->recs.push_back({k, a, b, bytes, units});
    }
  }
};

template <typename T>
static void stage_impl(const DevTables& t, DevWork& w, const PhysParams& p, const StagePtrs& sdh,
                       const StagePtrs& su, const StageOut& c_in, hipStream_t s, Timer* tm,
                       const DevLattice* lat) {
  // A stage array that is the stage input itself (the first stage reads y as x) is read once.
  StageOut c = c_in;
  if (sdh.y == sdh.x && su.y == su.x) {
    c.c1 += c.a1; c.a1 = 0.0;
    c.c2 += c.a2; c.a2 = 0.0;
  }
  if (sdh.acc == sdh.x && su.acc == su.x) {
    c.c1 += c.b1; c.b1 = 0.0;
    c.c2 += c.b2; c.b2 = 0.0;
  }
  T* qv = static_cast<T*>(w.qv);
  T* B = static_cast<T*>(w.B);
  double* F = static_cast<double*>(w.F);
  double* G = total_flux(w, p);
  T* qe = static_cast<T*>(w.qe);
  // the lattice kernel evaluates the inviscid rotating shallow-water form only
  const bool use_lat = lat && lat->ok && p.nu == 0.0 && !p.adv;
  // table-driven kernels: the whole level, or only the rim left by the lattice tiles
  const int32_t* tl = use_lat ? lat->sup_tris : nullptr;
  const int32_t* el = use_lat ? lat->sup_elems : nullptr;
  const int32_t* rl = use_lat ? lat->rim : nullptr;
  const int64_t nt = use_lat ? lat->n_sup_tris : t.T;
  const int64_t ne = use_lat ? lat->n_sup_elems : t.N;
  const int64_t nr = use_lat ? lat->n_rim : t.N;
  // Algorithmic bytes of each launch: every table entry, input and output element once.
  // Per triangle: 3+3 indices, 3+3 weights, f (80 B), its share of the state read (16 B) and
  // q_v.  Per element: the cell/edge tables (edge_cell 120 B, tend 480 B), the state or the
  // intermediates it reads, and the Runge-Kutta arrays of the stage (8 B per array per dof).
  const double sz = double(sizeof(T));
  auto epi = [](const StageOut& c, const StagePtrs& q, bool count_x) {
    int r = 0;
    if (c.a1 != 0.0 || c.a2 != 0.0) ++r;
    if (c.b1 != 0.0 || c.b2 != 0.0) ++r;
    if (count_x && (c.c1 != 0.0 || c.c2 != 0.0)) ++r;
    if (q.o1) ++r;
    if (q.o2) ++r;
    return 8.0 * r;
  };
  const double e_dof = epi(c, sdh, true);
  // the rim lists are short (a few tens of thousands of points): small workgroups spread their
  // gathers over every CU
  const int bs = use_lat ? 64 : BS;
  auto grid = [bs](int64_t n) { return unsigned((n + bs - 1) / bs); };
  {
    TimedLaunch tl_(tm, K_VERTEX, s, double(nt) * (80.0 + 16.0 + sz), nt);
    k_vertex<T><<<grid(nt), bs, 0, s>>>(nt, tl, t, sdh.x, su.x, p.H, qv);
  }
  {
    TimedLaunch tl_(tm, K_EDGE_CELL, s, double(ne) * (120.0 + 32.0 + 24.0 + 6.0 * sz), ne);
    k_edge_cell<T><<<grid(ne), bs, 0, s>>>(ne, el, t, sdh.x, su.x, qv, p, B, F, G, qe);
  }
  {
    TimedLaunch tl_(tm, K_TEND, s, double(nr) * (480.0 + 24.0 + 4.0 * sz + 4.0 * e_dof), nr);
    k_tend<T><<<grid(nr), bs, 0, s>>>(nr, t.n_elem, rl, t.c_e, t.c_div, t.e_c, t.inv_d, t.ecp, t.wl, B, F, G,
                                      qe, sdh, su, c, t, p.nu, p.adv);
  }
  HIPCHK(hipGetLastError());
  if (use_lat) {
    // stage input read once (dh + 3 u), the stage arrays, and the shared geometry of the
    // regular tile positions once for all 10 lozenges (58 values per position)
    const double nreg = double(lat->n_reg_elems);
    TimedLaunch tl_(tm, K_LATTICE, s, nreg * (32.0 + 4.0 * epi(c, sdh, false)) + nreg / 10.0 * 58.0 * 8.0,
                    lat->n_reg_elems);
    LatArgs a = lat->args;
    a.g = p.g;
    a.H = p.H;
    launch_lattice(a, std::is_same<T, float>::value, sdh, su, c, s);
  }
}

void launch_lattice_masked(const DevLattice& lat, DevWork& w, const uint8_t* na, const uint8_t* ea,
                           const uint8_t* tflag, int64_t flagged, const PhysParams& p, bool fp32, const StagePtrs& sdh,
                           const StagePtrs& su, const StageOut& c_in, hipStream_t s, Timer* tm, bool inter) {
  if (!lat.ok) throw std::runtime_error("masked lattice stage: the level has no lattice form");
  if (p.nu != 0.0 || p.adv) throw std::runtime_error("masked lattice stage: inviscid shallow-water form only");
  // a stage array that is the stage input itself is read once (as in the uniform stage)
  StageOut c = c_in;
  if (sdh.y == sdh.x && su.y == su.x) {
    c.c1 += c.a1; c.a1 = 0.0;
    c.c2 += c.a2; c.a2 = 0.0;
  }
  if (sdh.acc == sdh.x && su.acc == su.x) {
    c.c1 += c.b1; c.b1 = 0.0;
    c.c2 += c.b2; c.b2 = 0.0;
  }
  // algorithmic bytes per element of the flagged tiles (all tiles without flags): the uniform
  // kernel's (stage input, Runge-Kutta arrays, the shared geometry's share) plus the four mask
  // bytes and the stored F (3 doubles), Q (3) and B (1)
  int r = 0;
  if (c.a1 != 0.0 || c.a2 != 0.0) ++r;
  if (c.b1 != 0.0 || c.b2 != 0.0) ++r;
  if (sdh.o1) ++r;
  if (sdh.o2) ++r;
  const double sz = fp32 ? 4.0 : 8.0;
  const int64_t units = tflag ? flagged * LT_TI * LT_TJ : lat.n_reg_elems;
  const double nreg = double(units);
  // (+ 8 B of the stored divergence); the intermediates-only form: the stage input, the
  // geometry's share and the stored F, Q, B
  TimedLaunch tl_(tm, inter ? K_LATTICE_INTER : K_LATTICE_ML, s,
                  inter ? nreg * (32.0 + 24.0 + 4.0 * sz) + nreg / 10.0 * 58.0 * 8.0
                        : nreg * (32.0 + 4.0 * 8.0 * r + 4.0 + 24.0 + 4.0 * sz + 8.0) + nreg / 10.0 * 58.0 * 8.0,
                  units);
  LatArgs a = lat.args;
  a.g = p.g;
  a.H = p.H;
  LatML m;
  m.na = na;
  m.ea = ea;
  m.tflag = tflag;
  m.F = static_cast<double*>(w.F);
  m.Q = w.Q;
  m.B = w.B;
  m.c = inter ? nullptr : w.c;
  launch_lattice(a, fp32, sdh, su, c, s, &m, inter);
}

template <typename T>
static void intermediates_impl(const DevTables& t, DevWork& w, const PhysParams& p, const StagePtrs& sdh,
                               const StagePtrs& su, hipStream_t s, const int32_t* tri_list, int64_t nt,
                               const int32_t* elem_list, int64_t ne) {
  T* qv = static_cast<T*>(w.qv);
  if (nt)
    k_vertex<T><<<nblk(nt), BS, 0, s>>>(nt, tri_list, t, sdh.x, su.x, p.H, qv);
  if (ne)
    k_edge_cell<T><<<nblk(ne), BS, 0, s>>>(ne, elem_list, t, sdh.x, su.x, qv, p, static_cast<T*>(w.B),
                                           static_cast<double*>(w.F), total_flux(w, p), static_cast<T*>(w.qe));
  HIPCHK(hipGetLastError());
}

void launch_intermediates(const DevTables& t, DevWork& w, const PhysParams& p, bool fp32,
                          const StagePtrs& sdh, const StagePtrs& su, hipStream_t s, const int32_t* tri_list,
                          int64_t nt, const int32_t* elem_list, int64_t ne) {
  if (nt < 0) nt = t.T;
  if (ne < 0) ne = t.N;
  if (fp32)
    intermediates_impl<float>(t, w, p, sdh, su, s, tri_list, nt, elem_list, ne);
  else
    intermediates_impl<double>(t, w, p, sdh, su, s, tri_list, nt, elem_list, ne);
}

void launch_stage(const DevTables& t, DevWork& w, const PhysParams& p, bool fp32,
                  const StagePtrs& sdh, const StagePtrs& su, const StageOut& c, hipStream_t s,
                  Timer* tm, const DevLattice* lat) {
  if (fp32)
    stage_impl<float>(t, w, p, sdh, su, c, s, tm, lat);
  else
    stage_impl<double>(t, w, p, sdh, su, c, s, tm, lat);
}

// ------------------------------------------------------------------ diagnostics
constexpr int NRED = 7;
constexpr int RED_BLOCKS = 1024;

__global__ __launch_bounds__(BS) void k_diag_partial(
    int64_t N, int64_t n_elem, const double* __restrict__ A_i, const double* __restrict__ l_e,
    const double* __restrict__ d_e, const int32_t* __restrict__ e_c,
    const int32_t* __restrict__ e_v, const double* __restrict__ f_v,
    const double* __restrict__ dh, const double* __restrict__ u, double g, double H,
    double* __restrict__ part) {
  __shared__ double sh[NRED][BS];
  double acc[NRED] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
  for (int64_t id = int64_t(blockIdx.x) * BS + threadIdx.x; id < N; id += int64_t(gridDim.x) * BS) {
    double h = H + dh[id];
    acc[0] += A_i[id] * h;
    acc[1] += 0.5 * A_i[id] * (g * h) * (g * h);
    acc[2] = fmax(acc[2], fabs(dh[id]));
    if (!isfinite(dh[id])) acc[4] += 1.0;
    if (id < n_elem) {
      for (int d = 0; d < 3; ++d) {
        int64_t e = 3 * id + d;
        double ue = u[e];
        double he = 0.5 * ((H + dh[e_c[2 * e]]) + (H + dh[e_c[2 * e + 1]]));
        acc[1] += g * 0.5 * l_e[e] * d_e[e] * he * ue * ue;
        acc[3] = fmax(acc[3], fabs(ue));
        if (!isfinite(ue)) acc[4] += 1.0;
        double fe = 0.5 * (f_v[e_v[2 * e]] + f_v[e_v[2 * e + 1]]);
        double kw = M_PI / d_e[e];
        acc[5] = fmax(acc[5], sqrt(fe * fe + g * he * kw * kw));
        if (fabs(ue) > 0.0) acc[6] = fmin(acc[6], d_e[e] / fabs(ue));
      }
    }
  }
  for (int q = 0; q < NRED; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int st = BS / 2; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) {
      for (int q = 0; q < 2; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + st];
      sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + st]);
      sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + st]);
      sh[4][threadIdx.x] += sh[4][threadIdx.x + st];
      sh[5][threadIdx.x] = fmax(sh[5][threadIdx.x], sh[5][threadIdx.x + st]);
      sh[6][threadIdx.x] = fmin(sh[6][threadIdx.x], sh[6][threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < NRED; ++q) part[q * RED_BLOCKS + blockIdx.x] = sh[q][0];
}

__global__ __launch_bounds__(BS) void k_diag_final(const double* __restrict__ part,
                                                   double* __restrict__ out) {
  __shared__ double sh[NRED][BS];
  double acc[NRED] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
  for (int b = threadIdx.x; b < RED_BLOCKS; b += BS) {
    acc[0] += part[0 * RED_BLOCKS + b];
    acc[1] += part[1 * RED_BLOCKS + b];
    acc[2] = fmax(acc[2], part[2 * RED_BLOCKS + b]);
    acc[3] = fmax(acc[3], part[3 * RED_BLOCKS + b]);
    acc[4] += part[4 * RED_BLOCKS + b];
    acc[5] = fmax(acc[5], part[5 * RED_BLOCKS + b]);
    acc[6] = fmin(acc[6], part[6 * RED_BLOCKS + b]);
  }
  for (int q = 0; q < NRED; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int st = BS / 2; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) {
      for (int q = 0; q < 2; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + st];
      sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + st]);
      sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + st]);
      sh[4][threadIdx.x] += sh[4][threadIdx.x + st];
      sh[5][threadIdx.x] = fmax(sh[5][threadIdx.x], sh[5][threadIdx.x + st]);
      sh[6][threadIdx.x] = fmin(sh[6][threadIdx.x], sh[6][threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < NRED; ++q) out[q] = sh[q][0];
}

void launch_diagnostics(const DevTables& t, DevWork& w, const PhysParams& p, hipStream_t s,
                        double* host_out, const double* dh, const double* u) {
  double* part = w.red;
  double* out = w.red + NRED * RED_BLOCKS;
  k_diag_partial<<<RED_BLOCKS, BS, 0, s>>>(t.N, t.n_elem, t.A_i, t.l_e, t.d_e, t.e_c, t.e_v, t.f_v,
                                           dh ? dh : w.dh, u ? u : w.u, p.g, p.H, part);
  k_diag_final<<<1, BS, 0, s>>>(part, out);
  HIPCHK(hipGetLastError());
  double r[NRED];
  HIPCHK(hipMemcpyAsync(r, out, sizeof(r), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // energy: subtract the rest-state term c^4 A_S / 2, c^2 = g * mass / A_S (Sec. 7.2)
  for (int q = 0; q < NRED; ++q) host_out[q] = r[q];
}

// ------------------------------------------------------------------ table upload
template <typename X>
static X* dev_upload(const std::vector<X>& v) {
  X* p = nullptr;
  HIPCHK(wt::dmalloc(&p, v.size() * sizeof(X)));
  HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice));
  return p;
}

void upload_tables(const Level& L, const std::vector<double>& A_i, DevTables& t) {
  if (int64_t(A_i.size()) != L.N) throw std::runtime_error("upload_tables: cell areas do not match the level");
  const int64_t N = L.N, E = L.E, T = L.T;
  t.N = N; t.E = E; t.T = T; t.n_elem = 10 * L.n * L.n;
  std::vector<int32_t> c_e(6 * N);
  std::vector<double> c_div(6 * N), c_ke(6 * N);
  for (int64_t i = 0; i < N; ++i)
    for (int k = 0; k < 6; ++k) {
      bool ok = k < L.c_deg[i];
      int32_t e = L.c_e[6 * i + (ok ? k : 0)];
      c_e[6 * i + k] = e;
      c_div[6 * i + k] = ok ? L.c_s[6 * i + k] * L.l_e[e] / A_i[i] : 0.0;
      c_ke[6 * i + k] = ok ? L.l_e[e] * L.d_e[e] / (4.0 * A_i[i]) : 0.0;
    }
  std::vector<double> inv_d(E), wl(10 * E);
  for (int64_t e = 0; e < E; ++e) {
    inv_d[e] = 1.0 / L.d_e[e];
    for (int k = 0; k < 10; ++k) wl[10 * e + k] = L.w[10 * e + k] * L.l_e[L.ecp[10 * e + k]] / L.d_e[e];
  }
  std::vector<double> t_curl(3 * T), t_R(3 * T);
  for (int64_t v = 0; v < T; ++v)
    for (int s = 0; s < 3; ++s) {
      t_curl[3 * v + s] = L.t_s[3 * v + s] * L.d_e[L.t_e[3 * v + s]] / L.A_v[v];
      t_R[3 * v + s] = L.kite[3 * v + s] / L.A_v[v];
    }
  t.c_e = dev_upload(c_e);
  t.c_div = dev_upload(c_div);
  t.c_ke = dev_upload(c_ke);
  t.e_c = dev_upload(L.e_c);
  t.e_v = dev_upload(L.e_v);
  t.inv_d = dev_upload(inv_d);
  t.ecp = dev_upload(L.ecp);
  t.wl = dev_upload(wl);
  t.t_n = dev_upload(L.t_n);
  t.t_e = dev_upload(L.t_e);
  t.t_curl = dev_upload(t_curl);
  t.t_R = dev_upload(t_R);
  t.f_v = dev_upload(L.f_v);
  t.A_i = dev_upload(A_i);
  t.l_e = dev_upload(L.l_e);
  t.d_e = dev_upload(L.d_e);
  auto f32 = [](const std::vector<double>& v) { return dev_upload(std::vector<float>(v.begin(), v.end())); };
  t.c_div_f = f32(c_div);
  t.c_ke_f = f32(c_ke);
  t.inv_d_f = f32(inv_d);
  t.wl_f = f32(wl);
  t.t_curl_f = f32(t_curl);
  t.t_R_f = f32(t_R);
  t.f_v_f = f32(L.f_v);
  t.l_e_f = f32(L.l_e);
}

void free_tables(DevTables& t) {
  void* ps[] = {t.c_e, t.c_div, t.c_ke, t.e_c, t.e_v, t.inv_d, t.ecp, t.wl,
                t.t_n, t.t_e, t.t_curl, t.t_R, t.f_v, t.A_i, t.l_e, t.d_e,
                t.c_div_f, t.c_ke_f, t.inv_d_f, t.wl_f, t.t_curl_f, t.t_R_f, t.f_v_f, t.l_e_f};
  for (void* p : ps)
    if (p) (void)wt::dfree(p);
  t = DevTables{};
}

}  // namespace wt
