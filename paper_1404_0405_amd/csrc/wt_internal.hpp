// Internal device structures and kernel launchers of libwt.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "wt_grid.hpp"

namespace wt {

// Device tables of one full level, laid out per element (canonical order): element `id`
// owns node id, edges 3id..3id+2 and triangles 2id, 2id+1 (the two poles own only a node).
struct DevTables {
  int64_t N = 0, E = 0, T = 0, n_elem = 0;  // n_elem = 10 n^2 (elements with edges)
  int32_t* c_e = nullptr;     // 6N edges of each cell (padded with a valid edge)
  double* c_div = nullptr;    // 6N  n_{e,i} l_e / A_i          (0 in padded slots)
  double* c_ke = nullptr;     // 6N  l_e d_e / (4 A_i)
  int32_t* e_c = nullptr;     // 2E  from / to node
  int32_t* e_v = nullptr;     // 2E  left / right triangle
  double* inv_d = nullptr;    // E   1/d_e
  int32_t* ecp = nullptr;     // 10E perpendicular-flux stencil
  double* wl = nullptr;       // 10E w_{e,e'} l_{e'} / d_e
  int32_t* t_n = nullptr;     // 3T  triangle nodes
  int32_t* t_e = nullptr;     // 3T  triangle edges
  double* t_curl = nullptr;   // 3T  t_{e,v} d_e / A_v
  double* t_R = nullptr;      // 3T  kite / A_v  (weights of h_v)
  double* f_v = nullptr;      // T   Coriolis parameter at the circumcentre
  double* A_i = nullptr;      // N
  double* l_e = nullptr;      // E
  double* d_e = nullptr;      // E
  // single-precision copies of the weights the single-precision stage reads (each the same
  // rounding as converting the FP64 value on load, so results are unchanged; half the bytes)
  float *c_div_f = nullptr, *c_ke_f = nullptr, *inv_d_f = nullptr, *wl_f = nullptr;
  float *t_curl_f = nullptr, *t_R_f = nullptr, *f_v_f = nullptr, *l_e_f = nullptr;
};

// A table value in the compute type T: the FP64 table for double, its single-precision copy
// for float.
template <typename T>
__host__ __device__ __forceinline__ T tv(const double* d, const float* f, int64_t i);
template <>
__host__ __device__ __forceinline__ double tv<double>(const double* d, const float*, int64_t i) { return d[i]; }
template <>
__host__ __device__ __forceinline__ float tv<float>(const double*, const float* f, int64_t i) { return f[i]; }

// Work buffers of one level (double unless noted).
struct DevWork {
  double *dh = nullptr, *u = nullptr;          // prognostic state y
  double *dh_acc = nullptr, *u_acc = nullptr;  // Runge-Kutta accumulator
  double *dh_s[2] = {nullptr, nullptr}, *u_s[2] = {nullptr, nullptr};  // stage inputs
  void *qv = nullptr, *B = nullptr, *F = nullptr, *qe = nullptr;     // T-typed intermediates
  void* Q = nullptr;                           // T-typed qF^perp (multilevel path)
  double* c = nullptr;                         // fine divergence (multilevel path)
  double* G = nullptr;                         // F - nu grad dh (viscous runs; the divergence and
                                               // the flux restriction read it instead of F)
  double* ddh = nullptr;                       // tendency output buffers (test hook)
  double* du = nullptr;
  double* red = nullptr;                       // reduction scratch
};

// Physical constants and form of the equations a stage evaluates: gravity g, mean depth H,
// viscosity nu of the dissipative form (Sec. 3.1; 0: inviscid) and adv != 0 for the advection
// form (Sec. 6.1: the height carried by the fixed velocity, du/dt = 0).
struct PhysParams {
  double g, H, nu;
  int32_t adv;
};

// The mass flux whose divergence a stage takes: F, or G = F - nu grad dh in the viscous form.
inline double* total_flux(const DevWork& w, const PhysParams& p) {
  return p.nu != 0.0 ? w.G : static_cast<double*>(w.F);
}

// Generic Runge-Kutta epilogue evaluated at every point after the tendency k:
//   o1 = a1*y + b1*acc + c1*x + d1*k     (if o1 != null)
//   o2 = a2*y + b2*acc + c2*x + d2*k     (if o2 != null)
struct StageOut {
  double a1, b1, c1, d1, a2, b2, c2, d2;
};
struct StagePtrs {
  const double *y, *acc, *x;
  double *o1, *o2;
};

enum KernelId { K_VERTEX = 0, K_EDGE_CELL, K_TEND, K_LATTICE, K_LATTICE_ML, K_LATTICE_INTER, K_COUNT };
extern const char* const kKernelNames[K_COUNT];

struct Timer {
  bool enabled = false;
  struct Rec {
    int k;
    hipEvent_t a, b;
    double bytes;   // algorithmic bytes of the launch
    int64_t units;  // elements (node + its three edges) or triangles the launch processes
  };
  std::vector<Rec> recs;
};

// device tables of level L with cell areas A_i (the effective areas below jmax)
void upload_tables(const Level& L, const std::vector<double>& A_i, DevTables& t);
void free_tables(DevTables& t);

struct DevLattice;

// One tendency evaluation on stage input (x_dh, x_u) followed by the RK epilogue; with a
// lattice, the regular tiles go through the fused lattice kernel and only the rim through the
// table-driven kernels.
void launch_stage(const DevTables& t, DevWork& w, const PhysParams& p, bool fp32,
                  const StagePtrs& sdh, const StagePtrs& su, const StageOut& c,
                  hipStream_t s, Timer* tm, const DevLattice* lat = nullptr);

// The tile elements of the finest level of an adaptive grid through the masked lattice kernel:
// tendencies zero at inactive points (na, ea), F, Q, B of every tile element stored for the
// restriction.  tflag (10 per tile; null: every tile) limits it to the tiles of each lozenge that
// hold support points, `flagged` of them (for the byte count).  The rim round the lozenge
// corners is left to the listed kernels.  inter: F, Q, B alone (no tendency, no stage output; the
// level's tendencies follow the restriction from the level above).
void launch_lattice_masked(const DevLattice& lat, DevWork& w, const uint8_t* na, const uint8_t* ea,
                           const uint8_t* tflag, int64_t flagged, const PhysParams& p, bool fp32,
                           const StagePtrs& sdh, const StagePtrs& su, const StageOut& c, hipStream_t s, Timer* tm,
                           bool inter = false);

// q_v, B, F, q_e of one level (no tendency, no stage output): every triangle / element, or the
// listed ones (nt, ne < 0: the whole level).
void launch_intermediates(const DevTables& t, DevWork& w, const PhysParams& p, bool fp32,
                          const StagePtrs& sdh, const StagePtrs& su, hipStream_t s,
                          const int32_t* tri_list = nullptr, int64_t nt = -1, const int32_t* elem_list = nullptr,
                          int64_t ne = -1);

// Diagnostics: out[0]=mass, out[1]=energy, out[2]=max|dh|, out[3]=max|u|, out[4]=non-finite
// count, out[5]=omega_max, out[6]=min d_e/|u_e|.
void launch_diagnostics(const DevTables& t, DevWork& w, const PhysParams& p, hipStream_t s,
                        double* host_out, const double* dh = nullptr, const double* u = nullptr);

}  // namespace wt
