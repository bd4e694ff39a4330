// Per-point bodies of the adaptive stage (Sec. 3.1, 4.1-4.4): one function per kernel of the
// multilevel Runge-Kutta step, evaluated at one node, edge or triangle.  The one-launch-per-kernel
// path (wt_ml.hip, wt_kernels.hip) and the batched ensemble step (wt_batch.hip) both call these,
// so the two give identical results.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wt_ml.hpp"

namespace wt {

// ------------------------------------------------------------------ inter-scale predictions
// The velocity prediction sums are evaluated in the compute type T (float in the single-precision
// mode, with the coarse values and weights rounded to it); a prediction is then combined with the
// stored values (detail = value - prediction, value = detail + prediction) in double, so the
// state keeps double precision and the forward and inverse transforms stay exact inverses of
// each other.  The height transform stays in double in both modes: its prediction is part of the
// area-weighted restriction R_h (eq. (Rh)), and the partial transform of a step replaces coarse
// heights by R_h of the fine ones, which conserves mass to round-off only when R_h inverts the
// adapt's reconstruction exactly (a single-precision height prediction left 1e-10 relative mass
// drift after 20 steps).

// velocity difference of the two half-edges of coarse edge e predicted from the coarse
// velocities of its two triangles' stencils
template <typename T>
__device__ __forceinline__ T pair_pred(const DevPair& P, int64_t e, const int32_t* __restrict__ e_v,
                                       const double* __restrict__ uc) {
  int32_t tl = e_v[2 * e], tr = e_v[2 * e + 1];
  T s = T(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) s += tv<T>(P.w_pl, P.w_pl_f, 9 * e + k) * T(uc[P.v_sten[9 * tl + k]]);
#pragma unroll
  for (int k = 0; k < 9; ++k) s += tv<T>(P.w_pr, P.w_pr_f, 9 * e + k) * T(uc[P.v_sten[9 * tr + k]]);
  return s;
}

// interior fine edge s of coarse triangle t predicted from the triangle's coarse stencil
template <typename T>
__device__ __forceinline__ T int_pred(const DevPair& P, int64_t t, int s, const double* __restrict__ uc) {
  T v = T(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) v += tv<T>(P.w_int, P.w_int_f, 27 * t + 9 * s + k) * T(uc[P.v_sten[9 * t + k]]);
  return v;
}

// the same from the column copies of the tables (identical arithmetic)
template <typename T>
__device__ __forceinline__ T int_pred_c(const DevPair& P, int64_t t, int s, const double* __restrict__ uc) {
  T v = T(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) v += tv<T>(P.w_int_c, P.w_int_cf, P.ct(9 * s + k, t)) * T(uc[P.v_sten_c[P.ct(k, t)]]);
  return v;
}

// height at the midpoint of coarse edge e predicted from its four even fine neighbours
// (s~-weighted mean, eq. (WTpred))
__device__ __forceinline__ double h_pred(const DevPair& P, int64_t e, const double* __restrict__ hf) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) s += P.st[4 * e + c] * hf[P.even[P.cells[4 * e + c]]];
  return s;
}

// height detail at the midpoint of coarse edge e: fine value minus the prediction (subtracted
// term by term)
__device__ __forceinline__ double h_detail(const DevPair& P, int64_t e, const double* __restrict__ hf) {
  double s = hf[P.mid[e]];
#pragma unroll
  for (int c = 0; c < 4; ++c) s -= P.st[4 * e + c] * hf[P.even[P.cells[4 * e + c]]];
  return s;
}

// ------------------------------------------------------------------ prolongation (one pair)
// Inactive even node: the coarse value; inactive odd node: s~-weighted mean of its four even
// fine neighbours; inactive half-edges: u^j -+ (p1-p2)/2; inactive interior edges: prediction.
__device__ __forceinline__ void body_prolong_even(int64_t k, const DevPair& P, const uint8_t* __restrict__ naf,
                                                  const double* __restrict__ hc, double* __restrict__ hf) {
  int32_t f = P.even[k];
  if (!naf[f]) hf[f] = hc[k];
}

template <typename T>
__device__ __forceinline__ void body_prolong_odd_pair(int64_t e, const DevPair& P, const uint8_t* __restrict__ naf,
                                                      const uint8_t* __restrict__ eaf,
                                                      const int32_t* __restrict__ e_v_c,
                                                      const double* __restrict__ uc, double* __restrict__ hf,
                                                      double* __restrict__ uf) {
  int32_t m = P.mid[e];
  if (!naf[m]) hf[m] = h_pred(P, e, hf);
  int32_t h1 = P.h1[e], h2 = P.h2[e];
  bool a1 = eaf[h1], a2 = eaf[h2];
  if (!a1 || !a2) {
    const double half = 0.5 * double(pair_pred<T>(P, e, e_v_c, uc));
    if (!a1) uf[h1] = uc[e] + half;
    if (!a2) uf[h2] = uc[e] - half;
  }
}

template <typename T>
__device__ __forceinline__ void body_prolong_int(int64_t t, const DevPair& P, const uint8_t* __restrict__ eaf,
                                                 const double* __restrict__ uc, double* __restrict__ uf) {
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    int32_t f = P.int_e[3 * t + s];
    if (!eaf[f]) uf[f] = double(int_pred<T>(P, t, s, uc));
  }
}

// ------------------------------------------------------------------ TRiSK intermediates (one level)
// q_v = (zeta_v + f_v) / h_v at triangle t
template <typename T>
__device__ __forceinline__ void body_vertex(int64_t t, const DevTables& tb, const double* __restrict__ dh,
                                            const double* __restrict__ u, double H, T* __restrict__ qv) {
  T z = T(0), hv = T(0);
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    z += tv<T>(tb.t_curl, tb.t_curl_f, 3 * t + s) * T(u[tb.t_e[3 * t + s]]);
    hv += tv<T>(tb.t_R, tb.t_R_f, 3 * t + s) * (T(H) + T(dh[tb.t_n[3 * t + s]]));
  }
  qv[t] = (z + tv<T>(tb.f_v, tb.f_v_f, t)) / hv;
}

// B_i = g dh_i + K_i at node id; F_e = h_e u_e and q_e at its three edges.  Viscous form
// (Sec. 3.1): B_i - nu (div u)_i and, into G, the total mass flux F_e - nu (grad dh)_e, so that
// -div G = -div F + nu div grad dh and -grad B = -grad B + nu grad div u.
template <typename T>
__device__ __forceinline__ void body_edge_cell(int64_t id, const DevTables& tb, const double* __restrict__ dh,
                                               const double* __restrict__ u, const T* __restrict__ qv,
                                               const PhysParams& ph, T* __restrict__ B, double* __restrict__ F,
                                               double* __restrict__ G, T* __restrict__ qe) {
  T K = T(0), D = T(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    T ue = T(u[tb.c_e[6 * id + k]]);
    K += tv<T>(tb.c_ke, tb.c_ke_f, 6 * id + k) * ue * ue;
    if (ph.nu != 0.0) D += tv<T>(tb.c_div, tb.c_div_f, 6 * id + k) * ue;
  }
  T b = T(ph.g) * T(dh[id]) + K;
  if (ph.nu != 0.0) b -= T(ph.nu) * D;
  B[id] = b;
  if (id >= tb.n_elem) return;
  const double H = ph.H;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int64_t e = 3 * id + d;
    const double ha = dh[tb.e_c[2 * e]], hb = dh[tb.e_c[2 * e + 1]];
    T he = T(0.5) * ((T(H) + T(ha)) + (T(H) + T(hb)));
    const double f = double(he * T(u[e]));  // the mass flux is stored in double in both precisions
    F[e] = f;
    if (ph.nu != 0.0) G[e] = f - ph.nu * ((hb - ha) * tb.inv_d[e]);
    qe[e] = T(0.5) * (qv[tb.e_v[2 * e]] + qv[tb.e_v[2 * e + 1]]);
  }
}

// relative vorticity of triangle v (circulation / area)
template <typename T>
__device__ __forceinline__ T tri_curl(int64_t v, const DevTables& tb, const double* __restrict__ u) {
  T z = T(0);
#pragma unroll
  for (int s = 0; s < 3; ++s) z += tv<T>(tb.t_curl, tb.t_curl_f, 3 * v + s) * T(u[tb.t_e[3 * v + s]]);
  return z;
}

// Q_e = sum over the perpendicular-flux stencil of w l'/d F' (q_e + q_e')/2.  Viscous form: plus
// nu (grad^perp curl u)_e = nu (zeta_left - zeta_right) / l_e, the adjoint of the discrete curl
// (so that -grad^perp curl dissipates enstrophy), with u the stage input.
template <typename T>
__device__ __forceinline__ void body_Q(int64_t e, const DevTables& tb, const double* __restrict__ F,
                                       const T* __restrict__ qe, T* __restrict__ Q, double nu,
                                       const double* __restrict__ u) {
  T q0 = qe[e], s = T(0);
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    int32_t ep = tb.ecp[10 * e + k];
    s += tv<T>(tb.wl, tb.wl_f, 10 * e + k) * T(F[ep]) * (T(0.5) * (q0 + qe[ep]));
  }
  if (nu != 0.0)
    s += T(nu) * (tri_curl<T>(tb.e_v[2 * e], tb, u) - tri_curl<T>(tb.e_v[2 * e + 1], tb, u)) / tv<T>(tb.l_e, tb.l_e_f, e);
  Q[e] = s;
}

// ------------------------------------------------------------------ restriction (one pair)
// fine divergence c_i (integrated form, used by the flux restriction)
__device__ __forceinline__ void body_div(int64_t i, const DevTables& tf, const double* __restrict__ F,
                                         double* __restrict__ c) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) s += tf.c_div[6 * i + k] * F[tf.c_e[6 * i + k]];
  c[i] = s;
}

// F^j = R_F(F^{j+1}, c^{j+1}) and Q^j = mean of the half-edges at non-leaf coarse edge e
template <typename T>
__device__ __forceinline__ void body_restrict_edges(int64_t e, const DevPair& P, const uint8_t* __restrict__ eaf,
                                                    const double* __restrict__ l_f, const double* __restrict__ l_c,
                                                    const double* __restrict__ Ff, const double* __restrict__ cf,
                                                    const T* __restrict__ Qf, double* __restrict__ Fc,
                                                    T* __restrict__ Qc) {
  int32_t h1 = P.h1[e], h2 = P.h2[e];
  if (!(eaf[h1] && eaf[h2])) return;
  double phi = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int32_t f = P.rf_f[3 * e + k];
    phi += P.rf_fw[3 * e + k] * (l_f[f] * Ff[f]);
  }
#pragma unroll
  for (int k = 0; k < RF_NC; ++k) phi += P.rf_cw[RF_NC * e + k] * cf[P.rf_c[RF_NC * e + k]];
  Fc[e] = phi / l_c[e];
  Qc[e] = T(0.5) * (Qf[h1] + Qf[h2]);
}

// B^j = B^{j+1} at non-leaf coarse node k
template <typename T>
__device__ __forceinline__ void body_restrict_B(int64_t k, const DevPair& P, const uint8_t* __restrict__ naf,
                                                const T* __restrict__ Bf, T* __restrict__ Bc) {
  int32_t f = P.even[k];
  if (naf[f]) Bc[k] = Bf[f];
}

// ------------------------------------------------------------------ tendencies (one level)
// Runge-Kutta stage combination at point i after the tendency k
__device__ __forceinline__ void rk_out(int64_t i, double k, const StagePtrs& p, const StageOut& c) {
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

// Tendencies at node id and its edges with the level's (possibly restricted) F, Q, B, zero at
// inactive points, then the stage combination.  F is the total mass flux (G of a viscous run);
// adv != 0: the advection form, whose velocity does not change.
template <typename T>
__device__ __forceinline__ void body_tend_ml(int64_t id, const DevTables& tb, const uint8_t* __restrict__ na,
                                             const uint8_t* __restrict__ ea, const T* __restrict__ B,
                                             const double* __restrict__ F, const T* __restrict__ Q,
                                             const StagePtrs& pdh, const StagePtrs& pu, const StageOut& c,
                                             int32_t adv) {
  double k = 0.0;
  if (na[id]) {
    double div = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) div += tb.c_div[6 * id + q] * F[tb.c_e[6 * id + q]];
    k = -div;
  }
  rk_out(id, k, pdh, c);
  if (id >= tb.n_elem) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int64_t e = 3 * id + d;
    double ku = 0.0;
    if (ea[e] && !adv) ku = double(-Q[e] - (B[tb.e_c[2 * e + 1]] - B[tb.e_c[2 * e]]) * tv<T>(tb.inv_d, tb.inv_d_f, e));
    rk_out(e, ku, pu, c);
  }
}

// ------------------------------------------------------------------ partial height transform
// Two passes per pair.  First, for every coarse edge e: whether the height-prediction stencil of
// its odd fine node is active (the node and its four even neighbours), and where it is, that
// node's detail (each detail is used by the 2-4 coarse cells sharing area with the odd node, so
// it is computed once here rather than once per cell).  Mask bytes are combined without early
// exits, so their loads are issued together.
__device__ __forceinline__ void body_partial_d(int64_t e, const DevPair& P, const uint8_t* __restrict__ naf,
                                               const double* __restrict__ hf, double* __restrict__ det,
                                               uint8_t* __restrict__ act) {
  const uint8_t a = naf[P.mid[e]] & naf[P.even[P.cells[4 * e]]] & naf[P.even[P.cells[4 * e + 1]]] &
                    naf[P.even[P.cells[4 * e + 2]]] & naf[P.even[P.cells[4 * e + 3]]];
  act[e] = a;
  if (a) det[e] = h_detail(P, e, hf);
}

// Then h^j_k <- R_h(h^{j+1})_k at complete coarse node k: every stencil of its odd nodes is
// active and every coarse edge of the node is non-leaf (the same sum, in the same order, as
// R_h written out with the details).
__device__ __forceinline__ void body_partial_h(int64_t k, const DevPair& P, const int32_t* __restrict__ c_e_c,
                                               const uint8_t* __restrict__ nac, const uint8_t* __restrict__ naf,
                                               const uint8_t* __restrict__ eaf, const double* __restrict__ det,
                                               const uint8_t* __restrict__ act, const double* __restrict__ hf,
                                               double* __restrict__ hc) {
  const int32_t ev = P.even[k];
  int32_t ecs[MK_MAX];
#pragma unroll
  for (int q = 0; q < MK_MAX; ++q) ecs[q] = P.mk[P.cn(q, k)];   // valid entries first, then -1
  uint32_t ok = nac[k] & naf[ev];
#pragma unroll
  for (int q = 0; q < MK_MAX; ++q)
    if (ecs[q] >= 0) ok &= act[ecs[q] >> 2];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int32_t e = c_e_c[6 * k + q];
    ok &= eaf[P.h1[e]] & eaf[P.h2[e]];
  }
  if (!ok) return;
  double s = hf[ev];
#pragma unroll
  for (int q = 0; q < MK_MAX; ++q)
    if (ecs[q] >= 0) s += P.s_upd[P.upd(ecs[q])] * det[ecs[q] >> 2];
  hc[k] = s;
}

}  // namespace wt
