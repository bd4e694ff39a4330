// Host precompute of the inter-scale tables between a coarse level j and a fine level j+1:
// nesting maps, height-transform weights from spherical overlap areas, velocity-prediction
// weights, and the flux-restriction weights.
#pragma once
#include <cstdint>
#include <vector>

#include "wt_grid.hpp"

namespace wt {

constexpr int RF_NC = 8;    // nonzero fine-divergence weights per coarse-edge flux restriction (at most 7; padded)
constexpr int MK_MAX = 12;  // odd fine nodes sharing area with one coarse cell

struct PairTables {
  int64_t Nc = 0, Ec = 0, Tc = 0, Nf = 0, Ef = 0;
  std::vector<int32_t> even;      // Nc: coarse node -> its fine copy
  std::vector<int32_t> mid;       // Ec: coarse edge -> fine midpoint node
  std::vector<int32_t> h1, h2;    // Ec: fine half-edges (oriented along the coarse edge)
  std::vector<int32_t> cells;     // 4Ec: a, b (ends), p (left), q (right opposite vertex)
  std::vector<double> area_geo;   // 4Ec: overlap areas A_cm (geometric)
  std::vector<double> st;         // 4Ec: s~_cm = A_cm / sum_c A_cm
  std::vector<double> aov;        // 4Ec: effective overlap areas s~_cm A^{j+1}_m
  std::vector<double> s_upd;      // 4Ec: s_km = aov / A^j_k
  std::vector<int32_t> mk;        // 12Nc: 4*edge + column of every odd node sharing area with k
  std::vector<int32_t> int_e;     // 3Tc: fine edges inside the coarse triangle
  std::vector<int32_t> v_sten;    // 9Tc: coarse edges of the triangle's prediction stencil
  std::vector<double> w_int;      // 27Tc: prediction weights of the 3 interior fine edges
  std::vector<double> w_pl, w_pr; // 9Ec each: (p1 - p2) weights on v_sten of left/right triangle
  std::vector<int32_t> rf_f;      // 3Ec: fine edges of the basic flux restriction
  std::vector<double> rf_fw;      // 3Ec: weights on l_f F_f
  std::vector<int32_t> rf_c;      // 8Ec: fine nodes whose divergence enters (nonzero weights first)
  std::vector<double> rf_cw;      // 8Ec: weights on c_n (integrated flux units; 0 on padding)
};

// Geometry-only part (maps, overlap areas, s~, velocity weights).
void build_pair(const Level& C, const Level& F, PairTables& P);
// Effective areas and everything that depends on them: A_c_eff from A_f_eff (fine level).
void finish_pair(const Level& C, const Level& F, const std::vector<double>& A_f_eff,
                 PairTables& P, std::vector<double>& A_c_eff);

double sph_overlap(const V3* P, int np, const V3* Q, int nq);  // unit-sphere area

}  // namespace wt
