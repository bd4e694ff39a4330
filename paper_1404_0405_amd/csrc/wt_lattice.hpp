// Lattice form of the uniform TRiSK stage.
//
// The 10 lozenges of the icosahedral grid are congruent under rotations of the icosahedron
// that map lattice coordinates to lattice coordinates, so every geometric quantity of a
// lattice position (i,j) -- areas, lengths, kite fractions, TRiSK weights -- is the same in all
// lozenges; only the Coriolis parameter differs, and it follows from the rotated circumcentre.
// One reference table (lozenge 0, padded by G positions across its sides) therefore serves all
// lozenges.  Tiles whose halo reaches a lozenge corner (the pentagons) are left to the
// table-driven kernels through index lists.
#pragma once
#include <cstdint>
#include <vector>

#include "wt_grid.hpp"

namespace wt {

constexpr int LT_G = 3;     // padding of the reference table
constexpr int LT_MARGIN = 5;  // lozenge corners must lie this far outside a regular tile
constexpr int LT_TI = 16;   // tile rows (i)
constexpr int LT_TJ = 32;   // tile columns (j)

// quantity index q in the reference table (value at padded position p is tab[q * W2 + p])
enum LatQ {
  LQ_INVA = 0,            // 1 / A_i
  LQ_KC = 1,              // 3: l_e d_e / 4 of frame edges d = 0,1,2
  LQ_LEN = 4,             // 3: l_e
  LQ_INVD = 7,            // 3: 1 / d_e
  LQ_CURL = 10,           // 6: t_{e,v} d_e / A_v for triangle t, side s (index 10 + 3t + s)
  LQ_R = 16,              // 6: kite / A_v for triangle t, corner s
  LQ_CC = 22,             // 6: circumcentre of triangle t, component c (unit sphere)
  LQ_WL = 28,             // 30: w_{e,e'} l_e' / d_e for frame edge d, stencil slot k (28 + 10d + k)
  LQ_COUNT = 58
};

struct LatticeHost {
  int J = 0;
  int64_t n = 0, W = 0, W2 = 0;
  std::vector<double> tab;            // LQ_COUNT * W2
  std::vector<double> frot;           // 10 x 3: f = sum_c frot[3L+c] * cc_ref[c]
  std::vector<int32_t> tiles;         // 2 per regular tile: i0, j0
  std::vector<int32_t> rim_elems;     // elements not covered by regular tiles (+ poles)
  std::vector<int32_t> sup_elems;     // elements whose B, F, q_e the rim needs
  std::vector<int32_t> sup_tris;      // triangles whose q_v the rim needs
};

// Halo addressing of the lattice kernel for a point (i,j) of lozenge L outside [0,n)^2:
// canonical node, the canonical edges of its three frame directions and their signs (edge -1
// if the rule would leave the neighbour lozenge).  Used to verify the kernel's indexing.
void kernel_halo_address(int L, int64_t i, int64_t j, int64_t n, int64_t& node, int64_t* edge, int* sign);

// Build the reference table, the tile list and the rim lists for level L (needs n >= 64).
bool build_lattice(const Level& L, LatticeHost& H);

}  // namespace wt
