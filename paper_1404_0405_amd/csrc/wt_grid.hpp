// Host-side construction of one level of the nested icosahedral C-grid: canonical numbering
// through the lozenge seam rules, spherical geometry, and the TRiSK operator tables.
//
// Grid (Sec. 2.2, Fig. 1): the icosahedron's 20 faces are paired into 10 lozenges; level J
// refines every lozenge into a 2^J x 2^J lattice by arc-midpoint bisection.  One element
// (Sec. 5.2) is one node, two triangles and three edges.
#pragma once
#include <cstdint>
#include <vector>

namespace wt {

struct V3 {
  double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
V3 unit(V3 a);
double arc(V3 a, V3 b);                    // great-circle angle
double tri_area(V3 a, V3 b, V3 c);         // signed spherical excess (Van Oosterom-Strackee)
V3 circumcentre(V3 a, V3 b, V3 c);         // of a counter-clockwise spherical triangle

// Lattice <-> canonical numbering for level J (n = 2^J):
//   node (L,i,j), 0<=i,j<n  ->  (L*n+i)*n+j ; poles 10n^2 (north), 10n^2+1 (south)
//   edge 3*node + d, d in {0:(1,0), 1:(1,1), 2:(0,1)}; triangle 2*node + t.
struct Lattice {
  int J;
  int64_t n, N, E, T;
  explicit Lattice(int J_);
  // canonical node of lattice point (L,i,j); the point may lie up to one lozenge side outside
  // [0,n)^2 (not in a corner wedge), in which case the seam rules map it into the neighbour.
  int64_t node(int L, int64_t i, int64_t j) const;
  bool decode(int64_t id, int& L, int64_t& i, int64_t& j) const;  // false for poles
  // canonical edge joining canonical nodes a,b; sign = +1 if it points from a to b.
  int64_t edge(int64_t a, int64_t b, int& sign) const;
};

struct Level {
  int J = 0;
  int64_t n = 0, N = 0, E = 0, T = 0;
  double radius = 0, omega = 0;
  std::vector<V3> pos;                         // unit node positions
  // topology
  std::vector<int32_t> e_c;                    // 2E: from-node (owner), to-node
  std::vector<int32_t> e_v;                    // 2E: left, right triangle
  std::vector<int32_t> t_n, t_e;               // 3T: nodes, edges (counter-clockwise)
  std::vector<int8_t> t_s;                     // 3T: +1 if edge circulates CCW around triangle
  std::vector<int32_t> c_e, c_t;               // 6N: edges, vertex between edge k and k+1
  std::vector<int8_t> c_s;                     // 6N: +1 if edge points out of the cell
  std::vector<uint8_t> c_deg;                  // 5 or 6
  // geometry (metres, square metres)
  std::vector<double> A_i, A_v, d_e, l_e, f_v;
  std::vector<double> kite;                    // 3T: kite of node s inside triangle
  std::vector<V3> cc;                          // circumcentres
  // TRiSK perpendicular-flux stencil (10 slots, padded with weight 0)
  std::vector<int32_t> ecp;                    // 10E
  std::vector<double> w;                       // 10E: w_{e,e'}
};

// Build level J; radius and omega in SI units.  Aborts on internal inconsistency.
void build_level(int J, double radius, double omega, Level& L);

}  // namespace wt
