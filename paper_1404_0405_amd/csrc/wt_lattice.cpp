// Reference geometry of the lozenge lattice, regular tiles and rim lists (Sec. 4.1, 5.2).
#include "wt_lattice.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace wt {

#define LAT_CHECK(c, msg)                                                         \
  do {                                                                            \
    if (!(c)) {                                                                   \
      std::fprintf(stderr, "wt lattice: %s (%s:%d)\n", msg, __FILE__, __LINE__);  \
      std::abort();                                                               \
    }                                                                             \
  } while (0)

namespace {
const int D0[3] = {1, 1, 0}, D1[3] = {0, 1, 1};  // delta_d = (D0[d], D1[d])
// vertex k of a cell C: triangle type, offset of its lattice origin from C, corner of C
const int VT[6] = {0, 1, 0, 1, 0, 1};
const int VOI[6] = {0, 0, -1, -1, -1, 0}, VOJ[6] = {0, 0, 0, -1, -1, -1};
const int VC[6] = {0, 0, 1, 1, 2, 2};
}  // namespace

// The lattice kernel's halo addressing, written the same way as in the kernel: one seam
// crossing, then the edge directions mapped by the lattice rotation of that seam.
void kernel_halo_address(int L, int64_t i, int64_t j, int64_t n, int64_t& node, int64_t* edge, int* sign) {
  const bool north = L < 5;
  const int k = north ? L : L - 5, km = (k + 4) % 5, kp = (k + 1) % 5;
  int L2 = L;
  int64_t i2 = i, j2 = j;
  int rot = 0;
  if (north) {
    if (i < 0) { L2 = km; i2 = n + i - j; j2 = n + i; rot = 1; }
    else if (j < 0) { L2 = 5 + km; j2 = n + j; }
    else if (i >= n) { L2 = 5 + k; i2 = i - n; }
    else if (j >= n) { L2 = kp; i2 = j - n; j2 = j - i; rot = -1; }
  } else {
    if (i < 0) { L2 = k; i2 = n + i; }
    else if (j < 0) { L2 = 5 + km; i2 = n + j; j2 = n + j - i; rot = -1; }
    else if (i >= n) { L2 = 5 + kp; i2 = i - j; j2 = i - n; rot = 1; }
    else if (j >= n) { L2 = kp; j2 = j - n; }
  }
  const int64_t id = (int64_t(L2) * n + i2) * n + j2;
  node = id;
  if (rot == 0) {
    for (int d = 0; d < 3; ++d) { edge[d] = 3 * id + d; sign[d] = 1; }
  } else if (rot == 1) {
    edge[0] = 3 * id + 1; sign[0] = 1;
    edge[1] = 3 * id + 2; sign[1] = 1;
    edge[2] = 3 * (id - n); sign[2] = -1;
  } else {
    edge[0] = 3 * (id - 1) + 2; sign[0] = -1;
    edge[1] = 3 * id; sign[1] = 1;
    edge[2] = 3 * id + 1; sign[2] = 1;
  }
  // the point one row above / one column left must lie in the same lozenge
  if (rot == 1 && i2 < 1) edge[2] = -1;
  if (rot == -1 && j2 < 1) edge[0] = -1;
}

bool build_lattice(const Level& Lv, LatticeHost& H) {
  const int64_t n = Lv.n;
  if (n < 64) return false;
  Lattice lat(Lv.J);
  const int G = LT_G;
  H.J = Lv.J;
  H.n = n;
  H.W = n + 2 * G;
  H.W2 = H.W * H.W;
  const int64_t W = H.W, W2 = H.W2;
  auto P = [&](int64_t i, int64_t j) { return (i + G) * W + (j + G); };
  auto inside = [&](int64_t i, int64_t j) { return i >= -G && i < n + G && j >= -G && j < n + G; };
  auto irregular = [&](int64_t i, int64_t j) {
    bool oi = i < 0 || i >= n, oj = j < 0 || j >= n;
    if (oi && oj) return true;  // corner wedge
    return (i == 0 || i == n) && (j == 0 || j == n);  // the four corners (pentagons / poles)
  };
  // positions of the padded frame of lozenge 0
  std::vector<V3> pos(W2, V3{0, 0, 0});
  std::vector<uint8_t> pv(W2, 0);
  for (int64_t i = -G; i < n + G; ++i)
    for (int64_t j = -G; j < n + G; ++j)
      if (!irregular(i, j)) {
        pos[P(i, j)] = Lv.pos[lat.node(0, i, j)];
        pv[P(i, j)] = 1;
      }
  auto pvalid = [&](int64_t i, int64_t j) { return inside(i, j) && pv[P(i, j)]; };
  // triangles: circumcentre, kites, area
  std::vector<V3> cc(2 * W2);
  std::vector<double> kite(6 * W2, 0.0), Av(2 * W2, 0.0);
  std::vector<uint8_t> tv(2 * W2, 0);
  const double R = Lv.radius, R2 = R * R;
  for (int64_t i = -G; i < n + G; ++i)
    for (int64_t j = -G; j < n + G; ++j)
      for (int t = 0; t < 2; ++t) {
        int64_t ci[3] = {i, i + 1, t == 0 ? i + 1 : i};
        int64_t cj[3] = {j, t == 0 ? j : j + 1, j + 1};
        bool ok = true;
        for (int s = 0; s < 3; ++s) ok = ok && pvalid(ci[s], cj[s]);
        if (!ok) continue;
        V3 a = pos[P(ci[0], cj[0])], b = pos[P(ci[1], cj[1])], c = pos[P(ci[2], cj[2])];
        V3 o = circumcentre(a, b, c);
        V3 v[3] = {a, b, c};
        double sum = 0;
        for (int s = 0; s < 3; ++s) {
          V3 p = v[s], q = v[(s + 1) % 3], r = v[(s + 2) % 3];
          double k = R2 * (tri_area(p, unit(p + q), o) + tri_area(p, o, unit(r + p)));
          kite[6 * P(i, j) + 3 * t + s] = k;
          sum += k;
        }
        cc[2 * P(i, j) + t] = o;
        Av[2 * P(i, j) + t] = sum;
        tv[2 * P(i, j) + t] = 1;
      }
  auto tvalid = [&](int64_t i, int64_t j, int t) { return inside(i, j) && tv[2 * P(i, j) + t]; };
  // cell areas and kite fractions
  std::vector<double> Ai(W2, 0.0), rho(6 * W2, 0.0);
  std::vector<uint8_t> cv(W2, 0);
  for (int64_t i = -G; i < n + G; ++i)
    for (int64_t j = -G; j < n + G; ++j) {
      bool ok = true;
      double k6[6];
      for (int k = 0; k < 6; ++k) {
        int64_t ti = i + VOI[k], tj = j + VOJ[k];
        if (!tvalid(ti, tj, VT[k])) { ok = false; break; }
        k6[k] = kite[6 * P(ti, tj) + 3 * VT[k] + VC[k]];
      }
      if (!ok) continue;
      double s = 0;
      for (int k = 0; k < 6; ++k) s += k6[k];
      Ai[P(i, j)] = s;
      for (int k = 0; k < 6; ++k) rho[6 * P(i, j) + k] = k6[k] / s;
      cv[P(i, j)] = 1;
    }
  auto cvalid = [&](int64_t i, int64_t j) { return inside(i, j) && cv[P(i, j)]; };
  // edges: d_e, l_e (adjacent triangles: E0: T0(P), T1(P-d2); E1: T0(P), T1(P); E2: T1(P), T0(P-d0))
  std::vector<double> de(3 * W2, 0.0), le(3 * W2, 0.0);
  std::vector<uint8_t> ev(3 * W2, 0);
  for (int64_t i = -G; i < n + G; ++i)
    for (int64_t j = -G; j < n + G; ++j)
      for (int d = 0; d < 3; ++d) {
        if (!pvalid(i, j) || !pvalid(i + D0[d], j + D1[d])) continue;
        int64_t ai = i, aj = j, bi = i, bj = j;
        int at = 0, bt = 1;
        if (d == 0) { bi = i; bj = j - 1; at = 0; bt = 1; }
        if (d == 1) { at = 0; bt = 1; }
        if (d == 2) { at = 1; bi = i - 1; bj = j; bt = 0; }
        if (!tvalid(ai, aj, at) || !tvalid(bi, bj, bt)) continue;
        de[3 * P(i, j) + d] = R * arc(pos[P(i, j)], pos[P(i + D0[d], j + D1[d])]);
        le[3 * P(i, j) + d] = R * arc(cc[2 * P(ai, aj) + at], cc[2 * P(bi, bj) + bt]);
        ev[3 * P(i, j) + d] = 1;
      }
  auto evalid = [&](int64_t i, int64_t j, int d) { return inside(i, j) && ev[3 * P(i, j) + d]; };
  // slot s of cell C -> frame edge (owner offset, direction)
  auto slot_edge = [&](int s, int64_t& oi, int64_t& oj, int& d) {
    if (s < 3) { oi = 0; oj = 0; d = s; }
    else { d = s - 3; oi = -D0[d]; oj = -D1[d]; }
  };
  H.tab.assign(size_t(LQ_COUNT) * W2, 0.0);
  auto T = [&](int q, int64_t p) -> double& { return H.tab[size_t(q) * W2 + p]; };
  for (int64_t i = -G; i < n + G; ++i)
    for (int64_t j = -G; j < n + G; ++j) {
      int64_t p = P(i, j);
      if (cvalid(i, j)) T(LQ_INVA, p) = 1.0 / Ai[p];
      for (int d = 0; d < 3; ++d)
        if (evalid(i, j, d)) {
          T(LQ_KC + d, p) = le[3 * p + d] * de[3 * p + d] / 4.0;
          T(LQ_LEN + d, p) = le[3 * p + d];
          T(LQ_INVD + d, p) = 1.0 / de[3 * p + d];
        }
      for (int t = 0; t < 2; ++t) {
        if (!tvalid(i, j, t)) continue;
        // sides: T0: E0(P) +, E2(P+d0) +, E1(P) - ; T1: E1(P) +, E0(P+d2) -, E2(P) -
        int64_t si[3], sj[3];
        int sd[3], sg[3];
        if (t == 0) {
          si[0] = i; sj[0] = j; sd[0] = 0; sg[0] = 1;
          si[1] = i + 1; sj[1] = j; sd[1] = 2; sg[1] = 1;
          si[2] = i; sj[2] = j; sd[2] = 1; sg[2] = -1;
        } else {
          si[0] = i; sj[0] = j; sd[0] = 1; sg[0] = 1;
          si[1] = i; sj[1] = j + 1; sd[1] = 0; sg[1] = -1;
          si[2] = i; sj[2] = j; sd[2] = 2; sg[2] = -1;
        }
        bool ok = true;
        for (int s = 0; s < 3; ++s) ok = ok && inside(si[s], sj[s]) && pvalid(si[s], sj[s]) &&
                                         pvalid(si[s] + D0[sd[s]], sj[s] + D1[sd[s]]);
        if (!ok) continue;
        for (int s = 0; s < 3; ++s) {
          double dd = R * arc(pos[P(si[s], sj[s])], pos[P(si[s] + D0[sd[s]], sj[s] + D1[sd[s]])]);
          T(LQ_CURL + 3 * t + s, p) = sg[s] * dd / Av[2 * p + t];
          T(LQ_R + 3 * t + s, p) = kite[6 * p + 3 * t + s] / Av[2 * p + t];
        }
        V3 o = cc[2 * p + t];
        T(LQ_CC + 3 * t + 0, p) = o.x;
        T(LQ_CC + 3 * t + 1, p) = o.y;
        T(LQ_CC + 3 * t + 2, p) = o.z;
      }
      // perpendicular-flux weights of frame edge d: cell A = P (edge in slot d), cell B = P+d_d
      // (edge in slot d+3); w = n_e n_e' (S - 1/2), S = kite/cell fractions passed.
      for (int d = 0; d < 3; ++d) {
        if (!evalid(i, j, d)) continue;
        int64_t bi = i + D0[d], bj = j + D1[d];
        if (!cvalid(i, j) || !cvalid(bi, bj)) continue;
        bool ok = true;
        double w[10], lk[10];
        for (int side = 0; side < 2 && ok; ++side) {
          int64_t ci = side ? bi : i, cj = side ? bj : j;
          int s0 = side ? d + 3 : d;
          double ne = side ? -1.0 : 1.0, S = 0;
          for (int step = 1; step < 6; ++step) {
            S += rho[6 * P(ci, cj) + (s0 + step - 1) % 6];
            int s = (s0 + step) % 6;
            int64_t oi, oj;
            int dd;
            slot_edge(s, oi, oj, dd);
            if (!evalid(ci + oi, cj + oj, dd)) { ok = false; break; }
            double nep = s < 3 ? 1.0 : -1.0;
            int k = side * 5 + step - 1;
            w[k] = ne * nep * (S - 0.5);
            lk[k] = le[3 * P(ci + oi, cj + oj) + dd];
          }
        }
        if (!ok) continue;
        for (int k = 0; k < 10; ++k) T(LQ_WL + 10 * d + k, p) = w[k] * lk[k] / de[3 * p + d];
      }
    }
  // rotation rows: lozenge 0 -> lozenge L maps corners c00, c10, c01 (columns) to those of L
  {
    auto corner_pos = [&](int L, int ci, int cj) { return Lv.pos[lat.node(L, ci * n, cj * n)]; };
    auto mat = [&](int L, double M[3][3]) {
      V3 c[3] = {corner_pos(L, 0, 0), corner_pos(L, 1, 0), corner_pos(L, 0, 1)};
      for (int r = 0; r < 3; ++r) {
        M[r][0] = r == 0 ? c[0].x : r == 1 ? c[0].y : c[0].z;
        M[r][1] = r == 0 ? c[1].x : r == 1 ? c[1].y : c[1].z;
        M[r][2] = r == 0 ? c[2].x : r == 1 ? c[2].y : c[2].z;
      }
    };
    double C0[3][3], inv[3][3];
    mat(0, C0);
    double det = C0[0][0] * (C0[1][1] * C0[2][2] - C0[1][2] * C0[2][1]) -
                 C0[0][1] * (C0[1][0] * C0[2][2] - C0[1][2] * C0[2][0]) +
                 C0[0][2] * (C0[1][0] * C0[2][1] - C0[1][1] * C0[2][0]);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
        inv[r][c] = (C0[r1][c1] * C0[r2][c2] - C0[r1][c2] * C0[r2][c1]) / det;
      }
    H.frot.assign(30, 0.0);
    for (int L = 0; L < 10; ++L) {
      double CL[3][3], RL[3][3];
      mat(L, CL);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double s = 0;
          for (int k = 0; k < 3; ++k) s += CL[r][k] * inv[k][c];
          RL[r][c] = s;
        }
      // check: a rotation that also maps corner c11
      V3 c11 = corner_pos(0, 1, 1), t = corner_pos(L, 1, 1);
      double m[3] = {RL[0][0] * c11.x + RL[0][1] * c11.y + RL[0][2] * c11.z,
                     RL[1][0] * c11.x + RL[1][1] * c11.y + RL[1][2] * c11.z,
                     RL[2][0] * c11.x + RL[2][1] * c11.y + RL[2][2] * c11.z};
      LAT_CHECK(std::fabs(m[0] - t.x) + std::fabs(m[1] - t.y) + std::fabs(m[2] - t.z) < 1e-12,
                "lozenges are not congruent");
      for (int c = 0; c < 3; ++c) H.frot[3 * L + c] = 2.0 * Lv.omega * RL[2][c];
    }
    // the kernel takes f from lozenge 0 for all northern lozenges and from lozenge 5 for all
    // southern ones: they are rotations of one another about the polar axis
    for (int L = 1; L < 10; ++L)
      if (L != 5)
        for (int c = 0; c < 3; ++c)
          LAT_CHECK(std::fabs(H.frot[3 * L + c] - H.frot[(L < 5 ? 0 : 15) + c]) < 1e-13 * 2.0 * Lv.omega,
                    "northern (southern) lozenges are not turned into one another about the polar axis");
  }
  // regular tiles: the halo (LT_G positions) contains no lozenge corner
  H.tiles.clear();
  std::vector<uint8_t> covered(10 * n * n, 0);
  for (int64_t i0 = 0; i0 + LT_TI <= n; i0 += LT_TI)
    for (int64_t j0 = 0; j0 + LT_TJ <= n; j0 += LT_TJ) {
      bool reg = true;
      const int M = LT_MARGIN;
      for (int64_t ci : {int64_t(0), n})
        for (int64_t cj : {int64_t(0), n})
          if (ci >= i0 - M && ci < i0 + LT_TI + M && cj >= j0 - M && cj < j0 + LT_TJ + M) reg = false;
      if (!reg) continue;
      // the halo addressing of the lattice kernel (seam rules in registers) must give the
      // canonical node and edges of every halo point, in bounds, in every lozenge
      for (int L = 0; L < 10; ++L)
        for (int64_t i = i0 - 2; i < i0 + LT_TI + 2; ++i)
          for (int64_t j = j0 - 2; j < j0 + LT_TJ + 2; ++j) {
            if (i >= 0 && i < n && j >= 0 && j < n) continue;
            int64_t node, edge[3];
            int sign[3];
            kernel_halo_address(L, i, j, n, node, edge, sign);
            LAT_CHECK(node == lat.node(L, i, j), "halo node address");
            for (int d = 0; d < 3; ++d) {
              LAT_CHECK(edge[d] >= 0 && edge[d] < 30 * n * n, "halo edge out of bounds");
              int sg;
              int64_t e = lat.edge(lat.node(L, i, j), lat.node(L, i + D0[d], j + D1[d]), sg);
              LAT_CHECK(e == edge[d] && sg == sign[d], "halo edge address");
            }
          }
      // every geometry quantity the tile reads must be defined
      for (int64_t i = i0 - 2; i < i0 + LT_TI + 2; ++i)
        for (int64_t j = j0 - 2; j < j0 + LT_TJ + 2; ++j)
          LAT_CHECK(pvalid(i, j), "regular tile reads an irregular point");
      for (int64_t i = i0 - 1; i < i0 + LT_TI + 1; ++i)
        for (int64_t j = j0 - 1; j < j0 + LT_TJ + 1; ++j)
          LAT_CHECK(cvalid(i, j) && evalid(i, j, 0) && evalid(i, j, 1) && evalid(i, j, 2),
                    "regular tile reads undefined geometry");
      H.tiles.push_back(int32_t(i0));
      H.tiles.push_back(int32_t(j0));
      for (int L = 0; L < 10; ++L)
        for (int64_t i = i0; i < i0 + LT_TI; ++i)
          for (int64_t j = j0; j < j0 + LT_TJ; ++j) covered[(int64_t(L) * n + i) * n + j] = 1;
    }
  // rim: uncovered elements and the poles; support rings over node adjacency
  std::vector<uint8_t> ring(Lv.N, 0);
  H.rim_elems.clear();
  for (int64_t id = 0; id < Lv.N; ++id)
    if (id >= 10 * n * n || !covered[id]) {
      H.rim_elems.push_back(int32_t(id));
      ring[id] = 1;
    }
  auto dilate = [&](std::vector<uint8_t>& r) {
    std::vector<uint8_t> o = r;
    for (int64_t id = 0; id < Lv.N; ++id) {
      if (!r[id]) continue;
      for (int k = 0; k < Lv.c_deg[id]; ++k) {
        int64_t e = Lv.c_e[6 * id + k];
        o[Lv.e_c[2 * e]] = 1;
        o[Lv.e_c[2 * e + 1]] = 1;
      }
    }
    r.swap(o);
  };
  dilate(ring);
  dilate(ring);
  H.sup_elems.clear();
  for (int64_t id = 0; id < Lv.N; ++id)
    if (ring[id]) H.sup_elems.push_back(int32_t(id));
  dilate(ring);
  H.sup_tris.clear();
  for (int64_t id = 0; id < 10 * n * n; ++id)
    if (ring[id]) {
      H.sup_tris.push_back(int32_t(2 * id));
      H.sup_tris.push_back(int32_t(2 * id + 1));
    }
  return !H.tiles.empty();
}

}  // namespace wt
