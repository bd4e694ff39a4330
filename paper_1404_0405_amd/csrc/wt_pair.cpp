// Inter-scale tables between levels j and j+1 (Sec. 2.2, 4.1-4.4).
#include "wt_pair.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <thread>

namespace wt {

#define PAIR_CHECK(c, msg)                                                       \
  do {                                                                           \
    if (!(c)) {                                                                  \
      std::fprintf(stderr, "wt pair: %s (%s:%d)\n", msg, __FILE__, __LINE__);   \
      std::abort();                                                              \
    }                                                                            \
  } while (0)

template <class F>
static void pfor(int64_t n, F f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 2048) nt = 1;
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t b = t * chunk, e = std::min<int64_t>(n, b + chunk);
    if (b >= e) break;
    th.emplace_back([=, &f] {
      for (int64_t k = b; k < e; ++k) f(k);
    });
  }
  for (auto& t : th) t.join();
}

// ---------------------------------------------------------------- spherical clipping
// Intersection of two convex spherical polygons (counter-clockwise, smaller than a
// hemisphere): the subject polygon is cut successively by the great-circle half-spaces
// {x : x . (q_j x q_j+1) >= 0} of the clip polygon's edges; the area of the result is a fan
// of spherical triangles.
double sph_overlap(const V3* P, int np, const V3* Q, int nq) {
  V3 buf[2][40];
  int n = np;
  for (int i = 0; i < np; ++i) buf[0][i] = P[i];
  int cur = 0;
  for (int j = 0; j < nq && n > 0; ++j) {
    V3 nrm = cross(Q[j], Q[(j + 1) % nq]);
    int m = 0;
    const V3* in = buf[cur];
    V3* out = buf[1 - cur];
    for (int i = 0; i < n; ++i) {
      V3 s = in[i], e = in[(i + 1) % n];
      double ds = dot(s, nrm), de = dot(e, nrm);
      bool si = ds >= 0.0, ei = de >= 0.0;
      if (si && m < 40) out[m++] = s;
      if (si != ei && m < 40) out[m++] = unit(std::fabs(de) * s + std::fabs(ds) * e);
    }
    n = m;
    cur = 1 - cur;
  }
  if (n < 3) return 0.0;
  double a = 0.0;
  for (int i = 1; i + 1 < n; ++i) a += tri_area(buf[cur][0], buf[cur][i], buf[cur][i + 1]);
  return a;
}

static void cell_poly(const Level& L, int64_t node, V3* out, int& n) {
  n = L.c_deg[node];
  for (int k = 0; k < n; ++k) out[k] = L.cc[L.c_t[6 * node + k]];
}

static int64_t third(const Level& L, int64_t t, int64_t a, int64_t b) {
  for (int s = 0; s < 3; ++s) {
    int64_t v = L.t_n[3 * t + s];
    if (v != a && v != b) return v;
  }
  PAIR_CHECK(false, "degenerate triangle");
  return -1;
}

// ---------------------------------------------------------------- velocity frames
// Linear tangent field V(xi) = a + G xi in gnomonic coordinates about a triangle's
// circumcentre; one design-matrix row per (point, tangent).
struct Frame {
  V3 c, b1, b2;
  double scale;
};
static Frame make_frame(V3 c) {
  Frame f;
  f.c = c;
  V3 ref = std::fabs(c.z) < 0.9 ? V3{0, 0, 1} : V3{1, 0, 0};
  f.b1 = unit(cross(ref, c));
  f.b2 = cross(c, f.b1);
  f.scale = 1.0;
  return f;
}
static void xi_of(const Frame& f, V3 x, double& x1, double& x2) {
  double cx = dot(x, f.c);
  x1 = dot(x, f.b1) / cx;
  x2 = dot(x, f.b2) / cx;
}
static void row_of(const Frame& f, V3 x, V3 t, double* r) {
  double x1, x2;
  xi_of(f, x, x1, x2);
  x1 /= f.scale;
  x2 /= f.scale;
  double t1 = dot(t, f.b1), t2 = dot(t, f.b2), nr = std::sqrt(t1 * t1 + t2 * t2);
  t1 /= nr;
  t2 /= nr;
  r[0] = t1; r[1] = t2; r[2] = t1 * x1; r[3] = t1 * x2; r[4] = t2 * x1; r[5] = t2 * x2;
}

// Solve the 6x6 normal equations M X = Phi^T for X (6x9) by Gaussian elimination with
// partial pivoting.
static void normal_solve(const double rows[9][6], double out[6][9]) {
  double M[6][6 + 9];
  for (int a = 0; a < 6; ++a) {
    for (int b = 0; b < 6; ++b) {
      double s = 0;
      for (int k = 0; k < 9; ++k) s += rows[k][a] * rows[k][b];
      M[a][b] = s;
    }
    for (int k = 0; k < 9; ++k) M[a][6 + k] = rows[k][a];
  }
  for (int col = 0; col < 6; ++col) {
    int piv = col;
    for (int r = col + 1; r < 6; ++r)
      if (std::fabs(M[r][col]) > std::fabs(M[piv][col])) piv = r;
    PAIR_CHECK(std::fabs(M[piv][col]) > 1e-300, "singular velocity fit");
    if (piv != col)
      for (int c = 0; c < 15; ++c) std::swap(M[piv][c], M[col][c]);
    for (int r = 0; r < 6; ++r) {
      if (r == col) continue;
      double f = M[r][col] / M[col][col];
      if (f == 0.0) continue;
      for (int c = col; c < 15; ++c) M[r][c] -= f * M[col][c];
    }
  }
  for (int a = 0; a < 6; ++a)
    for (int k = 0; k < 9; ++k) out[a][k] = M[a][6 + k] / M[a][a];
}

// ---------------------------------------------------------------- build
void build_pair(const Level& C, const Level& F, PairTables& P) {
  PAIR_CHECK(F.J == C.J + 1, "levels not consecutive");
  Lattice lc(C.J), lf(F.J);
  P.Nc = C.N; P.Ec = C.E; P.Tc = C.T; P.Nf = F.N; P.Ef = F.E;
  const int64_t nc = C.n, nf = F.n;
  static const int DI[3] = {1, 1, 0}, DJ[3] = {0, 1, 1};
  P.even.resize(C.N);
  pfor(C.N, [&](int64_t k) {
    int L;
    int64_t i, j;
    if (lc.decode(k, L, i, j))
      P.even[k] = int32_t((int64_t(L) * nf + 2 * i) * nf + 2 * j);
    else
      P.even[k] = int32_t(10 * nf * nf + (k - 10 * nc * nc));
  });
  P.mid.resize(C.E); P.h1.resize(C.E); P.h2.resize(C.E); P.cells.resize(4 * C.E);
  pfor(C.E, [&](int64_t e) {
    int64_t id = e / 3;
    int d = int(e % 3);
    int L;
    int64_t i, j;
    lc.decode(id, L, i, j);
    int64_t f0 = (int64_t(L) * nf + 2 * i) * nf + 2 * j;
    int64_t fm = (int64_t(L) * nf + 2 * i + DI[d]) * nf + 2 * j + DJ[d];
    P.mid[e] = int32_t(fm);
    P.h1[e] = int32_t(3 * f0 + d);
    P.h2[e] = int32_t(3 * fm + d);
    int64_t a = C.e_c[2 * e], b = C.e_c[2 * e + 1];
    P.cells[4 * e] = int32_t(a);
    P.cells[4 * e + 1] = int32_t(b);
    P.cells[4 * e + 2] = int32_t(third(C, C.e_v[2 * e], a, b));
    P.cells[4 * e + 3] = int32_t(third(C, C.e_v[2 * e + 1], a, b));
    PAIR_CHECK(F.e_c[2 * P.h1[e]] == P.even[a] && F.e_c[2 * P.h2[e] + 1] == P.even[b], "half-edge map");
  });
  // overlap areas of the fine hexagon of each odd node with its four coarse cells
  P.area_geo.resize(4 * C.E);
  P.st.resize(4 * C.E);
  const double R2 = C.radius * C.radius;
  pfor(C.E, [&](int64_t e) {
    V3 pm[6], pc[6];
    int npm, npc;
    cell_poly(F, P.mid[e], pm, npm);
    double s = 0;
    for (int c = 0; c < 4; ++c) {
      cell_poly(C, P.cells[4 * e + c], pc, npc);
      double a = R2 * sph_overlap(pm, npm, pc, npc);
      P.area_geo[4 * e + c] = a;
      s += a;
    }
    PAIR_CHECK(std::fabs(s / F.A_i[P.mid[e]] - 1.0) < 1e-9, "coarse cells do not cover the fine cell");
    for (int c = 0; c < 4; ++c) P.st[4 * e + c] = P.area_geo[4 * e + c] / s;
  });
  // odd nodes sharing area with each coarse node
  P.mk.assign(MK_MAX * C.N, -1);
  {
    std::vector<int> cnt(C.N, 0);
    for (int64_t e = 0; e < C.E; ++e)
      for (int c = 0; c < 4; ++c) {
        int64_t k = P.cells[4 * e + c];
        PAIR_CHECK(cnt[k] < MK_MAX, "too many odd nodes around a cell");
        P.mk[MK_MAX * k + cnt[k]++] = int32_t(4 * e + c);
      }
  }
  // interior fine edges of every coarse triangle
  P.int_e.resize(3 * C.T);
  pfor(C.T, [&](int64_t t) {
    for (int s = 0; s < 3; ++s) {
      int64_t ma = P.mid[C.t_e[3 * t + s]], mb = P.mid[C.t_e[3 * t + (s + 1) % 3]];
      int sg;
      P.int_e[3 * t + s] = int32_t(lf.edge(ma, mb, sg));
    }
  });
  // velocity prediction: 9-edge stencil, least-squares linear field per coarse triangle
  P.v_sten.resize(9 * C.T);
  P.w_int.resize(27 * C.T);
  std::vector<double> pinv(54 * C.T);
  std::vector<Frame> frames(C.T);
  auto emid = [](const Level& L, int64_t e) { return unit(L.pos[L.e_c[2 * e]] + L.pos[L.e_c[2 * e + 1]]); };
  auto etan = [](const Level& L, int64_t e) { return unit(L.pos[L.e_c[2 * e + 1]] - L.pos[L.e_c[2 * e]]); };
  pfor(C.T, [&](int64_t t) {
    int32_t* st = &P.v_sten[9 * t];
    for (int s = 0; s < 3; ++s) st[s] = C.t_e[3 * t + s];
    for (int s = 0; s < 3; ++s) {
      int64_t e = C.t_e[3 * t + s];
      int64_t nb = C.e_v[2 * e] == t ? C.e_v[2 * e + 1] : C.e_v[2 * e];
      int w = 0;
      for (int q = 0; q < 3; ++q)
        if (C.t_e[3 * nb + q] != e) st[3 + 2 * s + w++] = C.t_e[3 * nb + q];
      PAIR_CHECK(w == 2, "neighbour triangle");
    }
    Frame fr = make_frame(C.cc[t]);
    double sc = 0;
    for (int k = 0; k < 9; ++k) {
      double x1, x2;
      xi_of(fr, emid(C, st[k]), x1, x2);
      sc += std::sqrt(x1 * x1 + x2 * x2);
    }
    fr.scale = sc / 9.0;
    frames[t] = fr;
    double rows[9][6], X[6][9];
    for (int k = 0; k < 9; ++k) row_of(fr, emid(C, st[k]), etan(C, st[k]), rows[k]);
    normal_solve(rows, X);
    for (int a = 0; a < 6; ++a)
      for (int k = 0; k < 9; ++k) pinv[54 * t + 9 * a + k] = X[a][k];
    for (int s = 0; s < 3; ++s) {
      int64_t f = P.int_e[3 * t + s];
      double r[6];
      row_of(fr, emid(F, f), etan(F, f), r);
      for (int k = 0; k < 9; ++k) {
        double w = 0;
        for (int a = 0; a < 6; ++a) w += r[a] * X[a][k];
        P.w_int[27 * t + 9 * s + k] = w;
      }
    }
  });
  P.w_pl.resize(9 * C.E);
  P.w_pr.resize(9 * C.E);
  pfor(C.E, [&](int64_t e) {
    V3 x1 = emid(F, P.h1[e]), x2 = emid(F, P.h2[e]);
    V3 t1 = etan(F, P.h1[e]), t2 = etan(F, P.h2[e]);
    for (int side = 0; side < 2; ++side) {
      int64_t t = C.e_v[2 * e + side];
      double r1[6], r2[6];
      row_of(frames[t], x1, t1, r1);
      row_of(frames[t], x2, t2, r2);
      double* out = side == 0 ? &P.w_pl[9 * e] : &P.w_pr[9 * e];
      for (int k = 0; k < 9; ++k) {
        double w = 0;
        for (int a = 0; a < 6; ++a) w += (r1[a] - r2[a]) * pinv[54 * t + 9 * a + k];
        out[k] = 0.5 * w;
      }
    }
  });
}

// Terms of the flux restriction generated by the odd node of coarse edge e2 (routing of its
// small pieces and its corrective exchanges), as (coarse edge, fine node, weight) triples on
// integrated fluxes oriented along each coarse edge.
struct RFTerm {
  int64_t edge, node;
  double w;
};
static void odd_node_terms(const Lattice& lc, const PairTables& P, const std::vector<double>& Af,
                           int64_t e2, std::vector<RFTerm>& out) {
  const int32_t* cl = &P.cells[4 * e2];
  const double* A = &P.aov[4 * e2];
  const double Am = Af[P.mid[e2]];
  int64_t m = P.mid[e2];
  // small pieces in p (column 2) and q (column 3) flow to a and b in proportion A_a : A_b
  for (int col = 2; col < 4; ++col)
    for (int tgt = 0; tgt < 2; ++tgt) {
      int sg;
      int64_t e = lc.edge(cl[col], cl[tgt], sg);
      out.push_back({e, m, sg * A[col] * A[tgt] / (A[0] + A[1])});
    }
  // corrective exchanges between neighbouring overlapping cells
  static const int PR[5][2] = {{0, 1}, {0, 2}, {1, 2}, {0, 3}, {1, 3}};
  for (auto& pr : PR) {
    int sg;
    int64_t e = lc.edge(cl[pr[0]], cl[pr[1]], sg);
    double X = A[pr[0]] * A[pr[1]] / Am;
    out.push_back({e, P.even[cl[pr[0]]], sg * X});
    out.push_back({e, P.even[cl[pr[1]]], -sg * X});
  }
  // p and q are not neighbours: half of their exchange through a, half through b
  double Xpq = 0.5 * A[2] * A[3] / Am;
  for (int via = 0; via < 2; ++via) {
    int sg;
    int64_t e = lc.edge(cl[2], cl[via], sg);
    out.push_back({e, P.even[cl[2]], sg * Xpq});
    out.push_back({e, P.even[cl[3]], -sg * Xpq});
    e = lc.edge(cl[via], cl[3], sg);
    out.push_back({e, P.even[cl[2]], sg * Xpq});
    out.push_back({e, P.even[cl[3]], -sg * Xpq});
  }
}

void finish_pair(const Level& C, const Level& F, const std::vector<double>& Af, PairTables& P,
                 std::vector<double>& Ac) {
  Lattice lc(C.J), lf(F.J);
  P.aov.resize(4 * C.E);
  for (int64_t q = 0; q < 4 * C.E; ++q) P.aov[q] = P.st[q] * Af[P.mid[q / 4]];
  Ac.assign(C.N, 0.0);
  pfor(C.N, [&](int64_t k) {
    double s = Af[P.even[k]];
    for (int q = 0; q < MK_MAX; ++q) {
      int32_t ec = P.mk[MK_MAX * k + q];
      if (ec >= 0) s += P.aov[ec];
    }
    Ac[k] = s;
  });
  P.s_upd.resize(4 * C.E);
  for (int64_t q = 0; q < 4 * C.E; ++q) P.s_upd[q] = P.aov[q] / Ac[P.cells[q]];
  // flux restriction rows: every term on coarse edge e comes from the odd node of e or of
  // the four other edges of its two triangles
  P.rf_f.assign(3 * C.E, 0);
  P.rf_fw.assign(3 * C.E, 0.0);
  P.rf_c.assign(RF_NC * C.E, 0);
  P.rf_cw.assign(RF_NC * C.E, 0.0);
  pfor(C.E, [&](int64_t e) {
    const int32_t* cl = &P.cells[4 * e];
    int64_t a = cl[0], b = cl[1], p = cl[2], q = cl[3];
    int64_t m = P.mid[e];
    int sg;
    int64_t eap = lc.edge(a, p, sg), eaq = lc.edge(a, q, sg), ebp = lc.edge(b, p, sg),
            ebq = lc.edge(b, q, sg);
    // basic part: inflow into m through its three a-side fine edges + alpha A_m c_m
    int64_t xs[3] = {P.even[a], P.mid[eap], P.mid[eaq]};
    for (int k = 0; k < 3; ++k) {
      int64_t f = lf.edge(m, xs[k], sg);
      P.rf_f[3 * e + k] = int32_t(f);
      P.rf_fw[3 * e + k] = -double(sg);
    }
    std::map<int64_t, double> cw;
    const double* A = &P.aov[4 * e];
    cw[m] += A[0] / (A[0] + A[1]) * Af[m];
    std::vector<RFTerm> terms;
    for (int64_t e2 : {e, eap, eaq, ebp, ebq}) odd_node_terms(lc, P, Af, e2, terms);
    for (auto& t : terms)
      if (t.edge == e) cw[t.node] += t.w;
    // nodes whose terms cancel exactly carry no weight: drop them (the sum is unchanged)
    int k = 0;
    for (auto& kv : cw) {
      if (kv.second == 0.0) continue;
      PAIR_CHECK(k < RF_NC, "flux restriction stencil too wide");
      P.rf_c[RF_NC * e + k] = int32_t(kv.first);
      P.rf_cw[RF_NC * e + k] = kv.second;
      ++k;
    }
    for (; k < RF_NC; ++k) {
      P.rf_c[RF_NC * e + k] = int32_t(m);
      P.rf_cw[RF_NC * e + k] = 0.0;
    }
  });
}

}  // namespace wt
