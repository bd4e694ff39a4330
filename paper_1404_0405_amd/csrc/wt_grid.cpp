// Host construction of one grid level: positions by recursive arc bisection, topology through
// the lozenge seam rules, spherical geometry (Sec. 4.1) and TRiSK weights (Sec. 3.1).
#include "wt_grid.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <thread>

namespace wt {

#define WT_CHECK(c, msg)                                                   \
  do {                                                                     \
    if (!(c)) {                                                            \
      std::fprintf(stderr, "wt grid: %s (%s:%d)\n", msg, __FILE__, __LINE__); \
      std::abort();                                                        \
    }                                                                      \
  } while (0)

template <class F>
static void parallel_for(int64_t n, F f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 4096) nt = 1;
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

V3 unit(V3 a) {
  double s = std::sqrt(dot(a, a));
  return {a.x / s, a.y / s, a.z / s};
}

// Geometry of small figures on the unit sphere, written so that rounding is not amplified by
// the figure's size h: vertex differences of nearby points are exact (Sterbenz), so triple and
// cross products are formed from differences; and the normalised positions' residual length
// error |x|^2 - 1 (~1e-16, which a plane through three points would turn into an O(1e-16/h)
// tilt) is computed exactly with fma and removed from direction differences.
static double norm2_minus_one(V3 a) {
  const double v[3] = {a.x, a.y, a.z};
  double t[7];
  for (int k = 0; k < 3; ++k) {
    t[2 * k] = v[k] * v[k];
    t[2 * k + 1] = std::fma(v[k], v[k], -t[2 * k]);
  }
  t[6] = -1.0;
  double s = t[0], c = 0.0;  // Neumaier summation
  for (int k = 1; k < 7; ++k) {
    double u = s + t[k];
    c += std::fabs(s) >= std::fabs(t[k]) ? (s - u) + t[k] : (t[k] - u) + s;
    s = u;
  }
  return s + c;
}
// b/|b| - a/|a| to full relative precision for nearby nearly-unit vectors
static V3 dir_diff(V3 b, V3 a) {
  double sa = 0.5 * norm2_minus_one(a), sb = 0.5 * norm2_minus_one(b);
  return (b - a) + (sa * a - sb * b);
}
V3 circumcentre(V3 a, V3 b, V3 c) { return unit(cross(dir_diff(b, a), dir_diff(c, a))); }
double arc(V3 a, V3 b) {
  V3 c = cross(a - b, b);
  return std::atan2(std::sqrt(dot(c, c)), dot(a, b));
}
double tri_area(V3 a, V3 b, V3 c) {
  double num = dot(a - c, cross(b - c, c));
  double den = 1.0 + dot(a, b) + dot(b, c) + dot(c, a);
  return 2.0 * std::atan2(num, den);
}

// ------------------------------------------------------------------ lattice numbering
Lattice::Lattice(int J_) : J(J_) {
  n = int64_t(1) << J;
  N = 10 * n * n + 2;
  E = 30 * n * n;
  T = 20 * n * n;
}

// Seam rules.  Lozenge k (north, 0..4) has corners c00=U_k, c10=L_k, c11=U_k+1, c01=N;
// lozenge 5+k (south) has c00=L_k, c10=S, c11=L_k+1, c01=U_k+1.  Crossing a side either
// translates the lattice (same orientation) or rotates it by 60 degrees.
int64_t Lattice::node(int L, int64_t i, int64_t j) const {
  for (int it = 0; it < 4; ++it) {
    if (i >= 0 && i < n && j >= 0 && j < n) return (int64_t(L) * n + i) * n + j;
    const bool north = L < 5;
    const int k = north ? L : L - 5;
    const int km = (k + 4) % 5, kp = (k + 1) % 5;
    int64_t ni = i, nj = j;
    if (north) {
      if (i == 0 && j == n) return 10 * n * n;
      if (i < 0) { L = km; ni = n + i - j; nj = n + i; }
      else if (j < 0) { L = 5 + km; nj = n + j; }
      else if (i >= n) { L = 5 + k; ni = i - n; }
      else { L = kp; ni = j - n; nj = j - i; }
    } else {
      if (i == n && j == 0) return 10 * n * n + 1;
      if (i < 0) { L = k; ni = n + i; }
      else if (j < 0) { L = 5 + km; ni = n + j; nj = n + j - i; }
      else if (i >= n) { L = 5 + kp; ni = i - j; nj = i - n; }
      else { L = kp; nj = j - n; }
    }
    i = ni;
    j = nj;
  }
  WT_CHECK(false, "lattice point in a corner wedge");
  return -1;
}

bool Lattice::decode(int64_t id, int& L, int64_t& i, int64_t& j) const {
  if (id >= 10 * n * n) return false;
  L = int(id / (n * n));
  i = (id / n) % n;
  j = id % n;
  return true;
}

static const int DI[3] = {1, 1, 0}, DJ[3] = {0, 1, 1};

int64_t Lattice::edge(int64_t a, int64_t b, int& sign) const {
  int L;
  int64_t i, j;
  if (decode(a, L, i, j))
    for (int d = 0; d < 3; ++d)
      if (node(L, i + DI[d], j + DJ[d]) == b) { sign = 1; return 3 * a + d; }
  if (decode(b, L, i, j))
    for (int d = 0; d < 3; ++d)
      if (node(L, i + DI[d], j + DJ[d]) == a) { sign = -1; return 3 * b + d; }
  WT_CHECK(false, "no edge between nodes");
  return -1;
}

// ------------------------------------------------------------------ construction
static void corners(V3 c[10][4]) {
  const double s = 1.0 / std::sqrt(5.0), r = 2.0 / std::sqrt(5.0);
  V3 U[5], Lw[5];
  for (int k = 0; k < 5; ++k) {
    double a = 2.0 * M_PI * k / 5.0, b = a + M_PI / 5.0;
    U[k] = {r * std::cos(a), r * std::sin(a), s};
    Lw[k] = {r * std::cos(b), r * std::sin(b), -s};
  }
  const V3 Np{0, 0, 1}, Sp{0, 0, -1};
  for (int k = 0; k < 5; ++k) {
    int kp = (k + 1) % 5;
    c[k][0] = U[k]; c[k][1] = Lw[k]; c[k][2] = U[kp]; c[k][3] = Np;
    c[5 + k][0] = Lw[k]; c[5 + k][1] = Sp; c[5 + k][2] = Lw[kp]; c[5 + k][3] = U[kp];
  }
}

// positions of the closed lattice of one lozenge, refined J times
static void lozenge_positions(const V3 c[4], int J, std::vector<V3>& P) {
  int64_t m = 1;
  P = {c[0], c[3], c[1], c[2]};  // row-major (i,j): (0,0),(0,1),(1,0),(1,1)
  for (int lev = 0; lev < J; ++lev) {
    int64_t M = 2 * m, w = m + 1, W = M + 1;
    std::vector<V3> Q(W * W);
    for (int64_t i = 0; i <= M; ++i)
      for (int64_t j = 0; j <= M; ++j) {
        V3 v;
        if (i % 2 == 0 && j % 2 == 0) v = P[(i / 2) * w + j / 2];
        else if (j % 2 == 0) v = unit(P[(i / 2) * w + j / 2] + P[(i / 2 + 1) * w + j / 2]);
        else if (i % 2 == 0) v = unit(P[(i / 2) * w + j / 2] + P[(i / 2) * w + j / 2 + 1]);
        else v = unit(P[(i / 2) * w + j / 2] + P[(i / 2 + 1) * w + j / 2 + 1]);
        Q[i * W + j] = v;
      }
    P.swap(Q);
    m = M;
  }
}

void build_level(int J, double radius, double omega, Level& G) {
  Lattice lat(J);
  const int64_t n = lat.n, N = lat.N, E = lat.E, T = lat.T;
  G.J = J; G.n = n; G.N = N; G.E = E; G.T = T;
  G.radius = radius; G.omega = omega;
  WT_CHECK(T < (int64_t(1) << 31), "level too large for 32-bit tables");

  // positions
  G.pos.assign(N, V3{0, 0, 0});
  V3 c[10][4];
  corners(c);
  parallel_for(10, [&](int64_t L) {
    std::vector<V3> P;
    lozenge_positions(c[L], J, P);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) G.pos[(L * n + i) * n + j] = P[i * (n + 1) + j];
  });
  G.pos[10 * n * n] = {0, 0, 1};
  G.pos[10 * n * n + 1] = {0, 0, -1};

  // triangles (owned by elements)
  G.t_n.assign(3 * T, -1);
  G.t_e.assign(3 * T, -1);
  G.t_s.assign(3 * T, 0);
  parallel_for(10 * n * n, [&](int64_t id) {
    int L;
    int64_t i, j;
    lat.decode(id, L, i, j);
    int64_t p = id, p10 = lat.node(L, i + 1, j), p11 = lat.node(L, i + 1, j + 1),
            p01 = lat.node(L, i, j + 1);
    int64_t tri[2][3] = {{p, p10, p11}, {p, p11, p01}};
    for (int t = 0; t < 2; ++t)
      for (int s = 0; s < 3; ++s) {
        int64_t a = tri[t][s], b = tri[t][(s + 1) % 3];
        int sg;
        int64_t e = lat.edge(a, b, sg);
        G.t_n[3 * (2 * id + t) + s] = int32_t(a);
        G.t_e[3 * (2 * id + t) + s] = int32_t(e);
        G.t_s[3 * (2 * id + t) + s] = int8_t(sg);
      }
  });

  // edges: end nodes, adjacent triangles
  G.e_c.assign(2 * E, -1);
  G.e_v.assign(2 * E, -1);
  parallel_for(10 * n * n, [&](int64_t id) {
    int L;
    int64_t i, j;
    lat.decode(id, L, i, j);
    for (int d = 0; d < 3; ++d) {
      G.e_c[2 * (3 * id + d)] = int32_t(id);
      G.e_c[2 * (3 * id + d) + 1] = int32_t(lat.node(L, i + DI[d], j + DJ[d]));
    }
  });
  for (int64_t t = 0; t < T; ++t)
    for (int s = 0; s < 3; ++s) {
      int64_t e = G.t_e[3 * t + s];
      int slot = G.t_s[3 * t + s] > 0 ? 0 : 1;
      WT_CHECK(G.e_v[2 * e + slot] < 0, "edge with two triangles on one side");
      G.e_v[2 * e + slot] = int32_t(t);
    }

  // cells: edges in counter-clockwise lattice order; vertex k between edge k and k+1
  G.c_e.assign(6 * N, -1);
  G.c_s.assign(6 * N, 0);
  G.c_t.assign(6 * N, -1);
  G.c_deg.assign(N, 0);
  static const int SI[6] = {1, 1, 0, -1, -1, 0}, SJ[6] = {0, 1, 1, 0, -1, -1};
  auto fill_cell = [&](int64_t id, const int64_t* nb, int deg) {
    for (int k = 0; k < deg; ++k) {
      int sg;
      int64_t e = lat.edge(id, nb[k], sg);
      G.c_e[6 * id + k] = int32_t(e);
      G.c_s[6 * id + k] = int8_t(sg);
      G.c_t[6 * id + k] = G.e_v[2 * e + (sg > 0 ? 0 : 1)];
    }
    G.c_deg[id] = uint8_t(deg);
  };
  parallel_for(10 * n * n, [&](int64_t id) {
    int L;
    int64_t i, j;
    lat.decode(id, L, i, j);
    int64_t nb[6];
    int deg = 0;
    for (int k = 0; k < 6; ++k) {
      if (i == 0 && j == 0 && k == 4) continue;  // pentagon: no (-1,-1) neighbour
      nb[deg++] = lat.node(L, i + SI[k], j + SJ[k]);
    }
    fill_cell(id, nb, deg);
  });
  {
    int64_t nb[5];
    for (int k = 0; k < 5; ++k) nb[k] = (int64_t(k) * n + 0) * n + (n - 1);  // north: (0,n-1) of N_k
    fill_cell(10 * n * n, nb, 5);
    for (int k = 0; k < 5; ++k) nb[k] = (int64_t(5 + 4 - k) * n + (n - 1)) * n + 0;  // south: (n-1,0)
    fill_cell(10 * n * n + 1, nb, 5);
  }

  // consistency: each vertex k is also adjacent to edge k+1, triangles counter-clockwise
  parallel_for(N, [&](int64_t id) {
    int deg = G.c_deg[id];
    for (int k = 0; k < deg; ++k) {
      int kn = (k + 1) % deg;
      int64_t e = G.c_e[6 * id + kn];
      int32_t right = G.e_v[2 * e + (G.c_s[6 * id + kn] > 0 ? 1 : 0)];
      WT_CHECK(right == G.c_t[6 * id + k], "cell edges not counter-clockwise");
    }
  });

  // ---------------------------------------------------------------- geometry
  const double R = radius, R2 = radius * radius;
  G.cc.resize(T);
  G.f_v.resize(T);
  G.kite.resize(3 * T);
  G.A_v.resize(T);
  parallel_for(T, [&](int64_t t) {
    V3 a = G.pos[G.t_n[3 * t]], b = G.pos[G.t_n[3 * t + 1]], c3 = G.pos[G.t_n[3 * t + 2]];
    WT_CHECK(tri_area(a, b, c3) > 0, "triangle not counter-clockwise");
    V3 cc = circumcentre(a, b, c3);
    G.cc[t] = cc;
    G.f_v[t] = 2.0 * omega * cc.z;
    double sum = 0;
    for (int s = 0; s < 3; ++s) {
      V3 p = G.pos[G.t_n[3 * t + s]], q = G.pos[G.t_n[3 * t + (s + 1) % 3]],
         r = G.pos[G.t_n[3 * t + (s + 2) % 3]];
      double k = R2 * (tri_area(p, unit(p + q), cc) + tri_area(p, cc, unit(r + p)));
      WT_CHECK(k > 0, "circumcentre outside triangle");
      G.kite[3 * t + s] = k;
      sum += k;
    }
    G.A_v[t] = sum;
  });
  G.A_i.assign(N, 0.0);
  parallel_for(N, [&](int64_t id) {
    double s = 0;
    for (int k = 0; k < G.c_deg[id]; ++k) {
      int64_t t = G.c_t[6 * id + k];
      for (int q = 0; q < 3; ++q)
        if (G.t_n[3 * t + q] == id) s += G.kite[3 * t + q];
    }
    G.A_i[id] = s;
  });
  G.d_e.resize(E);
  G.l_e.resize(E);
  parallel_for(E, [&](int64_t e) {
    G.d_e[e] = R * arc(G.pos[G.e_c[2 * e]], G.pos[G.e_c[2 * e + 1]]);
    G.l_e[e] = R * arc(G.cc[G.e_v[2 * e]], G.cc[G.e_v[2 * e + 1]]);
  });

  // ---------------------------------------------------------------- TRiSK weights
  // Per cell, the outward fluxes are spread over the kites so that each kite carries its
  // area share of the divergence; the fluxes across the half dual edges that result give
  // w_{e,e'} = n_{e,i} n_{e',i} (S - 1/2), S = kite/cell fractions passed going
  // counter-clockwise from e to e'.  Antisymmetric, hence energy neutral.
  G.ecp.assign(10 * E, 0);
  G.w.assign(10 * E, 0.0);
  parallel_for(E, [&](int64_t e) {
    int fill = 0;
    for (int side = 0; side < 2; ++side) {
      int64_t cell = G.e_c[2 * e + side];
      int deg = G.c_deg[cell];
      int me = -1;
      for (int k = 0; k < deg; ++k)
        if (G.c_e[6 * cell + k] == e) me = k;
      WT_CHECK(me >= 0, "edge missing from its cell");
      double S = 0;
      int ne = G.c_s[6 * cell + me];
      for (int step = 1; step < deg; ++step) {
        int kp = (me + step - 1) % deg, kn = (me + step) % deg;
        int64_t t = G.c_t[6 * cell + kp];
        double kt = 0;
        for (int q = 0; q < 3; ++q)
          if (G.t_n[3 * t + q] == cell) kt = G.kite[3 * t + q];
        S += kt / G.A_i[cell];
        G.ecp[10 * e + fill] = G.c_e[6 * cell + kn];
        G.w[10 * e + fill] = double(ne * G.c_s[6 * cell + kn]) * (S - 0.5);
        ++fill;
      }
    }
    for (; fill < 10; ++fill) {
      G.ecp[10 * e + fill] = int32_t(e);
      G.w[10 * e + fill] = 0.0;
    }
  });
}

}  // namespace wt
