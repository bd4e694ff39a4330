// Fused lattice TRiSK stage for gfx950: one workgroup per (tile, lozenge), 512 threads.
//
// Phase A stages the stage input (dh and the three edge velocities of every element) of the
// tile and a 2-element halo into LDS, crossing lozenge sides through the seam rules.  Phase B
// computes q_v of both triangles of every element of the tile + 2/1 halo, phase C h_e, F, q_e
// and B = g dh + K on the tile + 1 halo, phase D the tendencies d(dh)/dt = -div F and
// du/dt = -qF^perp - grad B of the tile (eqs. (height), (velo)) fused with the Runge-Kutta
// stage combination.  Geometry comes from one reference table shared by all 10 lozenges; the
// Coriolis parameter from the rotated reference circumcentre.  Workgroups are ordered so that
// the 10 lozenge copies of a tile run back to back on the same XCD (workgroups are dealt to
// the 8 XCDs round-robin) and share that tile's geometry in the XCD's L2.
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "wt_lattice_dev.hpp"

namespace wt {

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)

constexpr int LBS = LT_TI * LT_TJ;  // 512 threads, one per tile element in phase D
constexpr int AI = LT_TI + 4, AJ = LT_TJ + 4, NA = AI * AJ;   // stage input, halo 2
constexpr int BI = LT_TI + 3, BJ = LT_TJ + 3, NB = BI * BJ;   // q_v, halo 2 below / 1 above
constexpr int CI = LT_TI + 2, CJ = LT_TJ + 2, NC = CI * CJ;   // F, q_e, B, halo 1
constexpr int DD0[3] = {1, 1, 0}, DD1[3] = {0, 1, 1};

// Seam rules of the lozenge lattice (one side crossed): new lozenge and coordinates, and the
// lattice map applied (0 translation, +1 the 60-degree map (a,b) -> (a-b, a), -1 its inverse).
__device__ __forceinline__ void seam(int L, int i, int j, int n, int& L2, int& i2, int& j2, int& rot) {
  const bool north = L < 5;
  const int k = north ? L : L - 5, km = (k + 4) % 5, kp = (k + 1) % 5;
  L2 = L; i2 = i; j2 = j; rot = 0;
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
}

// stencil slot k of the perpendicular-flux sum of frame edge d: owner offset and direction
__device__ __forceinline__ void ecp_slot(int d, int k, int& oi, int& oj, int& dd) {
  int ci = 0, cj = 0, s;
  if (k < 5) {
    s = (d + 1 + k) % 6;
  } else {
    ci = DD0[d];
    cj = DD1[d];
    s = (d + k - 1) % 6;
  }
  if (s < 3) { oi = ci; oj = cj; dd = s; }
  else { dd = s - 3; oi = ci - DD0[dd]; oj = cj - DD1[dd]; }
}

__device__ __forceinline__ void lat_out(int64_t i, double k, const StagePtrs& p, const StageOut& c) {
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
__global__ __launch_bounds__(LBS) void k_lattice(LatArgs a, StagePtrs pdh, StagePtrs pu, StageOut c) {
  __shared__ double s_dh[NA], s_u[3][NA];
  __shared__ T s_qv[2][NB];
  __shared__ double s_F[3][NC];
  __shared__ T s_qe[3][NC], s_B[NC];

  const int b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int L = slot % 10;
  const int t = (slot / 10) * 8 + xcd;
  if (t >= a.ntile) return;  // uniform per workgroup
  const int i0 = a.tiles[2 * t], j0 = a.tiles[2 * t + 1];
  const int n = a.n;
  const int64_t W = a.W, W2 = a.W2;
  const double* __restrict__ tab = a.tab;
  const double H = a.H, g = a.g;
  const double* __restrict__ xdh = pdh.x;
  const double* __restrict__ xu = pu.x;
  const int tid = threadIdx.x;

  // ---- phase A: stage input of tile + halo 2
  for (int idx = tid; idx < NA; idx += LBS) {
    const int ai = idx / AJ, aj = idx % AJ;
    const int i = i0 - 2 + ai, j = j0 - 2 + aj;
    if (i >= 0 && i < n && j >= 0 && j < n) {
      const int64_t id = (int64_t(L) * n + i) * n + j;
      s_dh[idx] = xdh[id];
      s_u[0][idx] = xu[3 * id];
      s_u[1][idx] = xu[3 * id + 1];
      s_u[2][idx] = xu[3 * id + 2];
    } else {
      int L2, i2, j2, rot;
      seam(L, i, j, n, L2, i2, j2, rot);
      const int64_t id = (int64_t(L2) * n + i2) * n + j2;
      s_dh[idx] = xdh[id];
      if (rot == 0) {
        s_u[0][idx] = xu[3 * id];
        s_u[1][idx] = xu[3 * id + 1];
        s_u[2][idx] = xu[3 * id + 2];
      } else if (rot == 1) {
        s_u[0][idx] = xu[3 * id + 1];
        s_u[1][idx] = xu[3 * id + 2];
        s_u[2][idx] = -xu[3 * (id - n)];          // E0 of the point one row above, reversed
      } else {
        s_u[0][idx] = -xu[3 * (id - 1) + 2];      // E2 of the point one column left, reversed
        s_u[1][idx] = xu[3 * id];
        s_u[2][idx] = xu[3 * id + 1];
      }
    }
  }
  __syncthreads();

  // ---- phase B: q_v of both triangles, positions [-2, TI+1) x [-2, TJ+1)
  const double f0 = a.frot[3 * L], f1 = a.frot[3 * L + 1], f2 = a.frot[3 * L + 2];
  for (int idx = tid; idx < NB; idx += LBS) {
    const int bi = idx / BJ, bj = idx % BJ;
    const int la = bi * AJ + bj;
    const int64_t p = int64_t(i0 - 2 + bi + LT_G) * W + (j0 - 2 + bj + LT_G);
    const T h0 = T(H) + T(s_dh[la]), h10 = T(H) + T(s_dh[la + AJ]), h11 = T(H) + T(s_dh[la + AJ + 1]),
            h01 = T(H) + T(s_dh[la + 1]);
    {
      T z = T(tab[(LQ_CURL + 0) * W2 + p]) * T(s_u[0][la]) + T(tab[(LQ_CURL + 1) * W2 + p]) * T(s_u[2][la + AJ]) +
            T(tab[(LQ_CURL + 2) * W2 + p]) * T(s_u[1][la]);
      T hv = T(tab[(LQ_R + 0) * W2 + p]) * h0 + T(tab[(LQ_R + 1) * W2 + p]) * h10 +
             T(tab[(LQ_R + 2) * W2 + p]) * h11;
      T f = T(f0 * tab[(LQ_CC + 0) * W2 + p] + f1 * tab[(LQ_CC + 1) * W2 + p] + f2 * tab[(LQ_CC + 2) * W2 + p]);
      s_qv[0][idx] = (z + f) / hv;
    }
    {
      T z = T(tab[(LQ_CURL + 3) * W2 + p]) * T(s_u[1][la]) + T(tab[(LQ_CURL + 4) * W2 + p]) * T(s_u[0][la + 1]) +
            T(tab[(LQ_CURL + 5) * W2 + p]) * T(s_u[2][la]);
      T hv = T(tab[(LQ_R + 3) * W2 + p]) * h0 + T(tab[(LQ_R + 4) * W2 + p]) * h11 +
             T(tab[(LQ_R + 5) * W2 + p]) * h01;
      T f = T(f0 * tab[(LQ_CC + 3) * W2 + p] + f1 * tab[(LQ_CC + 4) * W2 + p] + f2 * tab[(LQ_CC + 5) * W2 + p]);
      s_qv[1][idx] = (z + f) / hv;
    }
  }
  __syncthreads();

  // ---- phase C: F, q_e at the three edges and B at the node, positions [-1, TI+1) x [-1, TJ+1)
  for (int idx = tid; idx < NC; idx += LBS) {
    const int ci = idx / CJ, cj = idx % CJ;
    const int la = (ci + 1) * AJ + (cj + 1);
    const int lb = (ci + 1) * BJ + (cj + 1);
    const int64_t p = int64_t(i0 - 1 + ci + LT_G) * W + (j0 - 1 + cj + LT_G);
    const T h = T(H) + T(s_dh[la]);
    const T u0 = T(s_u[0][la]), u1 = T(s_u[1][la]), u2 = T(s_u[2][la]);
    s_F[0][idx] = double(T(0.5) * (h + (T(H) + T(s_dh[la + AJ]))) * u0);
    s_F[1][idx] = double(T(0.5) * (h + (T(H) + T(s_dh[la + AJ + 1]))) * u1);
    s_F[2][idx] = double(T(0.5) * (h + (T(H) + T(s_dh[la + 1]))) * u2);
    s_qe[0][idx] = T(0.5) * (s_qv[0][lb] + s_qv[1][lb - 1]);
    s_qe[1][idx] = T(0.5) * (s_qv[0][lb] + s_qv[1][lb]);
    s_qe[2][idx] = T(0.5) * (s_qv[1][lb] + s_qv[0][lb - BJ]);
    const T ua = T(s_u[0][la - AJ]), ub = T(s_u[1][la - AJ - 1]), uc = T(s_u[2][la - 1]);
    const T K = T(tab[LQ_INVA * W2 + p]) *
                (T(tab[(LQ_KC + 0) * W2 + p]) * u0 * u0 + T(tab[(LQ_KC + 1) * W2 + p]) * u1 * u1 +
                 T(tab[(LQ_KC + 2) * W2 + p]) * u2 * u2 + T(tab[(LQ_KC + 0) * W2 + p - W]) * ua * ua +
                 T(tab[(LQ_KC + 1) * W2 + p - W - 1]) * ub * ub + T(tab[(LQ_KC + 2) * W2 + p - 1]) * uc * uc);
    s_B[idx] = T(g) * T(s_dh[la]) + K;
  }
  __syncthreads();

  // ---- phase D: tendencies of the tile element of this thread and the stage combination
  {
    const int di = tid / LT_TJ, dj = tid % LT_TJ;
    const int i = i0 + di, j = j0 + dj;
    const int lc = (di + 1) * CJ + (dj + 1);
    const int64_t p = int64_t(i + LT_G) * W + (j + LT_G);
    const int64_t id = (int64_t(L) * n + i) * n + j;
    double div = tab[(LQ_LEN + 0) * W2 + p] * s_F[0][lc] + tab[(LQ_LEN + 1) * W2 + p] * s_F[1][lc] +
                 tab[(LQ_LEN + 2) * W2 + p] * s_F[2][lc] - tab[(LQ_LEN + 0) * W2 + p - W] * s_F[0][lc - CJ] -
                 tab[(LQ_LEN + 1) * W2 + p - W - 1] * s_F[1][lc - CJ - 1] -
                 tab[(LQ_LEN + 2) * W2 + p - 1] * s_F[2][lc - 1];
    lat_out(id, -tab[LQ_INVA * W2 + p] * div, pdh, c);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const T q0 = s_qe[d][lc];
      T Q = T(0);
#pragma unroll
      for (int k = 0; k < 10; ++k) {
        int oi, oj, dd;
        ecp_slot(d, k, oi, oj, dd);
        const int le = lc + oi * CJ + oj;
        Q += T(tab[(LQ_WL + 10 * d + k) * W2 + p]) * T(s_F[dd][le]) * (T(0.5) * (q0 + s_qe[dd][le]));
      }
      const int lo = lc + DD0[d] * CJ + DD1[d];
      const T gradB = (s_B[lo] - s_B[lc]) * T(tab[(LQ_INVD + d) * W2 + p]);
      lat_out(3 * id + d, double(-Q - gradB), pu, c);
    }
  }
}

void launch_lattice(const LatArgs& a, bool fp32, const StagePtrs& pdh, const StagePtrs& pu,
                    const StageOut& c, hipStream_t s) {
  const int nslots = (a.ntile + 7) / 8;        // tiles per XCD, rounded up
  const unsigned grid = unsigned(nslots) * 10u * 8u;
  if (fp32)
    k_lattice<float><<<grid, LBS, 0, s>>>(a, pdh, pu, c);
  else
    k_lattice<double><<<grid, LBS, 0, s>>>(a, pdh, pu, c);
  HIPCHK(hipGetLastError());
}

void upload_lattice(const LatticeHost& h, DevLattice& d) {
  auto up = [](const auto& v, auto** p) {
    using X = typename std::remove_reference<decltype(v)>::type::value_type;
    HIPCHK(hipMalloc(reinterpret_cast<void**>(p), v.size() * sizeof(X)));
    HIPCHK(hipMemcpy(*p, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice));
  };
  double* tab;
  int32_t *tiles, *rim, *se, *st;
  up(h.tab, &tab);
  up(h.tiles, &tiles);
  up(h.rim_elems, &rim);
  up(h.sup_elems, &se);
  up(h.sup_tris, &st);
  d.args.tab = tab;
  d.args.tiles = tiles;
  d.args.ntile = int(h.tiles.size() / 2);
  d.args.n = int(h.n);
  d.args.W = h.W;
  d.args.W2 = h.W2;
  for (int q = 0; q < 30; ++q) d.args.frot[q] = h.frot[q];
  d.rim = rim;
  d.n_rim = int64_t(h.rim_elems.size());
  d.sup_elems = se;
  d.n_sup_elems = int64_t(h.sup_elems.size());
  d.sup_tris = st;
  d.n_sup_tris = int64_t(h.sup_tris.size());
  d.n_reg_elems = int64_t(d.args.ntile) * LT_TI * LT_TJ * 10;
  d.table_bytes = int64_t(h.tab.size()) * 8;
  d.ok = true;
}

void free_lattice(DevLattice& d) {
  const void* ps[] = {d.args.tab, d.args.tiles, d.rim, d.sup_elems, d.sup_tris};
  for (const void* p : ps)
    if (p) (void)hipFree(const_cast<void*>(p));
  d = DevLattice{};
}

}  // namespace wt
