// Fused lattice TRiSK stage for gfx950: one workgroup of 512 threads per tile position, looping
// over the 10 lozenges.
//
// The 10 lozenges are congruent, so the geometry of a tile position is the same in all of them:
// each workgroup loads it once (into registers; the few halo positions beyond the first 512
// into LDS) and reuses it for the 10 lozenge copies of its tile.  Per lozenge, phase A stages
// the stage input (dh and the three edge velocities of every element) of the tile and a
// 2-element halo into LDS, crossing lozenge sides through the seam rules; the global loads of
// the next lozenge's input are issued one iteration ahead, so their latency hides behind the
// arithmetic.  Phase B computes q_v of both triangles of every element of the tile + 2/1 halo,
// phase C h_e, F, q_e and B = g dh + K on the tile + 1 halo, phase D the tendencies
// d(dh)/dt = -div F and du/dt = -qF^perp - grad B of the tile (eqs. (height), (velo)) fused
// with the Runge-Kutta stage combination.  The Coriolis parameter comes from the rotated
// reference circumcentre.
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
constexpr int NA2 = NA - LBS, NB2 = NB - LBS, NC2 = NC - LBS;  // positions beyond one per thread
static_assert(NA2 > 0 && NA2 <= LBS && NB2 > 0 && NB2 <= LBS && NC2 > 0 && NC2 <= LBS, "tile shape");
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

// Global addresses of the stage input of halo position idx of lozenge L: node, three edge
// velocities in the frame of L, and the sign of the first and third (a rotated seam turns an
// edge of the neighbour around).
struct AAddr {
  int64_t node, e0, e1, e2;
  int neg;   // bit 0: reverse e0, bit 1: reverse e2
};

__device__ __forceinline__ AAddr a_address(int idx, int L, int i0, int j0, int n) {
  const int ai = idx / AJ, aj = idx % AJ;
  const int i = i0 - 2 + ai, j = j0 - 2 + aj;
  AAddr r;
  r.neg = 0;
  if (i >= 0 && i < n && j >= 0 && j < n) {
    const int64_t id = (int64_t(L) * n + i) * n + j;
    r.node = id; r.e0 = 3 * id; r.e1 = 3 * id + 1; r.e2 = 3 * id + 2;
  } else {
    int L2, i2, j2, rot;
    seam(L, i, j, n, L2, i2, j2, rot);
    const int64_t id = (int64_t(L2) * n + i2) * n + j2;
    r.node = id;
    if (rot == 0) {
      r.e0 = 3 * id; r.e1 = 3 * id + 1; r.e2 = 3 * id + 2;
    } else if (rot == 1) {
      r.e0 = 3 * id + 1; r.e1 = 3 * id + 2; r.e2 = 3 * (id - n); r.neg = 2;   // E0 one row above, reversed
    } else {
      r.e0 = 3 * (id - 1) + 2; r.neg = 1; r.e1 = 3 * id; r.e2 = 3 * id + 1;   // E2 one column left, reversed
    }
  }
  return r;
}

// Epilogue variants: which of y and acc the stage combination reads from HBM (x comes from LDS).
enum { EPI_Y = 1, EPI_ACC = 2 };

template <typename T, int EPI>
__global__ __launch_bounds__(LBS) void k_lattice(LatArgs a, StagePtrs pdh, StagePtrs pu, StageOut c) {
  __shared__ double s_dh[NA], s_u[3][NA];
  __shared__ T s_qv[2][NB];
  __shared__ double s_F[3][NC];
  __shared__ T s_qe[3][NC], s_B[NC];
  __shared__ T s_gR[6][NB];          // kite weights of h_v, all B positions
  __shared__ double s_gcc[6][NB];     // circumcentres, all B positions
  __shared__ T s_gcurl[6][NB2];      // curl weights of the second B slot
  __shared__ T s_gc[6][NC2];         // kinetic-energy weights of the second C slot

  // Tiles are dealt to the 8 XCDs (workgroups go round-robin) in contiguous bands, so the
  // workgroups running together on one XCD hold neighbouring tiles and share halos in its L2.
  const int b = blockIdx.x;
  const int per = (a.ntile + 7) >> 3;
  const int t = (b & 7) * per + (b >> 3);
  if (t >= a.ntile) return;  // uniform per workgroup
  const int i0 = a.tiles[2 * t], j0 = a.tiles[2 * t + 1];
  const int n = a.n;
  const int64_t W = a.W, W2 = a.W2;
  const double* __restrict__ tab = a.tab;
  const double H = a.H, g = a.g;
  const double* __restrict__ xdh = pdh.x;
  const double* __restrict__ xu = pu.x;
  const int tid = threadIdx.x;
  auto TAB = [&](int q, int64_t p) { return tab[int64_t(q) * W2 + p]; };

  // ---- geometry of this tile position, shared by the 10 lozenges
  // phase B: curl weights of the first slot in registers, the rest in LDS
  T gcurl[6];
  auto pb = [&](int idx) { return int64_t(i0 - 2 + idx / BJ + LT_G) * W + (j0 - 2 + idx % BJ + LT_G); };
  {
    const int64_t p = pb(tid);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      gcurl[q] = T(TAB(LQ_CURL + q, p));
      s_gR[q][tid] = T(TAB(LQ_R + q, p));
      s_gcc[q][tid] = TAB(LQ_CC + q, p);
    }
  }
  if (tid < NB2) {
    const int idx = tid + LBS;
    const int64_t p = pb(idx);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      s_gcurl[q][tid] = T(TAB(LQ_CURL + q, p));
      s_gR[q][idx] = T(TAB(LQ_R + q, p));
      s_gcc[q][idx] = TAB(LQ_CC + q, p);
    }
  }
  // phase C: K_i = sum over the 6 cell edges of (l d / 4A) u^2, first slot registers, second LDS
  auto kc6 = [&](int64_t p, T* o) {
    const double ia = TAB(LQ_INVA, p);
    o[0] = T(ia * TAB(LQ_KC + 0, p));
    o[1] = T(ia * TAB(LQ_KC + 1, p));
    o[2] = T(ia * TAB(LQ_KC + 2, p));
    o[3] = T(ia * TAB(LQ_KC + 0, p - W));
    o[4] = T(ia * TAB(LQ_KC + 1, p - W - 1));
    o[5] = T(ia * TAB(LQ_KC + 2, p - 1));
  };
  T gke[6];
  kc6(int64_t(i0 - 1 + tid / CJ + LT_G) * W + (j0 - 1 + tid % CJ + LT_G), gke);
  if (tid < NC2) {
    const int idx = tid + LBS;
    T o[6];
    kc6(int64_t(i0 - 1 + idx / CJ + LT_G) * W + (j0 - 1 + idx % CJ + LT_G), o);
#pragma unroll
    for (int q = 0; q < 6; ++q) s_gc[q][tid] = o[q];
  }
  // phase D: divergence weights n l / A (FP64), perpendicular-flux weights, 1/d
  const int di = tid / LT_TJ, dj = tid % LT_TJ;
  const int64_t pd = int64_t(i0 + di + LT_G) * W + (j0 + dj + LT_G);
  double gdiv[6];
  T gwl[30], ginvd[3];
  {
    const double ia = TAB(LQ_INVA, pd);
    gdiv[0] = ia * TAB(LQ_LEN + 0, pd);
    gdiv[1] = ia * TAB(LQ_LEN + 1, pd);
    gdiv[2] = ia * TAB(LQ_LEN + 2, pd);
    gdiv[3] = -ia * TAB(LQ_LEN + 0, pd - W);
    gdiv[4] = -ia * TAB(LQ_LEN + 1, pd - W - 1);
    gdiv[5] = -ia * TAB(LQ_LEN + 2, pd - 1);
#pragma unroll
    for (int q = 0; q < 30; ++q) gwl[q] = T(TAB(LQ_WL + q, pd));
#pragma unroll
    for (int d = 0; d < 3; ++d) ginvd[d] = T(TAB(LQ_INVD + d, pd));
  }

  // ---- stage input of lozenge 0 into registers
  const int a1idx = tid < NA2 ? tid + LBS : tid;   // second A slot (threads without one repeat the first)
  double r_dh[2], r_u0[2], r_u1[2], r_u2[2];
  int r_neg[2];   // bit 0: reverse u0, bit 1: reverse u2
  auto issue_a = [&](int L) {
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const AAddr ad = a_address(sl == 0 ? tid : a1idx, L, i0, j0, n);
      r_dh[sl] = xdh[ad.node];
      r_u0[sl] = xu[ad.e0];
      r_u1[sl] = xu[ad.e1];
      r_u2[sl] = xu[ad.e2];
      r_neg[sl] = ad.neg;
    }
  };
  issue_a(0);

  const int la_d = (di + 2) * AJ + (dj + 2);   // tile element in the A layout
  const int lc = (di + 1) * CJ + (dj + 1);     // tile element in the C layout

  for (int L = 0; L < 10; ++L) {
    __syncthreads();   // the previous lozenge's phase D has read s_dh, s_u
    s_dh[tid] = r_dh[0];
    s_u[0][tid] = (r_neg[0] & 1) ? -r_u0[0] : r_u0[0];
    s_u[1][tid] = r_u1[0];
    s_u[2][tid] = (r_neg[0] & 2) ? -r_u2[0] : r_u2[0];
    if (tid < NA2) {
      s_dh[a1idx] = r_dh[1];
      s_u[0][a1idx] = (r_neg[1] & 1) ? -r_u0[1] : r_u0[1];
      s_u[1][a1idx] = r_u1[1];
      s_u[2][a1idx] = (r_neg[1] & 2) ? -r_u2[1] : r_u2[1];
    }
    // stage-combination operands of this lozenge, then the next lozenge's input
    const int64_t id = (int64_t(L) * n + i0 + di) * n + (j0 + dj);
    double ydh = 0, yu[3] = {0, 0, 0}, adh = 0, au[3] = {0, 0, 0};
    if (EPI & EPI_Y) {
      ydh = pdh.y[id];
      yu[0] = pu.y[3 * id]; yu[1] = pu.y[3 * id + 1]; yu[2] = pu.y[3 * id + 2];
    }
    if (EPI & EPI_ACC) {
      adh = pdh.acc[id];
      au[0] = pu.acc[3 * id]; au[1] = pu.acc[3 * id + 1]; au[2] = pu.acc[3 * id + 2];
    }
    if (L < 9) issue_a(L + 1);
    __syncthreads();

    // ---- phase B: q_v of both triangles, positions [-2, TI+1) x [-2, TJ+1)
    const double f0 = a.frot[3 * L], f1 = a.frot[3 * L + 1], f2 = a.frot[3 * L + 2];
    auto qv_at = [&](int idx, const T* cu) {
      const int bi = idx / BJ, bj = idx % BJ;
      const int la = bi * AJ + bj;
      const T h0 = T(H) + T(s_dh[la]), h10 = T(H) + T(s_dh[la + AJ]), h11 = T(H) + T(s_dh[la + AJ + 1]),
              h01 = T(H) + T(s_dh[la + 1]);
      const T z0 = cu[0] * T(s_u[0][la]) + cu[1] * T(s_u[2][la + AJ]) + cu[2] * T(s_u[1][la]);
      const T hv0 = s_gR[0][idx] * h0 + s_gR[1][idx] * h10 + s_gR[2][idx] * h11;
      const T fa = T(f0 * s_gcc[0][idx] + f1 * s_gcc[1][idx] + f2 * s_gcc[2][idx]);
      s_qv[0][idx] = (z0 + fa) / hv0;
      const T z1 = cu[3] * T(s_u[1][la]) + cu[4] * T(s_u[0][la + 1]) + cu[5] * T(s_u[2][la]);
      const T hv1 = s_gR[3][idx] * h0 + s_gR[4][idx] * h11 + s_gR[5][idx] * h01;
      const T fb = T(f0 * s_gcc[3][idx] + f1 * s_gcc[4][idx] + f2 * s_gcc[5][idx]);
      s_qv[1][idx] = (z1 + fb) / hv1;
    };
    qv_at(tid, gcurl);
    if (tid < NB2) {
      T cu[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) cu[q] = s_gcurl[q][tid];
      qv_at(tid + LBS, cu);
    }
    __syncthreads();

    // ---- phase C: F, q_e at the three edges and B at the node, positions [-1, TI+1) x [-1, TJ+1)
    auto c_at = [&](int idx, const T* ke) {
      const int ci = idx / CJ, cj = idx % CJ;
      const int la = (ci + 1) * AJ + (cj + 1);
      const int lb = (ci + 1) * BJ + (cj + 1);
      const T h = T(H) + T(s_dh[la]);
      const T u0 = T(s_u[0][la]), u1 = T(s_u[1][la]), u2 = T(s_u[2][la]);
      s_F[0][idx] = double(T(0.5) * (h + (T(H) + T(s_dh[la + AJ]))) * u0);
      s_F[1][idx] = double(T(0.5) * (h + (T(H) + T(s_dh[la + AJ + 1]))) * u1);
      s_F[2][idx] = double(T(0.5) * (h + (T(H) + T(s_dh[la + 1]))) * u2);
      s_qe[0][idx] = T(0.5) * (s_qv[0][lb] + s_qv[1][lb - 1]);
      s_qe[1][idx] = T(0.5) * (s_qv[0][lb] + s_qv[1][lb]);
      s_qe[2][idx] = T(0.5) * (s_qv[1][lb] + s_qv[0][lb - BJ]);
      const T ua = T(s_u[0][la - AJ]), ub = T(s_u[1][la - AJ - 1]), uc = T(s_u[2][la - 1]);
      const T K = ke[0] * u0 * u0 + ke[1] * u1 * u1 + ke[2] * u2 * u2 + ke[3] * ua * ua + ke[4] * ub * ub +
                  ke[5] * uc * uc;
      s_B[idx] = T(g) * T(s_dh[la]) + K;
    };
    c_at(tid, gke);
    if (tid < NC2) {
      T ke[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) ke[q] = s_gc[q][tid];
      c_at(tid + LBS, ke);
    }
    __syncthreads();

    // ---- phase D: tendencies of the tile element of this thread and the stage combination
    {
      const double div = gdiv[0] * s_F[0][lc] + gdiv[1] * s_F[1][lc] + gdiv[2] * s_F[2][lc] +
                         gdiv[3] * s_F[0][lc - CJ] + gdiv[4] * s_F[1][lc - CJ - 1] + gdiv[5] * s_F[2][lc - 1];
      const double k = -div;
      if (pdh.o1) pdh.o1[id] = c.d1 * k + c.a1 * ydh + c.b1 * adh + c.c1 * s_dh[la_d];
      if (pdh.o2) pdh.o2[id] = c.d2 * k + c.a2 * ydh + c.b2 * adh + c.c2 * s_dh[la_d];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const T q0 = s_qe[d][lc];
      T Q = T(0);
#pragma unroll
      for (int k = 0; k < 10; ++k) {
        int oi, oj, dd;
        ecp_slot(d, k, oi, oj, dd);
        const int le = lc + oi * CJ + oj;
        Q += gwl[10 * d + k] * T(s_F[dd][le]) * (T(0.5) * (q0 + s_qe[dd][le]));
      }
      const int lo = lc + DD0[d] * CJ + DD1[d];
      const T gradB = (s_B[lo] - s_B[lc]) * ginvd[d];
      const double k = double(-Q - gradB);
      const double x = s_u[d][la_d];
      if (pu.o1) pu.o1[3 * id + d] = c.d1 * k + c.a1 * yu[d] + c.b1 * au[d] + c.c1 * x;
      if (pu.o2) pu.o2[3 * id + d] = c.d2 * k + c.a2 * yu[d] + c.b2 * au[d] + c.c2 * x;
      // one edge at a time: keeps the scheduler from holding all 60 stencil operands at once
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

void launch_lattice(const LatArgs& a, bool fp32, const StagePtrs& pdh, const StagePtrs& pu,
                    const StageOut& c, hipStream_t s) {
  const unsigned grid = unsigned((a.ntile + 7) / 8) * 8u;
  const bool ry = c.a1 != 0.0 || c.a2 != 0.0, racc = c.b1 != 0.0 || c.b2 != 0.0;
  const int epi = (ry ? EPI_Y : 0) | (racc ? EPI_ACC : 0);
#define WT_LAT_LAUNCH(T_, E_) k_lattice<T_, E_><<<grid, LBS, 0, s>>>(a, pdh, pu, c)
  if (fp32) {
    switch (epi) {
      case 0: WT_LAT_LAUNCH(float, 0); break;
      case 1: WT_LAT_LAUNCH(float, 1); break;
      case 2: WT_LAT_LAUNCH(float, 2); break;
      default: WT_LAT_LAUNCH(float, 3); break;
    }
  } else {
    switch (epi) {
      case 0: WT_LAT_LAUNCH(double, 0); break;
      case 1: WT_LAT_LAUNCH(double, 1); break;
      case 2: WT_LAT_LAUNCH(double, 2); break;
      default: WT_LAT_LAUNCH(double, 3); break;
    }
  }
#undef WT_LAT_LAUNCH
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
