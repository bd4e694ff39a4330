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
// reference circumcentre.  On the finest level of an adaptive grid the same kernel runs the level
// whole (the masked form): tendencies are zero at inactive points, and F, Q and B of the tile
// elements are stored for the restriction to the coarser level (Sec. 4.1-4.3).
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>
#include <type_traits>

#include "wt_alloc.hpp"
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

// Stencil slot k of the perpendicular-flux sum of frame edge d (the five other edges of the
// element's cell, then the five of the cell across edge d, counter-clockwise): offset of the
// owning element and the owner's frame direction.
struct Slot {
  int oi, oj, dd;
};
constexpr Slot stencil_slot(int d, int k) {
  int ci = 0, cj = 0, s = 0;
  if (k < 5) {
    s = (d + 1 + k) % 6;
  } else {
    ci = DD0[d];
    cj = DD1[d];
    s = (d + k - 1) % 6;
  }
  if (s < 3) return Slot{ci, cj, s};
  return Slot{ci - DD0[s - 3], cj - DD1[s - 3], s - 3};
}

// The 30 slots of an element's three edges name 19 distinct edges (the six edges of the
// element's own cell serve several stencils): each distinct edge is read once and feeds every
// slot that names it.
struct StencilUnion {
  int count = 0;
  int oi[30] = {}, oj[30] = {}, dd[30] = {}, nuse[30] = {}, use[30][3] = {};
};
constexpr StencilUnion make_union() {
  StencilUnion t;
  for (int d = 0; d < 3; ++d)
    for (int k = 0; k < 10; ++k) {
      const Slot sl = stencil_slot(d, k);
      int f = -1;
      for (int u = 0; u < t.count; ++u)
        if (t.oi[u] == sl.oi && t.oj[u] == sl.oj && t.dd[u] == sl.dd) f = u;
      if (f < 0) {
        f = t.count++;
        t.oi[f] = sl.oi;
        t.oj[f] = sl.oj;
        t.dd[f] = sl.dd;
      }
      t.use[f][t.nuse[f]++] = 10 * d + k;
    }
  return t;
}
constexpr StencilUnion SU = make_union();
static_assert(SU.count == 19, "distinct edges of the three perpendicular-flux stencils");

// Halo addressing of the stage input, split into a lozenge-independent part computed once
// per workgroup and a cheap per-lozenge part.  A halo position (i,j) either lies inside the
// lozenge or crosses one side (side 1: i<0, 2: j<0, 3: i>=n, 4: j>=n, in the precedence of the
// seam rules); where it lands in the neighbour, and the lattice map, depend only on whether the
// lozenge is northern or southern, the neighbour's number on the lozenge.
struct ASlot {
  int offN, offS;   // i2*n + j2 in the neighbour for a northern / southern lozenge
  int code;         // side | (rotN+1) << 3 | (rotS+1) << 5
};

__device__ __forceinline__ ASlot a_slot(int idx, int i0, int j0, int n) {
  const int ai = idx / AJ, aj = idx % AJ;
  const int i = i0 - 2 + ai, j = j0 - 2 + aj;
  const int side = i < 0 ? 1 : j < 0 ? 2 : i >= n ? 3 : j >= n ? 4 : 0;
  int L2, iN, jN, rN, iS, jS, rS;
  seam(0, i, j, n, L2, iN, jN, rN);
  seam(5, i, j, n, L2, iS, jS, rS);
  return ASlot{iN * n + jN, iS * n + jS, side | ((rN + 1) << 3) | ((rS + 1) << 5)};
}

// Stage-input addresses of a halo slot in lozenge L: node, three edge velocities in the frame
// of L, and which of the first and third to reverse (a rotated seam turns the neighbour's edge
// around).
struct AAddr {
  int64_t node, e0, e1, e2;
  int neg;   // bit 0: reverse e0, bit 1: reverse e2
};

__device__ __forceinline__ AAddr a_address(const ASlot& sl, int L, int n) {
  const bool north = L < 5;
  const int k = north ? L : L - 5, km = (k + 4) % 5, kp = (k + 1) % 5;
  const int side = sl.code & 7;
  const int L2 = side == 0 ? L : side == 1 ? (north ? km : k) : side == 2 ? 5 + km
               : side == 3 ? (north ? 5 + k : 5 + kp) : kp;
  const int rot = ((sl.code >> (north ? 3 : 5)) & 3) - 1;
  const int64_t id = int64_t(L2) * n * n + (north ? sl.offN : sl.offS);
  AAddr r;
  r.node = id;
  r.neg = 0;
  if (rot == 0) {
    r.e0 = 3 * id; r.e1 = 3 * id + 1; r.e2 = 3 * id + 2;
  } else if (rot == 1) {
    r.e0 = 3 * id + 1; r.e1 = 3 * id + 2; r.e2 = 3 * (id - n); r.neg = 2;   // E0 one row above, reversed
  } else {
    r.e0 = 3 * (id - 1) + 2; r.neg = 1; r.e1 = 3 * id; r.e2 = 3 * id + 1;   // E2 one column left, reversed
  }
  return r;
}

// Epilogue variants: which of y and acc the stage combination reads from HBM (x comes from LDS)
// and whether there is a second output (the first is always written).  Keeping these out of
// run-time branches lets the compiler count outstanding memory operations exactly, so waiting
// for this lozenge's operands never waits for the next lozenge's prefetch.  EPI_INTER (masked
// form only): the intermediates alone -- F, Q and B stored, no tendency and no stage output -- for
// a level below the finest, whose tendencies wait for the restriction from the level above.
enum { EPI_Y = 1, EPI_ACC = 2, EPI_O2 = 4, EPI_INTER = 8 };

template <typename T, int EPI, bool ML>
__global__ __launch_bounds__(LBS) void k_lattice(LatArgs a, StagePtrs pdh, StagePtrs pu, StageOut c, LatML m) {
  __shared__ double s_dh[NA], s_u[3][NA];
  __shared__ T s_qv[2][NB];
  __shared__ T s_F[3][NC];           // mass flux (exactly a T value in both precisions)
  __shared__ T s_Fq[3][NC], s_B[NC];  // F q_e and the Bernoulli function
  __shared__ T s_gR[4][NB];          // kite weights of h_v (two per triangle; the third is 1 - both)
  __shared__ T s_gf[4][NB];          // Coriolis parameter of both triangles, northern / southern lozenges
  __shared__ T s_gcurl[6][NB2];      // curl weights of the second B slot
  __shared__ T s_gke[6][NC];         // kinetic-energy weights
  __shared__ uint8_t s_act[ML ? LBS : 1];   // masked form: activity bits of the tile elements

  // Tiles are dealt to the 8 XCDs (workgroups go round-robin) in contiguous bands, so the
  // workgroups running together on one XCD hold neighbouring tiles and share halos in its L2.
  const int b = blockIdx.x;
  const int per = (a.ntile + 7) >> 3;
  const int t = (b & 7) * per + (b >> 3);
  if (t >= a.ntile) return;  // uniform per workgroup
  // masked form: only the lozenges in which this tile holds a point of the support (all when
  // no flags are given)
  uint32_t lmask = 0x3ffu;
  if constexpr (ML) {
    if (m.tflag) {
      lmask = 0u;
      for (int L = 0; L < 10; ++L) lmask |= uint32_t(m.tflag[t * 10 + L] != 0) << L;
      if (lmask == 0u) return;  // uniform per workgroup
    }
  }
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
  // The northern lozenges are turned into one another by rotations about the polar axis, and so
  // are the southern ones: f = 2 Omega sin(latitude) of a lattice position takes one value in
  // all northern lozenges and one in all southern ones.
  auto coriolis = [&](int64_t p, int idx) {
#pragma unroll
    for (int tr = 0; tr < 2; ++tr) {
      const double c0 = TAB(LQ_CC + 3 * tr, p), c1 = TAB(LQ_CC + 3 * tr + 1, p), c2 = TAB(LQ_CC + 3 * tr + 2, p);
      s_gf[tr][idx] = T(a.frot[0] * c0 + a.frot[1] * c1 + a.frot[2] * c2);
      s_gf[2 + tr][idx] = T(a.frot[15] * c0 + a.frot[16] * c1 + a.frot[17] * c2);
    }
  };
  auto pb = [&](int idx) { return int64_t(i0 - 2 + idx / BJ + LT_G) * W + (j0 - 2 + idx % BJ + LT_G); };
  {
    const int64_t p = pb(tid);
#pragma unroll
    for (int q = 0; q < 6; ++q) gcurl[q] = T(TAB(LQ_CURL + q, p));
    coriolis(p, tid);
    s_gR[0][tid] = T(TAB(LQ_R + 0, p));
    s_gR[1][tid] = T(TAB(LQ_R + 1, p));
    s_gR[2][tid] = T(TAB(LQ_R + 3, p));
    s_gR[3][tid] = T(TAB(LQ_R + 4, p));
  }
  if (tid < NB2) {
    const int idx = tid + LBS;
    const int64_t p = pb(idx);
#pragma unroll
    for (int q = 0; q < 6; ++q) s_gcurl[q][tid] = T(TAB(LQ_CURL + q, p));
    coriolis(p, idx);
    s_gR[0][idx] = T(TAB(LQ_R + 0, p));
    s_gR[1][idx] = T(TAB(LQ_R + 1, p));
    s_gR[2][idx] = T(TAB(LQ_R + 3, p));
    s_gR[3][idx] = T(TAB(LQ_R + 4, p));
  }
  // phase C: K_i = sum over the 6 cell edges of (l d / 4A) u^2
  for (int idx = tid; idx < NC; idx += LBS) {
    const int64_t p = int64_t(i0 - 1 + idx / CJ + LT_G) * W + (j0 - 1 + idx % CJ + LT_G);
    const double ia = TAB(LQ_INVA, p);
    s_gke[0][idx] = T(ia * TAB(LQ_KC + 0, p));
    s_gke[1][idx] = T(ia * TAB(LQ_KC + 1, p));
    s_gke[2][idx] = T(ia * TAB(LQ_KC + 2, p));
    s_gke[3][idx] = T(ia * TAB(LQ_KC + 0, p - W));
    s_gke[4][idx] = T(ia * TAB(LQ_KC + 1, p - W - 1));
    s_gke[5][idx] = T(ia * TAB(LQ_KC + 2, p - 1));
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
  const ASlot aslot[2] = {a_slot(tid, i0, j0, n), a_slot(a1idx, i0, j0, n)};
  double r_dh[2], r_u0[2], r_u1[2], r_u2[2];
  int r_neg[2];   // bit 0: reverse u0, bit 1: reverse u2
  auto issue_a = [&](int L) {
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const AAddr ad = a_address(aslot[sl], L, n);
      r_dh[sl] = xdh[ad.node];
      r_u0[sl] = xu[ad.e0];
      r_u1[sl] = xu[ad.e1];
      r_u2[sl] = xu[ad.e2];
      r_neg[sl] = ad.neg;
    }
  };
  const int L0 = ML ? __builtin_ctz(lmask) : 0;
  issue_a(L0);

  const int la_d = (di + 2) * AJ + (dj + 2);   // tile element in the A layout
  const int lc = (di + 1) * CJ + (dj + 1);     // tile element in the C layout

  // One lozenge; the next lozenge's input is prefetched in all but the last.  The last is a
  // separate copy so that no memory operation sits under a run-time branch.
  auto lozenge = [&](int L, int Lnext, auto prefetch) {
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
    if constexpr (decltype(prefetch)::value) issue_a(Lnext);
    __syncthreads();

    // ---- phase B: q_v of both triangles, positions [-2, TI+1) x [-2, TJ+1)
    const int hf = L < 5 ? 0 : 2;
    auto qv_at = [&](int idx, const T* cu) {
      const int bi = idx / BJ, bj = idx % BJ;
      const int la = bi * AJ + bj;
      const T h0 = T(H) + T(s_dh[la]), h10 = T(H) + T(s_dh[la + AJ]), h11 = T(H) + T(s_dh[la + AJ + 1]),
              h01 = T(H) + T(s_dh[la + 1]);
      const T z0 = cu[0] * T(s_u[0][la]) + cu[1] * T(s_u[2][la + AJ]) + cu[2] * T(s_u[1][la]);
      const T R0 = s_gR[0][idx], R1 = s_gR[1][idx], R3 = s_gR[2][idx], R4 = s_gR[3][idx];
      const T hv0 = R0 * h0 + R1 * h10 + (T(1) - R0 - R1) * h11;
      const T fa = s_gf[hf][idx];
      s_qv[0][idx] = (z0 + fa) / hv0;
      const T z1 = cu[3] * T(s_u[1][la]) + cu[4] * T(s_u[0][la + 1]) + cu[5] * T(s_u[2][la]);
      const T hv1 = R3 * h0 + R4 * h11 + (T(1) - R3 - R4) * h01;
      const T fb = s_gf[hf + 1][idx];
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

    double ydh = 0, yu[3] = {0, 0, 0}, adh = 0, au[3] = {0, 0, 0};
    if (EPI & EPI_Y) {
      ydh = pdh.y[id];
      yu[0] = pu.y[3 * id]; yu[1] = pu.y[3 * id + 1]; yu[2] = pu.y[3 * id + 2];
    }
    if (EPI & EPI_ACC) {
      adh = pdh.acc[id];
      au[0] = pu.acc[3 * id]; au[1] = pu.acc[3 * id + 1]; au[2] = pu.acc[3 * id + 2];
    }
    // masked form: activity of the element's node and edges, parked in LDS until phase D
    if constexpr (ML && !(EPI & EPI_INTER))
      s_act[tid] = uint8_t(uint32_t(m.na[id] != 0) | uint32_t(m.ea[3 * id] != 0) << 1 |
                           uint32_t(m.ea[3 * id + 1] != 0) << 2 | uint32_t(m.ea[3 * id + 2] != 0) << 3);
    // ---- phase C: F, q_e at the three edges and B at the node, positions [-1, TI+1) x [-1, TJ+1)
    auto c_at = [&](int idx) {
      const int ci = idx / CJ, cj = idx % CJ;
      const int la = (ci + 1) * AJ + (cj + 1);
      const int lb = (ci + 1) * BJ + (cj + 1);
      const T h = T(H) + T(s_dh[la]);
      const T u0 = T(s_u[0][la]), u1 = T(s_u[1][la]), u2 = T(s_u[2][la]);
      const T F0 = T(0.5) * (h + (T(H) + T(s_dh[la + AJ]))) * u0;
      const T F1 = T(0.5) * (h + (T(H) + T(s_dh[la + AJ + 1]))) * u1;
      const T F2 = T(0.5) * (h + (T(H) + T(s_dh[la + 1]))) * u2;
      s_F[0][idx] = F0;
      s_F[1][idx] = F1;
      s_F[2][idx] = F2;
      s_Fq[0][idx] = F0 * (T(0.5) * (s_qv[0][lb] + s_qv[1][lb - 1]));
      s_Fq[1][idx] = F1 * (T(0.5) * (s_qv[0][lb] + s_qv[1][lb]));
      s_Fq[2][idx] = F2 * (T(0.5) * (s_qv[1][lb] + s_qv[0][lb - BJ]));
      const T ua = T(s_u[0][la - AJ]), ub = T(s_u[1][la - AJ - 1]), uc = T(s_u[2][la - 1]);
      const T K = s_gke[0][idx] * u0 * u0 + s_gke[1][idx] * u1 * u1 + s_gke[2][idx] * u2 * u2 +
                  s_gke[3][idx] * ua * ua + s_gke[4][idx] * ub * ub + s_gke[5][idx] * uc * uc;
      s_B[idx] = T(g) * T(s_dh[la]) + K;
    };
    c_at(tid);
    if (tid < NC2) c_at(tid + LBS);
    __syncthreads();

    // ---- phase D: tendencies of the tile element of this thread and the stage combination
    {
      if constexpr (!(EPI & EPI_INTER)) {
        const double div = gdiv[0] * double(s_F[0][lc]) + gdiv[1] * double(s_F[1][lc]) +
                           gdiv[2] * double(s_F[2][lc]) + gdiv[3] * double(s_F[0][lc - CJ]) +
                           gdiv[4] * double(s_F[1][lc - CJ - 1]) + gdiv[5] * double(s_F[2][lc - 1]);
        const uint32_t act = ML ? uint32_t(s_act[tid]) : 0xfu;
        const double k = (act & 1u) ? -div : 0.0;
        pdh.o1[id] = c.d1 * k + c.a1 * ydh + c.b1 * adh + c.c1 * s_dh[la_d];
        if (EPI & EPI_O2) pdh.o2[id] = c.d2 * k + c.a2 * ydh + c.b2 * adh + c.c2 * s_dh[la_d];
        if constexpr (ML) m.c[id] = div;   // the fine divergence of the restriction
      }
      if constexpr (ML) {
        static_cast<T*>(m.B)[id] = s_B[lc];
#pragma unroll
        for (int d = 0; d < 3; ++d) m.F[3 * id + d] = double(s_F[d][lc]);
      }
    }
    // Q_e = (1/d_e) sum_e' w l' F' (q_e + q_e')/2 = (q_e S1 + S2) / 2 with S1 = sum w l'/d F' and
    // S2 = sum w l'/d F' q_e', summed over the distinct stencil edges
    {
      T S1[3] = {T(0), T(0), T(0)}, S2[3] = {T(0), T(0), T(0)};
#pragma unroll
      for (int u = 0; u < SU.count; ++u) {
        const int le = lc + SU.oi[u] * CJ + SU.oj[u];
        const T F = s_F[SU.dd[u]][le], Fq = s_Fq[SU.dd[u]][le];
#pragma unroll
        for (int r = 0; r < SU.nuse[u]; ++r) {
          const int w = SU.use[u][r];
          S1[w / 10] += gwl[w] * F;
          S2[w / 10] += gwl[w] * Fq;
        }
        // a few distinct edges at a time: bounds the operands the scheduler keeps in flight
        if (u % 5 == 4) __builtin_amdgcn_sched_barrier(0);
      }
      const int lb = (di + 2) * BJ + (dj + 2);
      const uint32_t act = ML && !(EPI & EPI_INTER) ? uint32_t(s_act[tid]) : 0xfu;
      const T qe[3] = {T(0.5) * (s_qv[0][lb] + s_qv[1][lb - 1]), T(0.5) * (s_qv[0][lb] + s_qv[1][lb]),
                       T(0.5) * (s_qv[1][lb] + s_qv[0][lb - BJ])};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T Q = T(0.5) * (qe[d] * S1[d] + S2[d]);
        if constexpr (ML) static_cast<T*>(m.Q)[3 * id + d] = Q;
        if constexpr (!(EPI & EPI_INTER)) {
          const int lo = lc + DD0[d] * CJ + DD1[d];
          const T gradB = (s_B[lo] - s_B[lc]) * ginvd[d];
          const double k = (act & (2u << d)) ? double(-Q - gradB) : 0.0;
          const double x = s_u[d][la_d];
          pu.o1[3 * id + d] = c.d1 * k + c.a1 * yu[d] + c.b1 * au[d] + c.c1 * x;
          if (EPI & EPI_O2) pu.o2[3 * id + d] = c.d2 * k + c.a2 * yu[d] + c.b2 * au[d] + c.c2 * x;
        }
      }
    }
  };
  if constexpr (ML) {
    uint32_t rest = lmask & (lmask - 1u);   // the flagged lozenges after the first
    int L = L0;
    while (rest) {
      const int Ln = __builtin_ctz(rest);
      rest &= rest - 1u;
      lozenge(L, Ln, std::true_type{});
      L = Ln;
    }
    lozenge(L, 0, std::false_type{});
  } else {
    for (int L = 0; L < 9; ++L) lozenge(L, L + 1, std::true_type{});
    lozenge(9, 0, std::false_type{});
  }
}

// Tile flags of the masked form: flag[10 t + L] = 1 when tile t of lozenge L holds a node or an
// edge of the 5-ring support (sn, se); every point whose F, Q, B or tendency is read lies within
// four rings of an active point, so unflagged tiles have nothing to compute.  *count receives the
// number of flagged pairs (cleared here first).
__global__ void k_tile_count_clear(int32_t* count) {
  if (threadIdx.x == 0) *count = 0;
}

__global__ __launch_bounds__(LBS) void k_tile_flags(const int32_t* __restrict__ tiles, int n,
                                                    const uint8_t* __restrict__ sn, const uint8_t* __restrict__ se,
                                                    uint8_t* __restrict__ flag, int32_t* __restrict__ count) {
  const int t = blockIdx.x, L = blockIdx.y;
  const int i0 = tiles[2 * t], j0 = tiles[2 * t + 1];
  const int di = threadIdx.x / LT_TJ, dj = threadIdx.x % LT_TJ;
  const int64_t id = (int64_t(L) * n + i0 + di) * n + (j0 + dj);
  const int v = (sn[id] | se[3 * id] | se[3 * id + 1] | se[3 * id + 2]) != 0;
  const int any = __syncthreads_or(v);
  if (threadIdx.x == 0) {
    flag[10 * t + L] = uint8_t(any != 0);
    if (any) atomicAdd(count, 1);
  }
}

void lattice_tile_flags(const DevLattice& lat, const uint8_t* sn, const uint8_t* se, uint8_t* flag, int32_t* count,
                        hipStream_t s) {
  if (!lat.ok || lat.args.ntile <= 0) return;
  k_tile_count_clear<<<1, 64, 0, s>>>(count);
  k_tile_flags<<<dim3(unsigned(lat.args.ntile), 10u), LBS, 0, s>>>(lat.args.tiles, lat.args.n, sn, se, flag, count);
  HIPCHK(hipGetLastError());
}

void launch_lattice(const LatArgs& a, bool fp32, const StagePtrs& pdh, const StagePtrs& pu,
                    const StageOut& c, hipStream_t s, const LatML* ml, bool inter) {
  const unsigned grid = unsigned((a.ntile + 7) / 8) * 8u;
  const bool ry = c.a1 != 0.0 || c.a2 != 0.0, racc = c.b1 != 0.0 || c.b2 != 0.0;
  if (!pdh.x || !pu.x) throw std::runtime_error("lattice stage: needs the stage input");
  if (!inter && (!pdh.o1 || !pu.o1 || (pdh.o2 == nullptr) != (pu.o2 == nullptr)))
    throw std::runtime_error("lattice stage: needs the first output, and the second for both or neither of dh, u");
  const int epi = (ry ? EPI_Y : 0) | (racc ? EPI_ACC : 0) | (pdh.o2 ? EPI_O2 : 0);
  if (ml && (!ml->na || !ml->ea || !ml->F || !ml->Q || !ml->B))
    throw std::runtime_error("lattice stage: the masked form needs masks and the F, Q, B outputs");
  if (inter && !ml) throw std::runtime_error("lattice stage: the intermediates-only form is a masked form");
  if (ml && !inter && !ml->c) throw std::runtime_error("lattice stage: the masked form needs the divergence output");
  const LatML m = ml ? *ml : LatML{};
  if (inter) {
    if (fp32) k_lattice<float, EPI_INTER, true><<<grid, LBS, 0, s>>>(a, pdh, pu, c, m);
    else k_lattice<double, EPI_INTER, true><<<grid, LBS, 0, s>>>(a, pdh, pu, c, m);
    HIPCHK(hipGetLastError());
    return;
  }
  auto go = [&](auto tag, auto e) {
    using T = decltype(tag);
    if (ml) k_lattice<T, decltype(e)::value, true><<<grid, LBS, 0, s>>>(a, pdh, pu, c, m);
    else k_lattice<T, decltype(e)::value, false><<<grid, LBS, 0, s>>>(a, pdh, pu, c, m);
  };
  auto dispatch = [&](auto tag) {
    switch (epi) {
      case 0: go(tag, std::integral_constant<int, 0>{}); break;
      case 1: go(tag, std::integral_constant<int, 1>{}); break;
      case 2: go(tag, std::integral_constant<int, 2>{}); break;
      case 3: go(tag, std::integral_constant<int, 3>{}); break;
      case 4: go(tag, std::integral_constant<int, 4>{}); break;
      case 5: go(tag, std::integral_constant<int, 5>{}); break;
      case 6: go(tag, std::integral_constant<int, 6>{}); break;
      default: go(tag, std::integral_constant<int, 7>{}); break;
    }
  };
  if (fp32) dispatch(float{});
  else dispatch(double{});
  HIPCHK(hipGetLastError());
}

void upload_lattice(const LatticeHost& h, DevLattice& d) {
  auto up = [](const auto& v, auto** p) {
    using X = typename std::remove_reference<decltype(v)>::type::value_type;
    HIPCHK(wt::dmalloc(reinterpret_cast<void**>(p), v.size() * sizeof(X)));
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
  std::vector<int32_t> re;
  for (int32_t id : h.rim_elems)
    if (int64_t(id) < 10 * h.n * h.n)
      for (int q = 0; q < 3; ++q) re.push_back(3 * id + q);
  int32_t* rep;
  up(re, &rep);
  d.rim_edges = rep;
  d.n_rim_edges = int64_t(re.size());
  d.n_reg_elems = int64_t(d.args.ntile) * LT_TI * LT_TJ * 10;
  d.table_bytes = int64_t(h.tab.size()) * 8;
  d.ok = true;
}

void free_lattice(DevLattice& d) {
  const void* ps[] = {d.args.tab, d.args.tiles, d.rim, d.sup_elems, d.sup_tris, d.rim_edges};
  for (const void* p : ps)
    if (p) (void)wt::dfree(const_cast<void*>(p));
  d = DevLattice{};
}

}  // namespace wt
