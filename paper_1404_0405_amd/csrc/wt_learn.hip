// Learned adjacent zone: patch features and labels for the child-patch predictor, gating of
// the children rule by its proposals, and the threshold test that judges them after a step.
//
// Patches: at level j the lattice of every lozenge is cut into 8 x 8 element patches,
// patch (L, pi, pj) -> (L m + pi) m + pj with m = n / 8; quadrant c = 2 a + b of a patch holds the
// elements (8 pi + 4 a .. +3, 8 pj + 4 b .. +3), whose next-level children form the 8 x 8 patch
// (L, 2 pi + a, 2 pj + b) of level j+1.  The poles belong to no patch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>

#include "wt_learn.hpp"

namespace wt {

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)

constexpr int LB = 256;
static inline unsigned nb(int64_t n) { return unsigned((n + LB - 1) / LB); }
#define TID (int64_t(blockIdx.x) * LB + threadIdx.x)

// log2(|d| / eps) clamped to [-16, 4] and scaled by 1/8: the detail size relative to its threshold
__device__ __forceinline__ float rlog(double d, double eps) {
  if (!(eps > 0.0)) return 0.5f;
  const double r = fabs(d) / eps;
  float v = r > 0.0 ? float(log2(r)) : -16.f;
  v = fminf(fmaxf(v, -16.f), 4.f);
  return 0.125f * v;
}

// Detail size of every fine point of several pairs (each fine point carries at most one detail),
// in two launches: every pair's arrays filled with the floor, then every pair's edge and triangle
// entries (blockIdx.y = 2 pair for the edges, 2 pair + 1 for the triangles).
__global__ __launch_bounds__(LB) void k_fill_pr_b(PointRJobs J) {
  const PointRJob& jb = J.j[blockIdx.y >> 1];
  float* a = (blockIdx.y & 1) ? jb.re : jb.rn;
  const int64_t n = (blockIdx.y & 1) ? jb.P.Ef : jb.P.Nf;
  for (int64_t i = TID; i < n; i += int64_t(gridDim.x) * LB) a[i] = -2.f;
}

__global__ __launch_bounds__(LB) void k_point_r_b(PointRJobs J) {
  const PointRJob& jb = J.j[blockIdx.y >> 1];
  const DevPair& P = jb.P;
  const int64_t stride = int64_t(gridDim.x) * LB;
  if ((blockIdx.y & 1) == 0) {
    for (int64_t r = TID; r < jb.ne; r += stride) {
      int64_t e = r;
      if (jb.le) {
        e = jb.le[r];
        if (e < 0) continue;   // padding of a work list
      }
      jb.rn[P.mid[e]] = rlog(jb.dh[e], jb.eh);
      const float ru = rlog(jb.dp[e], jb.eu);
      jb.re[P.h1[e]] = ru;
      jb.re[P.h2[e]] = ru;
    }
  } else {
    for (int64_t r = TID; r < jb.nt; r += stride) {
      int64_t t = r;
      if (jb.lt) {
        t = jb.lt[r];
        if (t < 0) continue;
      }
#pragma unroll
      for (int s = 0; s < 3; ++s) jb.re[P.int_e[3 * t + s]] = rlog(jb.di[3 * t + s], jb.eu);
    }
  }
}

void learn_point_r_batch(const PointRJob* jobs, int njobs, hipStream_t s) {
  for (int k0 = 0; k0 < njobs; k0 += MAX_PR_JOBS) {
    PointRJobs J{};
    const int nk = njobs - k0 < MAX_PR_JOBS ? njobs - k0 : MAX_PR_JOBS;
    int64_t mf = 1, mp = 1;
    for (int k = 0; k < nk; ++k) {
      J.j[k] = jobs[k0 + k];
      mf = std::max<int64_t>(mf, J.j[k].P.Ef);
      mp = std::max<int64_t>(mp, std::max(J.j[k].ne, J.j[k].nt));
    }
    k_fill_pr_b<<<dim3(std::min(nb(mf), 8192u), 2 * nk), LB, 0, s>>>(J);
    k_point_r_b<<<dim3(std::min(nb(mp), 8192u), 2 * nk), LB, 0, s>>>(J);
    HIPCHK(hipGetLastError());
  }
}

PointRJob point_r_job(const DevPair& P, const double* dh, const double* dp, const double* di, double eh, double eu,
                      float* rn, float* re, Span le, Span lt) {
  PointRJob j{};
  j.P = P; j.dh = dh; j.dp = dp; j.di = di; j.eh = eh; j.eu = eu; j.rn = rn; j.re = re;
  j.le = le.idx; j.ne = le.idx ? le.n : P.Ec;
  j.lt = lt.idx; j.nt = lt.idx ? lt.n : P.Tc;
  return j;
}

// Per-patch statistics, one wavefront per patch (lane = element of the patch):
//  0..3   max detail size over the patch: level-j height, level-j velocity, level-(j+1) height,
//         level-(j+1) velocity
//  4..19  the same four per quadrant (4 + 4 k + c)
//  20..23 active fraction of the level-(j+1) nodes of each quadrant's child patch
//  24..27 significant level-j points (nodes and edges) of each quadrant
//  28     active fraction of the patch's level-j nodes
__global__ __launch_bounds__(LB) void k_patch_stats(int64_t npatch, int n, const float* __restrict__ rn,
                                                    const float* __restrict__ re, const float* __restrict__ rnf,
                                                    const float* __restrict__ ref, const uint8_t* __restrict__ na,
                                                    const uint8_t* __restrict__ naf, const uint8_t* __restrict__ sn,
                                                    const uint8_t* __restrict__ se, float* __restrict__ stats) {
  __shared__ float s_v[LB / 64][64][7];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  const int64_t p = int64_t(blockIdx.x) * (LB / 64) + w;
  if (p >= npatch) return;   // uniform per wavefront; wavefronts do not share LDS rows
  const int m = n / 8;
  const int L = int(p / (int64_t(m) * m)), pi = int((p / m) % m), pj = int(p % m);
  const int ei = 8 * pi + l / 8, ej = 8 * pj + l % 8;
  const int64_t id = (int64_t(L) * n + ei) * n + ej;
  const int nf = 2 * n;
  float bh = -2.f, bu = -2.f, actf = 0.f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t f = (int64_t(L) * nf + 2 * ei + a) * nf + 2 * ej + b;
      bh = fmaxf(bh, rnf[f]);
      bu = fmaxf(bu, fmaxf(ref[3 * f], fmaxf(ref[3 * f + 1], ref[3 * f + 2])));
      actf += naf[f] ? 1.f : 0.f;
    }
  float* v = s_v[w][l];
  v[0] = rn[id];
  v[1] = fmaxf(re[3 * id], fmaxf(re[3 * id + 1], re[3 * id + 2]));
  v[2] = bh;
  v[3] = bu;
  v[4] = actf;
  v[5] = float(sn[id] + se[3 * id] + se[3 * id + 1] + se[3 * id + 2]);
  v[6] = na[id] ? 1.f : 0.f;
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
  float* out = stats + p * LEARN_STATS;
  // lanes 0..3: whole-patch maxima; lanes 4..19: quadrant maxima; 20..23 child activity;
  // 24..27 significant counts; 28 active fraction
  if (l < 4) {
    float mx = -2.f;
    for (int k = 0; k < 64; ++k) mx = fmaxf(mx, s_v[w][k][l]);
    out[l] = mx;
  } else if (l < 28) {
    const int c = l % 4, kind = (l - 4) / 4;   // kind 0..3 maxima, 4 activity, 5 significant
    const int a = c / 2, b = c % 2;
    float acc = kind < 4 ? -2.f : 0.f;
    for (int r = 0; r < 4; ++r)
      for (int q = 0; q < 4; ++q) {
        const int k = (4 * a + r) * 8 + 4 * b + q;
        const float x = s_v[w][k][kind];
        acc = kind < 4 ? fmaxf(acc, x) : acc + x;
      }
    out[l] = kind == 4 ? acc / 64.f : acc;
  } else if (l == 28) {
    float s = 0.f;
    for (int k = 0; k < 64; ++k) s += s_v[w][k][6];
    out[28] = s / 64.f;
  } else if (l < LEARN_STATS) {
    out[l] = 0.f;
  }
}

// 64 features per patch from its statistics and those of its 8 lattice neighbours (a neighbour
// outside the lozenge is replaced by the patch itself).
__global__ __launch_bounds__(LB) void k_patch_features(int64_t npatch, int m, float level_pos,
                                                       const float* __restrict__ stats, float* __restrict__ X) {
  const int64_t p = TID;
  if (p >= npatch) return;
  const int64_t L = p / (int64_t(m) * m);
  const int pi = int((p / m) % m), pj = int(p % m);
  float* x = X + p * 64;
  const float* own = stats + p * LEARN_STATS;
  int k = 0;
  for (int di = -1; di <= 1; ++di)
    for (int dj = -1; dj <= 1; ++dj, ++k) {
      const int qi = pi + di, qj = pj + dj;
      const int64_t q = (qi >= 0 && qi < m && qj >= 0 && qj < m) ? (L * m + qi) * m + qj : p;
      const float* st = stats + q * LEARN_STATS;
      x[k] = st[0];
      x[9 + k] = st[1];
      x[18 + k] = st[2];
      x[27 + k] = st[3];
    }
  for (int c = 0; c < 16; ++c) x[36 + c] = own[4 + c];
  for (int c = 0; c < 4; ++c) x[52 + c] = own[20 + c];
  for (int c = 0; c < 4; ++c) x[56 + c] = own[24 + c] / 64.f;
  x[60] = own[28];
  x[61] = level_pos;
  x[62] = 1.f;
  x[63] = 0.f;
}

// Label: the quadrant holds a significant level-j point (the children rule needs its children).
__global__ __launch_bounds__(LB) void k_patch_labels(int64_t npatch, const float* __restrict__ stats,
                                                     float* __restrict__ Y) {
  const int64_t p = TID;
  if (p >= npatch) return;
  for (int c = 0; c < 4; ++c) Y[p * 4 + c] = stats[p * LEARN_STATS + 24 + c] > 0.f ? 1.f : 0.f;
}

// Gate of the children rule and the quadrants it drops (significant now but not proposed).
__global__ __launch_bounds__(LB) void k_gate(int64_t npatch, const float* __restrict__ P, float thr,
                                             const float* __restrict__ stats, uint8_t* __restrict__ allow,
                                             uint8_t* __restrict__ dropped) {
  const int64_t q = TID;
  if (q >= 4 * npatch) return;
  const int64_t p = q / 4;
  const int c = int(q % 4);
  const bool a = P[q] >= thr;
  allow[q] = a ? 1 : 0;
  dropped[q] = (!a && stats[p * LEARN_STATS + 24 + c] > 0.f) ? 1 : 0;
}

__global__ void k_force_drop(int64_t patch, const float* __restrict__ stats, uint8_t* __restrict__ allow,
                             uint8_t* __restrict__ dropped) {
  const int c = threadIdx.x;
  if (c >= 4) return;
  allow[4 * patch + c] = 0;
  dropped[4 * patch + c] = stats[patch * LEARN_STATS + 24 + c] > 0.f ? 1 : 0;
}

void learn_force_drop(int64_t npatch, int64_t patch, const float* stats, uint8_t* allow, uint8_t* dropped,
                      hipStream_t s) {
  if (patch < 0 || patch >= npatch) throw std::runtime_error("learn_force_drop: patch out of range");
  k_force_drop<<<1, 64, 0, s>>>(patch, stats, allow, dropped);
  HIPCHK(hipGetLastError());
}

// Threshold test after a step: a dropped quadrant that holds a significant point again.
__global__ __launch_bounds__(LB) void k_violations(int64_t npatch, const float* __restrict__ stats,
                                                   const uint8_t* __restrict__ dropped, uint8_t* __restrict__ viol) {
  const int64_t q = TID;
  if (q >= 4 * npatch) return;
  viol[q] = (dropped[q] && stats[(q / 4) * LEARN_STATS + 24 + q % 4] > 0.f) ? 1 : 0;
}

void learn_patch_stats(int64_t npatch, int n, const float* rn, const float* re, const float* rnf, const float* ref,
                       const uint8_t* na, const uint8_t* naf, const uint8_t* sn, const uint8_t* se, float* stats,
                       hipStream_t s) {
  if (npatch <= 0) return;
  k_patch_stats<<<unsigned((npatch + LB / 64 - 1) / (LB / 64)), LB, 0, s>>>(npatch, n, rn, re, rnf, ref, na, naf, sn,
                                                                           se, stats);
  HIPCHK(hipGetLastError());
}

void learn_features(int64_t npatch, int n, float level_pos, const float* stats, float* X, hipStream_t s) {
  if (npatch <= 0) return;
  k_patch_features<<<nb(npatch), LB, 0, s>>>(npatch, n / 8, level_pos, stats, X);
  HIPCHK(hipGetLastError());
}

void learn_labels(int64_t npatch, const float* stats, float* Y, hipStream_t s) {
  if (npatch <= 0) return;
  k_patch_labels<<<nb(npatch), LB, 0, s>>>(npatch, stats, Y);
  HIPCHK(hipGetLastError());
}

void learn_gate(int64_t npatch, const float* P, double thr, const float* stats, uint8_t* allow, uint8_t* dropped,
                hipStream_t s) {
  if (npatch <= 0) return;
  k_gate<<<nb(4 * npatch), LB, 0, s>>>(npatch, P, float(thr), stats, allow, dropped);
  HIPCHK(hipGetLastError());
}

void learn_violations(int64_t npatch, const float* stats, const uint8_t* dropped, uint8_t* viol, hipStream_t s) {
  if (npatch <= 0) return;
  k_violations<<<nb(4 * npatch), LB, 0, s>>>(npatch, stats, dropped, viol);
  HIPCHK(hipGetLastError());
}

}  // namespace wt
