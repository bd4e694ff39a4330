// Multilevel kernels for gfx950: prolongation of inactive points, flux / Q / B restriction,
// masked tendencies, partial height transform, wavelet details, adaptivity masks and the
// inverse transform (Sec. 2.2-2.3, 3.1, 4.1-4.4).  One thread per coarse node, edge or
// triangle of a level pair; every kernel is a gather, or a scatter of the value 1 into a byte
// mask (idempotent), so results do not depend on thread order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>
#include <string>

#include "wt_alloc.hpp"
#include "wt_body.hpp"
#include "wt_ml.hpp"

namespace wt {

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)

constexpr int BS = 256;
static inline unsigned nb(int64_t n) { return unsigned((n + BS - 1) / BS); }
#define TID (int64_t(blockIdx.x) * BS + threadIdx.x)
// thread index into an optional work list: the i-th listed index (padding entries are -1), or
// i itself
#define LISTED(var, count, lst)            \
  int64_t var = TID;                       \
  if (var >= (count)) return;              \
  if (lst) {                               \
    var = (lst)[var];                      \
    if (var < 0) return;                   \
  }
static inline int64_t span_n(const Span& sp, int64_t dense) { return sp.idx ? sp.n : dense; }

// ------------------------------------------------------------------ prolongation
__global__ __launch_bounds__(BS) void k_prolong_even(DevPair P, const uint8_t* __restrict__ naf,
                                                     const double* __restrict__ hc, double* __restrict__ hf,
                                                     const int32_t* __restrict__ lst, int64_t cnt) {
  LISTED(k, cnt, lst)
  body_prolong_even(k, P, naf, hc, hf);
}

// odd nodes / half-edges and interior edges of a pair in one launch (they do not read each
// other's outputs; both read the even nodes written before): blocks [0, bo) take the coarse
// edges, the rest the coarse triangles
template <typename T>
__global__ __launch_bounds__(BS) void k_prolong_odd_int(DevPair P, const uint8_t* __restrict__ naf,
                                                        const uint8_t* __restrict__ eaf,
                                                        const int32_t* __restrict__ e_v_c,
                                                        const double* __restrict__ uc, double* __restrict__ hf,
                                                        double* __restrict__ uf, const int32_t* __restrict__ le,
                                                        int64_t ne, int bo, const int32_t* __restrict__ lt,
                                                        int64_t nt) {
  if (int(blockIdx.x) < bo) {
    int64_t e = int64_t(blockIdx.x) * BS + threadIdx.x;
    if (e >= ne) return;
    if (le) {
      e = le[e];
      if (e < 0) return;
    }
    body_prolong_odd_pair<T>(e, P, naf, eaf, e_v_c, uc, hf, uf);
  } else {
    int64_t t = int64_t(int(blockIdx.x) - bo) * BS + threadIdx.x;
    if (t >= nt) return;
    if (lt) {
      t = lt[t];
      if (t < 0) return;
    }
    body_prolong_int<T>(t, P, eaf, uc, uf);
  }
}

void ml_prolong(const DevPair& P, const DevTables& tc, const uint8_t* naf, const uint8_t* eaf,
                const double* hc, const double* uc, double* hf, double* uf, bool fp32, hipStream_t s, Span ln,
                Span le, Span lt) {
  const int64_t nn = span_n(ln, P.Nc), ne = span_n(le, P.Ec), nt = span_n(lt, P.Tc);
  if (nn) k_prolong_even<<<nb(nn), BS, 0, s>>>(P, naf, hc, hf, ln.idx, nn);
  const int bo = int(nb(ne)), bt = int(nb(nt));
  if (bo + bt > 0) {
    if (fp32)
      k_prolong_odd_int<float><<<unsigned(bo + bt), BS, 0, s>>>(P, naf, eaf, tc.e_v, uc, hf, uf, le.idx, ne, bo,
                                                                lt.idx, nt);
    else
      k_prolong_odd_int<double><<<unsigned(bo + bt), BS, 0, s>>>(P, naf, eaf, tc.e_v, uc, hf, uf, le.idx, ne, bo,
                                                                 lt.idx, nt);
  }
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ Q, divergence, restriction
template <typename T>
__global__ __launch_bounds__(BS) void k_Q(int64_t E, DevTables tb, const double* __restrict__ F,
                                          const T* __restrict__ qe, T* __restrict__ Q, double nu,
                                          const double* __restrict__ u, const int32_t* __restrict__ lst) {
  LISTED(e, E, lst)
  body_Q<T>(e, tb, F, qe, Q, nu, u);
}

__global__ __launch_bounds__(BS) void k_div(int64_t N, DevTables tf, const double* __restrict__ F,
                                            double* __restrict__ c, const int32_t* __restrict__ lst) {
  LISTED(i, N, lst)
  body_div(i, tf, F, c);
}

template <typename T>
__global__ __launch_bounds__(BS) void k_restrict_edges(DevPair P, const uint8_t* __restrict__ eaf,
                                                       const double* __restrict__ l_f,
                                                       const double* __restrict__ l_c,
                                                       const double* __restrict__ Ff, const double* __restrict__ cf,
                                                       const T* __restrict__ Qf, double* __restrict__ Fc,
                                                       T* __restrict__ Qc, const int32_t* __restrict__ lst,
                                                       int64_t cnt) {
  LISTED(e, cnt, lst)
  body_restrict_edges<T>(e, P, eaf, l_f, l_c, Ff, cf, Qf, Fc, Qc);
}

template <typename T>
__global__ __launch_bounds__(BS) void k_restrict_B(DevPair P, const uint8_t* __restrict__ naf,
                                                   const T* __restrict__ Bf, T* __restrict__ Bc,
                                                   const int32_t* __restrict__ lst, int64_t cnt) {
  LISTED(k, cnt, lst)
  body_restrict_B<T>(k, P, naf, Bf, Bc);
}

// Tendencies at active points of one level with that level's (possibly restricted) F, Q, B,
// zero elsewhere, followed by the Runge-Kutta stage combination.
template <typename T>
__global__ __launch_bounds__(BS) void k_tend_ml(int64_t N, DevTables tb, const uint8_t* __restrict__ na,
                                                const uint8_t* __restrict__ ea, const T* __restrict__ B,
                                                const double* __restrict__ F, const T* __restrict__ Q,
                                                StagePtrs pdh, StagePtrs pu, StageOut c, int32_t adv,
                                                const int32_t* __restrict__ lst) {
  LISTED(id, N, lst)
  body_tend_ml<T>(id, tb, na, ea, B, F, Q, pdh, pu, c, adv);
}

template <typename T>
void ml_level_trisk_t(const DevTables& t, DevWork& w, const PhysParams& p, const double* xdh,
                      const double* xu, hipStream_t s);

void ml_level_intermediates(const DevTables& t, DevWork& w, const PhysParams& p, bool fp32,
                            const double* xdh, const double* xu, hipStream_t s, Span ltri, Span lel, Span led) {
  StagePtrs none{nullptr, nullptr, xdh, nullptr, nullptr};
  StagePtrs noneu{nullptr, nullptr, xu, nullptr, nullptr};
  // q_v, B, F, q_e through the uniform kernels (no stage output), then Q
  launch_intermediates(t, w, p, fp32, none, noneu, s, ltri.idx, span_n(ltri, t.T), lel.idx, span_n(lel, t.N));
  const int64_t ne = span_n(led, t.E);
  if (ne == 0) return;
  if (fp32)
    k_Q<float><<<nb(ne), BS, 0, s>>>(ne, t, static_cast<double*>(w.F), static_cast<float*>(w.qe),
                                     static_cast<float*>(w.Q), p.nu, xu, led.idx);
  else
    k_Q<double><<<nb(ne), BS, 0, s>>>(ne, t, static_cast<double*>(w.F), static_cast<double*>(w.qe),
                                      static_cast<double*>(w.Q), p.nu, xu, led.idx);
  HIPCHK(hipGetLastError());
}

void ml_restrict(const DevPair& P, const DevTables& tc, const DevTables& tf, DevWork& wc, DevWork& wf,
                 const uint8_t* naf, const uint8_t* eaf, const PhysParams& p, bool fp32, hipStream_t s, Span lfn,
                 Span lce, Span lcn) {
  const int64_t nf = span_n(lfn, tf.N), ne = span_n(lce, P.Ec), nn = span_n(lcn, P.Nc);
  double* Gf = total_flux(wf, p);
  double* Gc = total_flux(wc, p);
  if (fp32) {
    if (nf) k_div<<<nb(nf), BS, 0, s>>>(nf, tf, Gf, wf.c, lfn.idx);
    if (ne)
      k_restrict_edges<float><<<nb(ne), BS, 0, s>>>(P, eaf, tf.l_e, tc.l_e, Gf, wf.c, static_cast<float*>(wf.Q), Gc,
                                                    static_cast<float*>(wc.Q), lce.idx, ne);
    if (nn)
      k_restrict_B<float><<<nb(nn), BS, 0, s>>>(P, naf, static_cast<float*>(wf.B), static_cast<float*>(wc.B),
                                                lcn.idx, nn);
  } else {
    if (nf) k_div<<<nb(nf), BS, 0, s>>>(nf, tf, Gf, wf.c, lfn.idx);
    if (ne)
      k_restrict_edges<double><<<nb(ne), BS, 0, s>>>(P, eaf, tf.l_e, tc.l_e, Gf, wf.c, static_cast<double*>(wf.Q), Gc,
                                                     static_cast<double*>(wc.Q), lce.idx, ne);
    if (nn)
      k_restrict_B<double><<<nb(nn), BS, 0, s>>>(P, naf, static_cast<double*>(wf.B), static_cast<double*>(wc.B),
                                                 lcn.idx, nn);
  }
  HIPCHK(hipGetLastError());
}

void ml_tend(const DevTables& t, DevWork& w, const uint8_t* na, const uint8_t* ea, const PhysParams& p, bool fp32,
             const StagePtrs& sdh, const StagePtrs& su, const StageOut& c, hipStream_t s, Span lel) {
  const int64_t n = span_n(lel, t.N);
  if (n == 0) return;
  double* G = total_flux(w, p);
  if (fp32)
    k_tend_ml<float><<<nb(n), BS, 0, s>>>(n, t, na, ea, static_cast<float*>(w.B), G, static_cast<float*>(w.Q), sdh,
                                          su, c, p.adv, lel.idx);
  else
    k_tend_ml<double><<<nb(n), BS, 0, s>>>(n, t, na, ea, static_cast<double*>(w.B), G, static_cast<double*>(w.Q),
                                           sdh, su, c, p.adv, lel.idx);
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ restriction of the state
__global__ __launch_bounds__(BS) void k_restrict_h(DevPair P, const double* __restrict__ hf,
                                                   double* __restrict__ hc) {
  int64_t k = TID;
  if (k >= P.Nc) return;
  double s = hf[P.even[k]];
#pragma unroll
  for (int q = 0; q < MK_MAX; ++q) {   // valid entries first, then -1: same order as a break
    const int32_t ec = P.mk[P.cn(q, k)];
    if (ec >= 0) s += P.s_upd[P.upd(ec)] * h_detail(P, ec >> 2, hf);
  }
  hc[k] = s;
}

__global__ __launch_bounds__(BS) void k_restrict_u(DevPair P, const double* __restrict__ uf,
                                                   double* __restrict__ uc) {
  int64_t e = TID;
  if (e >= P.Ec) return;
  uc[e] = 0.5 * (uf[P.h1[e]] + uf[P.h2[e]]);
}

void ml_restrict_state(const DevPair& P, const double* hf, const double* uf, double* hc, double* uc,
                       hipStream_t s) {
  k_restrict_h<<<nb(P.Nc), BS, 0, s>>>(P, hf, hc);
  k_restrict_u<<<nb(P.Ec), BS, 0, s>>>(P, uf, uc);
  HIPCHK(hipGetLastError());
}

// Partial height transform at complete coarse nodes: the whole height-restriction stencil is
// active and every coarse edge of the node is non-leaf.
__global__ __launch_bounds__(BS) void k_partial_d(DevPair P, const uint8_t* __restrict__ naf,
                                                  const double* __restrict__ hf, double* __restrict__ det,
                                                  uint8_t* __restrict__ act) {
  const int64_t e = TID;
  if (e >= P.Ec) return;
  body_partial_d(e, P, naf, hf, det, act);
}

__global__ __launch_bounds__(BS) void k_partial_h(DevPair P, const int32_t* __restrict__ c_e_c,
                                                  const uint8_t* __restrict__ nac,
                                                  const uint8_t* __restrict__ naf,
                                                  const uint8_t* __restrict__ eaf,
                                                  const double* __restrict__ det, const uint8_t* __restrict__ act,
                                                  const double* __restrict__ hf, double* __restrict__ hc,
                                                  const int32_t* __restrict__ lst, int64_t cnt) {
  LISTED(k, cnt, lst)
  body_partial_h(k, P, c_e_c, nac, naf, eaf, det, act, hf, hc);
}

void ml_partial_h(const DevPair& P, const DevTables& tc, const uint8_t* nac, const uint8_t* naf,
                  const uint8_t* eaf, const double* hf, double* hc, double* det, uint8_t* act, hipStream_t s,
                  Span lcn) {
  const int64_t n = span_n(lcn, P.Nc);
  if (!n) return;
  // every coarse edge's stencil activity (so none is stale), then the listed coarse nodes
  k_partial_d<<<nb(P.Ec), BS, 0, s>>>(P, naf, hf, det, act);
  k_partial_h<<<nb(n), BS, 0, s>>>(P, tc.c_e, nac, naf, eaf, det, act, hf, hc, lcn.idx, n);
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ details
// ------------------------------------------------------------------ masks
// One ring in gather form: B = A and the same-level neighbours of A in the sense of R2 (a node
// joins if it, a neighbour node or an incident edge is in A; an edge joins if it, an end node or
// an edge of one of its triangles is in A).  No copy of A and no scatter.  Points away from the
// lozenge sides find their neighbours by lattice index arithmetic (only mask bytes are read);
// the others, and the poles, through the level's tables (a padded pentagon slot repeats an edge
// of the cell, which changes nothing here).
// One ring of same-level neighbours of the (an, ae) points: threads [0, N) do the nodes, [N, N+E)
// the edges.  Lattice-interior points use index arithmetic on the lozenge rows (n = 2^sh, ids fit
// in 32 bits up to level 11); the rest go through the tables.
__device__ __forceinline__ uint8_t ring_node(int32_t id, int sh, const int32_t* __restrict__ c_e,
                                             const int32_t* __restrict__ e_c, const uint8_t* __restrict__ an,
                                             const uint8_t* __restrict__ ae) {
  const int n = 1 << sh, mk = n - 1;
  uint8_t m = an[id];
  const int i = (id >> sh) & mk, j = id & mk;
  if ((id >> (2 * sh)) < 10 && i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2) {
    const int32_t r = n;   // next row
    m |= an[id + r] | an[id + r + 1] | an[id + 1] | an[id - r] | an[id - r - 1] | an[id - 1];
    m |= ae[3 * id] | ae[3 * id + 1] | ae[3 * id + 2] | ae[3 * (id - r)] | ae[3 * (id - r - 1) + 1] |
         ae[3 * (id - 1) + 2];
  } else {
    for (int q = 0; q < 6 && !m; ++q) {
      const int32_t e = c_e[6 * id + q];
      m = ae[e] | an[e_c[2 * e]] | an[e_c[2 * e + 1]];
    }
  }
  return m;
}

__device__ __forceinline__ uint8_t ring_edge(int32_t e, int sh, const int32_t* __restrict__ e_c,
                                             const int32_t* __restrict__ e_v, const int32_t* __restrict__ t_e,
                                             const uint8_t* __restrict__ an, const uint8_t* __restrict__ ae) {
  const int n = 1 << sh, mk = n - 1;
  const int32_t id = e / 3;
  const int d = e - 3 * id;
  const int i = (id >> sh) & mk, j = id & mk;
  uint8_t m;
  if (i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2) {
    const int32_t r = n;
    if (d == 0) {          // P -> P+(1,0): triangles (P, P+(1,0), P+(1,1)) and ((i,j-1), (i+1,j), P)
      m = an[id] | an[id + r] | ae[3 * id] | ae[3 * (id + r) + 2] | ae[3 * id + 1] | ae[3 * (id - 1) + 1] |
          ae[3 * (id - 1) + 2];
    } else if (d == 1) {   // P -> P+(1,1): triangles (P, P+(1,0), P+(1,1)) and (P, P+(1,1), P+(0,1))
      m = an[id] | an[id + r + 1] | ae[3 * id] | ae[3 * (id + r) + 2] | ae[3 * id + 1] | ae[3 * (id + 1)] |
          ae[3 * id + 2];
    } else {               // P -> P+(0,1): triangles (P, P+(1,1), P+(0,1)) and ((i-1,j), P, P+(0,1))
      m = an[id] | an[id + 1] | ae[3 * id + 1] | ae[3 * (id + 1)] | ae[3 * id + 2] | ae[3 * (id - r)] |
          ae[3 * (id - r) + 1];
    }
  } else {
    m = ae[e] | an[e_c[2 * e]] | an[e_c[2 * e + 1]];
    for (int side = 0; side < 2 && !m; ++side) {
      const int32_t t = e_v[2 * e + side];
      m = ae[t_e[3 * t]] | ae[t_e[3 * t + 1]] | ae[t_e[3 * t + 2]];
    }
  }
  return m;
}

// Levels with lozenge side below 8: one thread per node, then one per edge.
__global__ __launch_bounds__(BS) void k_ring_small(int32_t N, int32_t E, int sh, const int32_t* __restrict__ c_e,
                                                   const int32_t* __restrict__ e_c, const int32_t* __restrict__ e_v,
                                                   const int32_t* __restrict__ t_e, const uint8_t* __restrict__ an,
                                                   const uint8_t* __restrict__ ae, uint8_t* __restrict__ bn,
                                                   uint8_t* __restrict__ be) {
  const int32_t k = int32_t(blockIdx.x) * BS + int32_t(threadIdx.x);
  if (k < N) bn[k] = ring_node(k, sh, c_e, e_c, an, ae) ? 1 : 0;
  else if (k - N < E) be[k - N] = ring_edge(k - N, sh, e_c, e_v, t_e, an, ae) ? 1 : 0;
}

void ml_ring(const DevTables& t, int n, const uint8_t* an, const uint8_t* ae, uint8_t* bn, uint8_t* be,
             hipStream_t s) {
  if (n <= 0 || (n & (n - 1)) != 0) throw std::runtime_error("ml_ring: lozenge side must be a power of two");
  if (t.N + t.E >= (int64_t(1) << 31)) throw std::runtime_error("ml_ring: level too large for 32-bit ids");
  const int64_t lat = int64_t(10) * n * n;
  if (t.E != 3 * lat || t.N < lat || t.N - lat > BS)
    throw std::runtime_error("ml_ring: tables do not match the lattice size");
  const int sh = __builtin_ctz(unsigned(n));
  k_ring_small<<<nb(t.N + t.E), BS, 0, s>>>(int32_t(t.N), int32_t(t.E), sh, t.c_e, t.e_c, t.e_v, t.t_e, an, ae,
                                            bn, be);
  HIPCHK(hipGetLastError());
}

// One ring over the listed 8 x 8 node patches of several levels in one launch: blockIdx.y picks
// the level, whose first nblk blocks stride over its list, one block per patch (threads 0..63 the
// nodes, 64..255 their 192 edges); block 0 also does the poles.  The points of unlisted patches
// are not written (the caller cleared them).
// One ring over the listed patches of a level.  A patch away from the lozenge sides (patch rows
// and columns 1 .. m-2) stages the mask bytes of its 8 x 8 nodes and one ring of neighbours
// (rows and columns -1 .. 8: 10 node bytes and their 30 edge bytes a row) in LDS with coalesced
// byte loads, two per thread instead of 7-13 scattered ones, and evaluates the rule there with
// ring_node's and ring_edge's lattice-interior neighbours; a patch on a side takes the per-point
// rule (tables at the side).  The branch is uniform per block.  (Staging two patches per pass
// was slower: 342 against 245 us per ring on the turbulence's level 10.)
__global__ __launch_bounds__(BS) void k_ring_b(RingJobs J) {
  static_assert(BS == 256, "one block covers the 64 nodes and 192 edges of a patch");
  constexpr int SW = 10, EW = 30;   // staged row widths: node bytes, edge bytes
  __shared__ uint8_t s_n[SW * SW], s_e[SW * EW];
  const RingJob& jb = J.j[blockIdx.y];
  if (int(blockIdx.x) >= jb.nblk) return;
  const int sh = jb.sh, ps = sh - 3, m = 1 << ps;
  const int tid = threadIdx.x;
  const bool node = tid < 64;   // wave 0 the nodes of the patch, waves 1-3 their edges
  const int q = node ? tid : (tid - 64) / 3, d = node ? 0 : (tid - 64) - 3 * q;
  const int qi = q >> 3, qj = q & 7;
  const int ln = SW * (qi + 1) + (qj + 1), le = EW * (qi + 1) + 3 * (qj + 1);   // the point in LDS
  const int32_t cnt = *jb.pcount;
  uint8_t* __restrict__ out = node ? jb.bn : jb.be;
  for (int32_t b = blockIdx.x; b < cnt; b += jb.nblk) {
    const int32_t p = jb.plist[b];
    const int32_t L = p >> (2 * ps);
    const int pi = (p >> ps) & (m - 1), pj = p & (m - 1);
    const int32_t row0 = (L << sh) + 8 * pi;   // L n + i0
    const int32_t id = ((row0 + qi) << sh) + 8 * pj + qj;
    const int32_t x = node ? id : 3 * id + d;
    if (pi >= 1 && pi <= m - 2 && pj >= 1 && pj <= m - 2) {
      for (int t = tid; t < SW * (SW + EW); t += BS) {
        const int r = t / (SW + EW), w = t - (SW + EW) * r;
        const int32_t base = ((row0 - 1 + r) << sh) + 8 * pj - 1;   // node (i0 - 1 + r, j0 - 1)
        if (w < SW) s_n[SW * r + w] = jb.an[base + w];
        else s_e[EW * r + (w - SW)] = jb.ae[3 * base + (w - SW)];
      }
      __syncthreads();
      uint8_t v;
      if (node) {
        v = s_n[ln] | s_n[ln + SW] | s_n[ln + SW + 1] | s_n[ln + 1] | s_n[ln - SW] | s_n[ln - SW - 1] | s_n[ln - 1];
        v |= s_e[le] | s_e[le + 1] | s_e[le + 2] | s_e[le - EW] | s_e[le - EW - 2] | s_e[le - 1];
      } else if (d == 0) {
        v = s_n[ln] | s_n[ln + SW] | s_e[le] | s_e[le + EW + 2] | s_e[le + 1] | s_e[le - 2] | s_e[le - 1];
      } else if (d == 1) {
        v = s_n[ln] | s_n[ln + SW + 1] | s_e[le] | s_e[le + EW + 2] | s_e[le + 1] | s_e[le + 3] | s_e[le + 2];
      } else {
        v = s_n[ln] | s_n[ln + 1] | s_e[le + 1] | s_e[le + 3] | s_e[le + 2] | s_e[le - EW] | s_e[le - EW + 1];
      }
      out[x] = v ? 1 : 0;
      __syncthreads();   // the next patch's staging overwrites the LDS
    } else {
      out[x] = (node ? ring_node(x, sh, jb.c_e, jb.e_c, jb.an, jb.ae)
                     : ring_edge(x, sh, jb.e_c, jb.e_v, jb.t_e, jb.an, jb.ae)) ? 1 : 0;
    }
  }
  const int32_t pole = (10 << (2 * sh)) + tid;
  if (blockIdx.x == 0 && pole < jb.N) jb.bn[pole] = ring_node(pole, sh, jb.c_e, jb.e_c, jb.an, jb.ae) ? 1 : 0;
}

RingJob ring_job(const DevTables& t, int n, const uint8_t* an, const uint8_t* ae, uint8_t* bn, uint8_t* be,
                 const int32_t* plist) {
  if (n < 8 || (n & (n - 1)) != 0) throw std::runtime_error("ring_job: lozenge side must be 2^k >= 8");
  const int64_t lat = int64_t(10) * n * n;
  if (t.E != 3 * lat || t.N < lat || t.N - lat > BS || t.N + t.E >= (int64_t(1) << 31))
    throw std::runtime_error("ring_job: tables do not match the lattice size");
  const int64_t np = lat / 64;
  RingJob j{};
  j.N = int32_t(t.N);
  j.sh = __builtin_ctz(unsigned(n));
  j.nblk = int32_t(np < 2048 ? np : 2048);   // one round of workgroups at full occupancy (8 per CU)
  j.plist = plist;
  j.pcount = plist + np;
  j.c_e = t.c_e; j.e_c = t.e_c; j.e_v = t.e_v; j.t_e = t.t_e;
  j.an = an; j.ae = ae; j.bn = bn; j.be = be;
  return j;
}

void ml_ring_batch(const RingJob* jobs, int njobs, hipStream_t s) {
  for (int k0 = 0; k0 < njobs; k0 += MAX_LEVJOBS) {
    RingJobs J{};
    const int nk = njobs - k0 < MAX_LEVJOBS ? njobs - k0 : MAX_LEVJOBS;
    int grid = 1;
    for (int k = 0; k < nk; ++k) {
      J.j[k] = jobs[k0 + k];
      if (J.j[k].nblk > grid) grid = J.j[k].nblk;
    }
    k_ring_b<<<dim3(grid, nk), BS, 0, s>>>(J);
    HIPCHK(hipGetLastError());
  }
}

// Patch list for the ring dilation: pf[p] = the 8 x 8 node patch p (patch (L, pi, pj) ->
// (L m + pi) m + pj, m = n / 8) holds an active node or an active edge of its nodes; p is listed
// when some patch of its 3 x 3 neighbourhood in the lozenge is flagged, or p touches the lozenge
// border.  A node of an unlisted patch is more than 7 lattice steps from every active point (a
// path from another lozenge crosses the border, 8 steps away), so up to 7 rings leave it and its
// edges inactive.  The list order is the order of the appends (the ring does not depend on it).
// Several levels per launch (blockIdx.y picks the level; rows beyond a level's range exit).
// One thread per row of a patch (t = ((L m + pi) m + pj) 8 + r): the 8 mask bytes of its nodes and
// the 24 of their edges; the 8 lanes of a patch are combined by a wavefront ballot.
__global__ __launch_bounds__(BS) void k_patch_any_b(PatchJobs J) {
  const PatchJob& jb = J.j[blockIdx.y];
  const int sh = jb.sh, ps = sh - 3;
  const int64_t rows = int64_t(10) << (2 * sh - 3);
  if (int64_t(blockIdx.x) * BS >= rows) return;   // whole block out of range (uniform)
  const int64_t t = TID;
  if (t == 0) *jb.pcount = 0;
  const bool valid = t < rows;
  bool any = false;
  if (valid) {
    const int64_t p = t >> 3;
    const int m = 1 << ps, r = int(t & 7);
    const int64_t L = p >> (2 * ps);
    const int pi = int((p >> ps) & (m - 1)), pj = int(p & (m - 1));
    const int64_t id0 = ((L << sh) + 8 * pi + r) * (int64_t(1) << sh) + 8 * pj;
    const uint64_t a = *reinterpret_cast<const uint64_t*>(jb.an + id0);
    const uint64_t* ew = reinterpret_cast<const uint64_t*>(jb.ae + 3 * id0);
    any = (a | ew[0] | ew[1] | ew[2]) != 0;
  }
  const uint64_t bal = __ballot(any);
  const int lane = threadIdx.x & 63;
  if (valid && (lane & 7) == 0) jb.pf[t >> 3] = ((bal >> lane) & 0xffu) ? 1 : 0;
}

__global__ __launch_bounds__(BS) void k_patch_list_b(PatchJobs J) {
  const PatchJob& jb = J.j[blockIdx.y];
  const int ps = jb.sh - 3, m = 1 << ps;
  const int64_t p = TID;
  if (p >= int64_t(10) << (2 * ps)) return;
  const int64_t L = p >> (2 * ps);
  const int pi = int((p >> ps) & (m - 1)), pj = int(p & (m - 1));
  uint8_t v = (pi == 0 || pj == 0 || pi == m - 1 || pj == m - 1) ? 1 : 0;
  for (int di = -1; di <= 1 && !v; ++di)
    for (int dj = -1; dj <= 1 && !v; ++dj) v = jb.pf[((L << ps) + pi + di) * m + pj + dj];
  if (v) jb.plist[atomicAdd(jb.pcount, 1)] = int32_t(p);
}

void ml_patch_list_batch(const PatchJob* jobs, int njobs, hipStream_t s) {
  for (int k0 = 0; k0 < njobs; k0 += MAX_LEVJOBS) {
    PatchJobs J{};
    const int nk = njobs - k0 < MAX_LEVJOBS ? njobs - k0 : MAX_LEVJOBS;
    int64_t rows = 0;
    for (int k = 0; k < nk; ++k) {
      J.j[k] = jobs[k0 + k];
      if (J.j[k].sh < 3) throw std::runtime_error("ml_patch_list_batch: lozenge side must be 2^k >= 8");
      const int64_t r = int64_t(10) << (2 * J.j[k].sh - 3);
      if (r > rows) rows = r;
    }
    k_patch_any_b<<<dim3(nb(rows), nk), BS, 0, s>>>(J);
    k_patch_list_b<<<dim3(nb(rows / 8), nk), BS, 0, s>>>(J);
    HIPCHK(hipGetLastError());
  }
}


// ------------------------------------------------------------------ details and masks R1-R3
// Per-point bodies of the forward transform's details (eqs. (WTpred), velocity prediction) and
// of the rules R1 (significant points: active, |d| >= eps), R2 (same-level neighbours of
// significant nodes -- neighbour nodes, incident edges -- and edges -- end nodes, the edges of
// both triangles) and R3 (children on the next level of significant coarse nodes -- fine copy,
// its neighbours and incident fine edges -- and edges -- midpoint and the fine edges at it).
// The mask rules only set bytes to 1, so jobs of one launch may write the same mask.
template <typename T>
__device__ __forceinline__ void op_det_edge_t(int64_t e, const MaskJob& j) {
  const DevPair& P = j.P;
  j.dh[e] = h_detail(P, e, j.hf);
  j.dp[e] = (j.uf[P.h1[e]] - j.uf[P.h2[e]]) - double(pair_pred<T>(P, e, j.e_v, j.uc));
}

template <typename T>
__device__ __forceinline__ void op_det_int_t(int64_t t, const MaskJob& j) {
  const DevPair& P = j.P;
#pragma unroll
  for (int s = 0; s < 3; ++s) j.di[3 * t + s] = j.uf[P.int_e[3 * t + s]] - double(int_pred_c<T>(P, t, s, j.uc));
}

__device__ __forceinline__ void op_det_edge(int64_t e, const MaskJob& j) {
  if (j.fp32) op_det_edge_t<float>(e, j);
  else op_det_edge_t<double>(e, j);
}

__device__ __forceinline__ void op_det_int(int64_t t, const MaskJob& j) {
  if (j.fp32) op_det_int_t<float>(t, j);
  else op_det_int_t<double>(t, j);
}

__device__ __forceinline__ void op_sig_edge(int64_t e, const MaskJob& j) {
  const DevPair& P = j.P;
  const double eh = j.thr ? j.thr[0] : j.eh, eu = j.thr ? j.thr[1] : j.eu;
  const int32_t m = P.mid[e];
  if (j.a_n[m] && fabs(j.dh[e]) >= eh) j.o_n[m] = 1;
  const int32_t h1 = P.h1[e], h2 = P.h2[e];
  if (j.a_e[h1] && j.a_e[h2] && fabs(j.dp[e]) >= eu) {
    j.o_e[h1] = 1;
    j.o_e[h2] = 1;
  }
}

__device__ __forceinline__ void op_sig_int(int64_t t, const MaskJob& j) {
  const double eu = j.thr ? j.thr[1] : j.eu;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int32_t f = j.P.int_e[3 * t + s];
    if (j.a_e[f] && fabs(j.di[3 * t + s]) >= eu) j.o_e[f] = 1;
  }
}

__device__ __forceinline__ void op_r2_node(int64_t i, const MaskJob& j) {
  if (!j.a_n[i]) return;
  for (int q = 0; q < 6; ++q) {
    if (j.c_div[6 * i + q] == 0.0) continue;  // padded pentagon slot
    const int32_t e = j.c_e[6 * i + q];
    j.o_e[e] = 1;
    j.o_n[j.e_c[2 * e]] = 1;
    j.o_n[j.e_c[2 * e + 1]] = 1;
  }
}

__device__ __forceinline__ void op_r2_edge(int64_t e, const MaskJob& j) {
  if (!j.a_e[e]) return;
  j.o_n[j.e_c[2 * e]] = 1;
  j.o_n[j.e_c[2 * e + 1]] = 1;
  for (int side = 0; side < 2; ++side) {
    const int32_t t = j.e_v[2 * e + side];
    for (int s = 0; s < 3; ++s) j.o_e[j.t_e[3 * t + s]] = 1;
  }
}

__device__ __forceinline__ void mark_cell(int64_t f, const MaskJob& j, bool nbrs) {
  j.o_n[f] = 1;
  for (int q = 0; q < 6; ++q) {
    if (j.c_div[6 * f + q] == 0.0) continue;
    const int32_t e = j.c_e[6 * f + q];
    j.o_e[e] = 1;
    if (nbrs) {
      j.o_n[j.e_c[2 * e]] = 1;
      j.o_n[j.e_c[2 * e + 1]] = 1;
    }
  }
}

// Learned gate of the children rule: allow[4 patch + quadrant] for the element owning a coarse
// point (null: every point passes; the poles always pass).
__device__ __forceinline__ bool r3_allowed(const uint8_t* __restrict__ allow, int n, int64_t elem) {
  if (!allow || elem >= int64_t(10) * n * n) return true;
  const int64_t L = elem / (int64_t(n) * n);
  const int i = int((elem / n) % n), j = int(elem % n), m = n / 8;
  const int64_t patch = (L * m + i / 8) * m + j / 8;
  return allow[4 * patch + 2 * ((i % 8) / 4) + (j % 8) / 4] != 0;
}

__device__ __forceinline__ void op_r3_node(int64_t k, const MaskJob& j) {
  if (!j.a_n[k] || !r3_allowed(j.allow, j.nc, k)) return;
  mark_cell(j.P.even[k], j, true);
}

__device__ __forceinline__ void op_r3_edge(int64_t e, const MaskJob& j) {
  if (!j.a_e[e] || !r3_allowed(j.allow, j.nc, e / 3)) return;
  mark_cell(j.P.mid[e], j, false);
}

// Each job owns a range of workgroups, pre[j] <= blockIdx.x < pre[j+1], about one thread per
// entry (a list, padding -1 skipped, or 0..cnt), striding if the job has more entries.  Two
// instances: with the details (DET, every op) and without them (the mask rules only): the rules
// are byte gathers bound by load latency and run best at 6 waves per SIMD, which the register
// budget of the detail arithmetic would not allow.
template <bool DET>
__global__ __launch_bounds__(BS, DET ? 4 : 6) void k_mask_b(MaskJobs J) {
  const int32_t c = int32_t(blockIdx.x);
  int q = 0;
  while (q + 1 < J.n && J.pre[q + 1] <= c) ++q;
  const MaskJob& jb = J.j[q];
  const int64_t stride = int64_t(J.pre[q + 1] - J.pre[q]) * BS;
  if (jb.sparse) {
    // large whole-level rules, a wavefront at a time: each lane tests the significance bytes of 16
    // points with one load, a ballot collects the groups holding one (few: significant points are
    // sparse), and the wavefront then runs four such groups per pass, one point per lane.  The
    // last, partial group is always visited (its points are bounds-checked).
    const uint8_t* a = (jb.op == MO_R2_NODE || jb.op == MO_R3_NODE) ? jb.a_n : jb.a_e;
    const int64_t ng = (jb.cnt + 15) / 16;
    const int lane = threadIdx.x & 63;
    for (int64_t gb = int64_t(c - J.pre[q]) * BS + (threadIdx.x & ~63); gb < ng; gb += stride) {
      const int64_t g = gb + lane;
      bool hit = false;
      if (g < ng) {
        if (16 * g + 16 <= jb.cnt) {
          const uint4 w = *reinterpret_cast<const uint4*>(a + 16 * g);
          hit = (w.x | w.y | w.z | w.w) != 0u;
        } else {
          hit = true;
        }
      }
      uint64_t rem = __ballot(hit);
      while (rem) {
        int sel[4], k = 0;
        for (; k < 4 && rem; ++k) {
          sel[k] = __ffsll(static_cast<unsigned long long>(rem)) - 1;
          rem &= rem - 1;
        }
        const int sub = lane >> 4;
        if (sub < k) {
          const int64_t i = 16 * (gb + sel[sub]) + (lane & 15);
          if (i < jb.cnt) {
            switch (jb.op) {
              case MO_R2_NODE: op_r2_node(i, jb); break;
              case MO_R2_EDGE: op_r2_edge(i, jb); break;
              case MO_R3_NODE: op_r3_node(i, jb); break;
              default: op_r3_edge(i, jb); break;
            }
          }
        }
      }
    }
    return;
  }
  for (int64_t r = int64_t(c - J.pre[q]) * BS + threadIdx.x; r < jb.cnt; r += stride) {
    int64_t i = r;
    if (jb.lst) {
      i = jb.lst[r];
      if (i < 0) continue;
    }
    switch (jb.op) {
      case MO_DET_EDGE:
        if constexpr (DET) op_det_edge(i, jb);
        break;
      case MO_DET_INT:
        if constexpr (DET) op_det_int(i, jb);
        break;
      case MO_SIG_EDGE: op_sig_edge(i, jb); break;
      case MO_SIG_INT: op_sig_int(i, jb); break;
      case MO_R2_NODE: op_r2_node(i, jb); break;
      case MO_R2_EDGE: op_r2_edge(i, jb); break;
      case MO_R3_NODE: op_r3_node(i, jb); break;
      case MO_R3_EDGE: op_r3_edge(i, jb); break;
      default: break;
    }
  }
}

void ml_mask_ops(const MaskJob* jobs, int njobs, hipStream_t s) {
  constexpr int64_t kMaxBlocks = 16384;   // per job; more entries are strided over
  for (int k0 = 0; k0 < njobs; k0 += MAX_MASK_JOBS) {
    MaskJobs J{};
    int nk = 0;
    int64_t run = 0;
    bool det = false;
    for (int k = k0; k < njobs && k < k0 + MAX_MASK_JOBS; ++k) {
      if (jobs[k].cnt <= 0) continue;
      const MaskJob& jk = jobs[k];
      det |= jk.op == MO_DET_EDGE || jk.op == MO_DET_INT;
      if (jk.op >= MO_R2_NODE && jk.lst)
        throw std::runtime_error("ml_mask_ops: the mask rules run over whole levels");
      if (jk.op >= MO_R2_NODE &&
          (reinterpret_cast<uintptr_t>(jk.op == MO_R2_NODE || jk.op == MO_R3_NODE ? jk.a_n : jk.a_e) & 15))
        throw std::runtime_error("ml_mask_ops: significance masks must be 16-byte aligned");
      // rule jobs over large levels scan 16 points per lane (their significant points are
      // sparse); the others take one point per thread
      const bool sparse = jk.op >= MO_R2_NODE && jk.cnt >= (int64_t(1) << 21);
      const int64_t units = sparse ? (jk.cnt + 15) / 16 : jk.cnt;
      J.pre[nk] = int32_t(run);
      J.j[nk] = jk;
      J.j[nk++].sparse = sparse ? 1 : 0;
      run += std::min<int64_t>(kMaxBlocks, (units + BS - 1) / BS);
    }
    if (nk == 0) continue;
    J.pre[nk] = int32_t(run);
    J.n = nk;
    if (det)
      k_mask_b<true><<<unsigned(run), BS, 0, s>>>(J);
    else
      k_mask_b<false><<<unsigned(run), BS, 0, s>>>(J);
    HIPCHK(hipGetLastError());
  }
}

void ml_details_jobs(std::vector<MaskJob>& out, const DevPair& P, const DevTables& tc, const double* hf,
                     const double* uf, const double* uc, double* dh, double* dp, double* di, bool fp32, Span le,
                     Span lt) {
  MaskJob a{};
  a.P = P; a.e_v = tc.e_v; a.hf = hf; a.uf = uf; a.uc = uc; a.dh = dh; a.dp = dp; a.di = di;
  a.fp32 = fp32 ? 1 : 0;
  a.op = MO_DET_EDGE; a.cnt = span_n(le, P.Ec); a.lst = le.idx;
  out.push_back(a);
  a.op = MO_DET_INT; a.cnt = span_n(lt, P.Tc); a.lst = lt.idx;
  out.push_back(a);
}

void ml_significant_jobs(std::vector<MaskJob>& out, const DevPair& P, const uint8_t* naf, const uint8_t* eaf,
                         const double* dh, const double* dp, const double* di, double eh, double eu, uint8_t* sn,
                         uint8_t* se, Span le, Span lt) {
  MaskJob a{};
  a.P = P; a.a_n = naf; a.a_e = eaf; a.dh = const_cast<double*>(dh); a.dp = const_cast<double*>(dp);
  a.di = const_cast<double*>(di); a.eh = eh; a.eu = eu; a.o_n = sn; a.o_e = se;
  a.op = MO_SIG_EDGE; a.cnt = span_n(le, P.Ec); a.lst = le.idx;
  out.push_back(a);
  a.op = MO_SIG_INT; a.cnt = span_n(lt, P.Tc); a.lst = lt.idx;
  out.push_back(a);
}

void ml_r2_jobs(std::vector<MaskJob>& out, const DevTables& t, const uint8_t* sn, const uint8_t* se, uint8_t* nn,
                uint8_t* ne) {
  MaskJob a{};
  a.c_e = t.c_e; a.c_div = t.c_div; a.e_c = t.e_c; a.e_v = t.e_v; a.t_e = t.t_e;
  a.a_n = sn; a.a_e = se; a.o_n = nn; a.o_e = ne;
  a.op = MO_R2_NODE; a.cnt = t.N;
  out.push_back(a);
  a.op = MO_R2_EDGE; a.cnt = t.E;
  out.push_back(a);
}

void ml_r3_jobs(std::vector<MaskJob>& out, const DevPair& P, const DevTables& tf, const uint8_t* snc,
                const uint8_t* sec, uint8_t* nnf, uint8_t* nef, const uint8_t* allow, int nc) {
  MaskJob a{};
  a.P = P; a.c_e = tf.c_e; a.c_div = tf.c_div; a.e_c = tf.e_c;
  a.a_n = snc; a.a_e = sec; a.o_n = nnf; a.o_e = nef; a.allow = allow; a.nc = nc;
  a.op = MO_R3_NODE; a.cnt = P.Nc;
  out.push_back(a);
  a.op = MO_R3_EDGE; a.cnt = P.Ec;
  out.push_back(a);
}

// R4: edges at active nodes, then end nodes of active edges.
__global__ __launch_bounds__(BS) void k_r4_a(int64_t N, const int32_t* __restrict__ c_e,
                                             const double* __restrict__ c_div,
                                             const uint8_t* __restrict__ nn, uint8_t* __restrict__ ne) {
  int64_t i = TID;
  if (i >= N || !nn[i]) return;
  for (int q = 0; q < 6; ++q)
    if (c_div[6 * i + q] != 0.0) ne[c_e[6 * i + q]] = 1;
}

__global__ __launch_bounds__(BS) void k_r4_b(int64_t E, const int32_t* __restrict__ e_c,
                                             const uint8_t* __restrict__ ne, uint8_t* __restrict__ nn) {
  int64_t e = TID;
  if (e >= E || !ne[e]) return;
  nn[e_c[2 * e]] = 1;
  nn[e_c[2 * e + 1]] = 1;
}

void ml_r4(const DevTables& t, uint8_t* nn, uint8_t* ne, hipStream_t s) {
  k_r4_a<<<nb(t.N), BS, 0, s>>>(t.N, t.c_e, t.c_div, nn, ne);
  k_r4_b<<<nb(t.E), BS, 0, s>>>(t.E, t.e_c, ne, nn);
  HIPCHK(hipGetLastError());
}

// R5: prediction stencils on the coarse level of every active fine point.  Thread k takes coarse
// edge k, coarse node k and coarse triangle k (the three rules only set coarse mask bytes from
// the fine masks, so one launch holds them all).
__global__ __launch_bounds__(BS) void k_r5(DevPair P, const int32_t* __restrict__ e_v_c,
                                           const uint8_t* __restrict__ nnf, const uint8_t* __restrict__ nef,
                                           uint8_t* __restrict__ nnc, uint8_t* __restrict__ nec) {
  const int64_t k = TID;
  if (k < P.Ec) {
    const int64_t e = k;
    if (nnf[P.mid[e]])
      for (int c = 0; c < 4; ++c) nnc[P.cells[4 * e + c]] = 1;
    if (nef[P.h1[e]] || nef[P.h2[e]]) {
      nec[e] = 1;
      const int32_t tl = e_v_c[2 * e], tr = e_v_c[2 * e + 1];
      for (int q = 0; q < 9; ++q) {
        nec[P.v_sten[9 * tl + q]] = 1;
        nec[P.v_sten[9 * tr + q]] = 1;
      }
    }
  }
  if (k < P.Nc && nnf[P.even[k]]) nnc[k] = 1;
  if (k < P.Tc && (nef[P.int_e[3 * k]] || nef[P.int_e[3 * k + 1]] || nef[P.int_e[3 * k + 2]]))
    for (int q = 0; q < 9; ++q) nec[P.v_sten[9 * k + q]] = 1;
}

void ml_r5(const DevPair& P, const DevTables& tc, const uint8_t* nnf, const uint8_t* nef, uint8_t* nnc,
           uint8_t* nec, hipStream_t s) {
  int64_t m = P.Ec;
  if (P.Nc > m) m = P.Nc;
  if (P.Tc > m) m = P.Tc;
  k_r5<<<nb(m), BS, 0, s>>>(P, tc.e_v, nnf, nef, nnc, nec);
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ inverse transform
// Top-down, one pair at a time: kept details (points active before and after) or zero;
// even fine nodes h^j_k - sum_m s_km d_m, then odd nodes d_m + sum_c s~_cm h_even(c);
// half-edges u^j -+ ((p1-p2) + d)/2; interior edges d + prediction.
// the kept details of every coarse edge of several pairs (an even node's update reads up to 12
// of them): blockIdx.y picks the pair
__global__ __launch_bounds__(BS) void k_inv_keep_b(KeepJobs J) {
  const KeepJob& jb = J.j[blockIdx.y];
  for (int64_t e = TID; e < jb.Ec; e += int64_t(gridDim.x) * BS) {
    const int32_t m = jb.mid[e];
    jb.dk[e] = (jb.na_old[m] && jb.na_new[m]) ? jb.dh[e] : 0.0;
  }
}

__device__ __forceinline__ void inv_even(int64_t k, const DevPair& P, const double* __restrict__ dk,
                                         const double* __restrict__ hc, double* __restrict__ hf) {
  double s = hc[k];
#pragma unroll
  for (int q = 0; q < MK_MAX; ++q) {   // valid entries first, then -1: same order as a break
    const int32_t ec = P.mk[P.cn(q, k)];
    if (ec >= 0) s -= P.s_upd[P.upd(ec)] * dk[ec >> 2];
  }
  hf[P.even[k]] = s;
}

template <typename T>
__device__ __forceinline__ void inv_int(int64_t t, const DevPair& P, const uint8_t* __restrict__ ea_old,
                                        const uint8_t* __restrict__ ea_new, const double* __restrict__ di,
                                        const double* __restrict__ uc, double* __restrict__ uf) {
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int32_t f = P.int_e[3 * t + s];
    const bool keep = ea_old[f] && ea_new[f];
    uf[f] = (keep ? di[3 * t + s] : 0.0) + double(int_pred_c<T>(P, t, s, uc));
  }
}

// even nodes (heights) and interior fine edges (velocities) of a pair in one launch: they do not
// read each other's outputs; blocks [0, be) take the even nodes, the rest the coarse triangles
template <typename T>
__global__ __launch_bounds__(BS) void k_inv_even_int(DevPair P, const double* __restrict__ dk,
                                                     const double* __restrict__ hc, double* __restrict__ hf,
                                                     const int32_t* __restrict__ ln, int64_t nn, int be,
                                                     const uint8_t* __restrict__ ea_old,
                                                     const uint8_t* __restrict__ ea_new,
                                                     const double* __restrict__ di, const double* __restrict__ uc,
                                                     double* __restrict__ uf, const int32_t* __restrict__ lt,
                                                     int64_t nt) {
  if (int(blockIdx.x) < be) {
    int64_t k = int64_t(blockIdx.x) * BS + threadIdx.x;
    if (k >= nn) return;
    if (ln) {
      k = ln[k];
      if (k < 0) return;
    }
    inv_even(k, P, dk, hc, hf);
  } else {
    int64_t t = int64_t(int(blockIdx.x) - be) * BS + threadIdx.x;
    if (t >= nt) return;
    if (lt) {
      t = lt[t];
      if (t < 0) return;
    }
    inv_int<T>(t, P, ea_old, ea_new, di, uc, uf);
  }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_inv_odd_pair(DevPair P, const int32_t* __restrict__ e_v_c,
                                                     const uint8_t* __restrict__ ea_old,
                                                     const uint8_t* __restrict__ ea_new,
                                                     const double* __restrict__ dk,
                                                     const double* __restrict__ dp,
                                                     const double* __restrict__ uc, double* __restrict__ hf,
                                                     double* __restrict__ uf,
    const int32_t* __restrict__ lst, int64_t cnt) {
  LISTED(e, cnt, lst)
  double s = dk[e];
#pragma unroll
  for (int c = 0; c < 4; ++c) s += P.st[4 * e + c] * hf[P.even[P.cells[4 * e + c]]];
  hf[P.mid[e]] = s;
  int32_t h1 = P.h1[e], h2 = P.h2[e];
  bool keep = ea_old[h1] && ea_old[h2] && ea_new[h1] && ea_new[h2];
  const double half = 0.5 * (double(pair_pred<T>(P, e, e_v_c, uc)) + (keep ? dp[e] : 0.0));
  uf[h1] = uc[e] + half;
  uf[h2] = uc[e] - half;
}

void ml_inverse_keep_batch(const KeepJob* jobs, int njobs, hipStream_t s) {
  for (int k0 = 0; k0 < njobs; k0 += MAX_LEVJOBS) {
    KeepJobs J{};
    const int nk = njobs - k0 < MAX_LEVJOBS ? njobs - k0 : MAX_LEVJOBS;
    int64_t m = 1;
    for (int k = 0; k < nk; ++k) {
      J.j[k] = jobs[k0 + k];
      if (J.j[k].Ec > m) m = J.j[k].Ec;
    }
    const unsigned grid = nb(m) < 8192u ? nb(m) : 8192u;
    k_inv_keep_b<<<dim3(grid, nk), BS, 0, s>>>(J);
    HIPCHK(hipGetLastError());
  }
}

void ml_inverse_pair(const DevPair& P, const DevTables& tc, const uint8_t* ea_old, const uint8_t* ea_new,
                     const double* dp, const double* di, const double* dk, const double* hc, const double* uc,
                     double* hf, double* uf, bool fp32, hipStream_t s, Span ln, Span le, Span lt) {
  const int64_t nn = span_n(ln, P.Nc), ne = span_n(le, P.Ec), nt = span_n(lt, P.Tc);
  const int be = int(nb(nn)), bt = int(nb(nt));
  if (fp32) {
    if (be + bt > 0)
      k_inv_even_int<float><<<unsigned(be + bt), BS, 0, s>>>(P, dk, hc, hf, ln.idx, nn, be, ea_old, ea_new, di, uc,
                                                             uf, lt.idx, nt);
    if (ne) k_inv_odd_pair<float><<<nb(ne), BS, 0, s>>>(P, tc.e_v, ea_old, ea_new, dk, dp, uc, hf, uf, le.idx, ne);
  } else {
    if (be + bt > 0)
      k_inv_even_int<double><<<unsigned(be + bt), BS, 0, s>>>(P, dk, hc, hf, ln.idx, nn, be, ea_old, ea_new, di, uc,
                                                              uf, lt.idx, nt);
    if (ne)
      k_inv_odd_pair<double><<<nb(ne), BS, 0, s>>>(P, tc.e_v, ea_old, ea_new, dk, dp, uc, hf, uf, le.idx, ne);
  }
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ masked maxima
// Several masked maxima in one launch: blockIdx.y picks the job, gridDim.x blocks share its range.
// Each thread takes 8 consecutive points per pass (one 8-byte mask load, four 16-byte value loads,
// all independent of the mask so they are in flight together); the maximum is exact, so the
// result does not depend on the split.
__global__ __launch_bounds__(BS) void k_masked_max_b(MaxJobs J, double* __restrict__ part) {
  __shared__ double sh[BS];
  const MaxJob jb = J.j[blockIdx.y];
  const int64_t n8 = jb.n >> 3, stride = int64_t(gridDim.x) * BS;
  double m = 0.0;
  for (int64_t i = TID; i < n8; i += stride) {
    const uint2 a = reinterpret_cast<const uint2*>(jb.act)[i];
    const double2* v2 = reinterpret_cast<const double2*>(jb.v) + 4 * i;
    const double2 v0 = v2[0], v1 = v2[1], v2_ = v2[2], v3 = v2[3];
    const double w[8] = {v0.x, v0.y, v1.x, v1.y, v2_.x, v2_.y, v3.x, v3.y};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t byte = ((k < 4 ? a.x : a.y) >> (8 * (k & 3))) & 0xffu;
      if (byte) m = fmax(m, fabs(w[k]));
    }
  }
  for (int64_t i = (n8 << 3) + TID; i < jb.n; i += stride)
    if (jb.act[i]) m = fmax(m, fabs(jb.v[i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int st = BS / 2; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(BS) void k_max_final_b(int nblk, const double* __restrict__ part,
                                                    double* __restrict__ out) {
  __shared__ double sh[BS];
  double m = 0.0;
  for (int i = threadIdx.x; i < nblk; i += BS) m = fmax(m, part[int64_t(blockIdx.x) * nblk + i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int st = BS / 2; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__global__ void k_thresholds(const double* __restrict__ maxima, int nl, double eps, double* __restrict__ thr) {
  if (threadIdx.x != 0) return;
  double bh = 0.0, bu = 0.0;
  for (int q = 0; q < nl; ++q) {
    bh = fmax(bh, maxima[q]);
    bu = fmax(bu, maxima[nl + q]);
  }
  thr[0] = eps * bh;
  thr[1] = eps * bu;
}

void ml_thresholds(const double* maxima, int nl, double eps, double* thr, hipStream_t s) {
  k_thresholds<<<1, 64, 0, s>>>(maxima, nl, eps, thr);
  HIPCHK(hipGetLastError());
}

void ml_masked_max_batch(const MaxJobs& jobs, int njobs, double* scratch, double* out, hipStream_t s) {
  if (njobs <= 0) return;
  if (njobs > MAX_JOBS) throw std::runtime_error("ml_masked_max_batch: too many jobs");
  for (int k = 0; k < njobs; ++k)
    if ((reinterpret_cast<uintptr_t>(jobs.j[k].v) & 15) || (reinterpret_cast<uintptr_t>(jobs.j[k].act) & 7))
      throw std::runtime_error("ml_masked_max_batch: values must be 16-byte and masks 8-byte aligned");
  k_masked_max_b<<<dim3(MAX_BLOCKS, njobs), BS, 0, s>>>(jobs, scratch);
  k_max_final_b<<<njobs, BS, 0, s>>>(MAX_BLOCKS, scratch, out);
  HIPCHK(hipGetLastError());
}

// Byte fills and copies of up to MAX_JOBS buffers in one launch (blockIdx.y = job); 16-byte
// vector stores over the aligned body, bytes over the tail.
__global__ __launch_bounds__(BS) void k_bytes_b(ByteJobs J) {
  const ByteJob jb = J.j[blockIdx.y];
  const int64_t n16 = jb.n >> 4, stride = int64_t(gridDim.x) * BS;
  const uint32_t w = 0x01010101u * uint32_t(jb.val & 0xff);
  for (int64_t i = TID; i < n16; i += stride) {
    const uint4 v = jb.src ? reinterpret_cast<const uint4*>(jb.src)[i] : make_uint4(w, w, w, w);
    reinterpret_cast<uint4*>(jb.dst)[i] = v;
  }
  for (int64_t i = (n16 << 4) + TID; i < jb.n; i += stride) jb.dst[i] = jb.src ? jb.src[i] : uint8_t(jb.val);
}

void ml_bytes_batch(const ByteJob* jobs, int njobs, hipStream_t s) {
  for (int k0 = 0; k0 < njobs; k0 += MAX_JOBS) {
    ByteJobs J{};
    const int nk = njobs - k0 < MAX_JOBS ? njobs - k0 : MAX_JOBS;
    for (int k = 0; k < nk; ++k) {
      const ByteJob& jb = jobs[k0 + k];
      if ((reinterpret_cast<uintptr_t>(jb.dst) | reinterpret_cast<uintptr_t>(jb.src)) & 15)
        throw std::runtime_error("ml_bytes_batch: buffers must be 16-byte aligned");
      J.j[k] = jb;
    }
    k_bytes_b<<<dim3(256, nk), BS, 0, s>>>(J);
    HIPCHK(hipGetLastError());
  }
}

// ------------------------------------------------------------------ active counts
__global__ __launch_bounds__(BS) void k_count_part(int64_t n, const uint8_t* __restrict__ act,
                                                   double* __restrict__ part) {
  __shared__ double sh[BS];
  double c = 0.0;
  for (int64_t i = TID; i < n; i += int64_t(gridDim.x) * BS) c += act[i] ? 1.0 : 0.0;
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int st = BS / 2; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(BS) void k_sum_final(int n, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[BS];
  double c = 0.0;
  for (int i = threadIdx.x; i < n; i += BS) c += part[i];
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int st = BS / 2; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

void ml_count(int64_t n, const uint8_t* act, double* scratch, double* out, hipStream_t s) {
  const int nblk = 512;
  k_count_part<<<nblk, BS, 0, s>>>(n, act, scratch);
  k_sum_final<<<1, BS, 0, s>>>(nblk, scratch, out);
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ upload
template <typename X>
static const X* up(const std::vector<X>& v) {
  X* p = nullptr;
  HIPCHK(wt::dmalloc(&p, v.size() * sizeof(X)));
  HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice));
  return p;
}

// rows of w entries per element (element-major on the host) as columns (entry-major)
template <typename X>
static std::vector<X> columns(const std::vector<X>& v, int w) {
  const size_t n = v.size() / size_t(w);
  if (n * size_t(w) != v.size()) throw std::runtime_error("upload_pair: table is not a whole number of rows");
  std::vector<X> o(v.size());
  for (size_t x = 0; x < n; ++x)
    for (int q = 0; q < w; ++q) o[size_t(q) * n + x] = v[x * size_t(w) + size_t(q)];
  return o;
}

void upload_pair(const PairTables& P, DevPair& d) {
  d.Nc = P.Nc; d.Ec = P.Ec; d.Tc = P.Tc; d.Nf = P.Nf; d.Ef = P.Ef;
  if (int64_t(P.cells.size()) != 4 * P.Ec || int64_t(P.mk.size()) != MK_MAX * P.Nc ||
      int64_t(P.v_sten.size()) != 9 * P.Tc || int64_t(P.w_int.size()) != 27 * P.Tc ||
      int64_t(P.w_pl.size()) != 9 * P.Ec || int64_t(P.rf_cw.size()) != RF_NC * P.Ec)
    throw std::runtime_error("upload_pair: table sizes do not match the level pair");
  d.even = up(P.even); d.mid = up(P.mid); d.h1 = up(P.h1); d.h2 = up(P.h2); d.int_e = up(P.int_e);
  d.cells = up(P.cells); d.st = up(P.st); d.s_upd = up(columns(P.s_upd, 4));
  d.mk = up(columns(P.mk, MK_MAX)); d.v_sten = up(P.v_sten);
  d.rf_f = up(P.rf_f); d.rf_fw = up(P.rf_fw); d.rf_c = up(P.rf_c); d.rf_cw = up(P.rf_cw);
  d.w_int = up(P.w_int); d.w_pl = up(P.w_pl); d.w_pr = up(P.w_pr);
  auto f32 = [](const std::vector<double>& v) { return up(std::vector<float>(v.begin(), v.end())); };
  d.w_int_f = f32(P.w_int); d.w_pl_f = f32(P.w_pl); d.w_pr_f = f32(P.w_pr);
  const std::vector<double> wc = columns(P.w_int, 27);
  d.w_int_c = up(wc); d.w_int_cf = f32(wc); d.v_sten_c = up(columns(P.v_sten, 9));
}

void free_pair(DevPair& d) {
  const void* ps[] = {d.even, d.mid, d.h1, d.h2, d.cells, d.mk, d.int_e, d.v_sten, d.rf_f, d.rf_c,
                      d.st, d.s_upd, d.w_int, d.w_pl, d.w_pr, d.rf_fw, d.rf_cw, d.w_int_f, d.w_pl_f, d.w_pr_f, d.w_int_c, d.w_int_cf, d.v_sten_c};
  for (const void* p : ps)
    if (p) (void)wt::dfree(const_cast<void*>(p));
  d = DevPair{};
}

}  // namespace wt
