// Device tables of a level pair and launchers of the multilevel kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "wt_internal.hpp"
#include "wt_pair.hpp"

namespace wt {

// Optional work list of a launch: indices idx[0..n) (device), or every index when idx is null.
struct Span {
  const int32_t* idx = nullptr;
  int64_t n = 0;
};

// Inter-scale tables of a level pair on the device.  Most fixed-width rows keep one row per
// element (cells, st, w_pl, w_pr: per coarse edge; w_int, v_sten: per coarse triangle; rf_*):
// their kernels run over sparse support lists or gather the rows of other elements (an edge
// reads the stencils of its two triangles), and a lane then finds its whole row in one or two
// cache lines.  Column layouts (entry q of element x at q * count + x, so that the lanes of a
// wavefront, which take consecutive elements, read consecutive words of one column) serve the
// rest: mk (MK_MAX odd-node codes per coarse node) and s_upd (4 per coarse edge, reached through
// the codes ec = 4 e + c of mk), and column copies of w_int and v_sten for the passes over the
// dense triangle lists of the details and the inverse transform.  Each choice was measured;
// columns everywhere made the sparse-list kernels slower.
struct DevPair {
  int64_t Nc, Ec, Tc, Nf, Ef;
  const int32_t *even, *mid, *h1, *h2, *cells, *mk, *int_e, *v_sten, *rf_f, *rf_c;
  const double *st, *s_upd, *w_int, *w_pl, *w_pr, *rf_fw, *rf_cw;
  const float *w_int_f, *w_pl_f, *w_pr_f;   // single-precision copies of the velocity predictions
  // column copies of w_int (and its single-precision copy) and v_sten
  const double* w_int_c;
  const float* w_int_cf;
  const int32_t* v_sten_c;
  // column-layout positions
  __host__ __device__ int64_t ct(int q, int64_t t) const { return q * Tc + t; }   // per coarse triangle
  __host__ __device__ int64_t cn(int q, int64_t k) const { return q * Nc + k; }   // per coarse node
  __host__ __device__ int64_t upd(int32_t ec) const { return (ec & 3) * Ec + (ec >> 2); }   // s_upd of code ec
};

constexpr int MAX_LEVJOBS = 16;   // level or pair jobs per batched launch

void upload_pair(const PairTables& P, DevPair& d);
void free_pair(DevPair& d);

// Stage kernels take optional work lists (coarse nodes / edges / triangles of the pair; the
// level's triangles, elements, edges; fine nodes): only listed entities are processed.
// fp32: the predictions in single precision (stored in double)
void ml_prolong(const DevPair& P, const DevTables& tc, const uint8_t* naf, const uint8_t* eaf,
                const double* hc, const double* uc, double* hf, double* uf, bool fp32, hipStream_t s,
                Span ln = {}, Span le = {}, Span lt = {});
void ml_level_intermediates(const DevTables& t, DevWork& w, const PhysParams& p, bool fp32,
                            const double* xdh, const double* xu, hipStream_t s, Span ltri = {}, Span lel = {},
                            Span led = {});
void ml_restrict(const DevPair& P, const DevTables& tc, const DevTables& tf, DevWork& wc, DevWork& wf,
                 const uint8_t* naf, const uint8_t* eaf, const PhysParams& p, bool fp32, hipStream_t s,
                 Span lfn = {}, Span lce = {}, Span lcn = {});
void ml_tend(const DevTables& t, DevWork& w, const uint8_t* na, const uint8_t* ea, const PhysParams& p, bool fp32,
             const StagePtrs& sdh, const StagePtrs& su, const StageOut& c, hipStream_t s, Span lel = {});
void ml_restrict_state(const DevPair& P, const double* hf, const double* uf, double* hc, double* uc,
                       hipStream_t s);
// det (Ec doubles) and act (Ec bytes): scratch of the two passes (details and stencil activity
// of every coarse edge's odd node)
void ml_partial_h(const DevPair& P, const DevTables& tc, const uint8_t* nac, const uint8_t* naf,
                  const uint8_t* eaf, const double* hf, double* hc, double* det, uint8_t* act, hipStream_t s,
                  Span lcn = {});
// Details of a pair (edge and interior jobs), R1 significance of a pair, R2 of a level and R3 of
// a pair as jobs of ml_mask_ops, which runs any number of them, MAX_MASK_JOBS per launch
// (blockIdx.y = job): jobs of one call must not depend on each other (the mask rules only set
// bytes, so several may write one mask).
enum MaskOp : int32_t {
  MO_DET_EDGE = 0, MO_DET_INT, MO_SIG_EDGE, MO_SIG_INT, MO_R2_NODE, MO_R2_EDGE, MO_R3_NODE, MO_R3_EDGE
};
struct MaskJob {
  int32_t op, nc;      // nc: coarse lozenge side of the R3 gate
  int32_t sparse;      // set by ml_mask_ops: scan a large rule job 16 points per lane
  int32_t fp32;        // details: predictions in single precision
  int64_t cnt;         // entries: lst[0..cnt) (-1 padding skipped) or 0..cnt
  const int32_t* lst;
  DevPair P;
  const int32_t *c_e, *e_c, *e_v, *t_e;
  const double* c_div;
  const double *hf, *uf, *uc;
  double *dh, *dp, *di;
  const uint8_t *a_n, *a_e, *allow;
  uint8_t *o_n, *o_e;
  double eh, eu;
  const double* thr;   // R1: thresholds (eh, eu) on the device instead of eh, eu (null: use eh, eu)
};
constexpr int MAX_MASK_JOBS = 10;   // per launch (kernel argument size)
struct MaskJobs {
  MaskJob j[MAX_MASK_JOBS];
  int32_t pre[MAX_MASK_JOBS + 1];   // workgroup ranges of the jobs
  int32_t n;
};
void ml_mask_ops(const MaskJob* jobs, int njobs, hipStream_t s);
void ml_details_jobs(std::vector<MaskJob>& out, const DevPair& P, const DevTables& tc, const double* hf,
                     const double* uf, const double* uc, double* dh, double* dp, double* di, bool fp32,
                     Span le = {}, Span lt = {});
void ml_significant_jobs(std::vector<MaskJob>& out, const DevPair& P, const uint8_t* naf, const uint8_t* eaf,
                         const double* dh, const double* dp, const double* di, double eh, double eu, uint8_t* sn,
                         uint8_t* se, Span le = {}, Span lt = {});
void ml_r2_jobs(std::vector<MaskJob>& out, const DevTables& t, const uint8_t* sn, const uint8_t* se, uint8_t* nn,
                uint8_t* ne);
void ml_r3_jobs(std::vector<MaskJob>& out, const DevPair& P, const DevTables& tf, const uint8_t* snc,
                const uint8_t* sec, uint8_t* nnf, uint8_t* nef, const uint8_t* allow = nullptr, int nc = 0);
// (bn, be) = (an, ae) grown by one ring of same-level neighbours (the R2 relation, gather form)
// over a whole level of lozenge side n < 8 (larger levels: ml_ring_batch over patch lists).
void ml_ring(const DevTables& t, int n, const uint8_t* an, const uint8_t* ae, uint8_t* bn, uint8_t* be,
             hipStream_t s);
// allow (optional): learned gate per quadrant of the 8 x 8 patches of the coarse level (lattice size nc)
void ml_r4(const DevTables& t, uint8_t* nn, uint8_t* ne, hipStream_t s);
void ml_r5(const DevPair& P, const DevTables& tc, const uint8_t* nnf, const uint8_t* nef, uint8_t* nnc,
           uint8_t* nec, hipStream_t s);
// Inverse transform of the pairs, top-down: first the kept details of every pair (one batched
// launch; they depend only on the details and the old and new masks), then per pair the even
// nodes and interior edges (one launch), then the odd nodes and half-edges (they read the even
// nodes).
struct KeepJob {
  const int32_t* mid;
  int64_t Ec;
  const uint8_t *na_old, *na_new;
  const double* dh;
  double* dk;
};
struct KeepJobs {
  KeepJob j[MAX_LEVJOBS];
};
void ml_inverse_keep_batch(const KeepJob* jobs, int njobs, hipStream_t s);
void ml_inverse_pair(const DevPair& P, const DevTables& tc, const uint8_t* ea_old, const uint8_t* ea_new,
                     const double* dp, const double* di, const double* dk, const double* hc, const double* uc,
                     double* hf, double* uf, bool fp32, hipStream_t s, Span ln = {}, Span le = {}, Span lt = {});
// Several levels' support rings or patch lists in one launch (blockIdx.y = level job).
struct RingJob {
  int32_t N, sh, nblk;
  const int32_t *plist, *pcount, *c_e, *e_c, *e_v, *t_e;
  const uint8_t *an, *ae;
  uint8_t *bn, *be;
};
struct RingJobs {
  RingJob j[MAX_LEVJOBS];
};
// one ring of (an, ae) into (bn, be) over the listed patches of a level with lozenge side n >= 8
// (plist from ml_patch_list_batch of the set the ring chain starts from, at most 7 rings ago; the
// caller clears (bn, be) once before the chain)
RingJob ring_job(const DevTables& t, int n, const uint8_t* an, const uint8_t* ae, uint8_t* bn, uint8_t* be,
                 const int32_t* plist);
void ml_ring_batch(const RingJob* jobs, int njobs, hipStream_t s);
struct PatchJob {
  int32_t sh;   // lozenge side 2^sh >= 8
  const uint8_t *an, *ae;
  uint8_t* pf;
  int32_t *plist, *pcount;
};
struct PatchJobs {
  PatchJob j[MAX_LEVJOBS];
};
// 8 x 8 node patches within one patch of an active point of (an, ae) or on a lozenge border, per
// level: plist[0..count) with count = *pcount = plist[np], np = 10 (n/8)^2 (plist holds np + 1
// ints, pf np bytes of scratch)
void ml_patch_list_batch(const PatchJob* jobs, int njobs, hipStream_t s);
// max |v[i]| over act[i] != 0 for up to MAX_JOBS arrays at once; scratch holds
// MAX_JOBS * MAX_BLOCKS doubles, out[k] receives job k's maximum (0 when nothing is active)
constexpr int MAX_JOBS = 32, MAX_BLOCKS = 512;
struct MaxJob {
  const double* v;
  const uint8_t* act;
  int64_t n;
};
struct MaxJobs {
  MaxJob j[MAX_JOBS];
};
void ml_masked_max_batch(const MaxJobs& jobs, int njobs, double* scratch, double* out, hipStream_t s);
// thr[0] = eps * max(maxima[0..nl)), thr[1] = eps * max(maxima[nl..2 nl)) (maxima combined in index
// order from 0, as the host would), on the device
void ml_thresholds(const double* maxima, int nl, double eps, double* thr, hipStream_t s);
// dst[0..n) = src[0..n) (src non-null) or the byte val, for any number of 16-byte aligned
// buffers, MAX_JOBS per launch
struct ByteJob {
  uint8_t* dst;
  const uint8_t* src;
  int64_t n;
  int val;
};
struct ByteJobs {
  ByteJob j[MAX_JOBS];
};
void ml_bytes_batch(const ByteJob* jobs, int njobs, hipStream_t s);
void ml_count(int64_t n, const uint8_t* act, double* scratch, double* out, hipStream_t s);

}  // namespace wt
