// Batched persistent Runge-Kutta step of an ensemble (the phases and the work queue are
// described in wt_batch.hpp).
#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <stdexcept>
#include <string>

#include "wt_batch.hpp"
#include "wt_body.hpp"

namespace wt {

namespace cg = cooperative_groups;

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)

constexpr int BB = 256;

// entry i of a job
template <typename T>
__device__ __forceinline__ void batch_entry(const BatchJob& jb, int64_t i, const BatchLevel* __restrict__ LV,
                                            const BatchPair* __restrict__ PR) {
  const int s = jb.stage;
  switch (jb.kind) {
    case BK_PRO_EVEN: {
      const BatchPair& bp = PR[jb.a];
      const BatchLevel &C = LV[bp.c], &F = LV[bp.f];
      body_prolong_even(i, bp.P, F.na, C.pdh[s].x, const_cast<double*>(F.pdh[s].x));
      break;
    }
    case BK_PRO_ODD: {
      const BatchPair& bp = PR[jb.a];
      const BatchLevel &C = LV[bp.c], &F = LV[bp.f];
      body_prolong_odd_pair(i, bp.P, F.na, F.ea, C.t.e_v, C.pu[s].x, const_cast<double*>(F.pdh[s].x),
                            const_cast<double*>(F.pu[s].x));
      break;
    }
    case BK_PRO_INT: {
      const BatchPair& bp = PR[jb.a];
      const BatchLevel &C = LV[bp.c], &F = LV[bp.f];
      body_prolong_int(i, bp.P, F.ea, C.pu[s].x, const_cast<double*>(F.pu[s].x));
      break;
    }
    case BK_VERTEX: {
      const BatchLevel& L = LV[jb.a];
      body_vertex<T>(i, L.t, L.pdh[s].x, L.pu[s].x, L.H, static_cast<T*>(L.qv));
      break;
    }
    case BK_EDGE_CELL: {
      const BatchLevel& L = LV[jb.a];
      body_edge_cell<T>(i, L.t, L.pdh[s].x, L.pu[s].x, static_cast<const T*>(L.qv), L.g, L.H,
                        static_cast<T*>(L.B), static_cast<double*>(L.F), static_cast<T*>(L.qe));
      break;
    }
    case BK_Q: {
      const BatchLevel& L = LV[jb.a];
      body_Q<T>(i, L.t, static_cast<const double*>(L.F), static_cast<const T*>(L.qe), static_cast<T*>(L.Q));
      break;
    }
    case BK_DIV: {
      const BatchLevel& F = LV[jb.a];
      body_div(i, F.t, static_cast<const double*>(F.F), F.c);
      break;
    }
    case BK_RES_E: {
      const BatchPair& bp = PR[jb.a];
      const BatchLevel &C = LV[bp.c], &F = LV[bp.f];
      body_restrict_edges<T>(i, bp.P, F.ea, F.t.l_e, C.t.l_e, static_cast<const double*>(F.F), F.c,
                             static_cast<const T*>(F.Q), static_cast<double*>(C.F), static_cast<T*>(C.Q));
      break;
    }
    case BK_RES_B: {
      const BatchPair& bp = PR[jb.a];
      const BatchLevel &C = LV[bp.c], &F = LV[bp.f];
      body_restrict_B<T>(i, bp.P, F.na, static_cast<const T*>(F.B), static_cast<T*>(C.B));
      break;
    }
    case BK_TEND: {
      const BatchLevel& L = LV[jb.a];
      body_tend_ml<T>(i, L.t, L.na, L.ea, static_cast<const T*>(L.B), static_cast<const double*>(L.F),
                      static_cast<const T*>(L.Q), L.pdh[s], L.pu[s], L.so[s]);
      break;
    }
    case BK_PARTIAL_H: {
      const BatchPair& bp = PR[jb.a];
      const BatchLevel &C = LV[bp.c], &F = LV[bp.f];
      body_partial_h(i, bp.P, C.t.c_e, C.na, F.na, F.ea, F.dh, C.dh);
      break;
    }
    default:
      break;
  }
}

// Every workgroup takes chunks of the current phase from the phase's counter until none is left;
// the grid synchronises (with device-wide visibility of the writes) before the next phase.  The
// loop exits are uniform per workgroup, so every workgroup reaches every grid barrier.
__global__ __launch_bounds__(BB) void k_batch(const BatchLevel* __restrict__ LV, const BatchPair* __restrict__ PR,
                                              const BatchJob* __restrict__ JB, const BatchChunk* __restrict__ CH,
                                              const BatchPhase* __restrict__ PH, int nphase, int chunk,
                                              int32_t* __restrict__ ctr) {
  cg::grid_group grid = cg::this_grid();
  __shared__ int32_t s_c;
  for (int p = 0; p < nphase; ++p) {
    const BatchPhase ph = PH[p];
    for (;;) {
      if (threadIdx.x == 0) s_c = ph.c0 + atomicAdd(&ctr[p], 1);
      __syncthreads();
      const int32_t c = __builtin_amdgcn_readfirstlane(s_c);
      __syncthreads();   // the next grab rewrites s_c
      if (c >= ph.c1) break;
      const BatchChunk ck = CH[c];
      const BatchJob jb = JB[ck.job];
      const int64_t end = std::min<int64_t>(int64_t(ck.start) + chunk, jb.cnt);
      for (int64_t r = int64_t(ck.start) + threadIdx.x; r < end; r += BB) {
        int64_t i = r;
        if (jb.lst) {
          i = jb.lst[r];
          if (i < 0) continue;   // padding of a work list
        }
        if (jb.fp32) batch_entry<float>(jb, i, LV, PR);
        else batch_entry<double>(jb, i, LV, PR);
      }
    }
    __threadfence();
    grid.sync();
  }
}

template <typename X>
static X* upload_vec(const std::vector<X>& v, X* old, hipStream_t s) {
  if (old) HIPCHK(hipFree(old));
  X* d = nullptr;
  HIPCHK(hipMalloc(&d, std::max<size_t>(1, v.size()) * sizeof(X)));
  if (!v.empty()) HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice, s));
  return d;
}

void BatchPlan::upload(int chunk_entries, hipStream_t s) {
  if (chunk_entries < BB || chunk_entries % BB) throw std::runtime_error("batch plan: chunk must be a multiple of 256");
  std::vector<BatchChunk> ch;
  std::vector<BatchPhase> ph;
  for (const auto& pj : phase_jobs) {
    BatchPhase p{int32_t(ch.size()), 0};
    for (int32_t j : pj)
      for (int64_t st = 0; st < jobs[j].cnt; st += chunk_entries) ch.push_back(BatchChunk{j, int32_t(st)});
    p.c1 = int32_t(ch.size());
    ph.push_back(p);
  }
  if (ch.size() >= size_t(1) << 30) throw std::runtime_error("batch plan: too many chunks");
  // the previous tables may still be read by a queued launch
  HIPCHK(hipStreamSynchronize(s));
  d_levels = upload_vec(levels, d_levels, s);
  d_pairs = upload_vec(pairs, d_pairs, s);
  d_jobs = upload_vec(jobs, d_jobs, s);
  d_chunks = upload_vec(ch, d_chunks, s);
  d_phases = upload_vec(ph, d_phases, s);
  if (d_ctr) HIPCHK(hipFree(d_ctr));
  HIPCHK(hipMalloc(&d_ctr, std::max<size_t>(1, ph.size()) * sizeof(int32_t)));
  HIPCHK(hipStreamSynchronize(s));   // the host vectors of the copies are temporaries
  chunk = chunk_entries;
  nphase = int(ph.size());
  nchunk = int64_t(ch.size());
}

void BatchPlan::release() {
  void* ps[] = {d_levels, d_pairs, d_jobs, d_chunks, d_phases, d_ctr};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  d_levels = nullptr;
  d_pairs = nullptr;
  d_jobs = nullptr;
  d_chunks = nullptr;
  d_phases = nullptr;
  d_ctr = nullptr;
  nphase = 0;
  nchunk = 0;
  chunk = 0;
}

int batch_max_blocks_per_cu() {
  int n = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch, BB, 0));
  return n;
}

int batch_cu_count() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  int cus = 0;
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  return cus;
}

void batch_launch(BatchPlan& plan, int blocks_per_cu, hipStream_t s) {
  if (plan.nphase == 0) return;
  const int maxb = batch_max_blocks_per_cu();
  if (blocks_per_cu < 1 || blocks_per_cu > maxb)
    throw std::runtime_error("batch step: " + std::to_string(blocks_per_cu) + " workgroups per CU, at most " +
                             std::to_string(maxb) + " fit");
  HIPCHK(hipMemsetAsync(plan.d_ctr, 0, size_t(plan.nphase) * sizeof(int32_t), s));
  const BatchLevel* lv = plan.d_levels;
  const BatchPair* pr = plan.d_pairs;
  const BatchJob* jb = plan.d_jobs;
  const BatchChunk* ch = plan.d_chunks;
  const BatchPhase* ph = plan.d_phases;
  int nphase = plan.nphase, chunk = plan.chunk;
  int32_t* ctr = plan.d_ctr;
  void* args[] = {&lv, &pr, &jb, &ch, &ph, &nphase, &chunk, &ctr};
  const dim3 grid(unsigned(blocks_per_cu * batch_cu_count()));
  HIPCHK(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_batch), grid, dim3(BB), args, 0, s));
}

}  // namespace wt
