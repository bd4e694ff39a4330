// Batched persistent Runge-Kutta step of an ensemble (the phases and the work queue are
// described in wt_batch.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>
#include <string>

#include "wt_alloc.hpp"
#include "wt_batch.hpp"
#include "wt_body.hpp"

namespace wt {

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
      body_prolong_odd_pair<T>(i, bp.P, F.na, F.ea, C.t.e_v, C.pu[s].x, const_cast<double*>(F.pdh[s].x),
                            const_cast<double*>(F.pu[s].x));
      break;
    }
    case BK_PRO_INT: {
      const BatchPair& bp = PR[jb.a];
      const BatchLevel &C = LV[bp.c], &F = LV[bp.f];
      body_prolong_int<T>(i, bp.P, F.ea, C.pu[s].x, const_cast<double*>(F.pu[s].x));
      break;
    }
    case BK_VERTEX: {
      const BatchLevel& L = LV[jb.a];
      body_vertex<T>(i, L.t, L.pdh[s].x, L.pu[s].x, L.ph.H, static_cast<T*>(L.qv));
      break;
    }
    case BK_EDGE_CELL: {
      const BatchLevel& L = LV[jb.a];
      body_edge_cell<T>(i, L.t, L.pdh[s].x, L.pu[s].x, static_cast<const T*>(L.qv), L.ph, static_cast<T*>(L.B),
                        static_cast<double*>(L.F), L.G, static_cast<T*>(L.qe));
      break;
    }
    case BK_Q: {
      const BatchLevel& L = LV[jb.a];
      body_Q<T>(i, L.t, static_cast<const double*>(L.F), static_cast<const T*>(L.qe), static_cast<T*>(L.Q), L.ph.nu,
                L.pu[s].x);
      break;
    }
    case BK_DIV: {
      const BatchLevel& F = LV[jb.a];
      body_div(i, F.t, F.G, F.c);
      break;
    }
    case BK_RES_E: {
      const BatchPair& bp = PR[jb.a];
      const BatchLevel &C = LV[bp.c], &F = LV[bp.f];
      body_restrict_edges<T>(i, bp.P, F.ea, F.t.l_e, C.t.l_e, F.G, F.c, static_cast<const T*>(F.Q), C.G,
                             static_cast<T*>(C.Q));
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
      body_tend_ml<T>(i, L.t, L.na, L.ea, static_cast<const T*>(L.B), L.G, static_cast<const T*>(L.Q), L.pdh[s],
                      L.pu[s], L.so[s], L.ph.adv);
      break;
    }
    case BK_PARTIAL_D: {
      const BatchPair& bp = PR[jb.a];
      const BatchLevel& F = LV[bp.f];
      body_partial_d(i, bp.P, F.na, F.dh, bp.det, bp.act);
      break;
    }
    case BK_PARTIAL_H: {
      const BatchPair& bp = PR[jb.a];
      const BatchLevel &C = LV[bp.c], &F = LV[bp.f];
      body_partial_h(i, bp.P, C.t.c_e, C.na, F.na, F.ea, bp.det, bp.act, F.dh, C.dh);
      break;
    }
    default:
      break;
  }
}

// Grid barrier of phase p, a two-level tree: workgroups arrive on the counter of their group
// (blockIdx mod BAR_GROUPS), the last of a group on the phase's top counter, the last group sets
// the phase's done flag that every workgroup waits for.  Each phase has its own counters (zeroed
// before the launch), so nothing is reused.  The wait is bounded: past the limit the workgroup
// records the failure in *err and goes on (the host turns it into an error), and a workgroup
// that finds *err set does not wait at all, so the kernel always ends.
constexpr int BAR_GROUPS = 8, BAR_STRIDE = 32;   // counters one 128-byte line apart
constexpr int BAR_SLOTS = BAR_GROUPS + 2;        // group counters, top counter, done flag
constexpr uint32_t BAR_SPIN_LIMIT = 1u << 20;

__device__ __forceinline__ void batch_barrier(uint32_t* __restrict__ bar, int p, uint32_t* __restrict__ err) {
  // every wave waits for its own outstanding memory operations (all counters zero), so once the
  // workgroup barrier is passed the workgroup's stores sit in the caches, and one device-scope
  // release by the arriving thread (a write-back of its cache) covers them all
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    // release of this workgroup's writes; the counters themselves are relaxed, with acquire
    // fences where a thread learns that others have arrived and a release before it passes that on
    __threadfence();
    const uint32_t nwg = gridDim.x, g = blockIdx.x % BAR_GROUPS;
    const uint32_t gsize = nwg / BAR_GROUPS + (g < nwg % BAR_GROUPS ? 1u : 0u);
    const uint32_t ngroups = nwg < uint32_t(BAR_GROUPS) ? nwg : uint32_t(BAR_GROUPS);
    uint32_t* base = bar + size_t(p) * BAR_SLOTS * BAR_STRIDE;
    uint32_t* done = base + (BAR_GROUPS + 1) * BAR_STRIDE;
    if (__hip_atomic_fetch_add(base + g * BAR_STRIDE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gsize - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");   // the group's writes, passed on
      if (__hip_atomic_fetch_add(base + BAR_GROUPS * BAR_STRIDE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
          ngroups - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    // poll without cache maintenance; one acquire fence once the flag is seen
    uint32_t spins = 0;
    while (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
      if (++spins > BAR_SPIN_LIMIT) {
        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the caches this workgroup reads drop stale lines
  }
  __syncthreads();
}

// Block-wide chunk prefix of a phase's jobs: s_pre[j] = chunks of jobs 0..j-1 (s_pre[nj] = the
// phase's total), from each job's entry count (a work list's device count, or a whole level).
__device__ __forceinline__ int32_t phase_prefix(const BatchJob* __restrict__ JB, const BatchPhase& ph, int chunk,
                                                int32_t* s_pre, int32_t* s_tmp) {
  const int nj = ph.j1 - ph.j0, tid = threadIdx.x;
  int32_t v[BATCH_MAX_JOBS / BB], tsum = 0;
#pragma unroll
  for (int q = 0; q < BATCH_MAX_JOBS / BB; ++q) {
    const int j = (BATCH_MAX_JOBS / BB) * tid + q;
    v[q] = 0;
    if (j < nj) {
      const BatchJob& jb = JB[ph.j0 + j];
      const int64_t cnt = jb.dn ? *jb.dn : jb.cnt;
      v[q] = int32_t((cnt + chunk - 1) / chunk);
    }
    tsum += v[q];
  }
  s_tmp[tid] = tsum;
  __syncthreads();
  for (int off = 1; off < BB; off <<= 1) {   // inclusive scan of the per-thread sums
    const int32_t add = tid >= off ? s_tmp[tid - off] : 0;
    __syncthreads();
    s_tmp[tid] += add;
    __syncthreads();
  }
  int32_t run = s_tmp[tid] - tsum;
#pragma unroll
  for (int q = 0; q < BATCH_MAX_JOBS / BB; ++q) {
    const int j = (BATCH_MAX_JOBS / BB) * tid + q;
    if (j < nj) {
      run += v[q];
      s_pre[j + 1] = run;
    }
  }
  if (tid == 0) s_pre[0] = 0;
  __syncthreads();
  return s_pre[nj];
}

// Every workgroup takes chunks of the current phase until none is left -- from the phase's counter
// (queue != 0) or every gridDim-th chunk from its own index -- then waits at the phase's grid
// barrier.  The loop exits are uniform per workgroup, so every workgroup reaches every barrier.
__global__ __launch_bounds__(BB, 4) void k_batch(const BatchLevel* __restrict__ LV, const BatchPair* __restrict__ PR,
                                              const BatchJob* __restrict__ JB, const BatchPhase* __restrict__ PH,
                                              int nphase, int chunk, int queue, int32_t* __restrict__ ctr,
                                              uint32_t* __restrict__ bar, uint32_t* __restrict__ err) {
  __shared__ int32_t s_pre[BATCH_MAX_JOBS + 1], s_tmp[BB];
  __shared__ int32_t s_c;
  for (int p = 0; p < nphase; ++p) {
    const BatchPhase ph = PH[p];
    const int nj = ph.j1 - ph.j0;
    const int32_t total = phase_prefix(JB, ph, chunk, s_pre, s_tmp);
    for (int32_t k = 0;; ++k) {
      int32_t c;
      if (queue) {
        if (threadIdx.x == 0) s_c = atomicAdd(&ctr[p], 1);
        __syncthreads();
        c = __builtin_amdgcn_readfirstlane(s_c);
        __syncthreads();   // the next grab rewrites s_c
      } else {
        c = int32_t(blockIdx.x) + k * int32_t(gridDim.x);
      }
      if (c >= total) break;
      // the job of chunk c: the last j with s_pre[j] <= c (jobs without chunks are passed over)
      int lo = 0, hi = nj - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= c) lo = mid;
        else hi = mid - 1;
      }
      lo = __builtin_amdgcn_readfirstlane(lo);
      const BatchJob jb = JB[ph.j0 + lo];
      const int64_t cnt = jb.dn ? *jb.dn : jb.cnt;
      const int64_t start = int64_t(c - s_pre[lo]) * chunk;
      const int64_t end = std::min<int64_t>(start + chunk, cnt);
      for (int64_t r = start + threadIdx.x; r < end; r += BB) {
        int64_t i = r;
        if (jb.lst) {
          i = jb.lst[r];
          if (i < 0) continue;   // padding of a work list
        }
        if (jb.fp32) batch_entry<float>(jb, i, LV, PR);
        else batch_entry<double>(jb, i, LV, PR);
      }
    }
    batch_barrier(bar, p, err);
  }
}

// One phase as an ordinary launch: workgroup c runs entries [256 (c - pre[j]), +256) of the job j
// with pre[j] <= c < pre[j+1] (jobs without entries have no workgroup).
__global__ __launch_bounds__(BB) void k_phase(const BatchLevel* __restrict__ LV, const BatchPair* __restrict__ PR,
                                              const BatchJob* __restrict__ JB, PhaseArgs a) {
  const int32_t c = int32_t(blockIdx.x);
  int j = 0;
  while (j + 1 < a.nj && a.pre[j + 1] <= c) ++j;
  const BatchJob jb = JB[a.j0 + j];
  const int64_t r = int64_t(c - a.pre[j]) * BB + threadIdx.x;
  if (r >= jb.cnt) return;
  int64_t i = r;
  if (jb.lst) {
    i = jb.lst[r];
    if (i < 0) return;   // padding of a work list
  }
  if (jb.fp32) batch_entry<float>(jb, i, LV, PR);
  else batch_entry<double>(jb, i, LV, PR);
}

void phase_prepare(const BatchPlan& plan, std::vector<PhaseArgs>& out) {
  out.clear();
  for (const BatchPhase& ph : plan.phases) {
    PhaseArgs a{};
    if (ph.j0 < 0) {
      // a marker for a launch the caller makes itself (no jobs)
      a.j0 = ph.j0;
      out.push_back(a);
      continue;
    }
    a.j0 = ph.j0;
    a.nj = ph.j1 - ph.j0;
    if (a.nj > PHASE_MAX_JOBS) throw std::runtime_error("phase step: too many jobs in one phase");
    int64_t run = 0;
    for (int j = 0; j < a.nj; ++j) {
      a.pre[j] = int32_t(run);
      run += (plan.jobs[ph.j0 + j].cnt + BB - 1) / BB;
    }
    if (run >= (int64_t(1) << 31)) throw std::runtime_error("phase step: too many workgroups");
    a.pre[a.nj] = int32_t(run);
    a.total = int32_t(run);
    if (a.total > 0) out.push_back(a);
  }
}

void phase_launch(const BatchPlan& plan, const PhaseArgs& a, hipStream_t s) {
  if (a.total <= 0) return;
  k_phase<<<unsigned(a.total), BB, 0, s>>>(plan.d_levels, plan.d_pairs, plan.d_jobs, a);
  HIPCHK(hipGetLastError());
}

// One phase as an ordinary launch with the chunk prefix on the device: workgroup c runs entries
// [256 (c - pre[j]), +256) of the job j with pre[j] <= c < pre[j+1].
__global__ __launch_bounds__(BB) void k_phase_dev(const BatchLevel* __restrict__ LV, const BatchPair* __restrict__ PR,
                                                  const BatchJob* __restrict__ JB, int32_t j0, int32_t nj,
                                                  const int32_t* __restrict__ pre) {
  const int32_t c = int32_t(blockIdx.x);
  int lo = 0, hi = nj - 1;
  while (lo < hi) {   // the last j with pre[j] <= c (jobs without entries are passed over)
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  const BatchJob jb = JB[j0 + lo];
  const int64_t r = int64_t(c - pre[lo]) * BB + threadIdx.x;
  if (r >= jb.cnt) return;
  int64_t i = r;
  if (jb.lst) {
    i = jb.lst[r];
    if (i < 0) return;   // padding of a work list
  }
  if (jb.fp32) batch_entry<float>(jb, i, LV, PR);
  else batch_entry<double>(jb, i, LV, PR);
}

void phase_prepare_dev(BatchPlan& plan, std::vector<PhaseDev>& out, hipStream_t s) {
  out.clear();
  std::vector<int32_t> pre;
  for (const BatchPhase& ph : plan.phases) {
    if (ph.j0 < 0) throw std::runtime_error("ensemble step: a plan with marker phases");
    PhaseDev a{ph.j0, ph.j1 - ph.j0, 0, int32_t(pre.size())};
    int64_t run = 0;
    for (int j = 0; j < a.nj; ++j) {
      pre.push_back(int32_t(run));
      run += (plan.jobs[ph.j0 + j].cnt + BB - 1) / BB;
    }
    if (run >= (int64_t(1) << 31)) throw std::runtime_error("phase step: too many workgroups");
    pre.push_back(int32_t(run));
    a.total = int32_t(run);
    if (a.total > 0) out.push_back(a);
  }
  HIPCHK(hipStreamSynchronize(s));   // the previous table may still be read by a queued launch
  if (!plan.d_pre || plan.cap_pre < pre.size()) {
    if (plan.d_pre) HIPCHK(wt::dfree(plan.d_pre));
    plan.cap_pre = std::max<size_t>(1, pre.size() + pre.size() / 2);
    HIPCHK(wt::dmalloc(&plan.d_pre, plan.cap_pre * sizeof(int32_t)));
  }
  HIPCHK(hipMemcpyAsync(plan.d_pre, pre.data(), pre.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));   // pre is a local vector
}

void phase_launch_dev(const BatchPlan& plan, const PhaseDev& a, hipStream_t s) {
  if (a.total <= 0) return;
  k_phase_dev<<<unsigned(a.total), BB, 0, s>>>(plan.d_levels, plan.d_pairs, plan.d_jobs, a.j0, a.nj,
                                               plan.d_pre + a.off);
  HIPCHK(hipGetLastError());
}

// device words of a plan's counters: one work-queue counter per phase, BAR_SLOTS barrier lines
// per phase, the error flag
static size_t ctr_words(size_t nphase) {
  return ((nphase + BAR_STRIDE - 1) / BAR_STRIDE) * BAR_STRIDE + nphase * BAR_SLOTS * BAR_STRIDE + BAR_STRIDE;
}
static size_t ctr_bytes(size_t nphase) { return std::max<size_t>(1, ctr_words(nphase)) * sizeof(uint32_t); }

// copies v to the device buffer d (grown when too small; cap counts elements)
template <typename X>
static void upload_vec(const std::vector<X>& v, X*& d, size_t& cap, hipStream_t s) {
  if (!d || cap < v.size()) {
    if (d) HIPCHK(wt::dfree(d));
    cap = std::max<size_t>(1, v.size() + v.size() / 2);
    HIPCHK(wt::dmalloc(&d, cap * sizeof(X)));
  }
  if (!v.empty()) HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice, s));
}

void BatchPlan::upload(hipStream_t s) {
  for (const auto& ph : phases)
    if (ph.j1 - ph.j0 > BATCH_MAX_JOBS) throw std::runtime_error("batch plan: too many jobs in one phase");
  // the previous tables may still be read by a queued launch
  HIPCHK(hipStreamSynchronize(s));
  upload_vec(levels, d_levels, cap[0], s);
  upload_vec(pairs, d_pairs, cap[1], s);
  upload_vec(jobs, d_jobs, cap[2], s);
  upload_vec(phases, d_phases, cap[3], s);
  // work-queue counters, then the barrier slots of every phase, then the error flag
  if (!d_ctr || cap[4] < ctr_bytes(phases.size())) {
    if (d_ctr) HIPCHK(wt::dfree(d_ctr));
    cap[4] = ctr_bytes(phases.size() + phases.size() / 2);
    HIPCHK(wt::dmalloc(&d_ctr, cap[4]));
  }
  HIPCHK(hipStreamSynchronize(s));   // the host vectors of the copies may change afterwards
  nphase = int(phases.size());
}

void BatchPlan::release() {
  void* ps[] = {d_levels, d_pairs, d_jobs, d_phases, d_ctr, d_pre};
  for (void* p : ps)
    if (p) (void)wt::dfree(p);
  for (auto& c : cap) c = 0;
  d_levels = nullptr;
  d_pairs = nullptr;
  d_jobs = nullptr;
  d_phases = nullptr;
  d_ctr = nullptr;
  d_pre = nullptr;
  cap_pre = 0;
  nphase = 0;
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

void batch_launch(BatchPlan& plan, int blocks_per_cu, int chunk, bool queue, hipStream_t s) {
  if (plan.nphase == 0) return;
  const int maxb = batch_max_blocks_per_cu();
  if (blocks_per_cu < 1 || blocks_per_cu > maxb)
    throw std::runtime_error("batch step: " + std::to_string(blocks_per_cu) + " workgroups per CU, at most " +
                             std::to_string(maxb) + " fit");
  if (chunk < BB || chunk % BB) throw std::runtime_error("batch step: chunk must be a multiple of 256");
  for (const BatchPhase& ph : plan.phases)
    if (ph.j0 < 0) throw std::runtime_error("batch step: a plan with marker phases");
  HIPCHK(hipMemsetAsync(plan.d_ctr, 0, ctr_bytes(size_t(plan.nphase)), s));
  const BatchLevel* lv = plan.d_levels;
  const BatchPair* pr = plan.d_pairs;
  const BatchJob* jb = plan.d_jobs;
  const BatchPhase* ph = plan.d_phases;
  int nphase = plan.nphase, use_queue = queue ? 1 : 0;
  const size_t q0 = ((size_t(nphase) + BAR_STRIDE - 1) / BAR_STRIDE) * BAR_STRIDE;
  int32_t* ctr = plan.d_ctr;
  uint32_t* bar = reinterpret_cast<uint32_t*>(plan.d_ctr) + q0;
  uint32_t* err = bar + size_t(nphase) * BAR_SLOTS * BAR_STRIDE;
  void* args[] = {&lv, &pr, &jb, &ph, &nphase, &chunk, &use_queue, &ctr, &bar, &err};
  const dim3 grid(unsigned(blocks_per_cu * batch_cu_count()));
  // cooperative: the runtime refuses a grid whose workgroups cannot all be resident at once,
  // which the barriers need
  HIPCHK(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_batch), grid, dim3(BB), args, 0, s));
}

void batch_check(const BatchPlan& plan, hipStream_t s) {
  if (plan.nphase == 0) return;
  const size_t q0 = ((size_t(plan.nphase) + BAR_STRIDE - 1) / BAR_STRIDE) * BAR_STRIDE;
  const uint32_t* err = reinterpret_cast<const uint32_t*>(plan.d_ctr) + q0 + size_t(plan.nphase) * BAR_SLOTS * BAR_STRIDE;
  uint32_t h = 0;
  HIPCHK(hipMemcpyAsync(&h, err, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h) throw std::runtime_error("batch step: a grid barrier timed out (results of this step are invalid)");
}

}  // namespace wt
