// Batched Runge-Kutta step of an ensemble of adaptive grids: every member's whole multilevel step
// as one persistent cooperative launch over a global work queue.
//
// The step is a fixed sequence of phases (prolongation pair by pair top-down, the TRiSK
// intermediates of all levels, the restriction chain bottom-up, the tendencies, per stage; then the
// partial height transform).  A phase holds the (member, level or pair) jobs that can run at the
// same time; its work is cut into chunks of consecutive list entries of one job (the list lengths
// read on the device at the phase's start), handed out by an atomic counter (a work queue) or
// dealt round-robin, and the whole grid meets at a barrier between phases.  Each entry is evaluated by the
// same per-point code as the one-launch-per-kernel path, so results are identical.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "wt_ml.hpp"

namespace wt {

enum BatchKind : int32_t {
  BK_PRO_EVEN = 0, BK_PRO_ODD, BK_PRO_INT, BK_VERTEX, BK_EDGE_CELL, BK_Q, BK_DIV, BK_RES_E, BK_RES_B, BK_TEND,
  BK_PARTIAL_H, BK_PARTIAL_D
};

// one level of one member
struct BatchLevel {
  DevTables t;
  const uint8_t *na, *ea;
  void *qv, *B, *F, *qe, *Q;
  double *c, *dh;   // fine divergence, prognostic height
  double* G;        // total mass flux read by the divergence and the restriction (F if inviscid)
  PhysParams ph;
  int32_t fp32;
  StagePtrs pdh[4], pu[4];   // per Runge-Kutta stage
  StageOut so[4];
};

// one level pair of one member: coarse / fine entries of the level table
struct BatchPair {
  DevPair P;
  int32_t c, f;
  double* det;    // partial transform scratch: details and stencil activity of every coarse edge
  uint8_t* act;
};

// a job: kind, the level (a) or pair (a) it works on, the stage, the member's tendency precision
// and its entries: lst[0..*dn) of a work list (its count as the compaction left it on the
// device; cnt holds the list's padded bound when the plan was built), or 0..cnt of a whole level
// (lst and dn null)
struct BatchJob {
  int32_t kind, a, stage, fp32;
  const int32_t* lst;
  const int64_t* dn;
  int64_t cnt;
};

// the jobs of a phase: JB[j0..j1); j0 = j1 < 0 marks a launch the single-grid caller makes itself
// between phases (the masked lattice stage of a dense finest level, stage -1 - j0)
struct BatchPhase {
  int32_t j0, j1;
};

constexpr int BATCH_MAX_JOBS = 1024;   // jobs per phase (the kernel's chunk prefix lives in LDS)

// Host-built description of one ensemble step, uploaded once and launched every step until a
// member's levels, list or mask addresses, list use or time step change (the list lengths are
// read on the device, so new lists of the same predicates need no new plan).
struct BatchPlan {
  std::vector<BatchLevel> levels;
  std::vector<BatchPair> pairs;
  std::vector<BatchJob> jobs;     // phase by phase
  std::vector<BatchPhase> phases;
  BatchLevel* d_levels = nullptr;
  BatchPair* d_pairs = nullptr;
  BatchJob* d_jobs = nullptr;
  BatchPhase* d_phases = nullptr;
  int32_t* d_ctr = nullptr;   // work-queue counters, barrier slots and error flag of the phases
  size_t cap[5] = {0, 0, 0, 0, 0};   // allocated sizes of the five device buffers
  int nphase = 0;
  int32_t* d_pre = nullptr;   // chunk prefixes of the phases for ordinary launches (phase_prepare_dev)
  size_t cap_pre = 0;

  void upload(hipStream_t s);
  void release();
};

// One phase of a plan as an ordinary launch (a single grid's step, phase after phase in stream
// order): every job's entry count is its host-side cnt (a work list's padded bound: padding
// entries are skipped), one workgroup per 256 entries.  phase_prepare computes the per-phase
// chunk prefixes after the plan is built.
constexpr int PHASE_MAX_JOBS = 32;
struct PhaseArgs {
  int32_t j0, nj, total;
  int32_t pre[PHASE_MAX_JOBS + 1];
};
void phase_prepare(const BatchPlan& plan, std::vector<PhaseArgs>& out);
void phase_launch(const BatchPlan& plan, const PhaseArgs& a, hipStream_t s);
// The same for phases with any number of jobs (an ensemble's): the prefixes live on the device
// (uploaded here, synchronising s), the workgroup finds its job by binary search.
struct PhaseDev {
  int32_t j0, nj, total, off;   // off: start of the phase's prefix in plan.d_pre
};
void phase_prepare_dev(BatchPlan& plan, std::vector<PhaseDev>& out, hipStream_t s);
void phase_launch_dev(const BatchPlan& plan, const PhaseDev& a, hipStream_t s);

// Largest cooperative grid (workgroups per CU x CUs) the device holds for the batch kernel.
int batch_max_blocks_per_cu();
int batch_cu_count();
// One step: clears the counters and launches blocks_per_cu x CUs workgroups cooperatively;
// chunks of `chunk` entries (a multiple of 256) from the per-phase work queue (queue) or dealt
// round-robin.
void batch_launch(BatchPlan& plan, int blocks_per_cu, int chunk, bool queue, hipStream_t s);
// After a step: synchronises and throws if a grid barrier's bounded wait ran out.
void batch_check(const BatchPlan& plan, hipStream_t s);

}  // namespace wt
