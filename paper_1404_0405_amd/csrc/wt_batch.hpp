// Batched Runge-Kutta step of an ensemble of adaptive grids: every member's whole multilevel step
// as one persistent cooperative launch over a global work queue.
//
// The step is a fixed sequence of phases (prolongation pair by pair top-down, the TRiSK
// intermediates of all levels, the restriction chain bottom-up, the tendencies, per stage; then the
// partial height transform).  A phase holds the (member, level or pair) jobs that can run at the
// same time; its work is cut into chunks of consecutive list entries of one job, handed out by an
// atomic counter (a work queue) or dealt round-robin, and the whole grid meets at a barrier
// between phases.  Each entry is evaluated by the
// same per-point code as the one-launch-per-kernel path, so results are identical.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "wt_ml.hpp"

namespace wt {

enum BatchKind : int32_t {
  BK_PRO_EVEN = 0, BK_PRO_ODD, BK_PRO_INT, BK_VERTEX, BK_EDGE_CELL, BK_Q, BK_DIV, BK_RES_E, BK_RES_B, BK_TEND,
  BK_PARTIAL_H
};

// one level of one member
struct BatchLevel {
  DevTables t;
  const uint8_t *na, *ea;
  void *qv, *B, *F, *qe, *Q;
  double *c, *dh;   // fine divergence, prognostic height
  double g, H;
  int32_t fp32;
  StagePtrs pdh[4], pu[4];   // per Runge-Kutta stage
  StageOut so[4];
};

// one level pair of one member: coarse / fine entries of the level table
struct BatchPair {
  DevPair P;
  int32_t c, f;
};

// a job: kind, the level (a) or pair (a) it works on, the stage, the member's tendency precision
// and its entries lst[0..cnt) (-1 = padding) or 0..cnt
struct BatchJob {
  int32_t kind, a, stage, fp32;
  const int32_t* lst;
  int64_t cnt;
};

struct BatchChunk {
  int32_t job;
  int32_t start;   // first entry of the chunk
};

struct BatchPhase {
  int32_t c0, c1;   // chunk range
};

// Host-built description of one ensemble step, uploaded once and launched every step until the
// members' launch arguments change.
struct BatchPlan {
  std::vector<BatchLevel> levels;
  std::vector<BatchPair> pairs;
  std::vector<BatchJob> jobs;
  std::vector<std::vector<int32_t>> phase_jobs;   // jobs of each phase
  // device copies and the chunk tables for one chunk size
  BatchLevel* d_levels = nullptr;
  BatchPair* d_pairs = nullptr;
  BatchJob* d_jobs = nullptr;
  BatchChunk* d_chunks = nullptr;
  BatchPhase* d_phases = nullptr;
  int32_t* d_ctr = nullptr;   // work-queue counters, barrier slots and error flag of the phases
  size_t cap[6] = {0, 0, 0, 0, 0, 0};   // allocated sizes of the six device buffers
  int chunk = 0;              // entries per chunk the tables were cut for
  int nphase = 0;
  int64_t nchunk = 0;

  void upload(int chunk_entries, hipStream_t s);   // (re)builds the chunk tables for a chunk size
  void release();
};

// Largest cooperative grid (workgroups per CU x CUs) the device holds for the batch kernel.
int batch_max_blocks_per_cu();
int batch_cu_count();
// One step: clears the counters and launches blocks_per_cu x CUs workgroups cooperatively;
// queue: chunks from the per-phase work queue, else a fixed round-robin deal of the chunks.
void batch_launch(BatchPlan& plan, int blocks_per_cu, bool queue, hipStream_t s);
// After a step: synchronises and throws if a grid barrier's bounded wait ran out.
void batch_check(const BatchPlan& plan, hipStream_t s);

}  // namespace wt
