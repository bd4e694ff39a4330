// Work lists of the adaptive stage (index lists built by ballot / prefix-scan compaction).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "wt_ml.hpp"

namespace wt {

// idx[0..n) the listed indices in increasing order, idx[n..bound) = -1: launches cover `bound`
// entries (0 for an empty list, else a power of two with room to grow, kept while the count stays
// within it), so a launch sequence recorded for one list stays valid while later lists of the
// same predicate fit.
struct WorkList {
  int32_t* idx = nullptr;   // device
  int64_t n = 0, cap = 0, bound = 0;
  int64_t* dn = nullptr;    // device copy of n, written by the compaction (batched compaction only)
};

struct CompactScratch {
  int32_t* cnt = nullptr;
  int64_t* off = nullptr;
  int64_t cap = 0;
};

// L = { i < n : pred[i] != 0 } in increasing order.  With total_dev null the call synchronises
// and sets L.n; otherwise the count is written to total_dev (device) and L.n is left to the
// caller, who reads a batch of counts with one synchronisation.
void compact(const uint8_t* pred, int64_t n, WorkList& L, CompactScratch& sc, hipStream_t s,
             int64_t* total_dev = nullptr);
void free_list(WorkList& L);

// Many compactions in three launches and one read-back of the counts: add() the jobs, run().
struct CompactBatch {
  struct Job {
    const uint8_t* pred;
    int64_t n;
    WorkList* list;
  };
  std::vector<Job> jobs;
  void* d_jobs = nullptr;
  void* h_jobs = nullptr;
  int32_t* d_cnt = nullptr;
  int64_t *d_off = nullptr, *d_tot = nullptr, *h_tot = nullptr;
  int job_cap = 0;
  int64_t chunk_cap = 0;
  std::vector<unsigned char> uploaded;   // the job table on the device (skip the upload if equal)

  void add(const uint8_t* pred, int64_t n, WorkList& L);   // sizes L for n indices
  void run(hipStream_t s);   // compacts every job, sets the counts and bounds, pads with -1
  void release();
};
void free_scratch(CompactScratch& sc);

// Predicates of the work lists, for several levels and pairs in one launch: triangles with an edge
// in the edge support `se`; elements with a point in (sn, se); coarse nodes, edges, triangles of a
// pair with a fine point in the fine support (snf, sef).
enum PredKind : int32_t { PRED_TRI = 0, PRED_ELEM = 1, PRED_PAIR = 2 };
struct PredJob {
  int32_t kind, sh;   // sh: log2 of the lozenge side (triangles: the level; pairs: the coarse level)
  int64_t n, n_elem, Nc, Ec, Tc;
  const int32_t *a, *b, *c, *d, *e;
  const uint8_t *sn, *se;
  uint8_t *o1, *o2, *o3;
};
constexpr int MAX_PRED_JOBS = 24;   // per launch (kernel argument size)
struct PredJobs {
  PredJob j[MAX_PRED_JOBS];
};
PredJob pred_tri_job(int64_t T, int sh, const int32_t* t_e, const uint8_t* se, uint8_t* pt);
PredJob pred_elem_job(int64_t N, int64_t n_elem, const uint8_t* sn, const uint8_t* se, uint8_t* pe);
PredJob pred_pair_job(const DevPair& P, int shc, const uint8_t* snf, const uint8_t* sef, uint8_t* pn,
                      uint8_t* pe, uint8_t* pt);
void pred_batch(const PredJob* jobs, int njobs, hipStream_t s);

}  // namespace wt
