// Learned adjacent zone: launchers of the patch feature / label / gate / test kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wt_ml.hpp"

namespace wt {

constexpr int LEARN_STATS = 32;   // statistics per patch (layout in wt_learn.hip)

// rn[Nf], re[Ef]: detail size of every fine point of a pair (floor where there is none), for
// several pairs in two launches (the pairs' arrays are disjoint).  With work lists (le: coarse
// edges, lt: coarse triangles) only the listed points are read and every other point gets the
// floor: the points outside the lists are inactive with prolonged values, whose details vanish
// (up to rounding, far below the floor).
struct PointRJob {
  DevPair P;
  const double *dh, *dp, *di;
  double eh, eu;
  float *rn, *re;
  const int32_t *le, *lt;
  int64_t ne, nt;
};
constexpr int MAX_PR_JOBS = 12;   // per launch (kernel argument size)
struct PointRJobs {
  PointRJob j[MAX_PR_JOBS];
};
PointRJob point_r_job(const DevPair& P, const double* dh, const double* dp, const double* di, double eh, double eu,
                      float* rn, float* re, Span le = {}, Span lt = {});
void learn_point_r_batch(const PointRJob* jobs, int njobs, hipStream_t s);
// statistics of the npatch = 10 (n/8)^2 patches of a level with lattice size n: rn, re of the
// level (details of the pair below), rnf, ref of the level above, masks na (level), naf
// (level above), significant points sn, se of the level
void learn_patch_stats(int64_t npatch, int n, const float* rn, const float* re, const float* rnf, const float* ref,
                       const uint8_t* na, const uint8_t* naf, const uint8_t* sn, const uint8_t* se, float* stats,
                       hipStream_t s);
void learn_features(int64_t npatch, int n, float level_pos, const float* stats, float* X, hipStream_t s);
void learn_labels(int64_t npatch, const float* stats, float* Y, hipStream_t s);
void learn_gate(int64_t npatch, const float* P, double thr, const float* stats, uint8_t* allow, uint8_t* dropped,
                hipStream_t s);
// Test hook: the children rule of patch `patch` is withheld from all four quadrants (allow = 0;
// dropped where the quadrant is significant), whatever the network proposed.
void learn_force_drop(int64_t npatch, int64_t patch, const float* stats, uint8_t* allow, uint8_t* dropped,
                      hipStream_t s);
void learn_violations(int64_t npatch, const float* stats, const uint8_t* dropped, uint8_t* viol, hipStream_t s);

}  // namespace wt
