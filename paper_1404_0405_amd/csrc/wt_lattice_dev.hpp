// Device side of the lattice stage: kernel arguments and launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wt_internal.hpp"
#include "wt_lattice.hpp"

namespace wt {

struct LatArgs {
  const double* tab = nullptr;   // LQ_COUNT x W2 reference geometry
  const int32_t* tiles = nullptr;
  int ntile = 0, n = 0;
  int64_t W = 0, W2 = 0;
  double g = 0, H = 0;
  double frot[30] = {};
};

struct DevLattice {
  bool ok = false;
  LatArgs args;
  const int32_t *rim = nullptr, *sup_elems = nullptr, *sup_tris = nullptr;
  const int32_t* rim_edges = nullptr;   // the three edges of every rim element (not the poles)
  int64_t n_rim = 0, n_sup_elems = 0, n_sup_tris = 0, n_rim_edges = 0, n_reg_elems = 0, table_bytes = 0;
};

// Finest level of an adaptive grid: the tendencies are zero at inactive points (masks na, ea),
// and the kernel also stores what the restriction chain to the coarser level reads: the mass
// flux F (double), qF^perp Q and the Bernoulli function B (compute type) of every tile element,
// and (not in the intermediates-only form) the divergence of F at every tile node.
struct LatML {
  const uint8_t* na = nullptr;
  const uint8_t* ea = nullptr;
  const uint8_t* tflag = nullptr;   // per (tile, lozenge): 1 if it holds support points (null: all)
  double* F = nullptr;
  void* Q = nullptr;
  void* B = nullptr;
  double* c = nullptr;   // div F of every tile node (the fine divergence the restriction reads)
};

// flag[10 t + L] = 1 when tile t of lozenge L holds a point of the support (sn, se); *count the
// number of flagged pairs.
void lattice_tile_flags(const DevLattice& lat, const uint8_t* sn, const uint8_t* se, uint8_t* flag, int32_t* count,
                        hipStream_t s);
void upload_lattice(const LatticeHost& h, DevLattice& d);
void free_lattice(DevLattice& d);
// ml null: the uniform stage; otherwise the masked form above.  inter (masked form only): the
// intermediates F, Q, B alone, no tendency and no stage output (pdh.o*, pu.o* unused).
void launch_lattice(const LatArgs& a, bool fp32, const StagePtrs& pdh, const StagePtrs& pu,
                    const StageOut& c, hipStream_t s, const LatML* ml = nullptr, bool inter = false);

}  // namespace wt
