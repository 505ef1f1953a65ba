// Persistent projected PCG (kernels_pcg.hip): one cooperative launch runs the
// iterations of an interface solve, with grid-wide barriers between the phases
// of an iteration instead of kernel boundaries.
#pragma once

#include "kernels.h"

namespace feti {

// Grid barrier state (device memory, zero-initialised).  gen counts completed
// barriers; abort is raised by a block whose wait exceeds the spin limit, and
// every block then leaves the launch at its next barrier.
#ifndef FETI_BAR_GROUP
#define FETI_BAR_GROUP 192
#endif
constexpr int PCG_BAR_GROUP = FETI_BAR_GROUP;  // blocks per first-level arrival counter
constexpr int PCG_BAR_STRIDE = 64;   // uint32 words between counters (own 256-byte line)
constexpr int PCG_BAR_MAXGRP = 64;
struct GridBarrier {
  uint32_t count;
  uint32_t gen;
  int32_t abort;
  int32_t pad[PCG_BAR_STRIDE - 3];
  uint32_t grp[PCG_BAR_MAXGRP * PCG_BAR_STRIDE];  // first-level counters
};

constexpr int PCG_BLOCK = 512;   // threads per block of the persistent launch (two GEMV tiles at once)
constexpr int PCG_NPART = 24;    // partial sums per block
constexpr int PCG_NC_LOCAL = 192;  // coarse sizes applied redundantly in every block
constexpr int PCG_MAX_GRID = 256;  // largest grid of the single-problem launch (stopping-test staging)

struct PcgArgs {
  DevMesh m;
  const void* fm = nullptr;  // interface blocks (K_s^+)_bb (offsets m.sofs, leading dims m.ldb)
  int fm32 = 0;              // 1: float
  const void* mm = nullptr;  // preconditioner blocks (S_bb or K_bb), same layout
  int mm32 = 0;
  const double* Cinv = nullptr;  // (G^T G)^{-1}, n_c x n_c
  const double* H = nullptr;     // optional G (G^T G)^{-1}, n_c x N_lambda (coarse-index major)
  int nc = 0;
  double *lam = nullptr, *r = nullptr, *w = nullptr, *z = nullptr, *y = nullptr, *p = nullptr,
         *q = nullptr, *qraw = nullptr, *yb = nullptr, *zb = nullptr, *g = nullptr;
  const double* mdiag = nullptr;
  double* part = nullptr;  // 2 x grid x PCG_NPART (two alternating buffers)
  double* sc = nullptr;
  int32_t* ist = nullptr;
  GridBarrier* bar = nullptr;
  const int32_t* tile_sub = nullptr;   // GEMV row tiles (64 rows) over the interface blocks
  const int32_t* tile_row0 = nullptr;
  int ntile = 0;
  long long* tstamp = nullptr;  // optional: block 0 records the wall clock after each barrier
  int tstamp_iters = 0;         // iterations recorded (7 stamps each, 10 slots apart)
};

// One problem of a batch (device array): its mesh tables, operators and vectors.
struct ProbArgs {
  DevMesh m;
  const void* fm = nullptr;  // interface blocks (K_s^+)_bb
  const void* mm = nullptr;  // preconditioner blocks
  const double* Cinv = nullptr;
  int nc = 0;
  int nrow_items = 0;        // chunks of PCG_BLOCK multiplier rows
  double *lam = nullptr, *r = nullptr, *w = nullptr, *z = nullptr, *y = nullptr, *p = nullptr,
         *q = nullptr, *qraw = nullptr, *yb = nullptr, *zb = nullptr, *g = nullptr;
  const double* mdiag = nullptr;
  double* part = nullptr;    // nrow_items x PCG_NPART partial sums
  double* sc = nullptr;
  int32_t* ist = nullptr;
};

// The interface iterations of many independent problems in one cooperative launch.
// Work lists span all problems; each problem keeps its own scalars (published by the
// block with blockIdx = problem mod grid between barriers).
struct BatchArgs {
  const ProbArgs* probs = nullptr;
  int P = 0;
  int f32 = 0;  // every problem stores its blocks in float (1) or double (0)
  const int32_t *tile_prob = nullptr, *tile_sub = nullptr, *tile_row0 = nullptr;
  int ntile = 0;
  const int32_t *row_prob = nullptr, *row_chunk = nullptr;  // chunks of PCG_BLOCK rows
  int nrow = 0;
  const int32_t *flt_prob = nullptr, *flt_f = nullptr;      // floating subdomains
  int nflt = 0;
  double *alpha = nullptr, *beta = nullptr, *rho = nullptr;  // per problem
  int32_t* done = nullptr;    // per problem
  int32_t* iters = nullptr;   // per problem: iterations of this launch
  int32_t* status = nullptr;  // per problem: status at the end of this launch
  int32_t* ndone = nullptr;   // problems finished
  int32_t* cnt = nullptr;     // per problem: chunk counters of the reductions of phases C, D and G
  GridBarrier* bar = nullptr;
  int max_nb = 0;
  long long* tstamp = nullptr;  // optional: block 0 records the wall clock after each barrier
  int tstamp_iters = 0;         // iterations recorded (8 stamps each, 12 slots apart)
};
size_t pcg_batch_shmem(int max_nb);
int pcg_batch_max_grid(int max_nb);
hipError_t launch_pcg_batch(const BatchArgs& a, int grid, hipStream_t st);
// register, LDS and occupancy figures of the batch kernel (diagnostics)
void pcg_batch_describe(int max_nb, char* buf, size_t n);

// dynamic LDS bytes of the launch
size_t pcg_shmem(const DevMesh& m);
// largest co-resident grid of the persistent kernel on the current device (0: none)
int pcg_max_grid(const DevMesh& m);
hipError_t launch_pcg_persistent(const PcgArgs& a, int grid, hipStream_t st);
// H = G (G^T G)^{-1} from Cinv
void launch_build_h(const DevMesh& m, const double* Cinv, int nc, double* H, hipStream_t st);

}  // namespace feti
