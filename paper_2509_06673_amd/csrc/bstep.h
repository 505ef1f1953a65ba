// Device tables of the batched time step (feti_batch_step): every kernel of the solve
// set-up, the recovery and the refinement residual runs once for all problems of a
// batch, with the problem index in the last grid dimension, instead of once per
// problem.
#pragma once

#include "kernels.h"

namespace feti {

// Vectors of one problem, addressed by role so that one launch can name the same
// vector of every problem.
enum BVec {
  BV_U = 0, BV_F, BV_D, BV_YTMP, BV_LAM, BV_DLAM, BV_R, BV_W, BV_Z, BV_Y, BV_P, BV_Q, BV_YB, BV_ZB,
  BV_G, BV_GD, BV_GQ, BV_AC, BV_TL, BV_RF, BV_CJ, BV_DU, BV_LAMP, BV_LAMP2, BV_DLAMP, BV_DLAMS,
  BV_LALT, BV_RALT, BV_WALT, BV_COUNT
};
constexpr int BV_NONE = -1;

// Lengths of the vectors a launch works on.
enum BLen { BL_LAMBDA = 0, BL_TORN = 1 };

// Matrices of the local GEMVs.
enum BMat { BM_KINV = 0, BM_SPLUS = 1, BM_SBB = 2 };

// One problem of a batch (device array, rewritten only when a context's buffers move).
struct BProb {
  DevMesh m;
  MatParams mpP, mpE;
  const void* kinv = nullptr;   // K_s^+ (dense blocks at m.kofs, leading dims m.ld)
  const void* splus = nullptr;  // (K_s^+)_bb (m.sofs, m.ldb)
  const void* sbb = nullptr;    // preconditioner blocks
  int f32 = 0;                  // the three are float
  SymArgs sym;                  // packed lower tiles of K_s^+
  const double* H = nullptr;    // G (G^T G)^{-1}, n_c x N_lambda (n_c > 0)
  const double* Cinv = nullptr;
  int nc = 0;
  const double* mdiag = nullptr;
  double* v[BV_COUNT] = {};
  double* sc = nullptr;
  int32_t* ist = nullptr;
  double* part = nullptr;       // RED_NBLK x NPART partial sums of the reductions
};

// Per-step data of one problem (device array, one host-to-device copy per step).
struct BStepVals {
  LoadDev L;
  double a_prev = 0.0, b_prev2 = 0.0;  // start lam = a lam_prev + b lam_prev2
  int cand = 0;                        // 1: the first correction compares the previous step's total
};

// Block counts of the batched launches: the largest need over the problems.
struct BDims {
  int P = 0;
  int nl_blk = 0;      // (N_lambda + 255) / 256
  int nl64_blk = 0;    // (N_lambda + 63) / 64
  int ns_blk = 0;      // (sum n_s + 255) / 256
  int nb_blk = 0;      // (sum n_b + 255) / 256
  int red_blk = 0;     // blocks of a reduction over the multipliers
  int jump_blk = 0;    // (N_lambda + 255) / 256 + n_float
  int nflt = 0;        // floating subdomains
  int nc_blk = 0;      // (n_c + 3) / 4
  int elem_blk = 0;    // (n_elem + 127) / 128
  int erow_blk = 0;    // (n_elem edof + 255) / 256
  int max_ns = 0;      // LDS of the GEMVs
  // work items (problem, subdomain, 64-row tile) of the GEMVs with the full local blocks
  // and with the interface blocks, 3 int32 each (device)
  const int32_t* full_items = nullptr;
  const int32_t* iface_items = nullptr;
  int n_full_items = 0, n_iface_items = 0;
  // packed tiles: (problem, stored tile) of every tile and of the tiles the recovery
  // product reads, 2 int32 each; (problem, subdomain, block of 256 rows) of the row sums
  const int32_t* sym_items = nullptr;
  const int32_t* sym_kb_items = nullptr;
  const int32_t* sum_items = nullptr;
  int n_sym_items = 0, n_sym_kb_items = 0, n_sum_items = 0;
};

struct BGemv {
  int mat = BM_KINV;
  int full = 1;           // n = n_s (torn vectors) or n_b (interface space)
  int xbase = BV_NONE;
  int v = BV_NONE;        // multipliers gathered into the interface part
  int gmode = 0;
  double gcoef = -1.0;
  int y = BV_NONE;
  int alpha_c = BV_NONE;
  int kb_only = 0;
  int ybase = BV_NONE;
};

// launchers (kernels_iface.hip, kernels_fem.hip, kernels_sym.hip)
void launchb_axpby(const BProb* P, const BDims& d, int len, double a, int x, double b, int y, int z, hipStream_t st);
void launchb_start(const BProb* P, const BStepVals* V, const BDims& d, hipStream_t st);
void launchb_sgemv(const BProb* P, const BDims& d, const BGemv& g, int f32, hipStream_t st);
void launchb_jump(const BProb* P, const BDims& d, int yb, int from_torn, int out, int scaled, int g, hipStream_t st);
void launchb_coarse_g(const BProb* P, const BDims& d, int v, int base, double gsign, int g, hipStream_t st);
void launchb_coarse_apply(const BProb* P, const BDims& d, int g, int a, double scale, hipStream_t st);
void launchb_coarse_correct(const BProb* P, const BDims& d, int a, double scale, int vin, int v, hipStream_t st);
void launchb_h_project(const BProb* P, const BDims& d, int a, int b, int g1, int g2, int out, int r_out, int out2,
                       hipStream_t st);
void launchb_reduce(const BProb* P, const BDims& d, int x, int y, int nrm, int phase, hipStream_t st);
void launchb_init_scalars(const BProb* P, const BDims& d, double tol, double utol, int maxit, hipStream_t st);
void launchb_copy_scalar(const BProb* P, const BDims& d, int src, int dst, hipStream_t st);
void launchb_pick_start(const BProb* P, const BStepVals* V, const BDims& d, int alt, int lam, int alt2, int dst2,
                        int alt3, int dst3, hipStream_t st);
void launchb_sub_gather(const BProb* P, const BDims& d, int lam, int r, hipStream_t st);
void launchb_rhs(const BProb* P, const BStepVals* V, const BDims& d, hipStream_t st);
// y = K^+ x from the packed tiles (kb = 0, x a torn vector), or the recovery product
// y = ybase + K^+ [0; gcoef B^T v] (+ R alpha_c) (kb = 1)
void launchb_sym_gemv(const BProb* P, const BDims& d, int kb, int x, int v, double gcoef, int ybase, int alpha_c,
                      int y, int f32, hipStream_t st);
void launchb_elem_matvec(const BProb* P, const BDims& d, int x, int y, hipStream_t st);

}  // namespace feti
