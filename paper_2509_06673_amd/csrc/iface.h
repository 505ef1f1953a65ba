// Constants and launchers of the interface kernels (kernels_iface.hip).
#pragma once

#include "kernels.h"

namespace feti {

constexpr int RED_BLOCK = 256;   // threads of the partial-sum kernels
constexpr int RED_NBLK = 256;    // partial-sum blocks (fixed: the reduction order is fixed)
constexpr int NPART = 16;        // partial sums per block

// device scalar slots (double)
enum {
  SC_RHO = 0, SC_ALPHA = 1, SC_BETA = 2, SC_TOL = 3, SC_RES0 = 4, SC_RES = 5,
  SC_EREF = 6,  // reference of the dual-energy norm: max(|P d|_M, |w^(0)|_M)
  SC_REF = 8,   // 6 per-kind references max(|P d|_k, |w^(0)|_k)
  SC_EK = 16,   // 6 per-kind reference energies |P d|_{M,k}^2
  SC_COUNT = 24
};
// device integer slots
enum { IS_DONE = 0, IS_ITERS = 1, IS_STATUS = 2, IS_MAXIT = 3, IS_COUNT = 4 };
// scalar phases
enum { PH_REFNORM = 0, PH_INIT = 1, PH_ALPHA = 2, PH_CONV = 3, PH_BETA = 4 };

void launch_sgemv(const DevMesh& m, const GemvArgs& a, hipStream_t st);
void launch_jump(const DevMesh& m, const double* yb, int from_torn, double* out, int scaled,
                 const int32_t* skip, hipStream_t st);
void launch_coarse_g(const DevMesh& m, const double* v, const double* base, double gsign, double* g,
                     const int32_t* skip, hipStream_t st);
void launch_coarse_apply(int nc, const double* Cinv, const double* g, double* a, double scale,
                         const int32_t* skip, hipStream_t st);
void launch_coarse_correct(const DevMesh& m, const double* a, double scale, const double* vin,
                           double* v, const int32_t* skip, hipStream_t st);
void launch_gtg(const DevMesh& m, double* C, int nc, hipStream_t st);
// per-block partial sums: [0] (x, y); [2+k] |nrm|^2 and [8+k] sum |mdiag_j| nrm_j^2 over
// the rows of kind k
void launch_partials(const DevMesh& m, const double* x, const double* y, const double* nrm,
                     const double* mdiag, double* part, int nblk, const int32_t* done,
                     hipStream_t st);
// diagonal of the preconditioner M^{-1} = D B S B^T D from the S_bb blocks
void launch_precond_diag(const DevMesh& m, const double* S, double* mdiag, hipStream_t st);
void launch_scalar(const double* part, int nblk, double* sc, int32_t* ist, int phase,
                   hipStream_t st);
void launch_cg_lam(int64_t n, const double* sc, const int32_t* ist, const double* p,
                   const double* qraw, const double* q, double* lam, double* r, double* w,
                   hipStream_t st);
void launch_cg_p(int64_t n, const double* sc, const int32_t* ist, const double* y, double* p,
                 hipStream_t st);
void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z,
                  hipStream_t st);
void launch_sub_gather(const DevMesh& m, const double* lam, double* r, hipStream_t st);
void launch_kind_maxabs(const DevMesh& m, const double* x, const double* y, double* part, int nblk,
                        hipStream_t st);
void launch_copy_block(int nsub, int maxn, const int64_t* src_ofs, const int32_t* src_ld,
                       const int32_t* src_at, const int64_t* dst_ofs, const int32_t* dst_ld,
                       const int32_t* cnt, const double* src, double* dst, hipStream_t st);

}  // namespace feti
