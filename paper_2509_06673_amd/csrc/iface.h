// Constants and launchers of the interface kernels (kernels_iface.hip).
#pragma once

#include "kernels.h"

namespace feti {

constexpr int RED_BLOCK = 256;   // threads of the partial-sum kernels
constexpr int RED_NBLK = 512;    // cap on the blocks of a reduction over the multipliers
constexpr int NPART = 32;        // partial sums per block
constexpr int UPD_WIN = 3;       // updates summed by the update test

// device scalar slots (double)
enum {
  SC_RHO = 0, SC_ALPHA = 1, SC_BETA = 2, SC_TOL = 3, SC_RES0 = 4, SC_RES = 5,
  SC_EREF = 6,  // reference of the dual-energy norm: max(|P d|_M, |w^(0)|_M)
  SC_REF = 8,   // 6 per-kind references max(|P d|_k, |w^(0)|_k)
  SC_EK = 16,   // 6 per-kind reference energies |P d|_{M,k}^2
  SC_ERAT = 23, // current dual-energy ratio
  SC_KRAT = 24, // 6 current per-kind ratios (diagnostics)
  SC_UTOL = 32, // tolerance of the update test (0: off)
  SC_URING = 33, // UPD_WIN x 6 per-kind update sizes |alpha| |p|_k of the last updates
  SC_SEL0 = 51,  // start selection: residual norms of the current start and of a candidate
  SC_SEL1 = 52,
  SC_ULAM = 53,  // 6 per-kind |lambda|_k at the last update test (graph path; diagnostics)
  SC_COUNT = 64
};
// device integer slots (IS_CNT0.. : counters of the last-block reductions)
enum { IS_DONE = 0, IS_ITERS = 1, IS_STATUS = 2, IS_MAXIT = 3, IS_CNT0 = 4, IS_COUNT = 12 };
// scalar phases
enum { PH_REFNORM = 0, PH_INIT = 1, PH_ALPHA = 2, PH_CONV = 3, PH_BETA = 4 };

void launch_sgemv(const DevMesh& m, const GemvArgs& a, hipStream_t st);
// scalar state of a solve (residual tolerance, update tolerance, iteration cap, everything
// else zero)
void launch_init_scalars(double* sc, int32_t* ist, double tol, double utol, int maxit, hipStream_t st);
void launch_zero(int64_t n, double* z, hipStream_t st);
// out[node] = x at the first torn DOF of every code of the given kind
void launch_field_scatter(const DevMesh& m, const double* x, int kind, double* out, hipStream_t st);
// sc[dst] = sc[src]
void launch_copy_scalar(double* sc, int src, int dst, hipStream_t st);
// lam = alt where sc[SC_SEL1] < sc[SC_SEL0] (the candidate's residual is the smaller)
// (flag, when given, receives 1 if the candidate was taken, else 0; alt2/dst2 and
// alt3/dst3, when given, are copied along with it)
void launch_pick_start(int64_t n, const double* sc, const double* alt, double* lam, int32_t* flag, hipStream_t st,
                       const double* alt2 = nullptr, double* dst2 = nullptr, const double* alt3 = nullptr,
                       double* dst3 = nullptr);
// Projection with H = G (G^T G)^{-1} (coarse-index major, nc x n, nc <= HPROJ_NC_MAX):
// v = a - b, out = v - H (g1 - g2) (b, g2 may be null); r_out (optional) = v, out2
// (optional) = out.  With g1 - g2 = G^T v this is out = P v.
constexpr int HPROJ_NC_MAX = 192;
void launch_h_project(int64_t n, int nc, const double* H, const double* a, const double* b, const double* g1,
                      const double* g2, double* out, double* r_out, double* out2, hipStream_t st);
// out = jump (or (B B^T)^{-1}-weighted jump) of yb; with g, also g = G^T out
void launch_jump(const DevMesh& m, const double* yb, int from_torn, double* out, int scaled,
                 double* g, const int32_t* skip, hipStream_t st);
void launch_coarse_g(const DevMesh& m, const double* v, const double* base, double gsign, double* g,
                     const int32_t* skip, hipStream_t st);
void launch_coarse_apply(int nc, const double* Cinv, const double* g, double* a, double scale,
                         const int32_t* skip, hipStream_t st);
void launch_coarse_correct(const DevMesh& m, const double* a, double scale, const double* vin,
                           double* v, const int32_t* skip, hipStream_t st);
void launch_gtg(const DevMesh& m, double* C, int nc, hipStream_t st);
// reductions over the multipliers finished by the last block, which runs the scalar phase;
// counter must be zero on entry (the last block resets it)
void launch_reduce(const DevMesh& m, const double* x, const double* y, const double* nrm,
                   const double* mdiag, double* part, int32_t* counter, double* sc, int32_t* ist,
                   int phase, hipStream_t st);
void launch_correct_dot(const DevMesh& m, const double* a, const double* vin, double* v,
                        const double* x, double* part, int32_t* counter, double* sc, int32_t* ist,
                        int phase, hipStream_t st);
void launch_cg_lam(const DevMesh& m, const double* p, const double* qraw, const double* q,
                   double* lam, double* r, double* w, const double* mdiag, double* part,
                   int32_t* counter, double* sc, int32_t* ist, hipStream_t st);
void launch_cg_p(int64_t n, const double* sc, const int32_t* ist, const double* y, double* p,
                 hipStream_t st);
void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z,
                  hipStream_t st);
// diagonal of the preconditioner M^{-1} = D B S B^T D from the S_bb blocks (double or float)
template <class MT>
void launch_precond_diag(const DevMesh& m, const MT* S, double* mdiag, hipStream_t st);
void launch_sub_gather(const DevMesh& m, const double* lam, double* r, hipStream_t st);
void launch_kind_maxabs(const DevMesh& m, const double* x, const double* y, double* part, int nblk,
                        hipStream_t st);
// part[b] = sum of x_i^2 over the grid-stride range of block b (nblk blocks)
void launch_sumsq(int64_t n, const double* x, double* part, int nblk, hipStream_t st);
// per subdomain: dst block (cnt x cnt) = src block at (src_at, src_at); TS, TD = double or float
template <class TS, class TD>
void launch_copy_block(int nsub, int maxn, const int64_t* src_ofs, const int32_t* src_ld,
                       const int32_t* src_at, const int64_t* dst_ofs, const int32_t* dst_ld,
                       const int32_t* cnt, const TS* src, TD* dst, hipStream_t st);
void launch_to_f32(int64_t n, const double* src, float* dst, hipStream_t st);
void launch_to_f64(int64_t n, const float* src, double* dst, hipStream_t st);

}  // namespace feti
