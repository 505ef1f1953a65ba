// Device-side tables and kernel launchers of the FETI library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fem_device.h"
#include "loads_device.h"

namespace feti {

// owners of a primal DOF: up to four in 2D, eight at a corner of the 3D subdomain grid
constexpr int PI_SLOTS = 8;

// Device copies of the mesh and numbering tables (see MeshHost).
struct DevMesh {
  int nsub = 0, order = 2, ncell = 0, edof = 0, nelem = 0;
  int64_t sum_ns = 0, sum_nb = 0, n_lambda = 0;
  int n_float = 0, max_ns = 0, max_nb = 0;
  // per subdomain
  int32_t* ns = nullptr;        // local size
  int32_t* nI = nullptr;        // interior size
  int32_t* nb = nullptr;        // interface size (fixed DOFs included, trailing)
  int32_t* nfix = nullptr;      // 0 or 3
  int64_t* soff = nullptr;      // torn offset
  int64_t* boff = nullptr;      // interface-space offset
  int64_t* kofs = nullptr;      // offset of the dense n_s x ld block
  int32_t* ld = nullptr;        // leading dimension of the dense block
  int64_t* sofs = nullptr;      // offset of the dense n_b x ldb interface blocks
  int32_t* ldb = nullptr;
  uint8_t* sub_poro = nullptr;
  int32_t* sub_float = nullptr; // index in the coarse space or -1
  // per local DOF (torn)
  int32_t* code = nullptr;
  uint8_t* first = nullptr;     // 1 at the first torn DOF (lowest subdomain) of each code
  double* rfull = nullptr;      // 3 per DOF
  // elements
  int32_t *el_sub = nullptr, *el_cell = nullptr, *el_type = nullptr, *el_ldof = nullptr,
          *el_code = nullptr;
  int32_t *adj_ptr = nullptr, *adj = nullptr;  // torn DOF -> element contributions
  double* ebuf = nullptr;                      // nelem x edof element contributions
  double* emat = nullptr;                      // nelem x edof x edof element matrices K_e (column-major)
  // interface space
  int32_t* bg_row = nullptr;    // 2 per b DOF
  double* bg_sign = nullptr;
  int32_t* bd_row = nullptr;    // 3 per b DOF
  double* bd_wt = nullptr;
  double* rb = nullptr;         // 3 per b DOF
  int32_t* b_sub = nullptr;     // owning subdomain of each b DOF
  int32_t* b_torn = nullptr;    // torn index of each b DOF
  // multipliers
  int32_t* jr_b = nullptr;      // 2 per row
  double* jr_sign = nullptr;
  int32_t* grp_start = nullptr;
  int32_t* grp_size = nullptr;
  double* dwt = nullptr;        // 3 per row
  int32_t* row_kind = nullptr;  // DOF kind of each row
  // coarse space
  int32_t* float_sub = nullptr;
  // decoupled scheme: the fluid nodes of the poroelastic region (P1 lattice indices), per
  // node its (element, vertex) entries e * 3 + v (CSR), pressure Dirichlet flags and the
  // torn index of its first xi_P copy
  int decoupled = 0, n_dec = 0;
  int32_t *dec_node = nullptr, *dec_ptr = nullptr, *dec_ent = nullptr, *dec_xi = nullptr;
  uint8_t* dec_pdir = nullptr;
  // dual-primal coupling: n_pi primal unknowns, per interface DOF its primal index (-1:
  // dual), per primal DOF the interface indices of its owners (PI_SLOTS slots, -1 = none), per
  // subdomain the number of primal DOFs (the trailing ones of its interface block)
  int n_pi = 0, max_npi = 0, nsub_x = 1, nsub_y = 1;
  int32_t *bpi = nullptr, *pi_own = nullptr, *npi = nullptr;
  // dual-primal coupling: the n_defl normal-flux vectors W that deflate the iteration; per
  // multiplier row two (column, weight) slots (column -1: unused), per column its rows and
  // weights (CSR).  With defl_col set, the coarse rows (G a)_j of the interface kernels are
  // (W a)_j.
  int n_defl = 0;
  int32_t *defl_col = nullptr, *defl_ptr = nullptr, *defl_rows = nullptr;
  double *defl_w = nullptr, *defl_rw = nullptr;
};

// assembly / right-hand side (kernels_fem.hip)
void launch_assemble(const DevMesh& m, double* K, MatParams mpP, MatParams mpE, hipStream_t st);
// f = torn right-hand side (overwriting f); with cache (nelem x (edof + 3) doubles), for
// loads and Dirichlet data that do not depend on time: cmode 1 also stores there the
// element contributions and the load parts of the p rows, cmode 2 rewrites only the p
// rows and gathers from the cache
void launch_rhs(const DevMesh& m, const double* eta_prev, double* f, MatParams mpP, MatParams mpE,
                const LoadDev& L, hipStream_t st, double* cache = nullptr, int cmode = 0);
void launch_init_eta(const DevMesh& m, double* u, const LoadDev& L, hipStream_t st);
// y_i = sum of the element contributions m.ebuf of torn DOF i, in element order
void launch_gather_elem(const DevMesh& m, double* y, hipStream_t st);
// d = 3 (kernels_fem3d.hip): K_e of every tetrahedron into m.emat; K_s += K_e in 48
// colours; the right-hand side of nodal (RAW) data into f
void launch_elem_store3d(const DevMesh& m, MatParams mpP, MatParams mpE, hipStream_t st);
void launch_assemble3d(const DevMesh& m, double* K, hipStream_t st);
void launch_rhs3d(const DevMesh& m, const double* eta_prev, double* f, MatParams mpP, const LoadDev& L,
                  hipStream_t st);
// load sampled at the node of every multiplier row (body force of u rows, source of eta, xi_P, p rows)
void launch_interface_load(const DevMesh& m, const LoadDev& L, double* out, hipStream_t st);
// y = K x (torn, element by element, overwriting y)
// K_e of every element into m.emat (once the materials and tau are known)
void launch_elem_store(const DevMesh& m, MatParams mpP, MatParams mpE, hipStream_t st);
// decoupled scheme (the explicit fluid step of the Remark after eq. (linalg-system)):
// per poroelastic element and vertex the contribution tau Z^n - tau A_f p of the fluid
// rows (and with me != null the lumped mass row sums); per fluid node the lumped mass;
// eta^n; the pressure from the momentum solution; the initial state; a field on the
// lattice
void launch_dec_fluid(const DevMesh& m, const MatParams& mpP, const LoadDev& L, const double* p_lat, double* ce,
                      double* me, hipStream_t st);
void launch_dec_mass(const DevMesh& m, const double* me, double* mass, hipStream_t st);
void launch_dec_update(const DevMesh& m, const LoadDev& L, double k1, double k2, const double* ce,
                       const double* mass, double* eta_lat, const double* xi_lat, hipStream_t st);
void launch_dec_pressure(const DevMesh& m, const LoadDev& L, double k1, double k2, const double* u, double* xi_lat,
                         double* p_lat, const double* eta_lat, hipStream_t st);
void launch_dec_init(const DevMesh& m, const LoadDev& L, double k1, double k2, double* eta_lat, double* p_lat,
                     double* xi_lat, hipStream_t st);
void launch_dec_field(const DevMesh& m, const double* src_lat, double* out, hipStream_t st);
void launch_elem_matvec(const DevMesh& m, const double* x, double* y, MatParams mpP, MatParams mpE,
                        hipStream_t st);

// batched Gauss-Jordan elimination (kernels_gj.hip); panels of GJ_PANEL pivots
constexpr int GJ_PANEL = 128;
struct GJPlan {
  int nmat = 0;          // matrices in the batch
  int nb = 32;           // panel width
  int nsteps = 0;        // panel steps (max over matrices)
  int max_n = 0;
  // per (step, matrix): panel start and width (0 = idle), flag bit 0 = snapshot after this step
  int32_t* pstart = nullptr;
  int32_t* pwidth = nullptr;
  int32_t* pflag = nullptr;
  // per matrix
  int64_t* aofs = nullptr;  // offset of the matrix
  int32_t* lda = nullptr;
  int32_t* n = nullptr;     // full size (rows/cols that are updated)
  int64_t* snap_ofs = nullptr;  // where the trailing block is copied at the snapshot (-1 = none)
  int32_t* snap_at = nullptr;   // first index of the snapshot block
  int32_t* snap_ld = nullptr;
  // workspace
  double* pinv = nullptr;   // nmat x nb x nb (FP64 for either element type)
  void* wrow = nullptr;     // nmat x nb x max_n of the element type
  int32_t* status = nullptr;  // per matrix: 0 ok, 1 singular pivot
};
// T = double (FP64) or float (FP32)
template <class T>
void launch_gj_step(const GJPlan& p, T* A, T* snap, int step, bool snap_now, hipStream_t st);
template <class T>
void launch_gj_finalize(const GJPlan& p, T* A, const int32_t* nswept, hipStream_t st);

// interface operators: see iface.h
enum GatherMode { G_NONE = 0, G_SIGNED = 1, G_SCALED = 2 };
struct GemvArgs {
  const void* A = nullptr;       // matrix base (double, or float when a_f32)
  int a_f32 = 0;
  const int64_t* aofs = nullptr; // per subdomain offset
  const int32_t* lda = nullptr;
  int which_n = 0;               // 0: n = ns (full local), 1: n = nb (interface block)
  const double* xbase = nullptr; // torn (full) or interface-space vector, or nullptr
  const double* v = nullptr;     // multiplier vector gathered into the interface part
  int gmode = G_NONE;
  double gcoef = -1.0;           // x_b = xbase_b + gcoef * gather(v)
  double* y = nullptr;           // output, torn (full) or interface space
  const double* alpha_c = nullptr;  // optional: y += R alpha_c (full only)
  const int32_t* skip = nullptr;    // optional: do nothing when *skip != 0
  int kb_only = 0;                  // 1: sum only over the interface columns (x_I = 0)
  const double* ybase = nullptr;    // optional: y = ybase + A x (+ R alpha_c)
  int pi_mode = 0;                  // 1: x at the primal DOFs = pi_v[primal index] (0 if null)
  const double* pi_v = nullptr;
  // interface blocks under the dual-primal coupling ([dual | primal], primal trailing): rows
  // 0 all, 1 the dual rows only, 2 the primal rows only (the others are not written);
  // columns 0 all, 1 the dual columns only (x is taken as zero at the primal DOFs)
  int rsel = 0, csel = 0;
};

// Local solves from the packed lower tiles of the symmetric K_s^+ (kernels_sym.hip).
struct SymArgs {
  int ntile = 0;
  const int32_t* t_sub = nullptr;   // per stored tile: subdomain, tile row I, tile column J <= I
  const int32_t* t_I = nullptr;
  const int32_t* t_J = nullptr;
  const int64_t* tbase = nullptr;   // per subdomain: first tile; tile (I, J) = tbase + I (I + 1) / 2 + J
  const int32_t* nt = nullptr;      // per subdomain: tile rows
  const void* P = nullptr;          // ntile x 64 x 64 column-major tiles (double, or float when f32)
  int f32 = 0;
  double* part = nullptr;           // ntile x 2 x 64 partial products
  // products with x_I = 0 (interface columns only): the stored tiles whose tile row I
  // reaches the interface block (I >= tb[s] = (n_s - n_b) / 64), and tb per subdomain
  const int32_t* kb_tiles = nullptr;
  int n_kb_tiles = 0;
  const int32_t* tb = nullptr;
  // dual-primal coupling: with pi_mode, x at the primal DOFs is pi_v[primal index] (0 if null)
  int pi_mode = 0;
  const double* pi_v = nullptr;
};
// packed tiles P from the dense row-major blocks K (offsets kofs, leading dims ld)
template <class T>
void launch_sym_pack(const SymArgs& a, const T* K, const int64_t* kofs, const int32_t* ld, const int32_t* ns, T* P,
                     hipStream_t st);
// y = K_s^+ x_s for every subdomain (torn vectors)
void launch_sym_gemv(const DevMesh& m, const SymArgs& a, const double* x, double* y, hipStream_t st);
// y = ybase + K_s^+ [0; gcoef B_s^T v] (+ R_s alpha_c on floating subdomains): the recovery
// product with the interface columns only, from the stored tiles that reach them
void launch_sym_gemv_kb(const DevMesh& m, const SymArgs& a, const double* v, double gcoef, const double* ybase,
                        const double* alpha_c, double* y, hipStream_t st);

// dual-primal coupling (kernels_dp.hip)
// out[k] = sum over the owners o of primal DOF k of t1[torn(o)] + t2[torn(o)] + cy yb[o]
// (t1, t2 torn vectors, yb interface-space; any may be null)
void launch_pi_gather(const DevMesh& m, const double* t1, const double* t2, const double* yb, double cy, double* out,
                      const int32_t* skip, hipStream_t st);
// u[torn index of every primal interface DOF] = upi[its primal index]
void launch_pi_scatter(const DevMesh& m, const double* upi, double* u, hipStream_t st);
// r at the owners of every primal DOF: the first owner receives their sum, the others zero
void launch_pi_fold(const DevMesh& m, double* r, hipStream_t st);
// S (n_pi x n_pi, row-major) -= the primal blocks of the compact interface blocks A
void launch_pi_assemble(const DevMesh& m, const double* A, double* S, hipStream_t st);
// deflation (normal-flux vectors W, n_defl columns): out = column c of W (length N_lambda);
// g = W^T v; g = (F W)^T z with FW column-major (N_lambda x n_defl); E = W^T FW symmetrised
void launch_defl_column(const DevMesh& m, int c, double* out, hipStream_t st);
void launch_defl_wt(const DevMesh& m, const double* v, double* g, const int32_t* skip, hipStream_t st);
// (part: n_defl x DEFL_CHUNKS partial sums of the chunked reduction)
constexpr int DEFL_CHUNKS = 16;
// a = E^{-1} (F W)^T z (the partials of (F W)^T z in part, n_defl x DEFL_CHUNKS)
void launch_defl_fwt_apply(const DevMesh& m, const double* FW, const double* z, const double* Einv, double* a,
                           double* part, const int32_t* skip, hipStream_t st);
void launch_defl_gram(const DevMesh& m, const double* FW, double* E, hipStream_t st);

}  // namespace feti
