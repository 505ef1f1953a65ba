// C ABI of the FETI library and the host orchestration of one time step.
//
// A step (Section 2.5 backward Euler, Section 3 FETI):
//   f_s        per-subdomain right-hand side (rows 1 and 4 of eq. (linalg-system))
//   d          = sum_s B_s K_s^+ f_s,  e_s = R_s^T f_s            (eq. (feti-system))
//   lambda_0   start: previous multipliers (Algorithm 1/2 warm start), made
//              admissible (G^T lambda = e) by one coarse solve
//   PCG        projected preconditioned CG on F lambda = d with the Dirichlet
//              preconditioner of eq. (feti_dirichlet_preconditioner)
//   recovery   u_s = K_s^+ (f_s - B_s^T lambda) + R_s alpha  (proof of Theorem 3.1)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "bstep.h"
#include "feti_internal.h"
#include "iface.h"
#include "kernels.h"
#include "pcg.h"

using namespace feti;

struct feti_ctx_s {
  hipStream_t stream = nullptr;
  std::string err;
  int state = 0;  // 0 created, 1 mesh, 2 assembled, 3 factored
  int device = -1;
  MeshHost mh;
  DevMesh dm;
  std::vector<void*> allocs;
  std::vector<void*> mat_allocs;
  // materials
  feti_material matP{}, matE{};
  MatParams mpP{}, mpE{};
  double lamP = 0, muP = 0, lamE = 0, muE = 0, tau = 0;
  int precision = FETI_FP64, precond = FETI_PRECOND_DIRICHLET;
  bool keep_assembled = true;  // false: the elimination runs in place in K
  // dense blocks
  int64_t k_total = 0, s_total = 0;
  double* K = nullptr;      // assembled local matrices
  double* Kinv = nullptr;   // K_s^+
  double* Sbb = nullptr;    // S_bb snapshots
  double* Splus = nullptr;  // (K_s^+)_bb
  double* Kbb = nullptr;    // K_bb (lumped preconditioner)
  double* Cinv = nullptr;   // (G^T G)^{-1}
  double* H = nullptr;      // G (G^T G)^{-1} (small coarse spaces)
  // FP32 factors (precision FETI_FP32_IR)
  float* Kinv32 = nullptr;
  float* Sbb32 = nullptr;
  float* Splus32 = nullptr;
  // packed lower 64 x 64 tiles of K_s^+ for the local solves (beside the dense blocks)
  SymArgs sym;
  // load parts of the element right-hand sides for time-independent loads, and the load
  // and material parameters they were computed for
  double* ecache = nullptr;
  bool ecache_valid = false;
  unsigned char ekey[sizeof(LoadDev) + 2 * sizeof(MatParams)] = {};
  int nc = 0;
  // vectors
  double *f = nullptr, *u = nullptr, *ytmp = nullptr, *yb = nullptr, *zb = nullptr;
  double *rf = nullptr, *du = nullptr, *dlam = nullptr, *cj = nullptr, *kpart = nullptr;
  double *dlam_sum = nullptr, *dlam_prev = nullptr;  // corrections of this and of the previous step
  double *u_save = nullptr, *f_save = nullptr;        // time-stepping state kept across feti_solve
  bool have_dlam_prev = false;
  int pcg_mode = FETI_PCG_AUTO;
  double* mdiag = nullptr;  // diagonal of the preconditioner (weights of the dual-energy norm)
  double* h_kpart = nullptr;
  double *lam = nullptr, *lam_prev = nullptr, *lam_prev2 = nullptr, *d = nullptr, *r = nullptr,
         *w = nullptr, *z = nullptr, *y = nullptr, *p = nullptr, *q = nullptr, *qraw = nullptr,
         *tl = nullptr;
  double *g = nullptr, *ac = nullptr;
  double *lam_given = nullptr, *lam_alt = nullptr;  // start set by feti_set_start; scratch
  double *r_alt = nullptr, *w_alt = nullptr, *gd = nullptr, *gq = nullptr;  // start comparison, G^T d, G^T F lam
  double *part = nullptr, *sc = nullptr;
  int32_t* ist = nullptr;
  int32_t* h_ist = nullptr;
  // per-solve records of a time step (status, iterations, residuals, phase events), read
  // after the step's single synchronisation
  static constexpr int NREC = 8;
  int32_t* h_rec_ist = nullptr;  // NREC x IS_COUNT (pinned)
  double* h_rec_sc = nullptr;    // NREC x SC_COUNT (pinned)
  hipEvent_t rec_ev[NREC][4] = {};
  int32_t* d_pick = nullptr;     // device-side start choices: [0] first correction, [1] first solve
  int32_t* h_pick = nullptr;     // (pinned copy)
  double* h_sc = nullptr;
  int64_t nstep = 0;
  bool have_prev = false, have_prev2 = false;
  hipEvent_t ev[8] = {};
  hipEvent_t ev_gj[2] = {};  // around the elimination kernels of the last factor_subdomains
  double t_gj_ms = 0.0;
  bool own_stream = false;
  // persistent PCG: interface GEMV row tiles, grid barrier, partial sums, grid size
  int32_t* tile_sub = nullptr;
  int32_t* tile_row0 = nullptr;
  int ntile = 0;
  GridBarrier* bar = nullptr;
  double* ppart = nullptr;
  int pgrid = 0;
  // decoupled scheme: eta, p and xi_P of the fluid nodes on the P1 lattice, the lumped mass
  // per fluid node, per-element fluid contributions, and the constants of row 3
  double *dec_eta = nullptr, *dec_p = nullptr, *dec_xi = nullptr, *dec_mass = nullptr, *dec_ce = nullptr;
  double dec_k1 = 0.0, dec_k2 = 0.0;
  // dual-primal coupling: the inverse of the primal coarse matrix S_PiPi (n_pi x n_pi), the
  // primal right-hand side and solution, and the local solution of the start
  bool dp = false;
  double *Spinv = nullptr, *cpi = nullptr, *upi = nullptr, *ydp = nullptr;
  // deflation of the dual-primal iteration: F W (N_lambda x n_defl, column-major), the
  // inverse of E = W^T F W, and the coarse vectors of one projection
  double *FW = nullptr, *Edinv = nullptr, *gdef = nullptr, *adef = nullptr, *dpart = nullptr;
  bool defl = false;
  // captured PCG iteration chunks, keyed by the multiplier buffer they update
  struct Graph {
    hipGraphExec_t exec = nullptr;
    const double* lam = nullptr;
    int chunk = 0;
  } graphs[12];
  int graph_next = 0;            // round-robin replacement among the captured chunks
  int prev_iters[NREC] = {};     // iterations of the last solve in each record slot
};

namespace {

int fail(feti_ctx c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return fail(ctx, FETI_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));     \
  } while (0)

template <class T>
int dalloc(feti_ctx ctx, T** p, size_t count, std::vector<void*>& list) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) return fail(ctx, FETI_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  list.push_back(*p);
  return FETI_OK;
}

template <class T>
int upload(feti_ctx ctx, T** p, const std::vector<T>& v) {
  int rc = dalloc(ctx, p, v.size(), ctx->allocs);
  if (rc) return rc;
  if (!v.empty()) HIPCHK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  return FETI_OK;
}

#define RC(expr)              \
  do {                        \
    int _rc = (expr);         \
    if (_rc) return _rc;      \
  } while (0)

void lame(const feti_material& m, double& lam, double& mu) {
  lam = m.E * m.nu / ((1.0 + m.nu) * (1.0 - 2.0 * m.nu));
  mu = m.lame_mode == 1 ? m.E / (1.0 + m.nu) : m.E / (2.0 * (1.0 + m.nu));
}

int64_t round8(int64_t n) { return (n + 7) / 8 * 8; }

constexpr int KMAX_NBLK = 128;  // blocks of the per-kind max-abs reduction

int upload_mesh(feti_ctx ctx) {
  const MeshHost& h = ctx->mh;
  DevMesh& m = ctx->dm;
  const int nsub = (int)h.subs.size();
  m.nsub = nsub;
  m.order = h.desc.order_u;
  m.ncell = h.desc.ncell;
  m.edof = h.edof;
  m.nelem = (int)h.el_sub.size();
  m.sum_ns = h.sum_ns;
  m.sum_nb = h.sum_nb;
  m.n_lambda = h.n_lambda;
  m.n_float = h.n_float;
  m.max_ns = h.max_ns;
  m.max_nb = h.max_nb;
  std::vector<int32_t> ns(nsub), nI(nsub), nb(nsub), nfix(nsub), ld(nsub), ldb(nsub), sfl(nsub);
  std::vector<int64_t> soff(nsub), boff(nsub), kofs(nsub), sofs(nsub);
  std::vector<uint8_t> poro(nsub);
  int64_t ko = 0, so = 0;
  for (int s = 0; s < nsub; ++s) {
    const SubHost& sh = h.subs[s];
    ns[s] = sh.ns; nI[s] = sh.nI; nb[s] = sh.nb; nfix[s] = sh.nfix;
    soff[s] = sh.off; boff[s] = sh.boff;
    ld[s] = (int32_t)round8(sh.ns);
    kofs[s] = ko;
    ko += (int64_t)sh.ns * ld[s];
    ldb[s] = (int32_t)round8(sh.nb);
    sofs[s] = so;
    so += (int64_t)sh.nb * ldb[s];
    poro[s] = sh.poro ? 1 : 0;
    sfl[s] = h.sub_float[s];
  }
  ctx->k_total = ko;
  ctx->s_total = so;
  std::vector<int32_t> code(h.sum_ns), b_sub(h.sum_nb), b_torn(h.sum_nb);
  for (const SubHost& sh : h.subs) {
    for (int i = 0; i < sh.ns; ++i) code[sh.off + i] = sh.codes[i];
    for (int i = 0; i < sh.nb; ++i) {
      b_sub[sh.boff + i] = sh.sid;
      b_torn[sh.boff + i] = (int32_t)(sh.off + sh.nI + i);
    }
  }
  std::vector<int32_t> row_kind(h.n_lambda);
  // (3D: the uz rows join the ux kind of the per-kind stopping test, which tracks six kinds)
  for (int64_t j = 0; j < h.n_lambda; ++j) row_kind[j] = h.rows[j].kind == K_UZ ? K_UX : h.rows[j].kind;
  RC(upload(ctx, &m.ns, ns));
  RC(upload(ctx, &m.nI, nI));
  RC(upload(ctx, &m.nb, nb));
  RC(upload(ctx, &m.nfix, nfix));
  RC(upload(ctx, &m.soff, soff));
  RC(upload(ctx, &m.boff, boff));
  RC(upload(ctx, &m.kofs, kofs));
  RC(upload(ctx, &m.ld, ld));
  RC(upload(ctx, &m.sofs, sofs));
  RC(upload(ctx, &m.ldb, ldb));
  RC(upload(ctx, &m.sub_poro, poro));
  RC(upload(ctx, &m.sub_float, sfl));
  RC(upload(ctx, &m.code, code));
  {
    // first occurrence of every code in torn (subdomain-major) order
    std::vector<uint8_t> first(h.sum_ns, 0);
    std::vector<int32_t> sorted(code);
    std::sort(sorted.begin(), sorted.end());
    sorted.erase(std::unique(sorted.begin(), sorted.end()), sorted.end());
    std::vector<uint8_t> seen(sorted.size(), 0);
    for (int64_t i = 0; i < h.sum_ns; ++i) {
      const size_t k = std::lower_bound(sorted.begin(), sorted.end(), code[i]) - sorted.begin();
      if (!seen[k]) { seen[k] = 1; first[i] = 1; }
    }
    RC(upload(ctx, &m.first, first));
  }
  RC(upload(ctx, &m.rfull, h.rfull));
  RC(upload(ctx, &m.el_sub, h.el_sub));
  RC(upload(ctx, &m.el_cell, h.el_cell));
  RC(upload(ctx, &m.el_type, h.el_type));
  RC(upload(ctx, &m.el_ldof, h.el_ldof));
  RC(upload(ctx, &m.el_code, h.el_code));
  RC(upload(ctx, &m.adj_ptr, h.adj_ptr));
  RC(upload(ctx, &m.adj, h.adj));
  RC(dalloc(ctx, &m.ebuf, (size_t)m.nelem * m.edof, ctx->allocs));
  RC(upload(ctx, &m.bg_row, h.bg_row));
  RC(upload(ctx, &m.bg_sign, h.bg_sign));
  RC(upload(ctx, &m.bd_row, h.bd_row));
  RC(upload(ctx, &m.bd_wt, h.bd_wt));
  RC(upload(ctx, &m.rb, h.rb));
  RC(upload(ctx, &m.b_sub, b_sub));
  RC(upload(ctx, &m.b_torn, b_torn));
  std::vector<int32_t> jr_b(h.jr_b.begin(), h.jr_b.end());
  RC(upload(ctx, &m.jr_b, jr_b));
  RC(upload(ctx, &m.jr_sign, h.jr_sign));
  RC(upload(ctx, &m.grp_start, h.grp_start));
  RC(upload(ctx, &m.grp_size, h.grp_size));
  RC(upload(ctx, &m.dwt, h.dwt));
  RC(upload(ctx, &m.row_kind, row_kind));
  RC(upload(ctx, &m.float_sub, h.float_sub));
  ctx->dp = h.desc.coupling == FETI_COUPLING_PRIMAL;
  static_assert(PI_SLOTS == PI_OWNERS, "the device owner table has the host's slots");
  m.nsub_x = h.desc.nsub_x;
  m.nsub_y = h.desc.nsub_y;
  m.n_pi = h.n_pi;
  m.max_npi = 0;
  if (ctx->dp) {
    std::vector<int32_t> npi(nsub, 0);
    for (int s = 0; s < nsub; ++s)
      for (int8_t c : h.subs[s].cats) npi[s] += c == C_BP ? 1 : 0;
    for (int v : npi) m.max_npi = std::max(m.max_npi, v);
    RC(upload(ctx, &m.npi, npi));
    RC(upload(ctx, &m.bpi, h.bpi));
    RC(upload(ctx, &m.pi_own, h.pi_own));
    RC(dalloc(ctx, &ctx->cpi, std::max(m.n_pi, 1), ctx->allocs));
    RC(dalloc(ctx, &ctx->upi, std::max(m.n_pi, 1), ctx->allocs));
    RC(dalloc(ctx, &ctx->ydp, h.sum_ns, ctx->allocs));
    m.n_defl = h.n_defl;
    if (h.n_defl > 0) {
      RC(upload(ctx, &m.defl_col, h.defl_col));
      RC(upload(ctx, &m.defl_w, h.defl_w));
      RC(upload(ctx, &m.defl_ptr, h.defl_ptr));
      RC(upload(ctx, &m.defl_rows, h.defl_rows));
      RC(upload(ctx, &m.defl_rw, h.defl_rw));
      RC(dalloc(ctx, &ctx->gdef, h.n_defl, ctx->allocs));
      RC(dalloc(ctx, &ctx->adef, h.n_defl, ctx->allocs));
      RC(dalloc(ctx, &ctx->dpart, (size_t)h.n_defl * DEFL_CHUNKS, ctx->allocs));
      ctx->defl = true;
    } else {
      m.n_defl = 0;
    }
  }
  m.decoupled = h.desc.scheme == FETI_SCHEME_DECOUPLED ? 1 : 0;
  m.n_dec = (int)h.dec_node.size();
  if (m.decoupled) {
    RC(upload(ctx, &m.dec_node, h.dec_node));
    RC(upload(ctx, &m.dec_ptr, h.dec_ptr));
    RC(upload(ctx, &m.dec_ent, h.dec_ent));
    RC(upload(ctx, &m.dec_xi, h.dec_xi));
    RC(upload(ctx, &m.dec_pdir, h.dec_pdir));
    const size_t n1n = (size_t)h.n1 * h.n1;
    RC(dalloc(ctx, &ctx->dec_eta, n1n, ctx->allocs));
    RC(dalloc(ctx, &ctx->dec_p, n1n, ctx->allocs));
    RC(dalloc(ctx, &ctx->dec_xi, n1n, ctx->allocs));
    RC(dalloc(ctx, &ctx->dec_mass, std::max(m.n_dec, 1), ctx->allocs));
    RC(dalloc(ctx, &ctx->dec_ce, (size_t)m.nelem * 3, ctx->allocs));
  }
  // vectors
  const int64_t nl = h.n_lambda;
  RC(dalloc(ctx, &ctx->f, h.sum_ns, ctx->allocs));
  RC(dalloc(ctx, &ctx->u, h.sum_ns, ctx->allocs));
  RC(dalloc(ctx, &ctx->ytmp, h.sum_ns, ctx->allocs));
  RC(dalloc(ctx, &ctx->yb, h.sum_nb, ctx->allocs));
  RC(dalloc(ctx, &ctx->zb, h.sum_nb, ctx->allocs));
  RC(dalloc(ctx, &ctx->rf, h.sum_ns, ctx->allocs));
  RC(dalloc(ctx, &ctx->du, h.sum_ns, ctx->allocs));
  RC(dalloc(ctx, &ctx->u_save, h.sum_ns, ctx->allocs));
  RC(dalloc(ctx, &ctx->f_save, h.sum_ns, ctx->allocs));
  RC(dalloc(ctx, &ctx->dlam, h.n_lambda, ctx->allocs));
  RC(dalloc(ctx, &ctx->dlam_sum, h.n_lambda, ctx->allocs));
  RC(dalloc(ctx, &ctx->dlam_prev, h.n_lambda, ctx->allocs));
  RC(dalloc(ctx, &ctx->cj, h.n_lambda, ctx->allocs));
  RC(dalloc(ctx, &ctx->mdiag, h.n_lambda, ctx->allocs));
  RC(dalloc(ctx, &ctx->kpart, (size_t)KMAX_NBLK * 12, ctx->allocs));
  RC(dalloc(ctx, &ctx->d_pick, 2, ctx->allocs));
  double** lv[] = {&ctx->lam, &ctx->lam_prev, &ctx->lam_prev2, &ctx->d, &ctx->r, &ctx->w,
                   &ctx->z, &ctx->y, &ctx->p, &ctx->q, &ctx->qraw, &ctx->tl, &ctx->lam_given, &ctx->lam_alt,
                   &ctx->r_alt, &ctx->w_alt};
  for (double** pp : lv) RC(dalloc(ctx, pp, nl, ctx->allocs));
  ctx->nc = 3 * h.n_float;
  RC(dalloc(ctx, &ctx->g, std::max(ctx->nc, 1), ctx->allocs));
  RC(dalloc(ctx, &ctx->ac, std::max(ctx->nc, 1), ctx->allocs));
  RC(dalloc(ctx, &ctx->gd, std::max(ctx->nc, 1), ctx->allocs));
  RC(dalloc(ctx, &ctx->gq, std::max(ctx->nc, 1), ctx->allocs));
  RC(dalloc(ctx, &ctx->part, (size_t)RED_NBLK * NPART, ctx->allocs));
  RC(dalloc(ctx, &ctx->sc, SC_COUNT, ctx->allocs));
  RC(dalloc(ctx, &ctx->ist, IS_COUNT, ctx->allocs));
  // persistent PCG: 64-row tiles of the interface blocks, barrier, grid size
  {
    std::vector<int32_t> ts, tr;
    for (int s = 0; s < (int)h.subs.size(); ++s)
      for (int r0 = 0; r0 < h.subs[s].nb; r0 += 64) { ts.push_back(s); tr.push_back(r0); }
    ctx->ntile = (int)ts.size();
    if (ts.empty()) { ts.push_back(0); tr.push_back(0); }
    RC(upload(ctx, &ctx->tile_sub, ts));
    RC(upload(ctx, &ctx->tile_row0, tr));
    GridBarrier* bar = nullptr;
    RC(dalloc(ctx, &bar, 1, ctx->allocs));
    ctx->bar = bar;
    HIPCHK(hipMemsetAsync(ctx->bar, 0, sizeof(GridBarrier), ctx->stream));
    int grid = pcg_max_grid(m);
    (void)hipGetLastError();  // an unsupported query leaves no sticky error behind
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      grid = std::min(grid, 2 * cus);
    // one 64-row interface tile per block when the chip holds that many
    grid = std::min(grid, 192);
    grid = std::min({grid, PCG_BAR_GROUP * PCG_BAR_MAXGRP, PCG_MAX_GRID});
    if (const char* e = std::getenv("FETI_PCG_GRID"))
      grid = std::min({pcg_max_grid(m), std::max(1, std::atoi(e)), PCG_BAR_GROUP * PCG_BAR_MAXGRP, PCG_MAX_GRID});
    ctx->pgrid = std::max(0, grid);
    RC(dalloc(ctx, &ctx->ppart, (size_t)2 * std::max(1, ctx->pgrid) * PCG_NPART, ctx->allocs));
  }
  HIPCHK(hipMemsetAsync(ctx->u, 0, h.sum_ns * sizeof(double), ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->lam_prev, 0, nl * sizeof(double), ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->lam_prev2, 0, nl * sizeof(double), ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->ist, 0, IS_COUNT * sizeof(int32_t), ctx->stream));
  if (!ctx->h_ist) {
    HIPCHK(hipHostMalloc((void**)&ctx->h_ist, IS_COUNT * sizeof(int32_t), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&ctx->h_sc, SC_COUNT * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&ctx->h_kpart, KMAX_NBLK * 12 * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&ctx->h_rec_ist, feti_ctx_s::NREC * IS_COUNT * sizeof(int32_t), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&ctx->h_rec_sc, feti_ctx_s::NREC * SC_COUNT * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&ctx->h_pick, 2 * sizeof(int32_t), hipHostMallocDefault));
    for (auto& r : ctx->rec_ev)
      for (auto& e : r)
        if (!e) HIPCHK(hipEventCreate(&e));
  }
  for (auto& e : ctx->ev)
    if (!e) HIPCHK(hipEventCreate(&e));
  for (auto& e : ctx->ev_gj)
    if (!e) HIPCHK(hipEventCreate(&e));
  return FETI_OK;
}

void drop_graphs(feti_ctx ctx) {
  for (auto& g : ctx->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = feti_ctx_s::Graph();
  }
}

void free_all(feti_ctx ctx) {
  drop_graphs(ctx);
  for (void* p : ctx->allocs) (void)hipFree(p);
  for (void* p : ctx->mat_allocs) (void)hipFree(p);
  ctx->allocs.clear();
  ctx->mat_allocs.clear();
  ctx->dm = DevMesh();
  ctx->K = ctx->Kinv = ctx->Sbb = ctx->Splus = ctx->Kbb = ctx->Cinv = ctx->H = nullptr;
  ctx->Kinv32 = ctx->Sbb32 = ctx->Splus32 = nullptr;
  ctx->sym = SymArgs();
  ctx->ecache = nullptr;
  ctx->ecache_valid = false;
}

LoadDev make_load(feti_ctx ctx, const feti_load* L) {
  LoadDev d{};
  d.kind = L->kind;
  d.layout = ctx->mh.desc.layout;
  d.t = L->t;
  for (int i = 0; i < 16; ++i) d.prm[i] = L->params[i];
  d.lamP = ctx->lamP; d.muP = ctx->muP; d.lamE = ctx->lamE; d.muE = ctx->muE;
  d.alpha = ctx->matP.alpha; d.c0 = ctx->matP.c0;
  d.kf = ctx->matP.K / ctx->matP.mu_f;
  if (L->kind == FETI_LOAD_RAW) {
    d.f_p = L->f_p; d.f_e = L->f_e; d.z = L->z; d.t_side = L->t_side; d.zw_side = L->zw_side;
    d.g_u = L->g_u; d.g_p = L->g_p; d.eta0 = L->eta0;
  }
  d.dir_u = ctx->mh.desc.dirichlet_u;
  d.dir_p = ctx->mh.desc.dirichlet_p;
  return d;
}

// ---- interface operators ----------------------------------------------------

// the factors of the current precision
struct Factors {
  const void* kinv;
  const void* sbb;
  const void* splus;
  int f32;
};
Factors factors(feti_ctx ctx) {
  if (ctx->precision == FETI_FP32_IR) return {ctx->Kinv32, ctx->Sbb32, ctx->Splus32, 1};
  return {ctx->Kinv, ctx->Sbb, ctx->Splus, 0};
}

void op_project(feti_ctx ctx, const double* in, double* out, const int32_t* skip) {
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  if (ctx->nc == 0) {
    if (out != in) launch_axpby(m.n_lambda, 1.0, in, 0.0, nullptr, out, st);
    return;
  }
  launch_coarse_g(m, in, nullptr, 1.0, ctx->g, skip, st);
  launch_coarse_apply(ctx->nc, ctx->Cinv, ctx->g, ctx->ac, 1.0, skip, st);
  launch_coarse_correct(m, ctx->ac, -1.0, in, out, skip, st);
}

// y_b = (K^+)_bb B^T x per subdomain; y = B y_b; with g: also g = G^T y (same pass).
// Dual-primal coupling (the interface blocks hold N_s = [[K_rr^{-1}, -K_rr^{-1} K_rPi],
// [-K_Pir K_rr^{-1}, -S_s]] over [dual | primal]): the primal coarse solve of
// K~ [u_r; u_Pi] = [B^T x; 0] first, u_Pi = S_PiPi^{-1} sum_s L_s^T (N_s [B_s^T x; 0])_Pi,
// then y = sum_s B_s (N_s [B_s^T x; L_s u_Pi])_dual = B K~^{-1} B^T x.
void op_F_raw(feti_ctx ctx, const double* x, double* y, double* g, const int32_t* skip) {
  DevMesh& m = ctx->dm;
  GemvArgs a;
  const Factors fc = factors(ctx);
  a.A = fc.splus; a.a_f32 = fc.f32; a.aofs = m.sofs; a.lda = m.ldb; a.which_n = 1;
  a.v = x; a.gmode = G_SIGNED; a.gcoef = 1.0; a.y = ctx->yb; a.skip = skip;
  if (ctx->dp && m.n_pi > 0) {
    // primal rows of N_s [B_s^T x; 0] (dual columns only), the coarse solve, then the dual
    // rows of N_s [B_s^T x; L_s u_Pi]
    a.rsel = 2; a.csel = 1;
    launch_sgemv(m, a, ctx->stream);
    launch_pi_gather(m, nullptr, nullptr, ctx->yb, 1.0, ctx->cpi, skip, ctx->stream);
    launch_coarse_apply(m.n_pi, ctx->Spinv, ctx->cpi, ctx->upi, 1.0, skip, ctx->stream);
    a.pi_mode = 1; a.pi_v = ctx->upi; a.rsel = 1; a.csel = 0;
  }
  launch_sgemv(m, a, ctx->stream);
  launch_jump(m, ctx->yb, 0, y, 0, g, skip, ctx->stream);
}

void op_F(feti_ctx ctx, const double* x, double* y, const int32_t* skip) {
  op_F_raw(ctx, x, y, nullptr, skip);
}

// z_b = S_bb (B^T D x)_s per subdomain; y = D B z_b; with g: also g = G^T y
void op_M_raw(feti_ctx ctx, const double* x, double* y, double* g, const int32_t* skip) {
  DevMesh& m = ctx->dm;
  if (ctx->precond == FETI_PRECOND_NONE) {
    launch_axpby(m.n_lambda, 1.0, x, 0.0, nullptr, y, ctx->stream);
    if (g) launch_coarse_g(m, y, nullptr, 1.0, g, skip, ctx->stream);
    return;
  }
  GemvArgs a;
  const Factors fc = factors(ctx);
  if (ctx->precond == FETI_PRECOND_LUMPED) { a.A = ctx->Kbb; a.a_f32 = 0; }
  else { a.A = fc.sbb; a.a_f32 = fc.f32; }
  a.aofs = m.sofs; a.lda = m.ldb; a.which_n = 1;
  a.v = x; a.gmode = G_SCALED; a.gcoef = 1.0; a.y = ctx->zb; a.skip = skip;
  // dual-primal: the jump reads the dual rows, and x is zero at the primal DOFs
  if (ctx->dp) { a.rsel = 1; a.csel = 1; }
  launch_sgemv(m, a, ctx->stream);
  launch_jump(m, ctx->zb, 0, y, 1, g, skip, ctx->stream);
}

void op_M(feti_ctx ctx, const double* x, double* y, const int32_t* skip) {
  op_M_raw(ctx, x, y, nullptr, skip);
}

// Dual-primal deflation: y = z - W E^{-1} (F W)^T z (a search direction F-orthogonal to W).
void op_defl_dir(feti_ctx ctx, const double* z, double* y, const int32_t* skip) {
  DevMesh& m = ctx->dm;
  launch_defl_fwt_apply(m, ctx->FW, z, ctx->Edinv, ctx->adef, ctx->dpart, skip, ctx->stream);
  launch_coarse_correct(m, ctx->adef, -1.0, z, y, skip, ctx->stream);
}

// Dual-primal deflation of a start: v += W E^{-1} W^T (d - F v), so that W^T (d - F v) = 0.
void op_defl_start(feti_ctx ctx, double* v) {
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  op_F(ctx, v, ctx->q, nullptr);
  launch_axpby(m.n_lambda, 1.0, ctx->d, -1.0, ctx->q, ctx->r, st);
  launch_defl_wt(m, ctx->r, ctx->gdef, nullptr, st);
  launch_coarse_apply(m.n_defl, ctx->Edinv, ctx->gdef, ctx->adef, 1.0, nullptr, st);
  launch_coarse_correct(m, ctx->adef, 1.0, v, v, nullptr, st);
}

// Scratch of feti_apply_F_noalloc: the interface-space products y_b of every subdomain,
// in a file-scope device array (each GPU that loads the library holds its own copy until
// the process ends).  Host code refers to it only through the per-device address that
// hipGetSymbolAddress returns; the array's name is a host-side stand-in.
constexpr int64_t FETI_NOALLOC_SCRATCH = 1 << 20;  // doubles (8 MiB)
static __device__ __align__(256) double scratch[FETI_NOALLOC_SCRATCH];
constexpr int FETI_MAX_DEVICES = 64;
static double* g_scratch_ptr[FETI_MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// Address of this device's scratch (dev must be current), looked up once per device.
int noalloc_scratch(feti_ctx ctx, int dev, double** out) {
  if (dev < 0 || dev >= FETI_MAX_DEVICES) return fail(ctx, FETI_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ctx, FETI_EHIP, "hipGetSymbolAddress returned no address for the scratch");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return FETI_OK;
}

int32_t* counter(feti_ctx ctx, int phase) { return ctx->ist + IS_CNT0 + phase; }

// One projected PCG iteration (kernels skip once the iteration has converged):
//   q_raw = F p, q = P q_raw, alpha = rho / (p, q); lam += alpha p, r -= alpha q_raw,
//   w -= alpha q; convergence test on w; z = M^{-1} w, y = P z, beta; p = y + beta p.
void pcg_iteration(feti_ctx ctx, double* lam, const int32_t* done) {
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  const bool coarse = ctx->nc > 0;
  op_F_raw(ctx, ctx->p, ctx->qraw, coarse ? ctx->g : nullptr, done);
  if (coarse) launch_coarse_apply(ctx->nc, ctx->Cinv, ctx->g, ctx->ac, 1.0, done, st);
  launch_correct_dot(m, coarse ? ctx->ac : nullptr, ctx->qraw, ctx->q, ctx->p, ctx->part,
                     counter(ctx, PH_ALPHA), ctx->sc, ctx->ist, PH_ALPHA, st);
  launch_cg_lam(m, ctx->p, ctx->qraw, ctx->q, lam, ctx->r, ctx->w, ctx->mdiag, ctx->part,
                counter(ctx, PH_CONV), ctx->sc, ctx->ist, st);
  op_M_raw(ctx, ctx->w, ctx->z, coarse ? ctx->g : nullptr, done);
  if (coarse) launch_coarse_apply(ctx->nc, ctx->Cinv, ctx->g, ctx->ac, 1.0, done, st);
  if (ctx->defl) {
    // y = z - W E^{-1} (F W)^T z with (w, y) in the same pass
    launch_defl_fwt_apply(m, ctx->FW, ctx->z, ctx->Edinv, ctx->adef, ctx->dpart, done, st);
  }
  launch_correct_dot(m, coarse ? ctx->ac : (ctx->defl ? ctx->adef : nullptr), ctx->z, ctx->y, ctx->w, ctx->part,
                     counter(ctx, PH_BETA), ctx->sc, ctx->ist, PH_BETA, st);
  launch_cg_p(m.n_lambda, ctx->sc, ctx->ist, ctx->y, ctx->p, st);
}

// Projected PCG on F lambda = d with d = sum_s B_s K_s^+ f_s - c (c: prescribed jump
// of the primal solution, nullptr = 0).  lam holds the start guess on entry (any
// vector) and the solution on exit; u receives the recovered torn primal solution.
// iters_out accumulates the PCG iterations.
// Dual-energy norm of the projected residual w = P (d - F lam) of an admissible lam.
// With slot >= 0 the norm stays on the device in sc[slot] (no synchronisation).
int start_residual(feti_ctx ctx, const double* lam, double* norm, int slot = -1) {
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  op_F(ctx, lam, ctx->q, nullptr);
  launch_axpby(m.n_lambda, 1.0, ctx->d, -1.0, ctx->q, ctx->r, st);
  op_project(ctx, ctx->r, ctx->w, nullptr);
  launch_reduce(m, nullptr, nullptr, ctx->w, ctx->mdiag, ctx->part, counter(ctx, PH_REFNORM), ctx->sc, ctx->ist,
                PH_REFNORM, st);
  if (slot >= 0) {
    launch_copy_scalar(ctx->sc, SC_EREF, slot, st);
    return FETI_OK;
  }
  HIPCHK(hipMemcpyAsync(ctx->h_sc, ctx->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *norm = ctx->h_sc[SC_EREF];
  return FETI_OK;
}

// First half of a torn solve (no host synchronisation): d = sum_s B_s K_s^+ f_s - c,
// the admissible start, the scalar state, the reference norms of P d, and r, w, y, p
// with rho = (w, y).  With a candidate start the choice between it and lam is made on
// the device; pick_flag (device, may be null) receives 1 if the candidate was taken.
int torn_begin(feti_ctx ctx, const feti_solve_opts* o, double tol, double utol, const double* f, const double* cj,
               double* lam, const double* cand = nullptr, int32_t* pick_flag = nullptr) {
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  const int64_t nl = m.n_lambda;
  // d = sum_s B_s K_s^+ f_s - c
  if (ctx->dp) {
    // dual-primal: ytmp = N_s [f_r; 0] (kept for the recovery), the primal solution of
    // K~ u = f~ at lambda = 0, u_Pi = S_PiPi^{-1} sum_s L_s^T (f_Pi + ytmp_Pi), its local
    // part ydp = N_s [f_r; L_s u_Pi] = ytmp + N_s [0; L_s u_Pi], and d = sum_s B_s ydp
    SymArgs sa = ctx->sym;
    sa.pi_mode = 1; sa.pi_v = nullptr;
    launch_sym_gemv(m, sa, f, ctx->ytmp, st);
    launch_pi_gather(m, f, ctx->ytmp, nullptr, 0.0, ctx->cpi, nullptr, st);
    launch_coarse_apply(m.n_pi, ctx->Spinv, ctx->cpi, ctx->upi, 1.0, nullptr, st);
    sa.pi_v = ctx->upi;
    launch_sym_gemv_kb(m, sa, nullptr, 0.0, ctx->ytmp, nullptr, ctx->ydp, st);
    launch_jump(m, ctx->ydp, 1, ctx->d, 0, nullptr, nullptr, st);
    if (cj) launch_axpby(nl, 1.0, ctx->d, -1.0, cj, ctx->d, st);
  } else {
    if (ctx->sym.P) {
      launch_sym_gemv(m, ctx->sym, f, ctx->ytmp, st);
    } else {
      GemvArgs a;
      const Factors fc = factors(ctx);
      a.A = fc.kinv; a.a_f32 = fc.f32; a.aofs = m.kofs; a.lda = m.ld; a.which_n = 0;
      a.xbase = f; a.y = ctx->ytmp;
      launch_sgemv(m, a, st);
    }
    launch_jump(m, ctx->ytmp, 1, ctx->d, 0, nullptr, nullptr, st);
    if (cj) launch_axpby(nl, 1.0, ctx->d, -1.0, cj, ctx->d, st);
  }
  // admissible start: lambda += G (G^T G)^{-1} (e - G^T lambda) (dual-primal: the
  // deflated component of the residual taken exactly)
  auto admissible = [&](double* v) {
    if (ctx->defl) { op_defl_start(ctx, v); return; }
    if (ctx->nc == 0) return;
    launch_coarse_g(m, v, f, -1.0, ctx->g, nullptr, st);
    launch_coarse_apply(ctx->nc, ctx->Cinv, ctx->g, ctx->ac, 1.0, nullptr, st);
    launch_coarse_correct(m, ctx->ac, 1.0, v, v, nullptr, st);
  };
  admissible(lam);
  int32_t* flag = pick_flag ? pick_flag : ctx->d_pick;
  if (ctx->H) {
    static_assert(HPROJ_NC_MAX >= PCG_NC_LOCAL, "H exists for every coarse size the projection kernel takes");
    // with H: a projection is one pass after G^T v (P v = v - H G^T v), and a compared
    // candidate keeps its r and w.  G^T r is summed from r itself: at a warm start r is
    // tiny, and G^T d - G^T F lam would cancel down to the rounding of G^T d, leaving w
    // a part outside the range of P that no iteration removes.
    launch_coarse_g(m, ctx->d, nullptr, 1.0, ctx->gd, nullptr, st);
    auto start_rw = [&](const double* v, double* r, double* w) {
      op_F(ctx, v, ctx->q, nullptr);
      launch_axpby(nl, 1.0, ctx->d, -1.0, ctx->q, r, st);
      launch_coarse_g(m, r, nullptr, 1.0, ctx->gq, nullptr, st);
      launch_h_project(nl, ctx->nc, ctx->H, r, nullptr, ctx->gq, nullptr, w, nullptr, nullptr, st);
    };
    start_rw(lam, ctx->r, ctx->w);
    if (cand) {
      // keep the candidate start if its projected residual (dual-energy norm) is smaller
      launch_axpby(nl, 1.0, cand, 0.0, nullptr, ctx->lam_alt, st);
      admissible(ctx->lam_alt);
      start_rw(ctx->lam_alt, ctx->r_alt, ctx->w_alt);
      launch_reduce(m, nullptr, nullptr, ctx->w, ctx->mdiag, ctx->part, counter(ctx, PH_REFNORM), ctx->sc, ctx->ist,
                    PH_REFNORM, st);
      launch_copy_scalar(ctx->sc, SC_EREF, SC_SEL0, st);
      launch_reduce(m, nullptr, nullptr, ctx->w_alt, ctx->mdiag, ctx->part, counter(ctx, PH_REFNORM), ctx->sc,
                    ctx->ist, PH_REFNORM, st);
      launch_copy_scalar(ctx->sc, SC_EREF, SC_SEL1, st);
      launch_pick_start(nl, ctx->sc, ctx->lam_alt, lam, flag, st, ctx->r_alt, ctx->r, ctx->w_alt, ctx->w);
    }
    // tolerance reference: per-kind norms of P d
    launch_init_scalars(ctx->sc, ctx->ist, tol, utol, std::max(o->max_it, 0), st);
    launch_h_project(nl, ctx->nc, ctx->H, ctx->d, nullptr, ctx->gd, nullptr, ctx->tl, nullptr, nullptr, st);
    launch_reduce(m, nullptr, nullptr, ctx->tl, ctx->mdiag, ctx->part, counter(ctx, PH_REFNORM), ctx->sc,
                  ctx->ist, PH_REFNORM, st);
    // y = P M^{-1} w, p = y
    op_M_raw(ctx, ctx->w, ctx->z, ctx->gq, nullptr);
    launch_h_project(nl, ctx->nc, ctx->H, ctx->z, nullptr, ctx->gq, nullptr, ctx->y, nullptr, ctx->p, st);
    launch_reduce(m, ctx->w, ctx->y, ctx->w, ctx->mdiag, ctx->part, counter(ctx, PH_INIT), ctx->sc,
                  ctx->ist, PH_INIT, st);
    HIPCHK(hipGetLastError());
    return FETI_OK;
  }
  if (cand) {
    // keep the candidate start if its projected residual is smaller
    launch_axpby(nl, 1.0, cand, 0.0, nullptr, ctx->lam_alt, st);
    admissible(ctx->lam_alt);
    RC(start_residual(ctx, lam, nullptr, SC_SEL0));
    RC(start_residual(ctx, ctx->lam_alt, nullptr, SC_SEL1));
    launch_pick_start(nl, ctx->sc, ctx->lam_alt, lam, flag, st);
  }
  // tolerance reference: per-kind norms of P d
  launch_init_scalars(ctx->sc, ctx->ist, tol, utol, std::max(o->max_it, 0), st);
  op_project(ctx, ctx->d, ctx->tl, nullptr);
  launch_reduce(m, nullptr, nullptr, ctx->tl, ctx->mdiag, ctx->part, counter(ctx, PH_REFNORM), ctx->sc,
                ctx->ist, PH_REFNORM, st);
  // r = d - F lambda; w = P r; y = P M^{-1} w; p = y (dual-primal: y the deflated direction)
  op_F(ctx, lam, ctx->q, nullptr);
  launch_axpby(nl, 1.0, ctx->d, -1.0, ctx->q, ctx->r, st);
  op_project(ctx, ctx->r, ctx->w, nullptr);
  op_M(ctx, ctx->w, ctx->z, nullptr);
  if (ctx->defl) op_defl_dir(ctx, ctx->z, ctx->y, nullptr);
  else op_project(ctx, ctx->z, ctx->y, nullptr);
  launch_axpby(nl, 1.0, ctx->y, 0.0, nullptr, ctx->p, st);
  launch_reduce(m, ctx->w, ctx->y, ctx->w, ctx->mdiag, ctx->part, counter(ctx, PH_INIT), ctx->sc,
                ctx->ist, PH_INIT, st);
  HIPCHK(hipGetLastError());
  return FETI_OK;
}

// Second half of a torn solve: alpha_c = -(G^T G)^{-1} G^T r and the recovery
// u = K^+ (f - B^T lam) + R alpha_c, where K^+ f is still in ytmp from torn_begin.
// Dual-primal coupling: u = K~^{-1} (f~ - B^T lam), i.e. u_Pi = S_PiPi^{-1} sum_s L_s^T
// (f_Pi + ytmp_Pi - (N_s [B_s^T lam; 0])_Pi) and u_s = ytmp + N_s [-B_s^T lam; L_s u_Pi]
// with u_Pi copied to every owner of a primal DOF.
int torn_end(feti_ctx ctx, const double* lam, double* u, const double* f) {
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  if (ctx->dp) {
    GemvArgs a;
    a.A = ctx->Splus; a.aofs = m.sofs; a.lda = m.ldb; a.which_n = 1;
    a.v = lam; a.gmode = G_SIGNED; a.gcoef = 1.0; a.y = ctx->yb; a.rsel = 2; a.csel = 1;
    launch_sgemv(m, a, st);
    launch_pi_gather(m, f, ctx->ytmp, ctx->yb, -1.0, ctx->cpi, nullptr, st);
    launch_coarse_apply(m.n_pi, ctx->Spinv, ctx->cpi, ctx->upi, 1.0, nullptr, st);
    SymArgs sa = ctx->sym;
    sa.pi_mode = 1; sa.pi_v = ctx->upi;
    launch_sym_gemv_kb(m, sa, lam, -1.0, ctx->ytmp, nullptr, u, st);
    launch_pi_scatter(m, ctx->upi, u, st);
    HIPCHK(hipGetLastError());
    return FETI_OK;
  }
  if (ctx->nc > 0) {
    launch_coarse_g(m, ctx->r, nullptr, 1.0, ctx->g, nullptr, st);
    launch_coarse_apply(ctx->nc, ctx->Cinv, ctx->g, ctx->ac, -1.0, nullptr, st);
  }
  const Factors fc = factors(ctx);
  if (!fc.kinv) {
    // in-place factors: the packed tiles that the interface columns reach
    launch_sym_gemv_kb(m, ctx->sym, lam, -1.0, ctx->ytmp, ctx->nc > 0 ? ctx->ac : nullptr, u, st);
    HIPCHK(hipGetLastError());
    return FETI_OK;
  }
  GemvArgs a;
  a.A = fc.kinv; a.a_f32 = fc.f32; a.aofs = m.kofs; a.lda = m.ld; a.which_n = 0;
  a.kb_only = 1; a.ybase = ctx->ytmp;
  a.v = lam; a.gmode = G_SIGNED; a.gcoef = -1.0;
  a.y = u; a.alpha_c = ctx->nc > 0 ? ctx->ac : nullptr;
  launch_sgemv(m, a, st);
  HIPCHK(hipGetLastError());
  return FETI_OK;
}

// Enqueues one torn solve; its status, iterations, residuals and phase events go to
// record slot (read by finish_solve once the stream has been synchronised).  Returns
// only launch failures.
int solve_torn(feti_ctx ctx, const feti_solve_opts* o, double tol, double utol, const double* f, const double* cj,
               double* lam, double* u, int slot, const double* cand = nullptr, int32_t* pick_flag = nullptr) {
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  hipEvent_t* ev = ctx->rec_ev[slot];
  HIPCHK(hipEventRecord(ev[0], st));
  RC(torn_begin(ctx, o, tol, utol, f, cj, lam, cand, pick_flag));
  HIPCHK(hipEventRecord(ev[1], st));
  const int32_t* done = ctx->ist + IS_DONE;
  const int base_chunk = std::max(1, o->check_every);
  static const bool trace = std::getenv("FETI_TRACE") != nullptr;
  static const bool use_graph = std::getenv("FETI_NO_GRAPH") == nullptr;
  static const bool use_persist = std::getenv("FETI_NO_PERSIST") == nullptr;
  // (the persistent kernel projects with H = G (G^T G)^{-1}, built when n_c <= PCG_NC_LOCAL)
  const bool persist = use_persist && !trace && !ctx->dp && ctx->pcg_mode == FETI_PCG_AUTO && ctx->pgrid > 0 &&
                       ctx->nc <= PCG_NC_LOCAL && (ctx->nc == 0 || ctx->H != nullptr) &&
                       ctx->precond != FETI_PRECOND_NONE;
  if (persist) {
    // every iteration of the solve in one cooperative launch (a solve converged at
    // its start leaves the launch at once)
    {
      HIPCHK(hipMemsetAsync(ctx->bar, 0, sizeof(GridBarrier), st));
      const Factors fc = factors(ctx);
      PcgArgs pa;
      pa.m = m;
      pa.fm = fc.splus; pa.fm32 = fc.f32;
      if (ctx->precond == FETI_PRECOND_LUMPED) { pa.mm = ctx->Kbb; pa.mm32 = 0; }
      else { pa.mm = fc.sbb; pa.mm32 = fc.f32; }
      pa.Cinv = ctx->Cinv; pa.H = ctx->H; pa.nc = ctx->nc;
      pa.lam = lam; pa.r = ctx->r; pa.w = ctx->w; pa.z = ctx->z; pa.y = ctx->y; pa.p = ctx->p;
      pa.q = ctx->q; pa.qraw = ctx->qraw; pa.yb = ctx->yb; pa.zb = ctx->zb; pa.g = ctx->g;
      pa.mdiag = ctx->mdiag; pa.part = ctx->ppart; pa.sc = ctx->sc; pa.ist = ctx->ist; pa.bar = ctx->bar;
      pa.tile_sub = ctx->tile_sub; pa.tile_row0 = ctx->tile_row0; pa.ntile = ctx->ntile;
      static const bool ptrace = std::getenv("FETI_PCG_TRACE") != nullptr;
      long long* ts = nullptr;
      const int nts = 64;
      if (ptrace) {
        HIPCHK(hipMalloc(&ts, nts * 10 * sizeof(long long)));
        HIPCHK(hipMemsetAsync(ts, 0, nts * 10 * sizeof(long long), st));
        pa.tstamp = ts; pa.tstamp_iters = nts;
      }
      HIPCHK(launch_pcg_persistent(pa, ctx->pgrid, st));
      if (ptrace) {
        // stamps per iteration: 0 start, 1..6 after the barriers of phases A, B, D, E (with
        // the stopping test), F, G (stamp 0 of a later iteration = stamp 6 before)
        const int np = 6;
        std::vector<long long> h(nts * 10);
        HIPCHK(hipMemcpyAsync(h.data(), ts, h.size() * sizeof(long long), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        (void)hipFree(ts);
        int rate_khz = 0, dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
        double sum[6] = {0}; int cnt = 0;
        for (int it = 0; it < nts; ++it) {
          if (h[it * 10 + np] == 0) break;
          for (int k = 0; k < np; ++k) {
            const long long a0 = k > 0 ? h[it * 10 + k] : (it == 0 ? h[0] : h[(it - 1) * 10 + np]);
            sum[k] += (double)(h[it * 10 + k + 1] - a0);
          }
          ++cnt;
        }
        if (cnt > 0 && rate_khz > 0) {
          const double us = 1e3 / rate_khz / cnt;
          std::fprintf(stderr, "[pcg] grid %d, %d iterations, us per phase:", ctx->pgrid, cnt);
          for (int k = 0; k < np; ++k) std::fprintf(stderr, " %.2f", sum[k] * us);
          std::fprintf(stderr, "\n");
        }
      }
    }
  }
  for (; !persist;) {
    HIPCHK(hipMemcpyAsync(ctx->h_ist, ctx->ist, IS_COUNT * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (trace)
      HIPCHK(hipMemcpyAsync(ctx->h_sc, ctx->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (trace) {
      std::fprintf(stderr,
                   "[feti] tol %.1e it %d res %.3e rho %.3e status %d energy %.2e kinds %.2e %.2e %.2e "
                   "%.2e %.2e %.2e\n",
                   ctx->h_sc[SC_TOL], ctx->h_ist[IS_ITERS], ctx->h_sc[SC_RES], ctx->h_sc[SC_RHO],
                   ctx->h_ist[IS_STATUS], ctx->h_sc[SC_ERAT], ctx->h_sc[SC_KRAT], ctx->h_sc[SC_KRAT + 1],
                   ctx->h_sc[SC_KRAT + 2], ctx->h_sc[SC_KRAT + 3], ctx->h_sc[SC_KRAT + 4],
                   ctx->h_sc[SC_KRAT + 5]);
      if (ctx->h_sc[SC_UTOL] > 0.0) {
        // per kind: recent update sizes / |lambda|_k (the update test passes when all are <= utol)
        std::fprintf(stderr, "[feti]   update ratios");
        for (int k = 0; k < 6; ++k) {
          double s = 0.0;
          for (int i = 0; i < UPD_WIN; ++i) s += ctx->h_sc[SC_URING + i * 6 + k];
          const double l = ctx->h_sc[SC_ULAM + k];
          std::fprintf(stderr, " %.2e(|l| %.1e)", l > 0.0 ? s / l : 0.0, l);
        }
        std::fprintf(stderr, "\n");
      }
    }
    if (ctx->h_ist[IS_DONE] || ctx->h_ist[IS_ITERS] >= o->max_it) break;
    // The iterations of a chunk that follow convergence are launched and return at once
    // (a few microseconds per kernel), so a chunk is sized from the iteration count of the
    // last solve in the same record slot: the largest power of two within what that count
    // leaves (at most check_every), or check_every once this solve has run past it.  The
    // arithmetic is that of any chunking.
    int chunk = base_chunk;
    {
      const int left = ctx->prev_iters[slot] - ctx->h_ist[IS_ITERS];
      if (left > 0) {
        const int cap = std::min(left, base_chunk);
        chunk = 1;
        while (2 * chunk <= cap) chunk *= 2;
        if (cap == base_chunk) chunk = base_chunk;
      }
    }
    // one chunk of iterations, replayed from a captured graph
    feti_ctx_s::Graph* gr = nullptr;
    if (use_graph) {
      for (auto& g : ctx->graphs)
        if (g.exec && g.lam == lam && g.chunk == chunk) gr = &g;
      if (!gr) {
        gr = nullptr;
        for (auto& g : ctx->graphs)
          if (!gr && g.exec == nullptr) gr = &g;
        if (!gr) {
          constexpr int NG = (int)(sizeof(ctx->graphs) / sizeof(ctx->graphs[0]));
          gr = &ctx->graphs[ctx->graph_next];
          ctx->graph_next = (ctx->graph_next + 1) % NG;
        }
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        *gr = feti_ctx_s::Graph();
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int it = 0; it < chunk; ++it) pcg_iteration(ctx, lam, done);
        HIPCHK(hipStreamEndCapture(st, &graph));
        HIPCHK(hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0));
        (void)hipGraphDestroy(graph);
        gr->lam = lam;
        gr->chunk = chunk;
      }
      HIPCHK(hipGraphLaunch(gr->exec, st));
    } else {
      for (int it = 0; it < chunk; ++it) pcg_iteration(ctx, lam, done);
    }
  }
  HIPCHK(hipEventRecord(ev[2], st));
  RC(torn_end(ctx, lam, u, f));
  HIPCHK(hipEventRecord(ev[3], st));
  HIPCHK(hipMemcpyAsync(ctx->h_rec_ist + slot * IS_COUNT, ctx->ist, IS_COUNT * sizeof(int32_t),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(ctx->h_rec_sc + slot * SC_COUNT, ctx->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                        st));
  return FETI_OK;
}

// Outcome of the solve recorded in slot (the stream has been synchronised since):
// accumulates its iterations and phase times, returns its status (with the message).
int finish_solve(feti_ctx ctx, int slot, feti_stats* stats, int* iters_out, double* res0, double* res) {
  const int32_t* hi = ctx->h_rec_ist + slot * IS_COUNT;
  const double* hs = ctx->h_rec_sc + slot * SC_COUNT;
  const int status = hi[IS_STATUS];
  ctx->prev_iters[slot] = hi[IS_ITERS];
  if (iters_out) *iters_out += hi[IS_ITERS];
  if (res0) *res0 = hs[SC_RES0];
  if (res) *res = hs[SC_RES];
  if (stats) {
    const hipEvent_t* ev = ctx->rec_ev[slot];
    for (int k = 0; k < 3; ++k) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      stats->t_ms[1 + k] += ms;
    }
  }
  if (status == FETI_EHIP) return fail(ctx, status, "persistent PCG: grid barrier timed out");
  if (status == FETI_ENOTCONV) return fail(ctx, status, "PCG did not converge within max_it");
  if (status == FETI_EBREAKDOWN) return fail(ctx, status, "PCG breakdown");
  if (status == FETI_ENAN) return fail(ctx, status, "non-finite value in the interface iteration");
  return FETI_OK;
}

// Torn-system residual of (u, lam) for right-hand side f: rf = f - K u - B^T lam,
// cj = -sum_s B_s u_s (the jump a correction must add).
void torn_residual(feti_ctx ctx, const double* f, const double* u, const double* lam) {
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  launch_elem_matvec(m, u, ctx->ytmp, ctx->mpP, ctx->mpE, st);
  launch_axpby(m.sum_ns, 1.0, f, -1.0, ctx->ytmp, ctx->rf, st);
  launch_sub_gather(m, lam, ctx->rf, st);
  // dual-primal: a primal row's residual is the sum over its owners (kept in the first)
  if (ctx->dp) launch_pi_fold(m, ctx->rf, st);
  launch_jump(m, u, 1, ctx->cj, 0, nullptr, nullptr, st);
  launch_axpby(m.n_lambda, -1.0, ctx->cj, 0.0, nullptr, ctx->cj, st);
}

// One FETI solve followed by up to nref FP64 refinement corrections.  history: a time
// step (its total correction is kept for the next step's first correction, and the
// multiplier history is advanced).  The stream is synchronised once at the end, and
// between corrections only when a later one may be skipped (nref > 1).
int solve_refined(feti_ctx ctx, const feti_solve_opts* o, int nref, feti_stats* stats,
                  const double* cand = nullptr, int* took_cand = nullptr, bool history = false) {
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  const double tol_first =
      (ctx->precision == FETI_FP32_IR && o->tol_inner > 0.0) ? std::max(o->tol, o->tol_inner) : o->tol;
  // status of the step: that of the last solve (a first solve that ran out of iterations
  // is repaired by the corrections), but a breakdown, a non-finite value or a barrier
  // timeout in any solve is kept
  int nrec = 0, nfin = 0, rc = FETI_OK, hard = FETI_OK, last = FETI_OK, iters = 0, iters_first = 0, done_ir = 0;
  double res0 = 0, res = 0, r0c = 0, rc_ = 0, corr = 0.0;
  int it_corr[feti_ctx_s::NREC] = {0};
  // the first solve's start choice goes to d_pick[1] (d_pick[0] serves the corrections)
  RC(solve_torn(ctx, o, tol_first, 0.0, ctx->f, nullptr, ctx->lam, ctx->u, nrec++, cand, ctx->d_pick + 1));
  if (cand) HIPCHK(hipMemcpyAsync(ctx->h_pick + 1, ctx->d_pick + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  // outcome of every enqueued solve not read yet (after a synchronisation)
  auto finish = [&]() {
    for (; nfin < nrec; ++nfin) {
      int its = 0;
      const int s = nfin == 0 ? finish_solve(ctx, 0, stats, &its, &res0, &res)
                              : finish_solve(ctx, nfin, stats, &its, &r0c, &rc_);
      if (nfin == 0) iters_first = its;
      else it_corr[nfin - 1] = its;
      iters += its;
      last = s;
      if (s != FETI_OK && s != FETI_ENOTCONV && hard == FETI_OK) hard = s;
    }
    rc = hard != FETI_OK ? hard : last;
  };
  auto correction_size = [&]() {
    double mx[12] = {0};
    for (int b = 0; b < KMAX_NBLK; ++b)
      for (int c = 0; c < 12; ++c) mx[c] = std::max(mx[c], ctx->h_kpart[b * 12 + c]);
    double cs = 0.0;
    for (int kk = 0; kk < 6; ++kk)
      if (mx[6 + kk] > 0.0) cs = std::max(cs, mx[kk] / mx[6 + kk]);
    return cs;
  };
  HIPCHK(hipEventRecord(ctx->ev[6], st));
  bool warm_used = false;
  for (int k = 0; k < nref && nrec < feti_ctx_s::NREC; ++k) {
    torn_residual(ctx, ctx->f, ctx->u, ctx->lam);
    HIPCHK(hipMemsetAsync(ctx->dlam, 0, m.n_lambda * sizeof(double), st));
    // the first correction of a time step may start from the previous step's total
    // correction, kept only if its projected residual beats the zero start (chosen on
    // the device)
    const bool warm = history && k == 0 && o->corr_start == FETI_CORR_PREVIOUS && ctx->have_dlam_prev;
    RC(solve_torn(ctx, o, o->tol_corr, o->tol_upd, ctx->rf, ctx->cj, ctx->dlam, ctx->du, nrec++,
                  warm ? ctx->dlam_prev : nullptr, nullptr));
    if (warm) {
      HIPCHK(hipMemcpyAsync(ctx->h_pick, ctx->d_pick, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      warm_used = true;
    }
    launch_axpby(m.sum_ns, 1.0, ctx->u, 1.0, ctx->du, ctx->u, st);
    launch_axpby(m.n_lambda, 1.0, ctx->lam, 1.0, ctx->dlam, ctx->lam, st);
    launch_axpby(m.n_lambda, 1.0, ctx->dlam, k == 0 ? 0.0 : 1.0, k == 0 ? nullptr : ctx->dlam_sum, ctx->dlam_sum,
                 st);
    // size of the correction per DOF kind
    launch_kind_maxabs(m, ctx->du, ctx->u, ctx->kpart, KMAX_NBLK, st);
    HIPCHK(hipMemcpyAsync(ctx->h_kpart, ctx->kpart, KMAX_NBLK * 12 * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    ++done_ir;
    if (k + 1 < nref) {
      // a later correction runs only if this one still changed the fields
      HIPCHK(hipStreamSynchronize(st));
      finish();
      if (hard != FETI_OK) break;
      corr = correction_size();
      if (corr <= o->ir_tol) break;
    }
  }
  if (history) {
    // multiplier history for the next step's start
    std::swap(ctx->lam_prev2, ctx->lam_prev);
    launch_axpby(m.n_lambda, 1.0, ctx->lam, 0.0, nullptr, ctx->lam_prev, st);
    HIPCHK(hipEventRecord(ctx->ev[5], st));
  }
  HIPCHK(hipEventRecord(ctx->ev[7], st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  finish();
  if (took_cand) *took_cand = cand ? ctx->h_pick[1] : 0;
  if (done_ir > 0) corr = correction_size();
  if (history) {
    // the step's total correction, for the next step
    if (done_ir > 0 && rc == FETI_OK) std::swap(ctx->dlam_prev, ctx->dlam_sum);
    ctx->have_dlam_prev = done_ir > 0 && rc == FETI_OK;
  }
  if (stats) {
    stats->iters = iters;
    stats->iters_first = iters_first;
    stats->ir_steps = done_ir;
    for (int k = 0; k < 4 && k < done_ir; ++k) stats->iters_corr[k] = it_corr[k];
    stats->corr_warm = warm_used ? *ctx->h_pick : 0;
    stats->res0 = res0;
    stats->res = res;
    stats->rho = corr;
    stats->status = rc;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev[6], ctx->ev[7]);
    stats->t_ms[4] = ms;
  }
  return rc;
}

// Stored tiles of the packed K_s^+ of every subdomain, in storage order: subdomain s
// holds tile rows I < ceil(n_s / 64) and columns J <= I (tile index tbase[s] +
// I (I + 1) / 2 + J).  kb: the tiles of tile rows I >= tb[s] = (n_s - n_b) / 64 (those
// the interface columns reach).  Any output may be null.
void sym_tiles(const MeshHost& mh, std::vector<int32_t>* ts, std::vector<int32_t>* ti, std::vector<int32_t>* tj,
               std::vector<int32_t>* nt, std::vector<int64_t>* tbase, std::vector<int32_t>* kb,
               std::vector<int32_t>* tb) {
  int64_t t = 0;
  for (int s = 0; s < (int)mh.subs.size(); ++s) {
    const int T = (mh.subs[s].ns + 63) / 64;
    const int b0 = (mh.subs[s].ns - mh.subs[s].nb) / 64;
    if (nt) (*nt)[s] = T;
    if (tbase) (*tbase)[s] = t;
    if (tb) (*tb)[s] = b0;
    for (int I = 0; I < T; ++I)
      for (int J = 0; J <= I; ++J, ++t) {
        if (ts) ts->push_back(s);
        if (ti) ti->push_back(I);
        if (tj) tj->push_back(J);
        if (kb && I >= b0) kb->push_back((int32_t)t);
      }
  }
}

// Tile tables (once per mesh) and the packed lower tiles of K_s^+ in the precision of the
// factors.
int build_sym(feti_ctx ctx, bool f32) {
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  SymArgs& a = ctx->sym;
  if (!a.t_sub) {
    const int nsub = m.nsub;
    std::vector<int32_t> ts, ti, tj, nt(nsub), kb, tbs(nsub);
    std::vector<int64_t> tb(nsub);
    sym_tiles(ctx->mh, &ts, &ti, &tj, &nt, &tb, &kb, &tbs);
    int32_t *d_ts = nullptr, *d_ti = nullptr, *d_tj = nullptr, *d_nt = nullptr, *d_kb = nullptr, *d_tbs = nullptr;
    int64_t* d_tb = nullptr;
    RC(upload(ctx, &d_ts, ts));
    RC(upload(ctx, &d_ti, ti));
    RC(upload(ctx, &d_tj, tj));
    RC(upload(ctx, &d_nt, nt));
    RC(upload(ctx, &d_tb, tb));
    RC(upload(ctx, &d_kb, kb));
    RC(upload(ctx, &d_tbs, tbs));
    RC(dalloc(ctx, &a.part, ts.size() * 128, ctx->allocs));
    HIPCHK(hipStreamSynchronize(st));  // the host tables leave scope
    a.ntile = (int)ts.size();
    a.t_sub = d_ts; a.t_I = d_ti; a.t_J = d_tj; a.nt = d_nt; a.tbase = d_tb;
    a.kb_tiles = d_kb; a.n_kb_tiles = (int)kb.size(); a.tb = d_tbs;
  }
  if (a.P && a.f32 != (int)f32) {
    auto it = std::find(ctx->mat_allocs.begin(), ctx->mat_allocs.end(), const_cast<void*>(a.P));
    if (it != ctx->mat_allocs.end()) ctx->mat_allocs.erase(it);
    HIPCHK(hipFree(const_cast<void*>(a.P)));
    a.P = nullptr;
  }
  const size_t ne = (size_t)a.ntile * 4096;
  if (f32) {
    float* P = (float*)a.P;
    if (!P) RC(dalloc(ctx, &P, ne, ctx->mat_allocs));
    launch_sym_pack(a, (const float*)ctx->Kinv32, m.kofs, m.ld, m.ns, P, st);
    a.P = P;
  } else {
    double* P = (double*)a.P;
    if (!P) RC(dalloc(ctx, &P, ne, ctx->mat_allocs));
    launch_sym_pack(a, (const double*)ctx->Kinv, m.kofs, m.ld, m.ns, P, st);
    a.P = P;
  }
  a.f32 = f32 ? 1 : 0;
  HIPCHK(hipGetLastError());
  return FETI_OK;
}

int build_gj_plan(feti_ctx ctx, GJPlan& P, std::vector<int32_t>& host_flag, int nmat,
                  const std::vector<int>& n, const std::vector<int>& nI, const std::vector<int>& nsw,
                  const std::vector<int64_t>& aofs, const std::vector<int32_t>& lda,
                  const std::vector<int64_t>& snap_ofs, const std::vector<int32_t>& snap_ld,
                  int nb, std::vector<void*>& list) {
  P = GJPlan();
  P.nmat = nmat;
  P.nb = nb;
  std::vector<std::vector<std::pair<int, int>>> panels(nmat);
  std::vector<int> snap_step(nmat, -1);
  for (int mI = 0; mI < nmat; ++mI) {
    P.max_n = std::max(P.max_n, n[mI]);
    for (int k = 0; k < nI[mI]; k += nb) panels[mI].push_back({k, std::min(nb, nI[mI] - k)});
    if (snap_ofs[mI] >= 0) snap_step[mI] = (int)panels[mI].size() - 1;
    for (int k = nI[mI]; k < nsw[mI]; k += nb) panels[mI].push_back({k, std::min(nb, nsw[mI] - k)});
    P.nsteps = std::max(P.nsteps, (int)panels[mI].size());
  }
  std::vector<int32_t> ps((size_t)P.nsteps * nmat, 0), pw((size_t)P.nsteps * nmat, 0),
      pf((size_t)P.nsteps * nmat, 0);
  for (int mI = 0; mI < nmat; ++mI)
    for (int s = 0; s < (int)panels[mI].size(); ++s) {
      ps[(size_t)s * nmat + mI] = panels[mI][s].first;
      pw[(size_t)s * nmat + mI] = panels[mI][s].second;
      if (s == snap_step[mI]) pf[(size_t)s * nmat + mI] = 1;
    }
  host_flag.assign(P.nsteps, 0);
  for (int s = 0; s < P.nsteps; ++s)
    for (int mI = 0; mI < nmat; ++mI) host_flag[s] |= pf[(size_t)s * nmat + mI];
  std::vector<int32_t> nn(n.begin(), n.end()), snap_at(nI.begin(), nI.end());
  auto up = [&](auto** p, const auto& v) {
    int rc = dalloc(ctx, p, v.size(), list);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(*p, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice, ctx->stream);
    return e == hipSuccess ? FETI_OK : fail(ctx, FETI_EHIP, hipGetErrorString(e));
  };
  RC(up(&P.pstart, ps));
  RC(up(&P.pwidth, pw));
  RC(up(&P.pflag, pf));
  RC(up(&P.aofs, aofs));
  RC(up(&P.lda, lda));
  RC(up(&P.n, nn));
  RC(up(&P.snap_ofs, snap_ofs));
  RC(up(&P.snap_at, snap_at));
  RC(up(&P.snap_ld, snap_ld));
  RC(dalloc(ctx, &P.pinv, (size_t)nmat * nb * nb, list));
  double* wrow = nullptr;  // sized for FP64, enough for either element type
  RC(dalloc(ctx, &wrow, (size_t)nmat * nb * P.max_n, list));
  P.wrow = wrow;
  RC(dalloc(ctx, &P.status, nmat, list));
  HIPCHK(hipMemsetAsync(P.status, 0, nmat * sizeof(int32_t), ctx->stream));
  return FETI_OK;
}

}  // namespace

// ============================================================================
extern "C" {

int feti_create(feti_ctx* out, void* hip_stream) {
  if (!out) return FETI_EINVAL;
  feti_ctx ctx = new (std::nothrow) feti_ctx_s();
  if (!ctx) return FETI_ENOMEM;
  ctx->stream = (hipStream_t)hip_stream;
  *out = ctx;
  return FETI_OK;
}

int feti_destroy(feti_ctx ctx) {
  if (!ctx) return FETI_EINVAL;
  if (ctx->state >= 2) {
    (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    for (auto& e : ctx->ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : ctx->ev_gj)
      if (e) (void)hipEventDestroy(e);
    if (ctx->h_ist) (void)hipHostFree(ctx->h_ist);
    if (ctx->h_sc) (void)hipHostFree(ctx->h_sc);
    if (ctx->h_kpart) (void)hipHostFree(ctx->h_kpart);
    if (ctx->h_rec_ist) (void)hipHostFree(ctx->h_rec_ist);
    if (ctx->h_rec_sc) (void)hipHostFree(ctx->h_rec_sc);
    if (ctx->h_pick) (void)hipHostFree(ctx->h_pick);
    for (auto& r : ctx->rec_ev)
      for (auto& e : r)
        if (e) (void)hipEventDestroy(e);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
  return FETI_OK;
}

const char* feti_last_error(feti_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int feti_setup_mesh(feti_ctx ctx, const feti_mesh_desc* mesh) {
  if (!ctx || !mesh) return FETI_EINVAL;
  if (ctx->state != 0) return fail(ctx, FETI_ESTATE, "setup_mesh must be the first call");
  std::string e = build_mesh(*mesh, ctx->mh);
  if (!e.empty()) return fail(ctx, FETI_EINVAL, e);
  ctx->state = 1;
  return FETI_OK;
}

int feti_get_sizes(feti_ctx ctx, int64_t* s) {
  if (!ctx || !s) return FETI_EINVAL;
  if (ctx->state < 1) return fail(ctx, FETI_ESTATE, "no mesh");
  const MeshHost& h = ctx->mh;
  s[0] = (int64_t)h.subs.size();
  s[1] = h.sum_ns;
  s[2] = h.n_lambda;
  s[3] = 3 * h.n_float;
  s[4] = h.max_ns;
  s[5] = h.max_nb;
  s[6] = h.sum_nb;
  s[7] = h.n_p1_lat;
  s[8] = h.n_u_lat;
  s[9] = h.n_float;
  s[10] = h.n_pi;
  return FETI_OK;
}

int feti_export_indexing(feti_ctx ctx, int32_t* code, int32_t* sub_off, int32_t* sub_nb,
                         int32_t* brow_sub, int32_t* brow_local, int8_t* brow_sign) {
  if (!ctx) return FETI_EINVAL;
  if (ctx->state < 1) return fail(ctx, FETI_ESTATE, "no mesh");
  const MeshHost& h = ctx->mh;
  for (size_t s = 0; s < h.subs.size(); ++s) {
    const SubHost& sh = h.subs[s];
    if (code) std::memcpy(code + sh.off, sh.codes.data(), sh.ns * sizeof(int32_t));
    if (sub_off) sub_off[s] = (int32_t)sh.off;
    if (sub_nb) sub_nb[s] = sh.nb;
  }
  if (sub_off) sub_off[h.subs.size()] = (int32_t)h.sum_ns;
  for (int64_t j = 0; j < h.n_lambda; ++j)
    for (int e = 0; e < 2; ++e) {
      if (brow_sub) brow_sub[2 * j + e] = h.rows[j].sub[e];
      if (brow_local) brow_local[2 * j + e] = h.rows[j].loc[e];
      if (brow_sign) brow_sign[2 * j + e] = h.rows[j].sign[e];
    }
  return FETI_OK;
}

int feti_export_primal(feti_ctx ctx, int32_t* pi_code, int32_t* sub_npi) {
  if (!ctx) return FETI_EINVAL;
  if (ctx->state < 1) return fail(ctx, FETI_ESTATE, "no mesh");
  const MeshHost& h = ctx->mh;
  if (pi_code && h.n_pi > 0) std::memcpy(pi_code, h.pi_code.data(), h.n_pi * sizeof(int32_t));
  if (sub_npi)
    for (size_t s = 0; s < h.subs.size(); ++s) {
      int c = 0;
      for (int8_t cat : h.subs[s].cats) c += (h.n_pi > 0 && cat == C_BP) ? 1 : 0;
      sub_npi[s] = c;
    }
  return FETI_OK;
}

int feti_export_deflation(feti_ctx ctx, int32_t* col, double* w, int32_t* n_defl) {
  if (!ctx) return FETI_EINVAL;
  if (ctx->state < 1) return fail(ctx, FETI_ESTATE, "no mesh");
  const MeshHost& h = ctx->mh;
  const bool have = !h.defl_col.empty();
  for (int64_t j = 0; j < 2 * h.n_lambda; ++j) {
    if (col) col[j] = have ? h.defl_col[j] : -1;
    if (w) w[j] = have ? h.defl_w[j] : 0.0;
  }
  if (n_defl) *n_defl = h.n_defl;
  return FETI_OK;
}

int feti_assemble(feti_ctx ctx, const feti_material* P, const feti_material* E, double tau) {
  if (!ctx || !P || !E) return FETI_EINVAL;
  if (ctx->state < 1) return fail(ctx, FETI_ESTATE, "assemble before setup_mesh");
  if (!(tau > 0.0) || !(P->nu < 0.5) || !(E->nu < 0.5) || !(P->E > 0) || !(E->E > 0) ||
      !(P->c0 > 0) || !(P->K > 0) || !(P->mu_f > 0))
    return fail(ctx, FETI_EINVAL, "material parameters out of range (need E>0, nu<1/2, c0>0, K>0, tau>0)");
  if (ctx->state >= 2) {
    (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  ctx->device = dev;
  if (ctx->stream == nullptr) {
    // a stream of our own (blocking with respect to the null stream) so that the
    // iteration chunks can be captured into graphs
    HIPCHK(hipStreamCreate(&ctx->stream));
    ctx->own_stream = true;
  }
  ctx->matP = *P;
  ctx->matE = *E;
  ctx->tau = tau;
  lame(*P, ctx->lamP, ctx->muP);
  lame(*E, ctx->lamE, ctx->muE);
  const double den = P->alpha * P->alpha + P->c0 * ctx->lamP;
  ctx->mpP.mu = ctx->muP;
  ctx->mpP.kap1 = P->alpha / den;
  ctx->mpP.kap2 = ctx->lamP / den;
  ctx->mpP.kap3 = P->c0 / den;
  ctx->mpP.kf = P->K / P->mu_f;
  ctx->mpP.tau = tau;
  ctx->mpE.mu = ctx->muE;
  ctx->mpE.lam_inv = 1.0 / ctx->lamE;
  ctx->mpE.tau = tau;
  RC(upload_mesh(ctx));
  RC(dalloc(ctx, &ctx->dm.emat, (size_t)ctx->dm.nelem * ctx->dm.edof * ctx->dm.edof, ctx->allocs));
  const bool d3 = ctx->mh.dim == 3;
  if (d3) launch_elem_store3d(ctx->dm, ctx->mpP, ctx->mpE, ctx->stream);
  else launch_elem_store(ctx->dm, ctx->mpP, ctx->mpE, ctx->stream);
  RC(dalloc(ctx, &ctx->K, ctx->k_total, ctx->mat_allocs));
  HIPCHK(hipMemsetAsync(ctx->K, 0, ctx->k_total * sizeof(double), ctx->stream));
  if (d3) launch_assemble3d(ctx->dm, ctx->K, ctx->stream);
  else launch_assemble(ctx->dm, ctx->K, ctx->mpP, ctx->mpE, ctx->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->state = 2;
  ctx->nstep = 0;
  ctx->have_prev = ctx->have_prev2 = ctx->have_dlam_prev = false;
  return FETI_OK;
}

// In-place inverse of one dense symmetric n x n matrix A (device, row major) by the
// pivot-free sweep of the elimination; the plan's temporaries and the uploaded size are
// freed on every path.  FETI_ESINGULAR (with what) on a zero or non-finite pivot.
int invert_dense(feti_ctx ctx, double* A, int n, const char* what) {
  hipStream_t st = ctx->stream;
  GJPlan C;
  std::vector<int32_t> cflag;
  std::vector<void*> tmp;
  auto done = [&](int rc) {
    for (void* p : tmp) (void)hipFree(p);
    return rc;
  };
  int rc = build_gj_plan(ctx, C, cflag, 1, {n}, {0}, {n}, {0}, {n}, {-1}, {n}, GJ_PANEL, tmp);
  if (rc) return done(rc);
  for (int s = 0; s < C.nsteps; ++s) launch_gj_step(C, A, (double*)nullptr, s, false, st);
  int32_t* d_n = nullptr;
  if (hipMalloc(&d_n, sizeof(int32_t)) != hipSuccess) return done(fail(ctx, FETI_ENOMEM, "device allocation failed"));
  tmp.push_back(d_n);
  if (hipMemcpyAsync(d_n, &n, sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess)
    return done(fail(ctx, FETI_EHIP, "copy of the matrix size failed"));
  launch_gj_finalize(C, A, d_n, st);
  int32_t cs = 0;
  if (hipMemcpyAsync(&cs, C.status, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return done(fail(ctx, FETI_EHIP, std::string("inversion of the ") + what + " failed"));
  if (cs) return done(fail(ctx, FETI_ESINGULAR, std::string("zero or non-finite pivot in the ") + what));
  return done(FETI_OK);
}

int feti_factor_subdomains(feti_ctx ctx, int32_t precision, int32_t precond) {
  if (!ctx) return FETI_EINVAL;
  if (ctx->state < 2) return fail(ctx, FETI_ESTATE, "factor before assemble");
  if (precision != FETI_FP64 && precision != FETI_FP32_IR)
    return fail(ctx, FETI_EINVAL, "precision not supported");
  if (precond < 0 || precond > 2) return fail(ctx, FETI_EINVAL, "bad preconditioner");
  if (ctx->dp && precision != FETI_FP64) return fail(ctx, FETI_EINVAL, "the dual-primal coupling takes FP64 factors");
  ctx->precision = precision;
  ctx->precond = precond;
  drop_graphs(ctx);
  hipStream_t st = ctx->stream;
  const MeshHost& h = ctx->mh;
  DevMesh& m = ctx->dm;
  const int nsub = m.nsub;
  const bool f32 = precision == FETI_FP32_IR;
  if (!ctx->Kbb) RC(dalloc(ctx, &ctx->Kbb, ctx->s_total, ctx->mat_allocs));
  if (!ctx->keep_assembled && (ctx->state >= 3 || !ctx->K))
    return fail(ctx, FETI_ESTATE, "factors computed in place cannot be recomputed");
  if (!f32 && !ctx->Sbb) {
    RC(dalloc(ctx, &ctx->Sbb, ctx->s_total, ctx->mat_allocs));
    RC(dalloc(ctx, &ctx->Splus, ctx->s_total, ctx->mat_allocs));
  }
  if (!f32 && !ctx->Kinv) {
    if (ctx->keep_assembled) RC(dalloc(ctx, &ctx->Kinv, ctx->k_total, ctx->mat_allocs));
    else ctx->Kinv = ctx->K;  // eliminated in place
  }
  if (f32 && !ctx->Kinv32) {
    RC(dalloc(ctx, &ctx->Kinv32, ctx->k_total, ctx->mat_allocs));
    RC(dalloc(ctx, &ctx->Sbb32, ctx->s_total, ctx->mat_allocs));
    RC(dalloc(ctx, &ctx->Splus32, ctx->s_total, ctx->mat_allocs));
  }
  if (f32) launch_to_f32(ctx->k_total, ctx->K, ctx->Kinv32, st);
  else if (ctx->Kinv != ctx->K)
    HIPCHK(hipMemcpyAsync(ctx->Kinv, ctx->K, ctx->k_total * sizeof(double), hipMemcpyDeviceToDevice, st));
  // host copies of the per-subdomain geometry of the dense blocks
  std::vector<int> n(nsub), nI(nsub), nsw(nsub);
  std::vector<int64_t> aofs(nsub), sofs(nsub);
  std::vector<int32_t> lda(nsub), ldb(nsub), nbv(nsub), nIv(nsub), nfin(nsub);
  int64_t ko = 0, so = 0;
  for (int s = 0; s < nsub; ++s) {
    const SubHost& sh = h.subs[s];
    // pivots: every DOF but the fixed ones (dual coupling) or the primal ones (dual-primal
    // coupling); the final sign change covers the swept block, or (dual-primal) the whole
    // matrix, which then holds N_s = [[K_rr^{-1}, -K_rr^{-1} K_rPi], [-K_Pir K_rr^{-1}, -S_s]]
    int npi = 0;
    if (ctx->dp)
      for (int8_t c : sh.cats) npi += c == C_BP ? 1 : 0;
    n[s] = sh.ns; nI[s] = sh.nI; nsw[s] = sh.ns - (ctx->dp ? npi : sh.nfix);
    nfin[s] = ctx->dp ? sh.ns : nsw[s];
    lda[s] = (int32_t)round8(sh.ns); aofs[s] = ko; ko += (int64_t)sh.ns * lda[s];
    ldb[s] = (int32_t)round8(sh.nb); sofs[s] = so; so += (int64_t)sh.nb * ldb[s];
    nbv[s] = sh.nb; nIv[s] = sh.nI;
  }
  // lumped preconditioner block K_bb (Section 3.2) from the assembled matrix
  launch_copy_block(nsub, m.max_nb, m.kofs, m.ld, m.nI, m.sofs, m.ldb, m.nb, (const double*)ctx->K, ctx->Kbb,
                    st);
  std::vector<void*> tmp;
  GJPlan P;
  std::vector<int32_t> hflag;
  int rc = build_gj_plan(ctx, P, hflag, nsub, n, nI, nsw, aofs, lda, sofs, ldb, GJ_PANEL, tmp);
  if (rc) { for (void* p : tmp) (void)hipFree(p); return rc; }
  std::vector<int32_t> stat(nsub, 0);
  // the swept counts of the finalisation: a temporary like the plan's tables
  int32_t* d_nsw = nullptr;
  if (hipMalloc(&d_nsw, nfin.size() * sizeof(int32_t)) != hipSuccess) {
    for (void* p : tmp) (void)hipFree(p);
    return fail(ctx, FETI_ENOMEM, "device allocation failed");
  }
  tmp.push_back(d_nsw);
  if (hipMemcpyAsync(d_nsw, nfin.data(), nfin.size() * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess) {
    for (void* p : tmp) (void)hipFree(p);
    return fail(ctx, FETI_EHIP, "copy of the swept counts failed");
  }
  // S_bb of a subdomain without interior DOFs (a one-cell slab of a 3D decomposition) is
  // its K_bb: no interior pivot step takes that snapshot, so every interface block is
  // copied before the sweep (the snapshots of the other subdomains overwrite theirs)
  if (f32)
    launch_copy_block(nsub, m.max_nb, m.kofs, m.ld, m.nI, m.sofs, m.ldb, m.nb, (const float*)ctx->Kinv32,
                      ctx->Sbb32, st);
  else
    launch_copy_block(nsub, m.max_nb, m.kofs, m.ld, m.nI, m.sofs, m.ldb, m.nb, (const double*)ctx->Kinv, ctx->Sbb,
                      st);
  HIPCHK(hipEventRecord(ctx->ev_gj[0], st));
  if (f32) {
    for (int s = 0; s < P.nsteps; ++s) launch_gj_step(P, ctx->Kinv32, ctx->Sbb32, s, hflag[s] != 0, st);
    launch_gj_finalize(P, ctx->Kinv32, d_nsw, st);
    HIPCHK(hipEventRecord(ctx->ev_gj[1], st));
    launch_precond_diag(m, (const float*)ctx->Sbb32, ctx->mdiag, st);
    launch_copy_block(nsub, m.max_nb, m.kofs, m.ld, m.nI, m.sofs, m.ldb, m.nb, (const float*)ctx->Kinv32,
                      ctx->Splus32, st);
  } else {
    for (int s = 0; s < P.nsteps; ++s) launch_gj_step(P, ctx->Kinv, ctx->Sbb, s, hflag[s] != 0, st);
    launch_gj_finalize(P, ctx->Kinv, d_nsw, st);
    HIPCHK(hipEventRecord(ctx->ev_gj[1], st));
    // weights of the dual-energy residual norm: |diag| of the Dirichlet preconditioner
    launch_precond_diag(m, (const double*)ctx->Sbb, ctx->mdiag, st);
    // (K^+)_bb into the compact interface blocks
    launch_copy_block(nsub, m.max_nb, m.kofs, m.ld, m.nI, m.sofs, m.ldb, m.nb, (const double*)ctx->Kinv,
                      ctx->Splus, st);
  }
  // packed lower tiles of K_s^+ for the local solves (an in-place elimination keeps only
  // them: its dense blocks are released below)
  rc = build_sym(ctx, f32);
  if (rc) { for (void* p : tmp) (void)hipFree(p); return rc; }
  HIPCHK(hipMemcpyAsync(stat.data(), P.status, nsub * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev_gj[0], ctx->ev_gj[1]));
    ctx->t_gj_ms = ms;
  }
  for (void* p : tmp) (void)hipFree(p);
  if (!ctx->keep_assembled) {
    // an in-place elimination keeps K_s^+ only as packed tiles: the dense blocks (the
    // assembled matrices, eliminated in place for FP64; their FP32 copy for FP32) go
    auto release = [&](void* q) -> int {
      if (!q) return FETI_OK;
      auto it = std::find(ctx->mat_allocs.begin(), ctx->mat_allocs.end(), q);
      if (it != ctx->mat_allocs.end()) ctx->mat_allocs.erase(it);
      HIPCHK(hipFree(q));
      return FETI_OK;
    };
    RC(release(ctx->K));
    if (f32) RC(release(ctx->Kinv32));
    ctx->K = nullptr;
    ctx->Kinv = nullptr;
    ctx->Kinv32 = nullptr;
  }
  for (int s = 0; s < nsub; ++s)
    if (stat[s]) return fail(ctx, FETI_ESINGULAR, "zero or non-finite pivot in subdomain " + std::to_string(s));
  // dual-primal coupling: the primal coarse matrix S_PiPi = sum_s L_s^T S_s L_s from the
  // interface blocks (-S_s is their primal block) and its inverse, by the same pivot-free
  // sweep (the global primal order puts the U-type corners first: quasi-definite)
  if (ctx->dp && m.n_pi > 0) {
    const int np = m.n_pi;
    if (!ctx->Spinv) RC(dalloc(ctx, &ctx->Spinv, (size_t)np * np, ctx->mat_allocs));
    HIPCHK(hipMemsetAsync(ctx->Spinv, 0, (size_t)np * np * sizeof(double), st));
    launch_pi_assemble(m, ctx->Splus, ctx->Spinv, st);
    RC(invert_dense(ctx, ctx->Spinv, np, "primal coarse matrix"));
  }
  // deflation of the dual-primal iteration: F W column by column and E = W^T F W, inverted
  if (ctx->defl) {
    const int nd = m.n_defl;
    const int64_t nl = m.n_lambda;
    if (!ctx->FW) RC(dalloc(ctx, &ctx->FW, (size_t)nl * nd, ctx->mat_allocs));
    if (!ctx->Edinv) RC(dalloc(ctx, &ctx->Edinv, (size_t)nd * nd, ctx->mat_allocs));
    for (int c = 0; c < nd; ++c) {
      launch_defl_column(m, c, ctx->tl, st);
      op_F(ctx, ctx->tl, ctx->FW + (size_t)c * nl, nullptr);
    }
    launch_defl_gram(m, ctx->FW, ctx->Edinv, st);
    RC(invert_dense(ctx, ctx->Edinv, nd, "deflation matrix W^T F W"));
  }
  // coarse matrix G^T G and its inverse
  const int nc = ctx->nc;
  if (nc > 0) {
    if (!ctx->Cinv) RC(dalloc(ctx, &ctx->Cinv, (size_t)nc * nc, ctx->mat_allocs));
    launch_gtg(m, ctx->Cinv, nc, st);
    RC(invert_dense(ctx, ctx->Cinv, nc, "coarse matrix G^T G"));
    if (nc <= PCG_NC_LOCAL) {
      if (!ctx->H) RC(dalloc(ctx, &ctx->H, (size_t)nc * m.n_lambda, ctx->mat_allocs));
      launch_build_h(m, ctx->Cinv, nc, ctx->H, st);
    }
  }
  HIPCHK(hipGetLastError());
  ctx->state = 3;
  return FETI_OK;
}

int feti_init_state(feti_ctx ctx, const feti_load* load) {
  if (!ctx || !load) return FETI_EINVAL;
  if (ctx->state < 2) return fail(ctx, FETI_ESTATE, "init_state before assemble");
  DevMesh& m = ctx->dm;
  HIPCHK(hipMemsetAsync(ctx->u, 0, m.sum_ns * sizeof(double), ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->lam_prev, 0, m.n_lambda * sizeof(double), ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->lam_prev2, 0, m.n_lambda * sizeof(double), ctx->stream));
  LoadDev L = make_load(ctx, load);
  launch_init_eta(m, ctx->u, L, ctx->stream);
  if (m.decoupled) {
    // the fluid state on the lattice, and the lumped mass (from the stored element matrices)
    const double D = ctx->lamP * ctx->matP.c0 + ctx->matP.alpha * ctx->matP.alpha;
    if (!(D > 0.0) || ctx->matP.alpha == 0.0)
      return fail(ctx, FETI_EINVAL, "decoupled scheme needs alpha != 0 (p = k1 xi + k2 eta)");
    ctx->dec_k1 = ctx->matP.alpha / D;
    ctx->dec_k2 = ctx->lamP / D;
    const size_t n1n = (size_t)ctx->mh.n1 * ctx->mh.n1;
    launch_zero((int64_t)n1n, ctx->dec_eta, ctx->stream);
    launch_zero((int64_t)n1n, ctx->dec_p, ctx->stream);
    launch_zero((int64_t)n1n, ctx->dec_xi, ctx->stream);
    launch_dec_init(m, L, ctx->dec_k1, ctx->dec_k2, ctx->dec_eta, ctx->dec_p, ctx->dec_xi, ctx->stream);
    double* me = nullptr;
    HIPCHK(hipMalloc(&me, (size_t)m.nelem * 3 * sizeof(double)));
    launch_dec_fluid(m, ctx->mpP, L, ctx->dec_p, ctx->dec_ce, me, ctx->stream);
    launch_dec_mass(m, me, ctx->dec_mass, ctx->stream);
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(me);
    HIPCHK(e);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->nstep = 0;
  ctx->have_prev = ctx->have_prev2 = ctx->have_dlam_prev = false;
  return FETI_OK;
}

int feti_step(feti_ctx ctx, const feti_load* load, const feti_solve_opts* o, feti_stats* stats) {
  if (!ctx || !load || !o) return FETI_EINVAL;
  if (ctx->state < 3) return fail(ctx, FETI_ESTATE, "step before factor_subdomains");
  if (!(o->tol > 0.0) || o->max_it < 1 || o->corr_start < FETI_CORR_ZERO || o->corr_start > FETI_CORR_PREVIOUS)
    return fail(ctx, FETI_EINVAL, "bad solve options");
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  HIPCHK(hipEventRecord(ctx->ev[0], st));
  LoadDev L = make_load(ctx, load);
  const bool d3 = ctx->mh.dim == 3;
  if (d3 && (L.kind != FETI_LOAD_RAW || L.t_side || L.zw_side))
    return fail(ctx, FETI_EINVAL, "3D takes nodal (RAW) loads without side data");
  int cmode = 0;
  if (m.decoupled) {
    // explicit fluid step: eta^n from eta^{n-1}, p^{n-1} (and xi^{n-1} at pressure
    // Dirichlet nodes); the momentum rows then read eta^n through their prescribed eta
    // columns (no cached right-hand side: those columns change every step)
    launch_dec_fluid(m, ctx->mpP, L, ctx->dec_p, ctx->dec_ce, nullptr, st);
    launch_dec_update(m, L, ctx->dec_k1, ctx->dec_k2, ctx->dec_ce, ctx->dec_mass, ctx->dec_eta, ctx->dec_xi, st);
    L.eta_dec = ctx->dec_eta;
  } else if (L.kind == FETI_LOAD_MANUFACTURED || L.kind == FETI_LOAD_PATCH) {
    // these loads do not depend on t: the quadrature of a step repeats that of the last
    // step with the same load and material parameters
    unsigned char key[sizeof(ctx->ekey)];
    LoadDev Lk = L;
    Lk.t = 0.0;
    std::memcpy(key, &Lk, sizeof(LoadDev));
    std::memcpy(key + sizeof(LoadDev), &ctx->mpP, sizeof(MatParams));
    std::memcpy(key + sizeof(LoadDev) + sizeof(MatParams), &ctx->mpE, sizeof(MatParams));
    if (!ctx->ecache) RC(dalloc(ctx, &ctx->ecache, (size_t)m.nelem * (m.edof + 3), ctx->allocs));
    if (ctx->ecache_valid && std::memcmp(key, ctx->ekey, sizeof(key)) == 0) {
      cmode = 2;
    } else {
      cmode = 1;
      std::memcpy(ctx->ekey, key, sizeof(key));
      ctx->ecache_valid = true;
    }
  }
  if (d3) launch_rhs3d(m, ctx->u, ctx->f, ctx->mpP, L, st);
  else launch_rhs(m, ctx->u, ctx->f, ctx->mpP, ctx->mpE, L, st, ctx->ecache, cmode);
  // start vector
  int used = o->start;
  if (o->start == FETI_START_ZERO ||
      (o->start != FETI_START_GIVEN && o->start != FETI_START_BEST && !ctx->have_prev) ||
      (o->start == FETI_START_BEST && !ctx->have_prev)) {
    HIPCHK(hipMemsetAsync(ctx->lam, 0, m.n_lambda * sizeof(double), st));
    used = FETI_START_ZERO;
  }
  if (o->start == FETI_START_PREVIOUS && ctx->have_prev) {
    launch_axpby(m.n_lambda, 1.0, ctx->lam_prev, 0.0, nullptr, ctx->lam, st);
  } else if (o->start == FETI_START_EXTRAPOLATE && ctx->have_prev) {
    if (ctx->have_prev2) launch_axpby(m.n_lambda, 2.0, ctx->lam_prev, -1.0, ctx->lam_prev2, ctx->lam, st);
    else { launch_axpby(m.n_lambda, 1.0, ctx->lam_prev, 0.0, nullptr, ctx->lam, st); used = FETI_START_PREVIOUS; }
  }
  if (o->start == FETI_START_GIVEN) {
    launch_axpby(m.n_lambda, 1.0, ctx->lam_given, 0.0, nullptr, ctx->lam, st);
  } else if (o->start == FETI_START_BEST && ctx->have_prev) {
    launch_axpby(m.n_lambda, 1.0, ctx->lam_prev, 0.0, nullptr, ctx->lam, st);
    used = FETI_START_PREVIOUS;
  }
  HIPCHK(hipGetLastError());
  const bool cold = !ctx->have_prev && o->start != FETI_START_GIVEN;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int took = 0;
  const double* cand = (o->start == FETI_START_BEST) ? ctx->lam_given : nullptr;
  // (solve_refined advances the multiplier history and synchronises the stream)
  int rc = solve_refined(ctx, o, cold ? std::max(o->ir_cold, o->ir_max) : o->ir_max, stats, cand, &took, true);
  if (m.decoupled) {
    // pressure from row 3 (nodal): p^n = k1 xi^n + k2 eta^n
    launch_dec_pressure(m, L, ctx->dec_k1, ctx->dec_k2, ctx->u, ctx->dec_xi, ctx->dec_p, ctx->dec_eta, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
  }
  if (cand && took) used = FETI_START_GIVEN;
  ctx->have_prev2 = ctx->have_prev;
  ctx->have_prev = true;
  ctx->nstep += 1;
  if (stats) {
    stats->start_used = used;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev[0], ctx->rec_ev[0][0]);  // right-hand side, up to the first solve
    stats->t_ms[0] = ms;
    (void)hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[5]);
    stats->t_ms[5] = ms;
  }
  return rc;
}

int feti_solve(feti_ctx ctx, const double* f_dev, double* lambda_dev, double* u_dev,
               const feti_solve_opts* o, feti_stats* stats) {
  if (!ctx || !f_dev || !o) return FETI_EINVAL;
  if (ctx->state < 3) return fail(ctx, FETI_ESTATE, "solve before factor_subdomains");
  if (!(o->tol > 0.0) || o->max_it < 1 || o->corr_start < FETI_CORR_ZERO || o->corr_start > FETI_CORR_PREVIOUS)
    return fail(ctx, FETI_EINVAL, "bad solve options");
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  // the time-stepping state (eta^n inside u, the prepared right-hand side) survives the
  // solve: the solve works in the context's vectors and restores them afterwards
  HIPCHK(hipMemcpyAsync(ctx->u_save, ctx->u, m.sum_ns * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->f_save, ctx->f, m.sum_ns * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipEventRecord(ctx->ev[0], st));
  HIPCHK(hipMemcpyAsync(ctx->f, f_dev, m.sum_ns * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (o->start == FETI_START_GIVEN && lambda_dev)
    HIPCHK(hipMemcpyAsync(ctx->lam, lambda_dev, m.n_lambda * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    HIPCHK(hipMemsetAsync(ctx->lam, 0, m.n_lambda * sizeof(double), st));
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int rc = solve_refined(ctx, o, o->ir_max, stats);
  if (lambda_dev)
    HIPCHK(hipMemcpyAsync(lambda_dev, ctx->lam, m.n_lambda * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (u_dev) HIPCHK(hipMemcpyAsync(u_dev, ctx->u, m.sum_ns * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->u, ctx->u_save, m.sum_ns * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->f, ctx->f_save, m.sum_ns * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return rc;
}

int feti_get_solution(feti_ctx ctx, double* u_dev, double* lambda_dev) {
  if (!ctx) return FETI_EINVAL;
  if (ctx->state < 2) return fail(ctx, FETI_ESTATE, "no solution");
  DevMesh& m = ctx->dm;
  if (u_dev) HIPCHK(hipMemcpyAsync(u_dev, ctx->u, m.sum_ns * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  if (lambda_dev)
    HIPCHK(hipMemcpyAsync(lambda_dev, ctx->lam_prev, m.n_lambda * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return FETI_OK;
}

int feti_torn_residual(feti_ctx ctx, double* rho) {
  if (!ctx || !rho) return FETI_EINVAL;
  if (ctx->state < 3 || !ctx->have_prev) return fail(ctx, FETI_ESTATE, "torn_residual before a step");
  DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  // rf = f - K u - B^T lambda, cj = -B u for the last step's (u, lambda^n)
  torn_residual(ctx, ctx->f, ctx->u, ctx->lam_prev);
  launch_sumsq(m.sum_ns, ctx->rf, ctx->kpart, KMAX_NBLK, st);
  launch_sumsq(m.n_lambda, ctx->cj, ctx->kpart + KMAX_NBLK, KMAX_NBLK, st);
  launch_sumsq(m.sum_ns, ctx->f, ctx->kpart + 2 * KMAX_NBLK, KMAX_NBLK, st);
  HIPCHK(hipMemcpyAsync(ctx->h_kpart, ctx->kpart, 3 * KMAX_NBLK * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  double a = 0.0, b = 0.0, c = 0.0;
  for (int k = 0; k < KMAX_NBLK; ++k) {
    a += ctx->h_kpart[k];
    b += ctx->h_kpart[KMAX_NBLK + k];
    c += ctx->h_kpart[2 * KMAX_NBLK + k];
  }
  *rho = c > 0.0 ? std::sqrt((a + b) / c) : std::sqrt(a + b);
  return FETI_OK;
}

int feti_set_start(feti_ctx ctx, const double* lambda_dev) {
  if (!ctx || !lambda_dev) return FETI_EINVAL;
  if (ctx->state < 2) return fail(ctx, FETI_ESTATE, "set_start before assemble");
  HIPCHK(hipMemcpyAsync(ctx->lam_given, lambda_dev, ctx->dm.n_lambda * sizeof(double), hipMemcpyDeviceToDevice,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return FETI_OK;
}

int feti_state_size(feti_ctx ctx, int64_t* n_doubles) {
  if (!ctx || !n_doubles) return FETI_EINVAL;
  if (ctx->state < 2) return fail(ctx, FETI_ESTATE, "state_size before assemble");
  *n_doubles = ctx->dm.sum_ns + 3 * ctx->dm.n_lambda;
  if (ctx->dm.decoupled) *n_doubles += 3 * (int64_t)ctx->mh.n1 * ctx->mh.n1;  // eta, p, xi_P on the lattice
  return FETI_OK;
}

int feti_get_state(feti_ctx ctx, double* state_dev, int64_t* meta) {
  if (!ctx || !state_dev || !meta) return FETI_EINVAL;
  if (ctx->state < 2) return fail(ctx, FETI_ESTATE, "get_state before assemble");
  const DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  double* o = state_dev;
  HIPCHK(hipMemcpyAsync(o, ctx->u, m.sum_ns * sizeof(double), hipMemcpyDeviceToDevice, st));
  o += m.sum_ns;
  HIPCHK(hipMemcpyAsync(o, ctx->lam_prev, m.n_lambda * sizeof(double), hipMemcpyDeviceToDevice, st));
  o += m.n_lambda;
  HIPCHK(hipMemcpyAsync(o, ctx->lam_prev2, m.n_lambda * sizeof(double), hipMemcpyDeviceToDevice, st));
  o += m.n_lambda;
  HIPCHK(hipMemcpyAsync(o, ctx->dlam_prev, m.n_lambda * sizeof(double), hipMemcpyDeviceToDevice, st));
  o += m.n_lambda;
  if (m.decoupled) {
    const size_t n1n = (size_t)ctx->mh.n1 * ctx->mh.n1;
    for (const double* src : {(const double*)ctx->dec_eta, (const double*)ctx->dec_p, (const double*)ctx->dec_xi}) {
      HIPCHK(hipMemcpyAsync(o, src, n1n * sizeof(double), hipMemcpyDeviceToDevice, st));
      o += n1n;
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  meta[0] = ctx->nstep;
  meta[1] = ctx->have_prev ? 1 : 0;
  meta[2] = ctx->have_prev2 ? 1 : 0;
  meta[3] = ctx->have_dlam_prev ? 1 : 0;
  return FETI_OK;
}

int feti_set_state(feti_ctx ctx, const double* state_dev, const int64_t* meta) {
  if (!ctx || !state_dev || !meta) return FETI_EINVAL;
  if (ctx->state < 2) return fail(ctx, FETI_ESTATE, "set_state before assemble");
  if (meta[0] < 0 || meta[1] < 0 || meta[1] > 1 || meta[2] < 0 || meta[2] > 1 || meta[3] < 0 || meta[3] > 1 ||
      (meta[2] && !meta[1]))
    return fail(ctx, FETI_EINVAL, "inconsistent state flags");
  const DevMesh& m = ctx->dm;
  hipStream_t st = ctx->stream;
  const double* i = state_dev;
  HIPCHK(hipMemcpyAsync(ctx->u, i, m.sum_ns * sizeof(double), hipMemcpyDeviceToDevice, st));
  i += m.sum_ns;
  HIPCHK(hipMemcpyAsync(ctx->lam_prev, i, m.n_lambda * sizeof(double), hipMemcpyDeviceToDevice, st));
  i += m.n_lambda;
  HIPCHK(hipMemcpyAsync(ctx->lam_prev2, i, m.n_lambda * sizeof(double), hipMemcpyDeviceToDevice, st));
  i += m.n_lambda;
  HIPCHK(hipMemcpyAsync(ctx->dlam_prev, i, m.n_lambda * sizeof(double), hipMemcpyDeviceToDevice, st));
  i += m.n_lambda;
  if (m.decoupled) {
    const size_t n1n = (size_t)ctx->mh.n1 * ctx->mh.n1;
    for (double* dst : {ctx->dec_eta, ctx->dec_p, ctx->dec_xi}) {
      HIPCHK(hipMemcpyAsync(dst, i, n1n * sizeof(double), hipMemcpyDeviceToDevice, st));
      i += n1n;
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  ctx->nstep = meta[0];
  ctx->have_prev = meta[1] != 0;
  ctx->have_prev2 = meta[2] != 0;
  ctx->have_dlam_prev = meta[3] != 0;
  return FETI_OK;
}

int feti_get_field(feti_ctx ctx, int32_t field, double* out_dev) {
  if (!ctx || !out_dev) return FETI_EINVAL;
  if (ctx->state < 2) return fail(ctx, FETI_ESTATE, "get_field before assemble");
  const MeshHost& h = ctx->mh;
  if (field < FETI_FIELD_UX || field > FETI_FIELD_UZ || (field == FETI_FIELD_UZ && h.dim != 3))
    return fail(ctx, FETI_EINVAL, "unknown field");
  const DevMesh& m = ctx->dm;
  const bool ufield = field <= FETI_FIELD_UY || field == FETI_FIELD_UZ;
  const int64_t nlat = ufield ? h.n_u_lat : h.n_p1_lat;
  launch_zero(nlat, out_dev, ctx->stream);
  if (m.decoupled && (field == FETI_FIELD_ETA || field == FETI_FIELD_P))
    launch_dec_field(m, field == FETI_FIELD_ETA ? ctx->dec_eta : ctx->dec_p, out_dev, ctx->stream);
  else
    launch_field_scatter(m, ctx->u, field, out_dev, ctx->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return FETI_OK;
}

int feti_interface_load(feti_ctx ctx, const feti_load* load, double* out_dev) {
  if (!ctx || !load || !out_dev) return FETI_EINVAL;
  if (ctx->state < 2) return fail(ctx, FETI_ESTATE, "interface_load before assemble");
  if (ctx->mh.dim == 3) return fail(ctx, FETI_EINVAL, "interface_load is 2D only");
  launch_interface_load(ctx->dm, make_load(ctx, load), out_dev, ctx->stream);
  HIPCHK(hipGetLastError());
  return FETI_OK;
}

int feti_export_local(feti_ctx ctx, int32_t sub, int32_t which, double* out) {
  if (!ctx || !out) return FETI_EINVAL;
  if (ctx->state < 2 || (which != FETI_EXPORT_K && ctx->state < 3))
    return fail(ctx, FETI_ESTATE, "export before the stage that produces it");
  if (sub < 0 || sub >= (int)ctx->mh.subs.size()) return fail(ctx, FETI_EINVAL, "bad subdomain");
  const MeshHost& h = ctx->mh;
  int64_t ko = 0, so = 0;
  for (int s = 0; s < sub; ++s) {
    ko += (int64_t)h.subs[s].ns * round8(h.subs[s].ns);
    so += (int64_t)h.subs[s].nb * round8(h.subs[s].nb);
  }
  const SubHost& sh = h.subs[sub];
  if (which == FETI_EXPORT_K && (!ctx->K || (!ctx->keep_assembled && ctx->state >= 3)))
    return fail(ctx, FETI_ESTATE, "the assembled matrices were eliminated in place");
  if (which == FETI_EXPORT_KPLUS && !(ctx->precision == FETI_FP32_IR ? (void*)ctx->Kinv32 : (void*)ctx->Kinv))
    return fail(ctx, FETI_ESTATE, "factors eliminated in place are kept as packed tiles only");
  if (which != FETI_EXPORT_K && ctx->precision == FETI_FP32_IR) {
    // FP32 factors: widen the block to FP64 on the way out
    const bool sbb = which == FETI_EXPORT_SBB;
    const int64_t nn = sbb ? sh.nb : sh.ns;
    const int64_t ldv = round8(nn);
    const float* src = sbb ? ctx->Sbb32 + so : ctx->Kinv32 + ko;
    float* tmp32 = nullptr;
    HIPCHK(hipMalloc(&tmp32, nn * nn * sizeof(float)));
    hipError_t e = hipMemcpy2DAsync(tmp32, nn * sizeof(float), src, ldv * sizeof(float), nn * sizeof(float), nn,
                                    hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess) launch_to_f64(nn * nn, tmp32, out, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(tmp32);
    if (e != hipSuccess) return fail(ctx, FETI_EHIP, hipGetErrorString(e));
    return FETI_OK;
  }
  if (which == FETI_EXPORT_SBB) {
    HIPCHK(hipMemcpy2DAsync(out, sh.nb * sizeof(double), ctx->Sbb + so, round8(sh.nb) * sizeof(double),
                            sh.nb * sizeof(double), sh.nb, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    const double* src = which == FETI_EXPORT_K ? ctx->K : ctx->Kinv;
    HIPCHK(hipMemcpy2DAsync(out, sh.ns * sizeof(double), src + ko, round8(sh.ns) * sizeof(double),
                            sh.ns * sizeof(double), sh.ns, hipMemcpyDeviceToDevice, ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return FETI_OK;
}

int feti_apply_F(feti_ctx ctx, const double* x, double* y) {
  if (!ctx || !x || !y) return FETI_EINVAL;
  if (ctx->state < 3) return fail(ctx, FETI_ESTATE, "apply_F before factor_subdomains");
  op_F(ctx, x, y, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return FETI_OK;
}

int feti_apply_precond(feti_ctx ctx, const double* x, double* y) {
  if (!ctx || !x || !y) return FETI_EINVAL;
  if (ctx->state < 3) return fail(ctx, FETI_ESTATE, "apply_precond before factor_subdomains");
  op_M(ctx, x, y, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return FETI_OK;
}

int feti_apply_F_noalloc(feti_ctx ctx, const double* x, double* y) {
  if (!ctx || !x || !y) return FETI_EINVAL;
  if (ctx->state < 3) return fail(ctx, FETI_ESTATE, "apply_F_noalloc before factor_subdomains");
  DevMesh& m = ctx->dm;
  // scratch: the interface-space products, then (dual-primal coupling) the primal
  // right-hand side and solution of the coarse step
  const int64_t npi = ctx->dp ? m.n_pi : 0;
  if (m.sum_nb + 2 * npi > FETI_NOALLOC_SCRATCH)
    return fail(ctx, FETI_EINVAL, "interface space larger than the static scratch");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != ctx->device) return fail(ctx, FETI_EINVAL, "apply_F_noalloc called with another device current");
  double* yb = nullptr;
  RC(noalloc_scratch(ctx, dev, &yb));
  GemvArgs a;
  const Factors fc = factors(ctx);
  a.A = fc.splus; a.a_f32 = fc.f32; a.aofs = m.sofs; a.lda = m.ldb; a.which_n = 1;
  a.v = x; a.gmode = G_SIGNED; a.gcoef = 1.0; a.y = yb;
  // every entry of the scratch that a later kernel reads is written before it (the primal
  // rows by the first product, the dual rows by the second)
  if (npi > 0) {
    double* cpi = yb + m.sum_nb;
    double* upi = cpi + npi;
    a.rsel = 2; a.csel = 1;
    launch_sgemv(m, a, ctx->stream);
    launch_pi_gather(m, nullptr, nullptr, yb, 1.0, cpi, nullptr, ctx->stream);
    launch_coarse_apply(m.n_pi, ctx->Spinv, cpi, upi, 1.0, nullptr, ctx->stream);
    a.pi_mode = 1; a.pi_v = upi; a.rsel = 1; a.csel = 0;
  }
  launch_sgemv(m, a, ctx->stream);
  launch_jump(m, yb, 0, y, 0, nullptr, nullptr, ctx->stream);
  HIPCHK(hipGetLastError());
  return FETI_OK;
}

int feti_get_rhs(feti_ctx ctx, double* f_dev) {
  if (!ctx || !f_dev) return FETI_EINVAL;
  if (ctx->state < 2) return fail(ctx, FETI_ESTATE, "no right-hand side");
  HIPCHK(hipMemcpyAsync(f_dev, ctx->f, ctx->dm.sum_ns * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return FETI_OK;
}

int feti_time_kernel(feti_ctx ctx, int32_t which, int32_t reps, double* avg_ms, double* work) {
  if (!ctx || !avg_ms || !work) return FETI_EINVAL;
  if (ctx->state < 3) return fail(ctx, FETI_ESTATE, "time_kernel before factor_subdomains");
  if (which < 0 || which > 3 || reps < 1) return fail(ctx, FETI_EINVAL, "bad kernel id");
  DevMesh& m = ctx->dm;
  const MeshHost& h = ctx->mh;
  hipStream_t st = ctx->stream;
  double w = 0.0;
  if (which == FETI_KERNEL_ELIMINATION) {
    if (!ctx->keep_assembled) return fail(ctx, FETI_ESTATE, "in-place factors cannot be recomputed");
    // factor again; the figure is the time between the events around the elimination
    // kernels (pivots, panel rows, updates, panel writes, snapshot, finalisation) only
    RC(feti_factor_subdomains(ctx, ctx->precision, ctx->precond));
    for (const SubHost& sh : h.subs) w += (double)sh.ns * sh.ns * sh.ns;
    *avg_ms = ctx->t_gj_ms;
    *work = w;
    return FETI_OK;
  } else {
    GemvArgs a;
    const Factors fc = factors(ctx);
    const double esz = fc.f32 ? 4.0 : 8.0;  // bytes per matrix entry; vectors are FP64
    a.a_f32 = fc.f32;
    if (which == FETI_KERNEL_LOCAL_SOLVE) {
      a.A = fc.kinv; a.aofs = m.kofs; a.lda = m.ld; a.which_n = 0; a.xbase = ctx->f; a.y = ctx->ytmp;
      // with the packed tiles, the distinct entries of the symmetric K_s^+ are the work
      for (const SubHost& sh : h.subs)
        w += ctx->sym.P ? esz * 0.5 * sh.ns * (sh.ns + 1.0) + 16.0 * sh.ns : esz * sh.ns * sh.ns + 16.0 * sh.ns;
    } else {
      a.A = which == FETI_KERNEL_IFACE_GEMV ? fc.splus : fc.sbb;
      a.aofs = m.sofs; a.lda = m.ldb; a.which_n = 1; a.v = ctx->p;
      a.gmode = which == FETI_KERNEL_IFACE_GEMV ? G_SIGNED : G_SCALED; a.gcoef = 1.0;
      a.y = ctx->yb;
      for (const SubHost& sh : h.subs) w += esz * sh.nb * sh.nb + 16.0 * sh.nb;
    }
    const bool sym = which == FETI_KERNEL_LOCAL_SOLVE && ctx->sym.P;
    auto run = [&]() {
      if (sym) launch_sym_gemv(m, ctx->sym, ctx->f, ctx->ytmp, st);
      else launch_sgemv(m, a, st);
    };
    run();  // warm-up launch
    HIPCHK(hipEventRecord(ctx->ev[6], st));
    for (int i = 0; i < reps; ++i) run();
    HIPCHK(hipEventRecord(ctx->ev[7], st));
    HIPCHK(hipEventSynchronize(ctx->ev[7]));
  }
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, ctx->ev[6], ctx->ev[7]));
  *avg_ms = (double)ms / reps;
  *work = w;
  return FETI_OK;
}


int feti_set_pcg_mode(feti_ctx ctx, int32_t mode) {
  if (!ctx) return FETI_EINVAL;
  if (mode != FETI_PCG_AUTO && mode != FETI_PCG_GRAPH) return fail(ctx, FETI_EINVAL, "unknown PCG mode");
  ctx->pcg_mode = mode;
  return FETI_OK;
}

int feti_set_keep_assembled(feti_ctx ctx, int32_t keep) {
  if (!ctx) return FETI_EINVAL;
  if (ctx->state >= 3) return fail(ctx, FETI_ESTATE, "set_keep_assembled after factor_subdomains");
  ctx->keep_assembled = keep != 0;
  return FETI_OK;
}

}  // extern "C"

// ============================================================================
// Batches of independent problems

struct feti_batch_s {
  std::vector<feti_ctx> ctx;
  hipStream_t stream = nullptr;
  std::string err;
  int P = 0, f32 = 0, max_nb = 0;
  ProbArgs* d_main = nullptr;  // problem tables of the first solve (multipliers lam)
  ProbArgs* d_corr = nullptr;  // of the refinement corrections (multipliers dlam)
  int32_t *tile_prob = nullptr, *tile_sub = nullptr, *tile_row0 = nullptr;
  int32_t *row_prob = nullptr, *row_chunk = nullptr, *flt_prob = nullptr, *flt_f = nullptr;
  int ntile = 0, nrow = 0, nflt = 0;
  double *alpha = nullptr, *beta = nullptr, *rho = nullptr, *part = nullptr;
  int32_t *done = nullptr, *iters = nullptr, *status = nullptr, *ndone = nullptr, *cnt = nullptr;
  GridBarrier* bar = nullptr;
  int32_t* h_buf = nullptr;  // pinned: iterations and statuses of each launch of a step (2 P per slot)
  int nslot = 0;              // slots of h_buf
  int timed_slot = -1;        // launch of the current step timed for the autotuner
  int grid = 0;
  bool tuned = false;
  std::vector<int> cand;
  std::vector<double> cost;
  int trial = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<void*> allocs;
  // batched set-up, recovery and refinement residual: problem table (device, and the host
  // copy it was uploaded from), per-step values (device, and pinned staging) and launch
  // dimensions
  BProb* d_probs = nullptr;
  std::vector<BProb> h_probs;
  BStepVals* d_vals = nullptr;
  BStepVals* h_vals = nullptr;
  BDims dims;
  // the step captured as a graph (warm steps with a fixed grid), and the shape it holds
  bool use_graph = true;
  hipGraphExec_t gexec = nullptr;
  int g_nref = -1, g_cand = -1, g_grid = 0;
  feti_solve_opts g_opts{};  // options whose values the captured launches hold
  bool last_graph = false;   // the last step ran as a graph launch
  bool dense_kplus = true;   // every problem keeps its dense K^+ (else the recovery reads packed tiles)
};

namespace {

int bfail(feti_batch b, int code, const std::string& msg) {
  if (b) b->err = msg;
  return code;
}

#define BCHK(expr)                                                                           \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) return bfail(b, FETI_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)
#define BRC(expr)                                                                       \
  do {                                                                                  \
    int _rc = (expr);                                                                   \
    if (_rc != FETI_OK) return _rc;                                                     \
  } while (0)

template <class T>
int balloc(feti_batch b, T** p, size_t count) {
  *p = nullptr;
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return bfail(b, FETI_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  b->allocs.push_back(*p);
  return FETI_OK;
}

template <class T>
int bupload(feti_batch b, T** p, const std::vector<T>& v) {
  BRC(balloc(b, p, v.size()));
  if (!v.empty()) BCHK(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return FETI_OK;
}

// One cooperative launch of the interface iterations of every problem (enqueued only;
// the step reads the results after its single synchronisation).  Its iterations and
// statuses go to slot `slot` of the pinned record.  tune: this launch may be timed for
// the autotuner (first solves of a warm step only, so that every candidate is timed on
// the same kind of work).
int run_batch(feti_batch b, bool corr, bool tune, int slot) {
  hipStream_t st = b->stream;
  // fill kernels instead of memsets, so that a captured step holds no memset nodes (the
  // finished count is allocated as two words, one double)
  static_assert(sizeof(GridBarrier) % sizeof(double) == 0, "the barrier is cleared as doubles");
  launch_zero(sizeof(GridBarrier) / sizeof(double), reinterpret_cast<double*>(b->bar), st);
  launch_zero(1, reinterpret_cast<double*>(b->ndone), st);
  BatchArgs a;
  a.probs = corr ? b->d_corr : b->d_main;
  a.P = b->P; a.f32 = b->f32;
  a.tile_prob = b->tile_prob; a.tile_sub = b->tile_sub; a.tile_row0 = b->tile_row0; a.ntile = b->ntile;
  a.row_prob = b->row_prob; a.row_chunk = b->row_chunk; a.nrow = b->nrow;
  a.flt_prob = b->flt_prob; a.flt_f = b->flt_f; a.nflt = b->nflt;
  a.alpha = b->alpha; a.beta = b->beta; a.rho = b->rho;
  a.done = b->done; a.iters = b->iters; a.status = b->status; a.ndone = b->ndone; a.bar = b->bar; a.cnt = b->cnt;
  a.max_nb = b->max_nb;
  const bool timed = !b->tuned && tune;
  const int grid = timed ? b->cand[b->trial % b->cand.size()] : (b->tuned ? b->grid : b->cand[0]);
  static const bool ptrace = std::getenv("FETI_PCG_TRACE") != nullptr;
  long long* ts = nullptr;
  const int nts = 64;
  if (ptrace) {
    // diagnostics (host-launched steps only): block 0's clock after every barrier
    BCHK(hipMalloc(&ts, nts * 12 * sizeof(long long)));
    launch_zero(nts * 12, reinterpret_cast<double*>(ts), st);
    a.tstamp = ts;
    a.tstamp_iters = nts;
  }
  if (timed) BCHK(hipEventRecord(b->e0, st));
  BCHK(launch_pcg_batch(a, grid, st));
  if (timed) {
    BCHK(hipEventRecord(b->e1, st));
    b->timed_slot = slot;
  }
  if (ptrace) {
    std::vector<long long> h(nts * 12);
    BCHK(hipMemcpyAsync(h.data(), ts, h.size() * sizeof(long long), hipMemcpyDeviceToHost, st));
    BCHK(hipStreamSynchronize(st));
    (void)hipFree(ts);
    int rate_khz = 0, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
    constexpr int np = 7;
    double sum[np] = {0};
    int cnt = 0;
    std::string per_it;
    for (int it = 0; it < nts; ++it) {
      if (h[it * 12 + np] == 0) break;
      const long long s0 = it == 0 ? h[0] : h[(it - 1) * 12 + np];
      for (int k = 0; k < np; ++k) sum[k] += (double)(h[it * 12 + k + 1] - (k > 0 ? h[it * 12 + k] : s0));
      if (rate_khz > 0) per_it += " " + std::to_string((int)((h[it * 12 + np] - s0) * 1e3 / rate_khz));
      ++cnt;
    }
    if (cnt > 0 && rate_khz > 0) {
      const double us = 1e3 / rate_khz / cnt;
      std::fprintf(stderr, "[pcg batch] grid %d, %d iterations, us per phase (A B C D E F G):", grid, cnt);
      for (int k = 0; k < np; ++k) std::fprintf(stderr, " %.1f", sum[k] * us);
      std::fprintf(stderr, "\n[pcg batch] us per iteration:%s\n", per_it.c_str());
    }
  }
  int32_t* rec = b->h_buf + (size_t)slot * 2 * b->P;
  BCHK(hipMemcpyAsync(rec, b->iters, b->P * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  BCHK(hipMemcpyAsync(rec + b->P, b->status, b->P * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  return FETI_OK;
}

// After the step's synchronisation: each problem's iterations and worst status over the
// step's launches, and the autotuner's record of a timed launch.
int collect_batch(feti_batch b, int nlaunch, std::vector<feti_stats>& acc) {
  const int P = b->P;
  for (int k = 0; k < nlaunch; ++k) {
    const int32_t* rec = b->h_buf + (size_t)k * 2 * P;
    for (int p = 0; p < P; ++p) {
      acc[p].iters += rec[p];
      if (k == 0) acc[p].iters_first = rec[p];
      if (rec[P + p] != 0 && acc[p].status == 0) acc[p].status = rec[P + p];
    }
  }
  if (b->timed_slot >= 0) {
    // autotuner: time per iteration-problem of each candidate grid, each timed twice on
    // the first solve of a warm step, then keep the best
    const int32_t* rec = b->h_buf + (size_t)b->timed_slot * 2 * P;
    int64_t total = 0;
    for (int p = 0; p < P; ++p) total += rec[p];
    b->timed_slot = -1;
    float ms = 0.f;
    BCHK(hipEventElapsedTime(&ms, b->e0, b->e1));
    b->cost[b->trial % b->cand.size()] += ms / (double)std::max<int64_t>(total, 1);
    b->trial += 1;
    if (b->trial >= (int)b->cand.size() * 2) {
      int best = 0;
      for (int k = 1; k < (int)b->cand.size(); ++k)
        if (b->cost[k] < b->cost[best]) best = k;
      b->grid = b->cand[best];
      b->tuned = true;
    }
  }
  return FETI_OK;
}

// The problem table of the batched launches from the contexts' current buffers.
BProb prob_of(feti_ctx c) {
  BProb a;
  const Factors fc = factors(c);
  a.m = c->dm;
  a.mpP = c->mpP;
  a.mpE = c->mpE;
  a.kinv = fc.kinv;
  a.splus = fc.splus;
  a.sbb = c->precond == FETI_PRECOND_LUMPED ? (const void*)c->Kbb : fc.sbb;
  a.f32 = fc.f32;
  a.sym = c->sym;
  a.H = c->H;
  a.Cinv = c->Cinv;
  a.nc = c->nc;
  a.mdiag = c->mdiag;
  double** v = a.v;
  v[BV_U] = c->u; v[BV_F] = c->f; v[BV_D] = c->d; v[BV_YTMP] = c->ytmp; v[BV_LAM] = c->lam; v[BV_DLAM] = c->dlam;
  v[BV_R] = c->r; v[BV_W] = c->w; v[BV_Z] = c->z; v[BV_Y] = c->y; v[BV_P] = c->p; v[BV_Q] = c->q;
  v[BV_YB] = c->yb; v[BV_ZB] = c->zb; v[BV_G] = c->g; v[BV_GD] = c->gd; v[BV_GQ] = c->gq; v[BV_AC] = c->ac;
  v[BV_TL] = c->tl; v[BV_RF] = c->rf; v[BV_CJ] = c->cj; v[BV_DU] = c->du; v[BV_LAMP] = c->lam_prev;
  v[BV_LAMP2] = c->lam_prev2; v[BV_DLAMP] = c->dlam_prev; v[BV_DLAMS] = c->dlam_sum; v[BV_LALT] = c->lam_alt;
  v[BV_RALT] = c->r_alt; v[BV_WALT] = c->w_alt;
  a.sc = c->sc;
  a.ist = c->ist;
  a.part = c->part;
  return a;
}

// Uploads the problem table again when a context's buffers have moved since the last
// upload (a single-problem step swaps the multiplier histories).
int sync_probs(feti_batch b) {
  bool same = (int)b->h_probs.size() == b->P;
  std::vector<BProb> now(b->P);
  for (int p = 0; p < b->P; ++p) {
    now[p] = prob_of(b->ctx[p]);
    const BProb& o = b->h_probs.empty() ? now[p] : b->h_probs[p];
    if (same)
      same = std::memcmp(now[p].v, o.v, sizeof(o.v)) == 0 && now[p].kinv == o.kinv && now[p].splus == o.splus &&
             now[p].sbb == o.sbb && now[p].f32 == o.f32 && now[p].H == o.H && now[p].Cinv == o.Cinv &&
             now[p].mdiag == o.mdiag && now[p].m.ebuf == o.m.ebuf && now[p].m.emat == o.m.emat &&
             now[p].sym.P == o.sym.P && now[p].sym.f32 == o.sym.f32;
  }
  if (same) return FETI_OK;
  b->h_probs = now;
  BCHK(hipMemcpyAsync(b->d_probs, b->h_probs.data(), b->P * sizeof(BProb), hipMemcpyHostToDevice, b->stream));
  BCHK(hipStreamSynchronize(b->stream));  // the host table may change before the next step
  return FETI_OK;
}

// Batched form of torn_begin (the projection through H = G (G^T G)^{-1}, which every
// problem of a batch has): d = sum_s B_s K_s^+ f_s - c, the admissible start, r, w = P r,
// the tolerance references from P d, z = M^{-1} w, y = P z, p = y and rho = (w, y).  With
// cand, the first correction compares the previous step's total correction as a start
// (problems whose step values have cand = 0 keep their own start).
void btorn_begin(feti_batch b, double tol, double utol, int maxit, int f, int cj, int lam, int cand) {
  const BProb* P = b->d_probs;
  const BDims& d = b->dims;
  hipStream_t st = b->stream;
  const int f32 = b->f32;
  // K^+ f from the packed tiles (every factored context has them)
  launchb_sym_gemv(P, d, 0, f, BV_NONE, 0.0, BV_NONE, BV_NONE, BV_YTMP, f32, st);
  launchb_jump(P, d, BV_YTMP, 1, BV_D, 0, BV_NONE, st);
  if (cj != BV_NONE) launchb_axpby(P, d, BL_LAMBDA, 1.0, BV_D, -1.0, cj, BV_D, st);
  auto admissible = [&](int v) {
    launchb_coarse_g(P, d, v, f, -1.0, BV_G, st);
    launchb_coarse_apply(P, d, BV_G, BV_AC, 1.0, st);
    launchb_coarse_correct(P, d, BV_AC, 1.0, v, v, st);
  };
  admissible(lam);
  launchb_coarse_g(P, d, BV_D, BV_NONE, 1.0, BV_GD, st);
  auto start_rw = [&](int v, int r, int w) {
    BGemv a;
    a.mat = BM_SPLUS; a.full = 0; a.v = v; a.gmode = G_SIGNED; a.gcoef = 1.0; a.y = BV_YB;
    launchb_sgemv(P, d, a, f32, st);
    launchb_jump(P, d, BV_YB, 0, BV_Q, 0, BV_NONE, st);
    launchb_axpby(P, d, BL_LAMBDA, 1.0, BV_D, -1.0, BV_Q, r, st);
    launchb_coarse_g(P, d, r, BV_NONE, 1.0, BV_GQ, st);
    launchb_h_project(P, d, r, BV_NONE, BV_GQ, BV_NONE, w, BV_NONE, BV_NONE, st);
  };
  start_rw(lam, BV_R, BV_W);
  if (cand != BV_NONE) {
    launchb_axpby(P, d, BL_LAMBDA, 1.0, cand, 0.0, BV_NONE, BV_LALT, st);
    admissible(BV_LALT);
    start_rw(BV_LALT, BV_RALT, BV_WALT);
    launchb_reduce(P, d, BV_NONE, BV_NONE, BV_W, PH_REFNORM, st);
    launchb_copy_scalar(P, d, SC_EREF, SC_SEL0, st);
    launchb_reduce(P, d, BV_NONE, BV_NONE, BV_WALT, PH_REFNORM, st);
    launchb_copy_scalar(P, d, SC_EREF, SC_SEL1, st);
    launchb_pick_start(P, b->d_vals, d, BV_LALT, lam, BV_RALT, BV_R, BV_WALT, BV_W, st);
  }
  launchb_init_scalars(P, d, tol, utol, std::max(maxit, 0), st);
  launchb_h_project(P, d, BV_D, BV_NONE, BV_GD, BV_NONE, BV_TL, BV_NONE, BV_NONE, st);
  launchb_reduce(P, d, BV_NONE, BV_NONE, BV_TL, PH_REFNORM, st);
  BGemv m;
  m.mat = BM_SBB; m.full = 0; m.v = BV_W; m.gmode = G_SCALED; m.gcoef = 1.0; m.y = BV_ZB;
  launchb_sgemv(P, d, m, f32, st);
  launchb_jump(P, d, BV_ZB, 0, BV_Z, 1, BV_GQ, st);
  launchb_h_project(P, d, BV_Z, BV_NONE, BV_GQ, BV_NONE, BV_Y, BV_NONE, BV_P, st);
  launchb_reduce(P, d, BV_W, BV_Y, BV_W, PH_INIT, st);
}

// Batched torn_end: alpha_c = -(G^T G)^{-1} G^T r and u = K^+ f - K^+ B^T lam + R alpha_c,
// with K^+ f still in ytmp.
void btorn_end(feti_batch b, int lam, int u) {
  const BProb* P = b->d_probs;
  const BDims& d = b->dims;
  hipStream_t st = b->stream;
  launchb_coarse_g(P, d, BV_R, BV_NONE, 1.0, BV_G, st);
  launchb_coarse_apply(P, d, BV_G, BV_AC, -1.0, st);
  if (!b->dense_kplus) {
    launchb_sym_gemv(P, d, 1, BV_NONE, lam, -1.0, BV_YTMP, BV_AC, u, b->f32, st);
    return;
  }
  BGemv g;
  g.mat = BM_KINV; g.full = 1; g.kb_only = 1; g.ybase = BV_YTMP; g.v = lam; g.gmode = G_SIGNED; g.gcoef = -1.0;
  g.y = u; g.alpha_c = BV_AC;
  launchb_sgemv(P, d, g, b->f32, st);
}

// Batched torn_residual: rf = f - K u - B^T lam, cj = -sum_s B_s u_s.
void btorn_residual(feti_batch b) {
  const BProb* P = b->d_probs;
  const BDims& d = b->dims;
  hipStream_t st = b->stream;
  launchb_elem_matvec(P, d, BV_U, BV_YTMP, st);
  launchb_axpby(P, d, BL_TORN, 1.0, BV_F, -1.0, BV_YTMP, BV_RF, st);
  launchb_sub_gather(P, d, BV_LAM, BV_RF, st);
  launchb_jump(P, d, BV_U, 1, BV_CJ, 0, BV_NONE, st);
  launchb_axpby(P, d, BL_LAMBDA, -1.0, BV_CJ, 0.0, BV_NONE, BV_CJ, st);
}

}  // namespace

extern "C" {

int feti_batch_create(feti_batch* out, feti_ctx* ctxs, int32_t nprob) {
  if (!out || !ctxs || nprob < 1) return FETI_EINVAL;
  *out = nullptr;
  feti_batch b = new feti_batch_s();
  // on failure the message goes to the first context (there is no batch handle)
  auto bad = [&](int rc, const std::string& msg) {
    for (void* p : b->allocs) (void)hipFree(p);
    if (b->h_buf) (void)hipHostFree(b->h_buf);
    if (b->h_vals) (void)hipHostFree(b->h_vals);
    delete b;
    if (ctxs[0] && !msg.empty()) ctxs[0]->err = "feti_batch_create: " + msg;
    return rc == FETI_OK ? FETI_EINVAL : rc;
  };
  b->P = nprob;
  for (int p = 0; p < nprob; ++p) {
    feti_ctx c = ctxs[p];
    if (!c || c->state < 3) return bad(FETI_ESTATE, "batch of contexts that are not factored");
    if (c->stream != ctxs[0]->stream)
      return bad(FETI_EINVAL, "batch contexts on different streams (create them on one non-default stream)");
    if (c->precision != ctxs[0]->precision) return bad(FETI_EINVAL, "batch contexts of different precision");
    if (c->precond == FETI_PRECOND_NONE) return bad(FETI_EINVAL, "batch needs a preconditioner");
    if (c->nc > PCG_NC_LOCAL) return bad(FETI_EINVAL, "coarse space too large for a batch");
    if (c->dm.decoupled) return bad(FETI_EINVAL, "a batch steps the coupled scheme only");
    if (c->dp) return bad(FETI_EINVAL, "a batch takes the dual coupling only");
    b->ctx.push_back(c);
  }
  b->stream = ctxs[0]->stream;
  b->f32 = ctxs[0]->precision == FETI_FP32_IR;
  std::vector<int32_t> tp, ts, tr, rp, rcn, fp, ff;
  std::vector<ProbArgs> pm(nprob), pc(nprob);
  std::vector<int64_t> part_off(nprob);
  int64_t npart = 0;
  for (int p = 0; p < nprob; ++p) {
    feti_ctx c = ctxs[p];
    const MeshHost& h = c->mh;
    for (int s = 0; s < (int)h.subs.size(); ++s)
      for (int r0 = 0; r0 < h.subs[s].nb; r0 += 64) { tp.push_back(p); ts.push_back(s); tr.push_back(r0); }
    const int nri = (int)((c->dm.n_lambda + PCG_BLOCK - 1) / PCG_BLOCK);
    for (int k = 0; k < nri; ++k) { rp.push_back(p); rcn.push_back(k); }
    if (c->nc > 0)
      for (int f = 0; f < c->dm.n_float; ++f) { fp.push_back(p); ff.push_back(f); }
    b->max_nb = std::max(b->max_nb, c->dm.max_nb);
    part_off[p] = npart;
    npart += (int64_t)nri * PCG_NPART;
    ProbArgs& a = pm[p];
    const Factors fc = factors(c);
    a.m = c->dm;
    a.fm = fc.splus;
    a.mm = c->precond == FETI_PRECOND_LUMPED ? (const void*)c->Kbb : fc.sbb;
    if (c->precond == FETI_PRECOND_LUMPED && b->f32) return bad(FETI_EINVAL, "lumped preconditioner in a FP32 batch");
    a.Cinv = c->Cinv; a.nc = c->nc; a.nrow_items = nri;
    a.lam = c->lam; a.r = c->r; a.w = c->w; a.z = c->z; a.y = c->y; a.p = c->p; a.q = c->q; a.qraw = c->qraw;
    a.yb = c->yb; a.zb = c->zb; a.g = c->g; a.mdiag = c->mdiag; a.sc = c->sc; a.ist = c->ist;
    pc[p] = a;
    pc[p].lam = c->dlam;
  }
  b->ntile = (int)tp.size(); b->nrow = (int)rp.size(); b->nflt = (int)fp.size();
  int rc = FETI_OK;
  if ((rc = balloc(b, &b->part, npart))) return bad(rc, "");
  for (int p = 0; p < nprob; ++p) { pm[p].part = b->part + part_off[p]; pc[p].part = pm[p].part; }
  if ((rc = bupload(b, &b->d_main, pm)) || (rc = bupload(b, &b->d_corr, pc)) ||
      (rc = bupload(b, &b->tile_prob, tp)) || (rc = bupload(b, &b->tile_sub, ts)) ||
      (rc = bupload(b, &b->tile_row0, tr)) || (rc = bupload(b, &b->row_prob, rp)) ||
      (rc = bupload(b, &b->row_chunk, rcn)) || (rc = bupload(b, &b->flt_prob, fp)) ||
      (rc = bupload(b, &b->flt_f, ff)) || (rc = balloc(b, &b->alpha, nprob)) || (rc = balloc(b, &b->beta, nprob)) ||
      (rc = balloc(b, &b->rho, nprob)) || (rc = balloc(b, &b->done, nprob)) || (rc = balloc(b, &b->iters, nprob)) ||
      (rc = balloc(b, &b->status, nprob)) || (rc = balloc(b, &b->ndone, 2)) || (rc = balloc(b, &b->bar, 1)) ||
      (rc = balloc(b, &b->cnt, 3 * nprob)))
    return bad(rc, "");
  b->nslot = 8;
  if (hipHostMalloc((void**)&b->h_buf, (size_t)b->nslot * 2 * nprob * sizeof(int32_t), hipHostMallocDefault) !=
      hipSuccess)
    return bad(FETI_ENOMEM, "");
  // batched launches: table, per-step values, dimensions and GEMV work items
  {
    BDims& d = b->dims;
    d.P = nprob;
    std::vector<int32_t> fi, ii, yi, ki, si;
    for (int p = 0; p < nprob; ++p) {
      feti_ctx c = ctxs[p];
      const DevMesh& m = c->dm;
      const int64_t nl = m.n_lambda;
      d.nl_blk = std::max(d.nl_blk, (int)((nl + 255) / 256));
      d.nl64_blk = std::max(d.nl64_blk, (int)((nl + 63) / 64));
      d.ns_blk = std::max(d.ns_blk, (int)((m.sum_ns + 255) / 256));
      d.nb_blk = std::max(d.nb_blk, (int)((m.sum_nb + 255) / 256));
      d.red_blk = std::max(d.red_blk, (int)std::max<int64_t>(1, std::min<int64_t>((nl + RED_BLOCK - 1) / RED_BLOCK,
                                                                                   RED_NBLK)));
      d.nflt = std::max(d.nflt, c->nc > 0 ? m.n_float : 0);
      d.nc_blk = std::max(d.nc_blk, (c->nc + 3) / 4);
      d.elem_blk = std::max(d.elem_blk, (m.nelem + 127) / 128);
      d.erow_blk = std::max(d.erow_blk, (int)(((int64_t)m.nelem * m.edof + 255) / 256));
      d.max_ns = std::max(d.max_ns, m.max_ns);
      const MeshHost& h = c->mh;
      for (int s = 0; s < (int)h.subs.size(); ++s) {
        for (int t = 0; t * 64 < h.subs[s].ns; ++t) { fi.push_back(p); fi.push_back(s); fi.push_back(t); }
        for (int t = 0; t * 64 < h.subs[s].nb; ++t) { ii.push_back(p); ii.push_back(s); ii.push_back(t); }
        for (int t = 0; t * 256 < h.subs[s].ns; ++t) { si.push_back(p); si.push_back(s); si.push_back(t); }
      }
      if (!c->sym.P) return bad(FETI_ESTATE, "a context of the batch has no packed factors");
      std::vector<int32_t> kb;
      sym_tiles(h, nullptr, nullptr, nullptr, nullptr, nullptr, &kb, nullptr);
      if ((int)kb.size() != c->sym.n_kb_tiles) return bad(FETI_EINVAL, "packed tile tables out of step");
      for (int t = 0; t < c->sym.ntile; ++t) { yi.push_back(p); yi.push_back(t); }
      for (int32_t t : kb) { ki.push_back(p); ki.push_back(t); }
      if (!factors(c).kinv) b->dense_kplus = false;
    }
    int32_t *dfi = nullptr, *dii = nullptr, *dyi = nullptr, *dki = nullptr, *dsi = nullptr;
    if ((rc = bupload(b, &dfi, fi)) || (rc = bupload(b, &dii, ii)) || (rc = bupload(b, &dyi, yi)) ||
        (rc = bupload(b, &dki, ki)) || (rc = bupload(b, &dsi, si)) || (rc = balloc(b, &b->d_probs, nprob)) ||
        (rc = balloc(b, &b->d_vals, nprob)))
      return bad(rc, "");
    d.full_items = dfi;
    d.iface_items = dii;
    d.n_full_items = (int)(fi.size() / 3);
    d.n_iface_items = (int)(ii.size() / 3);
    d.sym_items = dyi;
    d.sym_kb_items = dki;
    d.sum_items = dsi;
    d.n_sym_items = (int)(yi.size() / 2);
    d.n_sym_kb_items = (int)(ki.size() / 2);
    d.n_sum_items = (int)(si.size() / 3);
    if (hipHostMalloc((void**)&b->h_vals, nprob * sizeof(BStepVals), hipHostMallocDefault) != hipSuccess)
      return bad(FETI_ENOMEM, "");
  }
  if (hipEventCreate(&b->e0) != hipSuccess || hipEventCreate(&b->e1) != hipSuccess) return bad(FETI_EHIP, "");
  const int maxg = pcg_batch_max_grid(b->max_nb);
  (void)hipGetLastError();
  if (maxg < 1) return bad(FETI_EHIP, "cooperative launch unavailable for the batch kernel");
  if (std::getenv("FETI_TRACE")) {
    char desc[256];
    pcg_batch_describe(b->max_nb, desc, sizeof(desc));
    std::fprintf(stderr, "[batch] %d problems, largest n_b %d, %zu bytes of LDS per block, co-resident grid %d; %s\n",
                 nprob, b->max_nb, pcg_batch_shmem(b->max_nb), maxg, desc);
  }
  int cus = 0, dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  for (int g : {cus / 2, cus, 2 * cus, 3 * cus, 4 * cus})
    if (g >= 1 && g <= maxg && std::find(b->cand.begin(), b->cand.end(), g) == b->cand.end()) b->cand.push_back(g);
  if (b->cand.empty()) b->cand.push_back(maxg);
  b->cost.assign(b->cand.size(), 0.0);
  b->grid = b->cand[0];
  *out = b;
  return FETI_OK;
}

int feti_batch_destroy(feti_batch b) {
  if (!b) return FETI_EINVAL;
  (void)hipStreamSynchronize(b->stream);
  for (void* p : b->allocs) (void)hipFree(p);
  if (b->h_buf) (void)hipHostFree(b->h_buf);
  if (b->h_vals) (void)hipHostFree(b->h_vals);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->e0) (void)hipEventDestroy(b->e0);
  if (b->e1) (void)hipEventDestroy(b->e1);
  delete b;
  return FETI_OK;
}

const char* feti_batch_last_error(feti_batch b) { return b ? b->err.c_str() : "null batch"; }

int feti_batch_set_grid(feti_batch b, int32_t grid) {
  if (!b || grid < 0) return FETI_EINVAL;
  if (grid == 0) {
    b->tuned = false;
    b->trial = 0;
    b->cost.assign(b->cand.size(), 0.0);
    return FETI_OK;
  }
  const int maxg = pcg_batch_max_grid(b->max_nb);
  if (grid > maxg) return bfail(b, FETI_EINVAL, "grid larger than the co-resident maximum");
  b->grid = grid;
  b->tuned = true;
  return FETI_OK;
}

int feti_batch_info(feti_batch b, int32_t* info) {
  if (!b || !info) return FETI_EINVAL;
  info[0] = b->tuned ? b->grid : b->cand[b->trial % b->cand.size()];
  info[1] = b->tuned ? 1 : 0;
  info[2] = (int32_t)std::min<size_t>(b->cand.size(), 8);
  for (int k = 0; k < 8; ++k) info[3 + k] = k < info[2] ? b->cand[k] : 0;
  info[11] = b->last_graph ? 1 : 0;
  return FETI_OK;
}

int feti_batch_step(feti_batch b, const feti_load* loads, const feti_solve_opts* o, feti_stats* stats) {
  if (!b || !loads || !o) return FETI_EINVAL;
  if (!(o->tol > 0.0) || o->max_it < 1 || o->corr_start < FETI_CORR_ZERO || o->corr_start > FETI_CORR_PREVIOUS)
    return bfail(b, FETI_EINVAL, "bad solve options");
  if (o->start == FETI_START_GIVEN || o->start == FETI_START_BEST)
    return bfail(b, FETI_EINVAL, "a batch step starts from the previous, extrapolated or zero multipliers");
  const int P = b->P;
  std::vector<feti_stats> acc(P);
  for (auto& s : acc) std::memset(&s, 0, sizeof(s));
  hipStream_t st = b->stream;
  BRC(sync_probs(b));
  // per-problem step values: the load, the start of the first solve, the warm correction
  bool cold = false, any_cand = false;
  for (int p = 0; p < P; ++p) {
    feti_ctx ctx = b->ctx[p];
    BStepVals& v = b->h_vals[p];
    v.L = make_load(ctx, &loads[p]);
    int used = o->start;
    if (o->start == FETI_START_ZERO || !ctx->have_prev) {
      v.a_prev = 0.0; v.b_prev2 = 0.0;
      used = FETI_START_ZERO;
    } else if (o->start == FETI_START_EXTRAPOLATE && ctx->have_prev2) {
      v.a_prev = 2.0; v.b_prev2 = -1.0;
    } else {
      v.a_prev = 1.0; v.b_prev2 = 0.0;
      used = FETI_START_PREVIOUS;
    }
    v.cand = o->corr_start == FETI_CORR_PREVIOUS && ctx->have_dlam_prev ? 1 : 0;
    any_cand = any_cand || v.cand;
    acc[p].start_used = used;
    cold = cold || !ctx->have_prev;
  }
  const int nref = cold ? std::max(o->ir_cold, o->ir_max) : o->ir_max;
  const int nlaunch = 1 + std::max(nref, 0);
  if (nlaunch > b->nslot) {
    // a larger record of the launches (a captured step refers to the old one)
    BCHK(hipStreamSynchronize(st));
    int32_t* nb = nullptr;
    if (hipHostMalloc((void**)&nb, (size_t)nlaunch * 2 * P * sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
      return bfail(b, FETI_ENOMEM, "pinned record of the batch launches");
    (void)hipHostFree(b->h_buf);
    b->h_buf = nb;
    b->nslot = nlaunch;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  // The work of the step, in stream order (no host synchronisation inside).
  auto enqueue = [&]() -> int {
    const BProb* PT = b->d_probs;
    const BDims& dm = b->dims;
    BCHK(hipMemcpyAsync(b->d_vals, b->h_vals, P * sizeof(BStepVals), hipMemcpyHostToDevice, st));
    launchb_rhs(PT, b->d_vals, dm, st);
    launchb_start(PT, b->d_vals, dm, st);
    btorn_begin(b, o->tol, 0.0, o->max_it, BV_F, BV_NONE, BV_LAM, BV_NONE);
    BRC(run_batch(b, false, !cold, 0));
    btorn_end(b, BV_LAM, BV_U);
    for (int k = 0; k < nref; ++k) {
      btorn_residual(b);
      launchb_axpby(PT, dm, BL_LAMBDA, 0.0, BV_NONE, 0.0, BV_NONE, BV_DLAM, st);
      btorn_begin(b, o->tol_corr, o->tol_upd, o->max_it, BV_RF, BV_CJ, BV_DLAM,
                  k == 0 && any_cand ? BV_DLAMP : BV_NONE);
      BRC(run_batch(b, true, false, 1 + k));
      btorn_end(b, BV_DLAM, BV_DU);
      launchb_axpby(PT, dm, BL_TORN, 1.0, BV_U, 1.0, BV_DU, BV_U, st);
      launchb_axpby(PT, dm, BL_LAMBDA, 1.0, BV_LAM, 1.0, BV_DLAM, BV_LAM, st);
      launchb_axpby(PT, dm, BL_LAMBDA, 1.0, BV_DLAM, k == 0 ? 0.0 : 1.0, k == 0 ? BV_NONE : BV_DLAMS, BV_DLAMS, st);
    }
    // histories: this step's total correction, and lam_prev2 <- lam_prev <- lam
    if (nref > 0) launchb_axpby(PT, dm, BL_LAMBDA, 1.0, BV_DLAMS, 0.0, BV_NONE, BV_DLAMP, st);
    launchb_axpby(PT, dm, BL_LAMBDA, 1.0, BV_LAMP, 0.0, BV_NONE, BV_LAMP2, st);
    launchb_axpby(PT, dm, BL_LAMBDA, 1.0, BV_LAM, 0.0, BV_NONE, BV_LAMP, st);
    BCHK(hipGetLastError());
    return FETI_OK;
  };
  BCHK(hipEventRecord(b->ctx[0]->ev[0], st));
  // A warm step with a fixed grid runs as one graph launch; the graph is captured at the
  // first such step and again when the step's shape (corrections, warm correction start,
  // grid) changes.  The per-step values enter through the pinned staging copy it holds.
  const bool graph = b->use_graph && b->tuned && !cold && !std::getenv("FETI_PCG_TRACE");
  if (graph) {
    const int gc = any_cand ? 1 : 0;
    if (b->gexec && (b->g_nref != nref || b->g_cand != gc || b->g_grid != b->grid ||
                     std::memcmp(&b->g_opts, o, sizeof(*o)) != 0)) {
      (void)hipGraphExecDestroy(b->gexec);
      b->gexec = nullptr;
    }
    if (!b->gexec) {
      hipGraph_t g = nullptr;
      BCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      const int rc = enqueue();
      hipGraph_t gcap = nullptr;
      const hipError_t e = hipStreamEndCapture(st, &gcap);
      g = gcap;
      if (rc != FETI_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return bfail(b, FETI_EHIP, std::string("capture of the batch step: ") + hipGetErrorString(e));
      const hipError_t ei = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        b->gexec = nullptr;
        return bfail(b, FETI_EHIP, std::string("instantiation of the batch step: ") + hipGetErrorString(ei));
      }
      b->g_nref = nref;
      b->g_cand = gc;
      b->g_grid = b->grid;
      std::memcpy(&b->g_opts, o, sizeof(*o));
    }
    BCHK(hipGraphLaunch(b->gexec, st));
  } else {
    BRC(enqueue());
  }
  b->last_graph = graph;
  BCHK(hipEventRecord(b->ctx[0]->ev[5], st));
  BCHK(hipStreamSynchronize(st));
  BRC(collect_batch(b, nlaunch, acc));
  for (int p = 0; p < P; ++p) {
    feti_ctx ctx = b->ctx[p];
    ctx->have_dlam_prev = nref > 0;
    ctx->have_prev2 = ctx->have_prev;
    ctx->have_prev = true;
    ctx->nstep += 1;
    acc[p].ir_steps = nref;
  }
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, b->ctx[0]->ev[0], b->ctx[0]->ev[5]);
  int worst = FETI_OK;
  for (int p = 0; p < P; ++p) {
    acc[p].t_ms[5] = ms;
    if (acc[p].status != 0 && worst == FETI_OK) worst = acc[p].status;
    if (stats) stats[p] = acc[p];
  }
  if (worst != FETI_OK) return bfail(b, worst, "a problem of the batch did not converge");
  return FETI_OK;
}

int feti_batch_set_capture(feti_batch b, int32_t on) {
  if (!b) return FETI_EINVAL;
  b->use_graph = on != 0;
  if (!b->use_graph && b->gexec) {
    (void)hipStreamSynchronize(b->stream);
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  return FETI_OK;
}


}  // extern "C"
