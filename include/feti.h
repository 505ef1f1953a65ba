/*
 * feti.h -- C ABI of the MI355X FETI solver for the coupled poroelasticity /
 * elasticity model (Ge & Wang, arXiv 2509.06673).
 *
 * The library computes, for every backward-Euler step, the discrete solution
 * of the block system of eq. (linalg-system) (Section 2.5): the poroelastic
 * region carries (u, xi_P, eta, p) on P_k-P1-P1-P1 elements, the elastic region
 * (u, xi_E) on P_k-P1 elements, and a Lagrange multiplier glues the two
 * (Section 2.3, Problem 2).  The system is torn into subdomains and solved by
 * the FETI method of Section 3: the interface problem F lambda = d (eq.
 * (feti-system) / (sim-feti)) is solved by projected preconditioned CG with
 * the Dirichlet preconditioner of eq. (feti_dirichlet_preconditioner), after
 * which the subdomain fields are recovered (proof of Theorem 3.1).
 *
 * Conventions
 *  - Every function returns FETI_OK (0) or a negative FETI_E* code; the text of
 *    the last error of a context is returned by feti_last_error().
 *  - Pointers named *_dev are device pointers (HIP global memory, for example
 *    the data_ptr() of a torch tensor on cuda:0).  Pointers named *_host are
 *    host pointers.  Every pointer argument is owned by the caller; no call
 *    retains or frees caller memory.  Device buffers written by the library
 *    are written on the context's stream (stream-ordered): synchronise that
 *    stream before reading them on the host.
 *  - Calls follow create -> setup_mesh -> assemble -> factor_subdomains ->
 *    {step | solve}* -> destroy; a call out of this order returns FETI_ESTATE.
 *  - One context is used by one host thread at a time.
 *  - DOF numbering.  A DOF is identified by code = 8 * node + kind with kind
 *    0 ux, 1 uy (node on the displacement lattice of spacing h/k), 2 eta,
 *    3 xi_P, 4 p, 5 xi_E (node on the P1 lattice of spacing h); lattices are
 *    row-major with x fastest.  Each subdomain lists its DOFs in the order
 *    [interior U | interior P | interface U | interface P | fixed] (U = u, eta;
 *    P = xi, p), each block sorted by (field u, eta, xi, p; node; component).
 *    "Torn" vectors concatenate the subdomain vectors in subdomain order.
 */
#ifndef FETI_H
#define FETI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct feti_ctx_s* feti_ctx;

enum {
    FETI_OK = 0,
    FETI_EINVAL = -1,       /* bad argument or unsupported configuration */
    FETI_ESTATE = -2,       /* call out of order */
    FETI_ENOMEM = -3,       /* device or host allocation failed */
    FETI_EHIP = -4,         /* a HIP runtime call failed */
    FETI_ESINGULAR = -5,    /* zero or non-finite pivot in the local elimination */
    FETI_ENOTCONV = -6,     /* PCG hit max_it; the best iterate is still written */
    FETI_EBREAKDOWN = -7,   /* PCG denominator vanished; the iterate is still written */
    FETI_ENAN = -8          /* non-finite value in a load or in the iteration */
};

/* layouts of the poroelastic region in the unit square */
enum { FETI_XSPLIT = 0, FETI_YSPLIT = 1, FETI_CORE = 2 };
/* load kinds of feti_load */
enum { FETI_LOAD_MANUFACTURED = 0, FETI_LOAD_PERIODIC = 1, FETI_LOAD_POINT_SOURCE = 2,
       FETI_LOAD_PATCH = 3, FETI_LOAD_RAW = 4 };
/* precision of the subdomain factors: FP64, or FP32 elimination on the matrix
 * cores with FP32 storage of K_s^+, S_bb and the interface block, the FP64 torn
 * residual and FP64 interface vectors, dot products and coarse problem winning
 * the accuracy back by refinement (feti_solve_opts.ir_*) */
enum { FETI_FP64 = 0, FETI_FP32_IR = 1 };
/* preconditioner (Section 3.1 Dirichlet; Section 3.2 lumped) */
enum { FETI_PRECOND_DIRICHLET = 0, FETI_PRECOND_LUMPED = 1, FETI_PRECOND_NONE = 2 };
/* start vector of the interface iteration */
enum { FETI_START_PREVIOUS = 0, FETI_START_ZERO = 1, FETI_START_EXTRAPOLATE = 2,
       FETI_START_GIVEN = 3,
       /* the start set by feti_set_start (e.g. a learned prediction, feti_ws.h) if its
        * projected residual w = P (d - F lambda), made admissible, is smaller in the
        * dual-energy norm of the stopping test than that of the previous-step start */
       FETI_START_BEST = 4 };

/* Mesh and decomposition (Section 2.4 spaces on a structured right-triangle
 * mesh of the unit square; subdomains are an nsub_x x nsub_y grid of cell
 * blocks with cuts at floor(a * ncell / nsub_x), or at the caller's cuts). */
typedef struct {
    int32_t ncell;        /* cells per side, h = 1/ncell */
    int32_t order_u;      /* k of P_k for the displacement: 1 or 2 */
    int32_t layout;       /* FETI_XSPLIT | FETI_YSPLIT | FETI_CORE */
    int32_t nsub_x, nsub_y;
    uint32_t dirichlet_u; /* bit 0: x=0, 1: x=1, 2: y=0, 3: y=1 -- sides with u Dirichlet */
    uint32_t dirichlet_p; /* sides with p Dirichlet (where the poroelastic region touches them) */
    const int32_t* cut_x; /* host, nsub_x + 1 cell indices 0 = c_0 < c_1 < ... < c_nsub_x = ncell
                             (subdomain column a covers cells [c_a, c_a+1)); NULL = even cuts.
                             Read during feti_setup_mesh only.  FETI_EINVAL if not strictly
                             increasing from 0 to ncell, or if a subdomain straddles the
                             interface of the layout. */
    const int32_t* cut_y; /* the same for the rows */
    int32_t scheme;       /* FETI_SCHEME_COUPLED (eq. (linalg-system) at once) or
                             FETI_SCHEME_DECOUPLED (the explicit fluid step of the Remark
                             after eq. (linalg-system); see feti_step) */
    int32_t coupling;     /* FETI_COUPLING_DUAL or FETI_COUPLING_PRIMAL (below) */
    int32_t dim;          /* 2 (or 0): the unit square in triangles; 3: the unit cube in
                             tetrahedra (Section 2 allows d = 2, 3), see below */
    int32_t nsub_z;       /* 3D: subdomains along z */
} feti_mesh_desc;

/* d = 3: the unit cube, ncell^3 cubes each cut into the six Kuhn tetrahedra around its
 * main diagonal (vertices v0, v0 + h e_a, v0 + h (e_a + e_b), v0 + h (1, 1, 1) for the
 * axis permutations (a, b, c)), P_k displacement (k = 1, 2; P2 nodes at the vertices and
 * edge midpoints) and P1 scalars; poroelastic for x < 1/2 (layout FETI_XSPLIT only);
 * nsub_x x nsub_y x nsub_z subdomains at the even cuts (cut_x, cut_y NULL; nsub_x even);
 * lattices x fastest, then y, then z; DOF kinds as in 2D plus uz = 6; outer faces bit 0:
 * x = 0, 1: x = 1, 2: y = 0, 3: y = 1, 4: z = 0, 5: z = 1.  Takes the dual-primal
 * coupling, the coupled scheme and loads of kind FETI_LOAD_RAW (nodal body forces,
 * source, Dirichlet and initial data on the cube lattices: f_p, f_e, g_u of 3 x mu^3
 * doubles, z, g_p, eta0 of n1^3; no side data, t_side and zw_side NULL); FETI_EINVAL
 * otherwise. */

/* Gluing of the shared DOFs.  DUAL: every shared DOF is torn and glued by multipliers
 * (Section 3.1); the interface operator F is symmetric but indefinite, with one negative
 * eigenvalue per multiplier of xi_P, p or xi_E.  PRIMAL (dual-primal, the FETI-DP
 * structure that the Introduction cites for three-field Biot): the shared xi_P, p and xi_E
 * DOFs and every shared DOF at a corner of the subdomain grid (on a vertical and a
 * horizontal cut line, outer sides included) are global primal unknowns, and multipliers
 * glue only the other shared DOFs (u and eta on the cut edges).  With K~ the partially
 * assembled matrix (primal DOFs summed over their owners), F = B K~^{-1} B^T is
 * symmetric positive definite, no subdomain floats (n_c = 0), and every application of F
 * solves the primal coarse problem S_PiPi = K~_PiPi - K~_Pir K~_rr^{-1} K~_rPi (dense,
 * inverted once by feti_factor_subdomains).  The solution is the same (Theorem 3.1's
 * equivalence).  With more than one subdomain the iteration is deflated by one
 * normal-flux vector per face-sharing subdomain pair (feti_export_deflation).  PRIMAL
 * takes FETI_FP64 factors and single contexts (no batches), and both schemes in 2D (under
 * FETI_SCHEME_DECOUPLED the subdomains carry (u, xi) only, so xi and the grid corners are
 * primal and multipliers glue u); FETI_EINVAL from feti_setup_mesh if a subdomain without
 * Dirichlet data has fewer than two primal displacement nodes. */
enum { FETI_COUPLING_DUAL = 0, FETI_COUPLING_PRIMAL = 1 };

/* Time discretisation of a step.  DECOUPLED: the fluid content and the pressure leave the
 * subdomain unknowns, so a poroelastic subdomain carries (u_P, xi_P) like an elastic one
 * (u_E, xi_E) and no multiplier glues eta or p.  Each step first updates the fluid content
 * explicitly with the lumped mass and the previous pressure, m_i (eta^n_i - eta^{n-1}_i) =
 * tau (Z^n - A_f p^{n-1})_i (at pressure Dirichlet nodes eta^n = (p_D - k1 xi^{n-1}) / k2),
 * then solves the momentum balance with eta^n known, and sets p^n = k1 xi^n + k2 eta^n
 * nodally (p_D on Dirichlet nodes).  Explicit, hence stable for tau below the explicit
 * diffusion limit of the consolidation operator and for alpha^2 < c0 lambda_P. */
enum { FETI_SCHEME_COUPLED = 0, FETI_SCHEME_DECOUPLED = 1 };

/* Parameters of Table 2 for one region; lame_mode 0: mu = E/(2(1+nu)),
 * 1: mu = E/(1+nu) as printed in Table 3. */
typedef struct {
    double E, nu, alpha, c0, K, mu_f;
    int32_t lame_mode;
} feti_material;

/* Loads.  MANUFACTURED: the smooth solution of Section 4.1 (rotated to the
 * layout); PATCH: the polynomial solution (coefficients in params[0..13]:
 * ux(1,x,y,x^2,xy,y^2), uy(...), p(1,y)); PERIODIC: body force
 * amp sin(omega t + phase) (sin(pi x) sin(pi y), cos(pi x) sin(pi y)) and
 * source amp sin(omega t + phase) sin(pi x) sin(pi y), params = {amp, omega,
 * phase}; POINT_SOURCE: source sin(t) * Gaussian(centre, sigma) of unit
 * integral, params = {cx, cy, sigma}.  t is the time of the step. */
typedef struct {
    int32_t kind;
    double t;
    double params[16];
    /* FETI_LOAD_RAW: the caller's data of the step at time t, on the lattices (device
     * pointers, caller-owned, read during the call; NULL = zero data).  They enter as
     * the nodal interpolants in the finite element spaces:
     *   F_u = (f_h, theta) + <t_h, theta> on the sides without u Dirichlet data
     *         (eqs. (vf1), (vf4); the traction of BCTR / BCTRE),
     *   Z   = (z_h, phi) + <z_w,h, phi> on the poroelastic edges of the sides without p
     *         Dirichlet data (eq. (vf3); the flux of BCFR, entering with the sign of the
     *         weak form),
     * Dirichlet values g_u, g_p at the Dirichlet nodes, and eta^0 (feti_init_state).
     * mu = k ncell + 1 displacement lattice points per side, n1 = ncell + 1; lattices
     * row-major with x fastest; sides 0: x = 0, 1: x = 1, 2: y = 0, 3: y = 1, indexed
     * along the side by the lattice y index (x = const) or x index (y = const). */
    const double* f_p;     /* [2][mu*mu] body force used on poroelastic elements */
    const double* f_e;     /* [2][mu*mu] body force used on elastic elements */
    const double* z;       /* [n1*n1] fluid source */
    const double* t_side;  /* [2][4][2][mu] traction [region 0 P / 1 E][side][component][along] */
    const double* zw_side; /* [4][n1] flux data [side][along] */
    const double* g_u;     /* [2][mu*mu] displacement Dirichlet values */
    const double* g_p;     /* [n1*n1] pressure Dirichlet values */
    const double* eta0;    /* [n1*n1] initial fluid content (read by feti_init_state) */
} feti_load;

enum { FETI_CORR_ZERO = 0, FETI_CORR_PREVIOUS = 1 };

typedef struct {
    double tol;           /* interface tolerance of a solve, e.g. 1e-10, on w = P (d - F lambda):
                             |w_k| <= tol max(|P d|_k, |w^(0)|_k) for every constrained field
                             kind k (u, eta, xi_P, p, xi_E jumps) that carries load data, and
                             the dual-energy norm (sum_j |M_jj| w_j^2)^(1/2), M the Dirichlet
                             preconditioner, <= tol times its reference */
    double tol_corr;      /* interface tolerance of each refinement correction (e.g. 1e-2) */
    double ir_tol;        /* refinement stops once max_k |du_k|_inf / |u_k|_inf <= ir_tol */
    int32_t max_it;       /* PCG iteration cap per solve */
    int32_t start;        /* FETI_START_* */
    int32_t check_every;  /* iterations between host convergence checks (>= 1) */
    int32_t ir_max;       /* refinement corrections on a step with previous multipliers */
    int32_t ir_cold;      /* refinement corrections on a step without them */
    double tol_inner;     /* with FETI_FP32_IR factors: tolerance of the first solve of a step
                             (its operators carry FP32 rounding, so a tighter first solve buys
                             nothing that the FP64 corrections do not redo); 0 = tol */
    double tol_upd;       /* update test of the refinement corrections (0 = off): a correction
                             also stops once, for every field kind k with nonzero multipliers,
                             its last three updates |alpha| |p|_k sum to at most
                             tol_upd |dlambda|_k (e.g. 3e-3).  A correction only has to shrink
                             the first solve's error by a few orders, and its noise-driven
                             residual keeps wandering long after its solution has settled.
                             Every kind counts, also those whose correction is tiny: at
                             nu -> 1/2 the pressure p = kappa_1 xi + kappa_2 eta magnifies the
                             error of the xi and eta multipliers. */
    int32_t corr_start;   /* start of the first refinement correction of a step:
                             FETI_CORR_ZERO, or FETI_CORR_PREVIOUS = the previous step's total
                             correction (the rounding that the corrections undo comes from the
                             same factors applied to a slowly varying load), kept only if its
                             projected residual is smaller than the zero start's.  Any other
                             value: FETI_EINVAL. */
} feti_solve_opts;

typedef struct {
    int32_t iters;        /* PCG iterations (summed over refinement corrections) */
    int32_t iters_first;  /* PCG iterations of the first solve of the step */
    int32_t ir_steps;     /* refinement corrections performed */
    int32_t status;       /* FETI_OK or the failure code */
    int32_t start_used;   /* FETI_START_* actually used */
    double res0, res;     /* max over kinds of the relative interface residual, start / end */
    double rho;           /* size of the last refinement correction, max_k |du_k|/|u_k| (0 if none) */
    double t_ms[8];       /* phase times (ms): rhs, d + start, pcg, recovery, refinement, total */
    int32_t iters_corr[4]; /* PCG iterations of the first four refinement corrections */
    int32_t corr_warm;    /* 1: the first correction started from the previous step's correction
                             (feti_step only; a batch chooses on the device and reports 0) */
} feti_stats;

/* ---- lifetime ---------------------------------------------------------- */

/* Create a context bound to hip_stream (a hipStream_t, NULL = default stream).
 * No device memory is touched until feti_assemble. */
int feti_create(feti_ctx* out, void* hip_stream);
int feti_destroy(feti_ctx ctx);
const char* feti_last_error(feti_ctx ctx);

/* ---- setup (Sections 2.4 and 3.1) ------------------------------------------ */

/* Build the lattice, the subdomains, their local DOF orders, the signed Boolean
 * jump rows and the rigid modes of floating subdomains (host only). */
int feti_setup_mesh(feti_ctx ctx, const feti_mesh_desc* mesh);

/* sizes: [0] n_sub, [1] sum n_s, [2] N_lambda, [3] n_c (coarse size),
 * [4] max n_s, [5] max n_b, [6] sum n_b, [7] P1 lattice size, [8] u lattice size,
 * [9] n_floating, [10] number of primal unknowns (dual-primal coupling, else 0) */
int feti_get_sizes(feti_ctx ctx, int64_t* sizes_host);

/* Bit-exact export of the numbering (host buffers):
 * local_code[sum n_s]: DOF code of each local DOF, torn order;
 * sub_offset[n_sub+1]: start of each subdomain in torn order;
 * sub_nb[n_sub]: interface (b) size; the b DOFs are the trailing ones;
 * brow_sub/brow_local/brow_sign[2*N_lambda]: the two entries of each jump row. */
int feti_export_indexing(feti_ctx ctx, int32_t* local_code_host, int32_t* sub_offset_host,
                         int32_t* sub_nb_host, int32_t* brow_sub_host,
                         int32_t* brow_local_host, int8_t* brow_sign_host);

/* Dual-primal coupling (FETI_COUPLING_PRIMAL; host buffers): primal_code[n_primal] the
 * code of every primal unknown in global order (field order u, eta, xi, p, then node,
 * then kind: the U-type corners first), sub_npi[n_sub] the number of primal DOFs of each
 * subdomain, which are the trailing ones of its interface block.  Either may be NULL. */
int feti_export_primal(feti_ctx ctx, int32_t* primal_code_host, int32_t* sub_npi_host);

/* Dual-primal coupling: the normal-flux vectors that deflate the interface iteration, one
 * per pair of subdomains sharing a face (an edge in 2D).  Column c holds, on each
 * multiplier row of that pair whose DOF is the displacement component normal to the
 * face, the integral over the face of that node's basis function in units of the element
 * size (h in 2D, the face triangle area h^2 / 2 in 3D), so that q_c^T B u is the integral
 * of the jump of u . n across the face (sign of the rows).  The start of a solve takes the
 * residual's component in their span exactly, and every search direction is made
 * F-orthogonal to them.  A row belongs to at most two columns (a row of a 3D grid edge,
 * where the jump between two face neighbours is the sum of chained rows):
 * col_host[2 * N_lambda] and w_host[2 * N_lambda] hold two (column, weight) slots per row
 * (column -1: unused); n_defl_host receives the number of columns.  Any pointer may be
 * NULL. */
int feti_export_deflation(feti_ctx ctx, int32_t* col_host, double* w_host, int32_t* n_defl_host);

/* Element-parallel assembly of every dense local matrix K_s (rows 1-4 or 5-6
 * of eq. (linalg-system) restricted to the subdomain's elements, Dirichlet
 * DOFs removed).  tau is the time step. */
int feti_assemble(feti_ctx ctx, const feti_material* mat_p, const feti_material* mat_e,
                  double tau);

/* Batched local elimination: pivot-free symmetric Gauss-Jordan sweeps of each
 * K_s in its [I | b] order (the LDL^T pivots of Theorem 3.1's reduction), which
 * snapshots the interface Schur complement S_bb of eq. (reduced-system) after
 * the interior pivots and ends with the generalised inverse K_s^+ (fixed DOFs
 * of floating subdomains zeroed).  Also builds the coarse matrix G^T G.
 * precision: FETI_FP64 | FETI_FP32_IR; precond: FETI_PRECOND_*. */
int feti_factor_subdomains(feti_ctx ctx, int32_t precision, int32_t precond);

/* Memory: keep the assembled K_s after the elimination (keep = 1, the default) or
 * eliminate in place (keep = 0): the dense storage of the context halves, and K_s
 * can then neither be exported after feti_factor_subdomains nor eliminated again.
 * Call before feti_factor_subdomains. */
int feti_set_keep_assembled(feti_ctx ctx, int32_t keep);

/* How the interface iteration runs: FETI_PCG_AUTO (default) runs every iteration of
 * a solve in one cooperative persistent launch when the device allows it and the
 * coarse space is small enough, else replays graph-captured chunks of the kernel
 * chain of an iteration; FETI_PCG_GRAPH always takes the graph chain.  Both follow
 * Algorithms 1 and 2 with the same stopping tests.  May be called at any time. */
enum { FETI_PCG_AUTO = 0, FETI_PCG_GRAPH = 1 };
int feti_set_pcg_mode(feti_ctx ctx, int32_t mode);

/* Diagnostic environment variables (read once per process; none changes a result beyond
 * rounding order):
 *   FETI_TRACE       per-solve iteration counts and residuals on stderr; takes the
 *                    host-driven kernel chain instead of the persistent launch;
 *   FETI_PCG_TRACE   per-phase clock stamps of the persistent launch on stderr (this
 *                    allocates a small device buffer per solve);
 *   FETI_NO_PERSIST  never the persistent launch (as FETI_PCG_GRAPH);
 *   FETI_NO_GRAPH    launch the kernel chain directly instead of replaying its graph;
 *   FETI_PCG_GRID    blocks of the persistent launch (clamped to what is co-resident). */

/* ---- time stepping ----------------------------------------------------------- */

/* Set eta^0 (the initial fluid content) from a load's initial data: nodal
 * interpolation of c0 p0 + alpha div u0 (eq. (mreform)), and reset the step
 * counter and the multiplier history. */
int feti_init_state(feti_ctx ctx, const feti_load* load);

/* One backward-Euler step at time load->t: right-hand side (eq.
 * (linalg-system) rows 1 and 4 with eta^{n-1}), interface PCG, recovery of all
 * fields, eta^n kept for the next step.  stats may be NULL. */
int feti_step(feti_ctx ctx, const feti_load* load, const feti_solve_opts* opts,
              feti_stats* stats);

/* Solve the torn system K_s u_s + B_s^T lam = f_s, sum_s B_s u_s = 0 for a
 * caller-given torn right-hand side (device, sum n_s doubles).  lambda_dev
 * (N_lambda doubles) is the start on input when opts->start is
 * FETI_START_GIVEN and the solution on output; u_dev receives the torn primal
 * solution.  The time-stepping state (eta^n, the multiplier history and the
 * right-hand side returned by feti_get_rhs) is left as it was, so solves may be
 * interleaved with steps; feti_get_solution still returns the last step's. */
int feti_solve(feti_ctx ctx, const double* f_dev, double* lambda_dev, double* u_dev,
               const feti_solve_opts* opts, feti_stats* stats);

/* Copy the torn primal solution of the last step (sum n_s doubles) and the
 * multipliers (N_lambda doubles) to device buffers; either may be NULL. */
int feti_get_solution(feti_ctx ctx, double* u_dev, double* lambda_dev);

/* Relative FP64 residual of the torn system of the last step (eq. (feti-system): the
 * local equations K_s u_s + B_s^T lambda = f_s and the gluing sum_s B_s u_s = 0):
 *   rho = |[f - K u - B^T lambda ; -B u]|_2 / |f|_2   (|...|_2 over all subdomains),
 * for the step's (u, lambda^n) as returned by feti_get_solution.  It is an a-posteriori
 * check of a solve, evaluated element by element in FP64; it leaves the step state as it
 * was.  *rho_host: host.  FETI_ESTATE before the first step.  Synchronises. */
int feti_torn_residual(feti_ctx ctx, double* rho_host);

/* ---- checkpoint / resume and field export ------------------------------------ */

/* The backward-Euler scheme of Section 2.5 carries eta^n from one step to the next
 * (row 4 of eq. (linalg-system) reads eta^{n-1}); the solver also carries the
 * multipliers lambda^n, lambda^{n-1} of the last two steps (starts of the interface
 * iteration) and the last step's total refinement correction.  The state is a flat
 * device vector of feti_state_size() doubles:
 *   [ torn primal solution of the last step (sum n_s; its eta entries are eta^n)
 *   | lambda^n (N_lambda) | lambda^{n-1} (N_lambda) | total correction (N_lambda) ]
 * followed, for FETI_SCHEME_DECOUPLED, by eta^n, p^n and xi_P^n on the P1 lattice (3 x
 * (n1)^2; the torn solution then has no eta entries)
 * and four host integers meta = {steps taken, have lambda^n, have lambda^{n-1},
 * have a correction}.  feti_set_state on a context built with the same mesh,
 * materials and time step continues the trajectory bit for bit: steps 1..10 equal
 * steps 1..5, get_state, set_state (on a fresh context) and steps 6..10.  Both
 * synchronise the context stream.  set_state returns FETI_EINVAL on flags that
 * are not 0/1 or on lambda^{n-1} without lambda^n. */
int feti_state_size(feti_ctx ctx, int64_t* n_doubles_host);
int feti_get_state(feti_ctx ctx, double* state_dev, int64_t* meta_host);
int feti_set_state(feti_ctx ctx, const double* state_dev, const int64_t* meta_host);

/* Fields of the last step on their global lattice (outputs u_h^n, xi_h^n, eta_h^n,
 * p_h^n of eq. (linalg-system)): field = DOF kind (FETI_FIELD_UX, UY on the
 * displacement lattice of spacing h/k, (u_lattice)^2 doubles; ETA, XI_P, P, XI_E on
 * the P1 lattice of spacing h, (n1)^2 doubles; sizes [8] and [7] of feti_get_sizes).
 * A node shared by several subdomains takes the value of the lowest-numbered one
 * (the copies agree to the interface tolerance); nodes that carry no unknown of the
 * field (Dirichlet nodes, nodes outside the field's region) are set to 0.  With
 * FETI_SCHEME_DECOUPLED, ETA and P are the explicit step's eta^n and p^n at every node of
 * the poroelastic region (p^n = p_D on pressure Dirichlet nodes).
 * out_dev: device, caller-owned.  Synchronises the context stream. */
enum { FETI_FIELD_UX = 0, FETI_FIELD_UY = 1, FETI_FIELD_ETA = 2, FETI_FIELD_XI_P = 3, FETI_FIELD_P = 4,
       FETI_FIELD_XI_E = 5, FETI_FIELD_UZ = 6 /* 3D */ };
int feti_get_field(feti_ctx ctx, int32_t field, double* out_dev);

/* Set the multiplier start of the next step (used with FETI_START_GIVEN and
 * FETI_START_BEST). */
int feti_set_start(feti_ctx ctx, const double* lambda_dev);

/* The load of a step sampled at the node of every multiplier row (N_lambda doubles,
 * device): the body force component of a displacement row (of the region of the
 * row's first subdomain), the source for an eta, xi_P or p row, 0 for a xi_E row.
 * These are the load features of the learned warm start (feti_ws.h). */
int feti_interface_load(feti_ctx ctx, const feti_load* load, double* out_dev);

/* ---- batches of independent problems -------------------------------------------- */

/* A batch of factored contexts (same stream, same precision, Dirichlet or lumped
 * preconditioner, at most 64 floating subdomains each) whose interface iterations
 * run in one cooperative launch per solve: the work of every problem is spread over
 * the whole chip, each problem keeps its own scalars and stopping test, and a
 * finished problem drops out of the launch.  The contexts stay owned by the caller
 * and must outlive the batch. */
typedef struct feti_batch_s* feti_batch;
int feti_batch_create(feti_batch* out, feti_ctx* ctxs, int32_t nprob);  /* failure text: feti_last_error(ctxs[0]);
                                                                          contexts of the coupled scheme only */
int feti_batch_destroy(feti_batch b);
const char* feti_batch_last_error(feti_batch b);

/* One backward-Euler step of every problem (loads[nprob], stats[nprob] may be NULL):
 * right-hand sides, interface solves and recovery as feti_step, with the previous-
 * step, extrapolated or zero start and a fixed number of refinement corrections
 * (opts->ir_max, or ir_cold on a problem's first step; tol_upd and corr_start as in
 * feti_step, the start of each problem chosen on the device). */
int feti_batch_step(feti_batch b, const feti_load* loads, const feti_solve_opts* opts, feti_stats* stats);

/* Launch shape: grid > 0 fixes the number of blocks; grid = 0 (the default) lets the
 * autotuner time candidate grids on the first launches and keep the fastest per
 * iteration.  info (12 entries): [0] grid in use, [1] 1 once the choice is final,
 * [2] candidates, [3..10] the candidate grids (up to 8, zero-padded), [11] 1 if the last
 * step ran as a captured graph (feti_batch_set_capture). */
int feti_batch_set_grid(feti_batch b, int32_t grid);
int feti_batch_info(feti_batch b, int32_t* info_host);

/* Graph capture of the batch step (on by default).  Once the grid is fixed (set, or
 * chosen by the autotuner), every warm step runs as one hipGraph launch: the step's
 * kernels, its cooperative interface launches and its copies, captured at the first such
 * step and captured again when the number of corrections, the warm correction start,
 * the grid or any solve option changes.  The loads and starts of each step enter through
 * a pinned staging copy that the graph reads when it runs.  on = 0 runs every step from
 * the host, launch by launch (same kernels, same order, same results). */
int feti_batch_set_capture(feti_batch b, int32_t on);

/* ---- inspection (unit parity of each stage) ------------------------------- */

/* Dense local matrix K_s, its S_bb snapshot and K_s^+ of subdomain sub, row
 * major into a device buffer of n_s*n_s (K, K^+) or n_b*n_b (S_bb) doubles.  Under the
 * dual-primal coupling KPLUS gives N_s = [[K_rr^{-1}, -K_rr^{-1} K_rPi], [-K_Pir K_rr^{-1},
 * -S_s]] (r: every DOF but the primal ones, S_s = K_PiPi - K_Pir K_rr^{-1} K_rPi). */
int feti_export_local(feti_ctx ctx, int32_t sub, int32_t which, double* out_dev);
enum { FETI_EXPORT_K = 0, FETI_EXPORT_SBB = 1, FETI_EXPORT_KPLUS = 2 };

/* y = F x (F = sum_s B_s K_s^+ B_s^T; dual-primal coupling: F = B K~^{-1} B^T with its
 * primal coarse solve) and y = M^{-1} x (Dirichlet preconditioner; dual-primal: the
 * Schur complements restricted to the dual DOFs) on device vectors of N_lambda doubles. */
int feti_apply_F(feti_ctx ctx, const double* x_dev, double* y_dev);
int feti_apply_precond(feti_ctx ctx, const double* x_dev, double* y_dev);

/* y = F x as feti_apply_F, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * interface-space products live in a static per-GPU device array of 2^20 doubles
 * (8 MiB, held by every GPU that loads the library until the process ends) instead of
 * the context's buffers, and the call neither allocates nor frees anything.  It is
 * stream-ordered on the context stream and does not synchronise.  The context must be
 * factored and its device current.  FETI_EINVAL when the interface space (sum_s n_b,s),
 * plus twice the primal count under the dual-primal coupling (its coarse step keeps the
 * primal right-hand side and solution there too), exceeds 2^20 entries or another device
 * is current.  Calls that overlap on one GPU
 * (several streams or host threads) share the array and race; the result is the same
 * as feti_apply_F's, bit for bit. */
int feti_apply_F_noalloc(feti_ctx ctx, const double* x_dev, double* y_dev);

/* Torn right-hand side of the last prepared step (sum n_s doubles). */
int feti_get_rhs(feti_ctx ctx, double* f_dev);

/* ---- measurement ------------------------------------------------------------ */

/* Launch one stage reps times back to back on the context stream between two
 * HIP events and report its average duration in ms and its algorithmic work
 * per launch: bytes for the GEMV stages (matrix entries read once plus the
 * vector traffic), flops for the elimination (sum_s n_s^3, the count of a
 * symmetric inversion).  The stage's outputs are the same as in a step, so a
 * context stays valid.  Requires a factored context. */
enum { FETI_KERNEL_LOCAL_SOLVE = 0,    /* y_s = K_s^+ f_s, every subdomain */
       FETI_KERNEL_IFACE_GEMV = 1,     /* y_b = (K_s^+)_bb B_s^T x: the F application */
       FETI_KERNEL_PRECOND_GEMV = 2,   /* y_b = S_bb (B^T D x)_s: the preconditioner */
       FETI_KERNEL_ELIMINATION = 3 };  /* the whole batched elimination (reps forced to 1) */
int feti_time_kernel(feti_ctx ctx, int32_t which, int32_t reps, double* avg_ms_host,
                     double* work_host);

#ifdef __cplusplus
}
#endif
#endif /* FETI_H */
