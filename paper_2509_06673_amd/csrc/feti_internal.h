// Internal data structures of the FETI library (host side).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/feti.h"

namespace feti {

// DOF kinds (code = 8 * node + kind)
enum Kind { K_UX = 0, K_UY = 1, K_ETA = 2, K_XIP = 3, K_P = 4, K_XIE = 5, K_UZ = 6 };  // K_UZ: 3D

// Categories of the local order [I_U | I_P | b_U | b_P | fixed]
enum Cat { C_IU = 0, C_IP = 1, C_BU = 2, C_BP = 3, C_FIX = 4 };

struct SubHost {
  int sid = 0;
  bool poro = false;
  bool floating = false;
  int i0 = 0, i1 = 0, j0 = 0, j1 = 0;  // cell range [i0, i1) x [j0, j1)
  int k0 = 0, k1 = 0;                   // 3D: cell range in z
  std::vector<int32_t> codes;          // local order
  std::vector<int8_t> cats;
  int ns = 0, nI = 0, nb = 0, nfix = 0;  // nb includes the fixed DOFs
  int64_t off = 0;                      // offset in torn vectors
  int64_t boff = 0;                     // offset in the concatenated interface space
};

// One jump row: two entries (subdomain, local index, sign)
struct JumpRow {
  int32_t sub[2];
  int32_t loc[2];
  int8_t sign[2];
  int32_t code;
  int32_t mult;   // number of subdomains sharing the DOF
  int32_t kind;
};

// owners of a primal DOF (a corner of the 3D subdomain grid has eight)
constexpr int PI_OWNERS = 8;

// Element DOF table: up to 21 DOFs per element in 2D, 42 in 3D (P2 tetrahedra)
constexpr int MAX_EDOF = 42;

struct MeshHost {
  feti_mesh_desc desc{};
  int dim = 2;               // 2: triangles on the unit square, 3: tetrahedra on the unit cube
  int ratio = 2;             // displacement lattice refinement (1 for P1, 2 for P2)
  int mu = 0;                // displacement lattice points per side
  int n1 = 0;                // P1 lattice points per side
  int64_t n_u_lat = 0, n_p1_lat = 0;  // lattice sizes (mu^dim, n1^dim)
  std::vector<SubHost> subs;
  std::vector<JumpRow> rows;
  // per-multiplier block of D = (B B^T)^{-1}: group start and size, row of D
  std::vector<int32_t> grp_start, grp_size;
  std::vector<double> dwt;   // 3 per row: D[j, grp_start + 0..2]
  int64_t sum_ns = 0, sum_nb = 0, n_lambda = 0;
  int max_ns = 0, max_nb = 0, n_float = 0;
  // element tables (all subdomains concatenated, subdomain-major)
  int edof = 0;              // DOFs per element (padded to the poro count)
  std::vector<int32_t> el_sub, el_cell, el_type;
  std::vector<int32_t> el_ldof;   // edof per element: local index or -1
  std::vector<int32_t> el_code;   // edof per element: DOF code (for Dirichlet lifting)
  std::vector<int32_t> sub_el_off;   // n_sub + 1
  // element contributions of every torn DOF, in element order: adj_ptr[sum_ns + 1],
  // adj[...] = e * edof + element row
  std::vector<int32_t> adj_ptr, adj;
  // gather lists per interface DOF (global b index): up to 2 (row, sign)
  std::vector<int32_t> bg_row;    // 2 per b DOF (-1 = none)
  std::vector<double> bg_sign;    // 2 per b DOF
  // scaled gather (B^T D): up to 3 (row, weight)
  std::vector<int32_t> bd_row;    // 3 per b DOF
  std::vector<double> bd_wt;      // 3 per b DOF
  // jump: per row, the two global b indices and signs
  std::vector<int32_t> jr_b;      // 2 per row
  std::vector<double> jr_sign;    // 2 per row
  // coarse space: per floating subdomain index f -> sub id; rigid modes on b
  std::vector<int32_t> float_sub;     // n_float
  std::vector<int32_t> sub_float;     // n_sub: index in float list or -1
  std::vector<double> rb;             // sum_nb x 3 (zero rows for non-floating subdomains)
  // rigid modes on all local DOFs (torn, 3 per DOF) for the recovery
  std::vector<double> rfull;
  // decoupled scheme: the P1 lattice nodes of the poroelastic region (increasing), per node
  // its (element, vertex) entries e * 3 + v over the poroelastic elements (element order,
  // CSR), whether it carries pressure Dirichlet data, and the torn index of its first
  // xi_P copy (lowest subdomain)
  std::vector<int32_t> dec_node, dec_ptr, dec_ent, dec_xi;
  std::vector<uint8_t> dec_pdir;
  // dual-primal coupling: the primal codes in global order (the first n_pi_u of U type),
  // per interface DOF its primal index (-1: dual or no coupling), per primal DOF the
  // interface indices of its owners (PI_OWNERS slots, -1 = none)
  int n_pi = 0, n_pi_u = 0;
  std::vector<int32_t> pi_code, bpi, pi_own;
  // dual-primal coupling: the normal-flux vectors that deflate the interface iteration, one
  // per pair of subdomains sharing a face (an edge in 2D): per multiplier row two (column,
  // weight) slots (column -1: unused), and per column its rows and weights (CSR)
  int n_defl = 0;
  std::vector<int32_t> defl_col, defl_ptr, defl_rows;
  std::vector<double> defl_w, defl_rw;
};

// Builds the deflation vectors of the dual-primal coupling (after the jump rows).
void build_deflation(MeshHost& m);

// Builds every host-side table from the mesh description (the numbering that
// the exported indexing documents).  Returns an error string on failure.
std::string build_mesh(const feti_mesh_desc& d, MeshHost& m);

}  // namespace feti
