// Element-parallel kernels: assembly of the dense local matrices, the
// per-step right-hand side, the initial fluid content and the element-by-element
// matrix-vector product of the refinement residual.  Accumulation is
// deterministic without atomics: the assembly processes the elements of a
// subdomain in eight colours (cell parity in x and y, times the two triangles of
// a cell) whose elements share no node; the right-hand side and the product
// write per-element contributions that a second kernel sums per DOF in a fixed
// element order.
#include "bstep.h"
#include "kernels.h"
#include "fem_device.h"
#include "loads_device.h"

namespace feti {

constexpr int MAX_EDOF_DEV = 21;

__device__ inline int elem_colour(int cell, int type, int ncell) {
  const int i = cell % ncell, j = cell / ncell;
  return ((i & 1) | ((j & 1) << 1)) * 2 + type;
}

// One thread per (element of the colour, element row).  K_s += K_e.
__global__ void k_assemble(const int32_t* __restrict__ el_sub, const int32_t* __restrict__ el_cell,
                           const int32_t* __restrict__ el_type, const int32_t* __restrict__ el_ldof,
                           const uint8_t* __restrict__ sub_poro, const int64_t* __restrict__ kofs,
                           const int32_t* __restrict__ ld, double* __restrict__ K, int nelem,
                           int edof, int order, int ncell, int colour, MatParams mpP,
                           MatParams mpE) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t e = gid / edof;
  const int r = (int)(gid % edof);
  if (e >= nelem) return;
  const int cell = el_cell[e], type = el_type[e];
  if (elem_colour(cell, type, ncell) != colour) return;
  const int lr = el_ldof[e * edof + r];
  if (lr < 0) return;
  const int s = el_sub[e];
  const bool poro = sub_poro[s] != 0;
  ElemGeom g;
  elem_geom(cell, type, ncell, g);
  const MatParams& mp = poro ? mpP : mpE;
  double* Ks = K + kofs[s];
  const int lds = ld[s];
  for (int c = 0; c < edof; ++c) {
    const int lc = el_ldof[e * edof + c];
    if (lc < 0) continue;
    Ks[(int64_t)lr * lds + lc] += elem_entry(order, poro, g, mp, r, c);
  }
}

// Value of the Dirichlet datum attached to a DOF code at time L.t.
__device__ inline double dirichlet_value(const LoadDev& L, bool poro, int32_t code, int umu,
                                         double uh, int n1, double h) {
  const int kind = code & 7, node = code >> 3;
  if (kind == 2 && L.eta_dec) return L.eta_dec[node];  // decoupled scheme: eta^n of the step
  if (L.kind == FETI_LOAD_RAW) {
    if (kind <= 1) return L.g_u ? L.g_u[(int64_t)kind * umu * umu + node] : 0.0;
    if (kind == 4) return L.g_p ? L.g_p[node] : 0.0;
    return 0.0;
  }
  if (kind <= 1) {
    const double x = (node % umu) * uh, y = (node / umu) * uh;
    return exact_u(L, poro, kind, x, y);
  }
  const double x = (node % n1) * h, y = (node / n1) * h;
  if (kind == 4) return exact_p(L, x, y);
  return 0.0;
}

// RAW loads: the boundary terms of an element's edges on the sides of the square, with the
// 3-point Gauss-Legendre rule on the edge (exact for the products of P2 traces):
// <t_h, theta_a> on sides without u Dirichlet data (traction of the element's region) and,
// in poroelastic elements, -tau <z_w,h, phi_k> on sides without p Dirichlet data.  The
// vertices' P1 lattice nodes come from the codes of the element's first scalar DOFs.
__device__ inline void raw_boundary_terms(const LoadDev& L, bool poro, const int32_t* ec, int order, int ncell,
                                          int nloc, int nu, double tau, double* acc) {
  const bool trac = L.t_side != nullptr, flux = poro && L.zw_side != nullptr;
  if (!trac && !flux) return;
  const int umu = order * ncell + 1, n1 = ncell + 1;
  const double len = 1.0 / ncell;  // boundary edges are axis-parallel cell edges
  int vi[3], vj[3];
  for (int v = 0; v < 3; ++v) {
    const int node = ec[nu + v] >> 3;
    vi[v] = node % n1;
    vj[v] = node / n1;
  }
  const double gs = 0.38729833462074168852;  // sqrt(3/5) / 2
  const double gq[3] = {0.5 - gs, 0.5, 0.5 + gs}, gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  for (int k = 0; k < 3; ++k) {
    const int a = k, b = (k + 1) % 3;
    int side = -1;
    if (vi[a] == 0 && vi[b] == 0) side = 0;
    else if (vi[a] == ncell && vi[b] == ncell) side = 1;
    else if (vj[a] == 0 && vj[b] == 0) side = 2;
    else if (vj[a] == ncell && vj[b] == ncell) side = 3;
    if (side < 0) continue;
    if (trac && !((L.dir_u >> side) & 1)) {
      // displacement nodes of the edge: ends a, b and (P2) the midpoint 3 + k
      const int nn = order == 2 ? 3 : 2;
      const int loc[3] = {a, b, 3 + k};
      double tv[2][3];
      const int reg = poro ? 0 : 1;
      for (int n = 0; n < nn; ++n) {
        const int node = ec[2 * loc[n]] >> 3;
        const int along = side < 2 ? node / umu : node % umu;
        for (int c = 0; c < 2; ++c) tv[c][n] = L.t_side[((int64_t)(reg * 4 + side) * 2 + c) * umu + along];
      }
      for (int q = 0; q < 3; ++q) {
        const double s = gq[q], la = 1.0 - s, lb = s;
        double psi[3];
        if (order == 2) { psi[0] = la * (2 * la - 1); psi[1] = lb * (2 * lb - 1); psi[2] = 4 * la * lb; }
        else { psi[0] = la; psi[1] = lb; psi[2] = 0.0; }
        double th[2] = {0.0, 0.0};
        for (int n = 0; n < nn; ++n)
          for (int c = 0; c < 2; ++c) th[c] += tv[c][n] * psi[n];
        const double wl = gw[q] * len;
        for (int n = 0; n < nn; ++n)
          for (int c = 0; c < 2; ++c) acc[2 * loc[n] + c] += wl * th[c] * psi[n];
      }
    }
    if (flux && !((L.dir_p >> side) & 1)) {
      const double za = L.zw_side[side * n1 + (side < 2 ? vj[a] : vi[a])];
      const double zb = L.zw_side[side * n1 + (side < 2 ? vj[b] : vi[b])];
      for (int q = 0; q < 3; ++q) {
        const double s = gq[q], la = 1.0 - s, lb = s;
        const double zh = za * la + zb * lb, wl = gw[q] * len;
        acc[nu + 6 + a] -= tau * wl * zh * la;
        acc[nu + 6 + b] -= tau * wl * zh * lb;
      }
    }
  }
}

// One thread per element: the element's right-hand side contributions (rows 1 and 4
// of eq. (linalg-system): F_u = (f, theta) and -R eta^{n-1} - tau Z on the p rows,
// minus the Dirichlet lifting K_e[r, D] g_D) into ebuf[e][row].
// cmode 1 (loads and Dirichlet data that do not depend on time): cache (nelem x edof,
// then nelem x 3) also receives the element contributions and the load parts of the p
// rows of poroelastic elements (whose eta terms come before the lifting).  Rows without
// eta terms do not change from step to step; k_rhs_prows forms the p rows of later
// steps from their load parts with the same terms in the same order.
__device__ __forceinline__ void rhs_elem_body(const DevMesh& m, const double* __restrict__ eta_prev,
                                              const MatParams& mpP, const MatParams& mpE, const LoadDev& L,
                                              double* cache, int cmode, int bx) {
  const int64_t e = (int64_t)bx * blockDim.x + threadIdx.x;
  if (e >= m.nelem) return;
  const int edof = m.edof, order = m.order, ncell = m.ncell;
  const int s = m.el_sub[e];
  const bool poro = m.sub_poro[s] != 0;
  ElemGeom g;
  elem_geom(m.el_cell[e], m.el_type[e], ncell, g);
  const MatParams& mp = poro ? mpP : mpE;
  const int nloc = order == 2 ? 6 : 3, nu = 2 * nloc;
  double acc[MAX_EDOF_DEV];
  for (int r = 0; r < MAX_EDOF_DEV; ++r) acc[r] = 0.0;
  const int32_t* ec = m.el_code + e * edof;
  const int umu = order * ncell + 1, n1 = ncell + 1;
  const bool raw = L.kind == FETI_LOAD_RAW;
  // RAW: the element's nodal data (the interpolants are evaluated at the quadrature points)
  double rf[2][6] = {}, rz[3] = {};
  if (raw) {
    const double* fd = poro ? L.f_p : L.f_e;
    if (fd)
      for (int a = 0; a < nloc; ++a) {
        const int node = ec[2 * a] >> 3;
        rf[0][a] = fd[node];
        rf[1][a] = fd[(int64_t)umu * umu + node];
      }
    if (poro && L.z)
      for (int k = 0; k < 3; ++k) rz[k] = L.z[ec[nu + 3 + k] >> 3];
  }
  // loads at the 7 quadrature points
  for (int q = 0; q < 7; ++q) {
    double l0, l1, l2, w;
    radon_point(q, l0, l1, l2, w);
    const double x = l0 * g.x[0] + l1 * g.x[1] + l2 * g.x[2];
    const double y = l0 * g.y[0] + l1 * g.y[1] + l2 * g.y[2];
    const double wa = w * g.area;
    const double lam[3] = {l0, l1, l2};
    double phi[6];
    for (int a = 0; a < nloc; ++a) {
      if (order == 1) phi[a] = lam[a];
      else if (a < 3) phi[a] = lam[a] * (2 * lam[a] - 1);
      else phi[a] = 4 * lam[a - 3] * lam[(a - 2) % 3];
    }
    double fx = 0.0, fy = 0.0;
    if (raw) {
      for (int a = 0; a < nloc; ++a) {
        fx += rf[0][a] * phi[a];
        fy += rf[1][a] * phi[a];
      }
    } else {
      body_force(L, poro, x, y, fx, fy);
    }
    for (int a = 0; a < nloc; ++a) {
      acc[2 * a] += wa * fx * phi[a];
      acc[2 * a + 1] += wa * fy * phi[a];
    }
    if (poro) {
      const double z = raw ? rz[0] * l0 + rz[1] * l1 + rz[2] * l2 : source(L, x, y);
      for (int k = 0; k < 3; ++k) acc[nu + 6 + k] -= mp.tau * wa * z * lam[k];
    }
  }
  if (raw) raw_boundary_terms(L, poro, ec, order, ncell, nloc, nu, mp.tau, acc);
  double pload[3] = {0.0, 0.0, 0.0};  // load parts of the p rows
  if (poro)
    for (int k = 0; k < 3; ++k) pload[k] = acc[nu + 6 + k];
  const int32_t* ld = m.el_ldof + e * edof;
  if (poro && ld[nu + 3] >= 0) {  // (the decoupled scheme has no eta unknowns)
    const double* eta = eta_prev + m.soff[s];
    double ev[3];
    for (int b = 0; b < 3; ++b) ev[b] = eta[ld[nu + 3 + b]];
    for (int k = 0; k < 3; ++k)
      for (int b = 0; b < 3; ++b) acc[nu + 6 + k] -= moment2(g, k, b) * ev[b];
  }
  // Dirichlet lifting
  const double uh = 1.0 / (order * ncell), h = 1.0 / ncell;
  for (int c = 0; c < edof; ++c) {
    if (ld[c] >= 0) continue;
    const int32_t code = m.el_code[e * edof + c];
    if (code < 0) continue;
    const double gv = dirichlet_value(L, poro, code, umu, uh, ncell + 1, h);
    if (gv == 0.0) continue;
    // K_e[r][c] from the stored element matrices (the same values elem_entry gives)
    const double* Kc = m.emat ? m.emat + (e * edof + c) * edof : nullptr;
    for (int r = 0; r < edof; ++r)
      if (ld[r] >= 0) acc[r] -= (Kc ? Kc[r] : elem_entry(order, poro, g, mp, r, c)) * gv;
  }
  double* out = m.ebuf + e * edof;
  for (int r = 0; r < edof; ++r) out[r] = acc[r];
  if (cmode == 1) {
    for (int r = 0; r < edof; ++r) cache[e * edof + r] = acc[r];
    double* pl = cache + (int64_t)m.nelem * edof + e * 3;
    for (int k = 0; k < 3; ++k) pl[k] = pload[k];
  }
}

__global__ void __launch_bounds__(128) k_rhs_elem(DevMesh m, const double* __restrict__ eta_prev,
                                                  MatParams mpP, MatParams mpE, LoadDev L, double* cache,
                                                  int cmode) {
  rhs_elem_body(m, eta_prev, mpP, mpE, L, cache, cmode, blockIdx.x);
}

// A later step of a time-independent load (cmode 2): one thread per p row of every
// element (elastic elements return at once) rewrites that row of the cached element
// contributions from its load part: the eta moments, then the lifting columns in
// order, as k_rhs_elem, with K_e read from the stored element matrices.
__global__ void __launch_bounds__(256) k_rhs_prows(DevMesh m, const double* __restrict__ eta_prev, MatParams mpP,
                                                   LoadDev L, double* __restrict__ cache) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t e = gid / 3;
  const int k = (int)(gid % 3);
  if (e >= m.nelem) return;
  const int s = m.el_sub[e];
  if (m.sub_poro[s] == 0) return;
  const int edof = m.edof, order = m.order, ncell = m.ncell;
  const int nloc = order == 2 ? 6 : 3, nu = 2 * nloc;
  const int r = nu + 6 + k;
  const int32_t* ld = m.el_ldof + e * edof;
  double acc = cache[(int64_t)m.nelem * edof + e * 3 + k];
  ElemGeom g;
  elem_geom(m.el_cell[e], m.el_type[e], ncell, g);
  if (ld[nu + 3] >= 0) {  // (the decoupled scheme has no eta unknowns)
    const double* eta = eta_prev + m.soff[s];
    for (int b = 0; b < 3; ++b) acc -= moment2(g, k, b) * eta[ld[nu + 3 + b]];
  }
  if (ld[r] >= 0) {
    const int umu = order * ncell + 1;
    const double uh = 1.0 / (order * ncell), h = 1.0 / ncell;
    for (int c = 0; c < edof; ++c) {
      if (ld[c] >= 0) continue;
      const int32_t code = m.el_code[e * edof + c];
      if (code < 0) continue;
      const double gv = dirichlet_value(L, true, code, umu, uh, ncell + 1, h);
      if (gv == 0.0) continue;
      acc -= (m.emat ? m.emat[(e * edof + c) * edof + r] : elem_entry(order, true, g, mpP, r, c)) * gv;
    }
  }
  cache[e * edof + r] = acc;
}

// One thread per (element, row): ebuf[e][row] = (K_e x_e)[row]
// One thread per (element, row): row r of K_e into emat, column-major per element
// (entry (r, c) at (e edof + c) edof + r, so that the threads of consecutive rows read
// consecutive addresses); every entry, also those of Dirichlet DOFs, which the
// products skip
__global__ void k_elem_store(DevMesh m, MatParams mpP, MatParams mpE) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int edof = m.edof;
  const int64_t e = gid / edof;
  const int r = (int)(gid % edof);
  if (e >= m.nelem) return;
  const bool poro = m.sub_poro[m.el_sub[e]] != 0;
  ElemGeom g;
  elem_geom(m.el_cell[e], m.el_type[e], m.ncell, g);
  const MatParams& mp = poro ? mpP : mpE;
  double* col0 = m.emat + e * edof * edof + r;
  for (int c = 0; c < edof; ++c) col0[(int64_t)c * edof] = elem_entry(m.order, poro, g, mp, r, c);
}

// One thread per (element, row): ebuf[e][row] = (K_e x_e)[row], K_e read from emat
__device__ __forceinline__ void elem_matvec_body(const DevMesh& m, const double* __restrict__ x, int bx) {
  const int64_t gid = (int64_t)bx * blockDim.x + threadIdx.x;
  const int edof = m.edof;
  const int64_t e = gid / edof;
  const int r = (int)(gid % edof);
  if (e >= m.nelem) return;
  const int32_t* ld = m.el_ldof + e * edof;
  double acc = 0.0;
  if (ld[r] >= 0) {
    const double* xs = x + m.soff[m.el_sub[e]];
    const double* col0 = m.emat + e * edof * edof + r;
    for (int c = 0; c < edof; ++c) {
      const int lc = ld[c];
      if (lc >= 0) acc += col0[(int64_t)c * edof] * xs[lc];
    }
  }
  m.ebuf[gid] = acc;
}

__global__ void k_elem_matvec(DevMesh m, const double* __restrict__ x) { elem_matvec_body(m, x, blockIdx.x); }

// y_i = sum of the element contributions of torn DOF i, in element order
__device__ __forceinline__ void gather_elem_body(const DevMesh& m, const double* __restrict__ ebuf,
                                                 double* __restrict__ y, int bx) {
  const int64_t i = (int64_t)bx * blockDim.x + threadIdx.x;
  if (i >= m.sum_ns) return;
  double s = 0.0;
  for (int k = m.adj_ptr[i]; k < m.adj_ptr[i + 1]; ++k) s += ebuf[m.adj[k]];
  y[i] = s;
}

__global__ void k_gather_elem(DevMesh m, double* __restrict__ y) { gather_elem_body(m, m.ebuf, y, blockIdx.x); }

// eta^0 at every local eta DOF (nodal interpolation of c0 p0 + alpha div u0)
__global__ void k_init_eta(const int32_t* __restrict__ code, double* __restrict__ u, int64_t n,
                           int ncell, LoadDev L) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t c = code[i];
  if ((c & 7) != 2) return;
  const int node = c >> 3;
  if (L.kind == FETI_LOAD_RAW) {
    u[i] = L.eta0 ? L.eta0[node] : 0.0;
    return;
  }
  const double h = 1.0 / ncell;
  u[i] = initial_eta(L, (node % (ncell + 1)) * h, (node / (ncell + 1)) * h);
}

// load at the node of every multiplier row, read through the row's first interface DOF
__global__ void k_interface_load(DevMesh m, LoadDev L, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m.n_lambda) return;
  const int64_t gb = m.jr_b[2 * j];
  const int32_t code = m.code[m.b_torn[gb]];
  const int kind = code & 7, node = code >> 3;
  const bool poro = m.sub_poro[m.b_sub[gb]] != 0;
  double v = 0.0;
  if (L.kind == FETI_LOAD_RAW) {
    const int umu = m.order * m.ncell + 1;
    const double* fd = poro ? L.f_p : L.f_e;
    if (kind <= 1) v = fd ? fd[(int64_t)kind * umu * umu + node] : 0.0;
    else if (kind <= 4) v = L.z ? L.z[node] : 0.0;
    out[j] = v;
    return;
  }
  if (kind <= 1) {
    const int umu = m.order * m.ncell + 1;
    const double uh = 1.0 / (m.order * m.ncell);
    double fx, fy;
    body_force(L, poro, (node % umu) * uh, (node / umu) * uh, fx, fy);
    v = kind == 0 ? fx : fy;
  } else if (kind <= 4) {
    const int n1 = m.ncell + 1;
    const double h = 1.0 / m.ncell;
    v = source(L, (node % n1) * h, (node / n1) * h);
  }
  out[j] = v;
}

// ---- launchers ---------------------------------------------------------------

void launch_interface_load(const DevMesh& m, const LoadDev& L, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_interface_load, dim3((unsigned)((m.n_lambda + 255) / 256)), dim3(256), 0, st, m, L, out);
}


void launch_assemble(const DevMesh& m, double* K, MatParams mpP, MatParams mpE, hipStream_t st) {
  const int64_t nthreads = (int64_t)m.nelem * m.edof;
  const int blk = 256;
  const int grid = (int)((nthreads + blk - 1) / blk);
  for (int colour = 0; colour < 8; ++colour)
    hipLaunchKernelGGL(k_assemble, dim3(grid), dim3(blk), 0, st, m.el_sub, m.el_cell, m.el_type,
                       m.el_ldof, m.sub_poro, m.kofs, m.ld, K, m.nelem, m.edof, m.order, m.ncell,
                       colour, mpP, mpE);
}

void launch_rhs(const DevMesh& m, const double* eta_prev, double* f, MatParams mpP, MatParams mpE,
                const LoadDev& L, hipStream_t st, double* cache, int cmode) {
  if (cache && cmode == 2) {
    const int64_t nthreads = (int64_t)m.nelem * 3;
    hipLaunchKernelGGL(k_rhs_prows, dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0, st, m, eta_prev, mpP, L,
                       cache);
    DevMesh mc = m;  // the gather reads the cached element contributions
    mc.ebuf = cache;
    hipLaunchKernelGGL(k_gather_elem, dim3((unsigned)((m.sum_ns + 255) / 256)), dim3(256), 0, st, mc, f);
    return;
  }
  hipLaunchKernelGGL(k_rhs_elem, dim3((m.nelem + 127) / 128), dim3(128), 0, st, m, eta_prev, mpP, mpE, L, cache,
                     cache && cmode == 1 ? 1 : 0);
  hipLaunchKernelGGL(k_gather_elem, dim3((unsigned)((m.sum_ns + 255) / 256)), dim3(256), 0, st, m, f);
}

void launch_gather_elem(const DevMesh& m, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_elem, dim3((unsigned)((m.sum_ns + 255) / 256)), dim3(256), 0, st, m, y);
}

void launch_init_eta(const DevMesh& m, double* u, const LoadDev& L, hipStream_t st) {
  const int blk = 256;
  const int grid = (int)((m.sum_ns + blk - 1) / blk);
  hipLaunchKernelGGL(k_init_eta, dim3(grid), dim3(blk), 0, st, m.code, u, m.sum_ns, m.ncell, L);
}

void launch_elem_store(const DevMesh& m, MatParams mpP, MatParams mpE, hipStream_t st) {
  const int64_t nthreads = (int64_t)m.nelem * m.edof;
  hipLaunchKernelGGL(k_elem_store, dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0, st, m, mpP, mpE);
}

void launch_elem_matvec(const DevMesh& m, const double* x, double* y, MatParams mpP, MatParams mpE,
                        hipStream_t st) {
  (void)mpP;
  (void)mpE;
  const int64_t nthreads = (int64_t)m.nelem * m.edof;
  hipLaunchKernelGGL(k_elem_matvec, dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0, st, m, x);
  hipLaunchKernelGGL(k_gather_elem, dim3((unsigned)((m.sum_ns + 255) / 256)), dim3(256), 0, st, m, y);
}

// ---- decoupled scheme: the explicit fluid step ------------------------------------
// Remark after eq. (linalg-system): the fluid content is advanced by explicit Euler with
// the lumped mass and the previous pressure, m_i (eta^n_i - eta^{n-1}_i) = tau (Z^n -
// A_f p^{n-1})_i, before the momentum balance is solved with eta^n known; the pressure
// then follows nodally from row 3, p = k1 xi + k2 eta.  The element matrices stored at
// assembly hold the p rows of row 4: -R (eta columns) and -tau A_f (p columns).

// The load part of the fluid rows of element e: -tau (z, phi_k) over the 7-point rule
// (and the RAW flux terms), accumulated in the order of k_rhs_elem.
__device__ inline void fluid_load(const DevMesh& m, int64_t e, const LoadDev& L, const ElemGeom& g, double tau,
                                  double pl[3]) {
  const int edof = m.edof, order = m.order, nloc = order == 2 ? 6 : 3, nu = 2 * nloc;
  const int32_t* ec = m.el_code + e * edof;
  const bool raw = L.kind == FETI_LOAD_RAW;
  double rz[3] = {0.0, 0.0, 0.0};
  if (raw && L.z)
    for (int k = 0; k < 3; ++k) rz[k] = L.z[ec[nu + 3 + k] >> 3];
  double acc[MAX_EDOF_DEV];
  for (int r = 0; r < MAX_EDOF_DEV; ++r) acc[r] = 0.0;
  for (int q = 0; q < 7; ++q) {
    double l0, l1, l2, w;
    radon_point(q, l0, l1, l2, w);
    const double x = l0 * g.x[0] + l1 * g.x[1] + l2 * g.x[2];
    const double y = l0 * g.y[0] + l1 * g.y[1] + l2 * g.y[2];
    const double wa = w * g.area;
    const double lam[3] = {l0, l1, l2};
    const double z = raw ? rz[0] * l0 + rz[1] * l1 + rz[2] * l2 : source(L, x, y);
    for (int k = 0; k < 3; ++k) acc[nu + 6 + k] -= tau * wa * z * lam[k];
  }
  if (raw) raw_boundary_terms(L, true, ec, order, m.ncell, nloc, nu, tau, acc);
  for (int k = 0; k < 3; ++k) pl[k] = acc[nu + 6 + k];
}

// One thread per element (elastic elements return): ce[e][k] = tau Z_k - tau (A_f p)_k,
// and with me: me[e][k] = sum_b R_e[k][b].
__global__ void __launch_bounds__(128) k_dec_fluid(DevMesh m, MatParams mpP, LoadDev L,
                                                   const double* __restrict__ p_lat, double* __restrict__ ce,
                                                   double* __restrict__ me) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nelem) return;
  if (!m.sub_poro[m.el_sub[e]]) return;
  const int edof = m.edof, nloc = m.order == 2 ? 6 : 3, nu = 2 * nloc;
  ElemGeom g;
  elem_geom(m.el_cell[e], m.el_type[e], m.ncell, g);
  double pl[3];
  fluid_load(m, e, L, g, mpP.tau, pl);
  const int32_t* ec = m.el_code + e * edof;
  double pv[3];
  for (int b = 0; b < 3; ++b) pv[b] = p_lat[ec[nu + b] >> 3];  // vertex nodes from the xi codes
  const double* Ke = m.emat + e * edof * edof;                  // entry (r, c) at c * edof + r
  for (int k = 0; k < 3; ++k) {
    double v = -pl[k];
    for (int b = 0; b < 3; ++b) v += Ke[(nu + 6 + b) * edof + nu + 6 + k] * pv[b];
    ce[e * 3 + k] = v;
    if (me) {
      double s = 0.0;
      for (int b = 0; b < 3; ++b) s -= Ke[(nu + 3 + b) * edof + nu + 6 + k];
      me[e * 3 + k] = s;
    }
  }
}

// one thread per fluid node: the lumped mass, summed over the node's element entries
__global__ void k_dec_mass(DevMesh m, const double* __restrict__ me, double* __restrict__ mass) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m.n_dec) return;
  double s = 0.0;
  for (int q = m.dec_ptr[k]; q < m.dec_ptr[k + 1]; ++q) s += me[m.dec_ent[q]];
  mass[k] = s;
}

// one thread per fluid node: eta^n (explicit Euler with the lumped mass; at a pressure
// Dirichlet node from row 3 with the previous xi)
__global__ void k_dec_update(DevMesh m, LoadDev L, double k1, double k2, const double* __restrict__ ce,
                             const double* __restrict__ mass, double* __restrict__ eta_lat,
                             const double* __restrict__ xi_lat) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m.n_dec) return;
  const int node = m.dec_node[k];
  if (m.dec_pdir[k]) {
    const int umu = m.order * m.ncell + 1, n1 = m.ncell + 1;
    const double pD = dirichlet_value(L, true, 8 * node + 4, umu, 1.0 / (m.order * m.ncell), n1, 1.0 / m.ncell);
    eta_lat[node] = (pD - k1 * xi_lat[node]) / k2;
    return;
  }
  double s = 0.0;
  for (int q = m.dec_ptr[k]; q < m.dec_ptr[k + 1]; ++q) s += ce[m.dec_ent[q]];
  eta_lat[node] += s / mass[k];
}

// one thread per fluid node: xi^n from its first torn copy, p^n = k1 xi^n + k2 eta^n
// (p_D at pressure Dirichlet nodes)
__global__ void k_dec_pressure(DevMesh m, LoadDev L, double k1, double k2, const double* __restrict__ u,
                               double* __restrict__ xi_lat, double* __restrict__ p_lat,
                               const double* __restrict__ eta_lat) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m.n_dec) return;
  const int node = m.dec_node[k];
  const double xi = u[m.dec_xi[k]];
  xi_lat[node] = xi;
  if (m.dec_pdir[k]) {
    const int umu = m.order * m.ncell + 1, n1 = m.ncell + 1;
    p_lat[node] = dirichlet_value(L, true, 8 * node + 4, umu, 1.0 / (m.order * m.ncell), n1, 1.0 / m.ncell);
  } else {
    p_lat[node] = k1 * xi + k2 * eta_lat[node];
  }
}

// one thread per fluid node: eta^0 (R14), p^0 the interpolant of the initial pressure,
// xi^0 = (p^0 - k2 eta^0) / k1
__global__ void k_dec_init(DevMesh m, LoadDev L, double k1, double k2, double* __restrict__ eta_lat,
                           double* __restrict__ p_lat, double* __restrict__ xi_lat) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m.n_dec) return;
  const int node = m.dec_node[k];
  const int n1 = m.ncell + 1;
  const double h = 1.0 / m.ncell, x = (node % n1) * h, y = (node / n1) * h;
  double eta, p;
  if (L.kind == FETI_LOAD_RAW) {
    eta = L.eta0 ? L.eta0[node] : 0.0;
    p = 0.0;
  } else {
    eta = initial_eta(L, x, y);
    p = exact_p(L, x, y);
  }
  eta_lat[node] = eta;
  p_lat[node] = p;
  xi_lat[node] = (p - k2 * eta) / k1;
}

// out[node] = src[node] at every fluid node
__global__ void k_dec_field(DevMesh m, const double* __restrict__ src, double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m.n_dec) return;
  out[m.dec_node[k]] = src[m.dec_node[k]];
}

void launch_dec_fluid(const DevMesh& m, const MatParams& mpP, const LoadDev& L, const double* p_lat, double* ce,
                      double* me, hipStream_t st) {
  hipLaunchKernelGGL(k_dec_fluid, dim3((m.nelem + 127) / 128), dim3(128), 0, st, m, mpP, L, p_lat, ce, me);
}
void launch_dec_mass(const DevMesh& m, const double* me, double* mass, hipStream_t st) {
  if (m.n_dec == 0) return;
  hipLaunchKernelGGL(k_dec_mass, dim3((m.n_dec + 255) / 256), dim3(256), 0, st, m, me, mass);
}
void launch_dec_update(const DevMesh& m, const LoadDev& L, double k1, double k2, const double* ce,
                       const double* mass, double* eta_lat, const double* xi_lat, hipStream_t st) {
  if (m.n_dec == 0) return;
  hipLaunchKernelGGL(k_dec_update, dim3((m.n_dec + 255) / 256), dim3(256), 0, st, m, L, k1, k2, ce, mass, eta_lat,
                     xi_lat);
}
void launch_dec_pressure(const DevMesh& m, const LoadDev& L, double k1, double k2, const double* u, double* xi_lat,
                         double* p_lat, const double* eta_lat, hipStream_t st) {
  if (m.n_dec == 0) return;
  hipLaunchKernelGGL(k_dec_pressure, dim3((m.n_dec + 255) / 256), dim3(256), 0, st, m, L, k1, k2, u, xi_lat, p_lat,
                     eta_lat);
}
void launch_dec_init(const DevMesh& m, const LoadDev& L, double k1, double k2, double* eta_lat, double* p_lat,
                     double* xi_lat, hipStream_t st) {
  if (m.n_dec == 0) return;
  hipLaunchKernelGGL(k_dec_init, dim3((m.n_dec + 255) / 256), dim3(256), 0, st, m, L, k1, k2, eta_lat, p_lat,
                     xi_lat);
}
void launch_dec_field(const DevMesh& m, const double* src_lat, double* out, hipStream_t st) {
  if (m.n_dec == 0) return;
  hipLaunchKernelGGL(k_dec_field, dim3((m.n_dec + 255) / 256), dim3(256), 0, st, m, src_lat, out);
}

// ---- batched launches (problem = blockIdx.y) ----------------------------------

__global__ void __launch_bounds__(128) kb_rhs_elem(const BProb* __restrict__ P, const BStepVals* __restrict__ V) {
  const BProb& p = P[blockIdx.y];
  rhs_elem_body(p.m, p.v[BV_U], p.mpP, p.mpE, V[blockIdx.y].L, nullptr, 0, blockIdx.x);
}

__global__ void __launch_bounds__(256) kb_elem_matvec(const BProb* __restrict__ P, int x) {
  const BProb& p = P[blockIdx.y];
  elem_matvec_body(p.m, p.v[x], blockIdx.x);
}

__global__ void __launch_bounds__(256) kb_gather_elem(const BProb* __restrict__ P, int y) {
  const BProb& p = P[blockIdx.y];
  gather_elem_body(p.m, p.m.ebuf, p.v[y], blockIdx.x);
}

void launchb_rhs(const BProb* P, const BStepVals* V, const BDims& d, hipStream_t st) {
  hipLaunchKernelGGL(kb_rhs_elem, dim3(d.elem_blk, d.P), dim3(128), 0, st, P, V);
  hipLaunchKernelGGL(kb_gather_elem, dim3(d.ns_blk, d.P), dim3(256), 0, st, P, (int)BV_F);
}

void launchb_elem_matvec(const BProb* P, const BDims& d, int x, int y, hipStream_t st) {
  hipLaunchKernelGGL(kb_elem_matvec, dim3(d.erow_blk, d.P), dim3(256), 0, st, P, x);
  hipLaunchKernelGGL(kb_gather_elem, dim3(d.ns_blk, d.P), dim3(256), 0, st, P, y);
}

}  // namespace feti
