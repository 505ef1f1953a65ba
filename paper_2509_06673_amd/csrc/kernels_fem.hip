// Element-parallel kernels: assembly of the dense local matrices, the
// per-step right-hand side, the initial fluid content and the torn-system
// residual.  Accumulation is deterministic without atomics: the elements of
// a subdomain are processed in eight colours (cell parity in x and y, times
// the two triangles of a cell); elements of one colour share no node, so
// their scatter-adds never touch the same entry.
#include "kernels.h"
#include "fem_device.h"
#include "loads_device.h"

namespace feti {

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
  if (kind <= 1) {
    const double x = (node % umu) * uh, y = (node / umu) * uh;
    return exact_u(L, poro, kind, x, y);
  }
  const double x = (node % n1) * h, y = (node / n1) * h;
  if (kind == 4) return exact_p(L, x, y);
  return 0.0;
}

// One thread per (element of the colour, element row): f_s += load integral
// (rows 1 and 4 of eq. (linalg-system): F_u and -R eta^{n-1} - tau Z) minus
// the Dirichlet lifting K_e[r, D] g_D.
__global__ void k_rhs(const int32_t* __restrict__ el_sub, const int32_t* __restrict__ el_cell,
                      const int32_t* __restrict__ el_type, const int32_t* __restrict__ el_ldof,
                      const int32_t* __restrict__ el_code, const uint8_t* __restrict__ sub_poro,
                      const int64_t* __restrict__ soff, const double* __restrict__ eta_prev,
                      double* __restrict__ f, int nelem, int edof, int order, int ncell, int colour,
                      MatParams mpP, MatParams mpE, LoadDev L) {
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
  const int nu = order == 2 ? 12 : 6;
  double acc = 0.0;
  if (r < nu) {
    // consistent load (f, theta_r) with the 7-point rule
    const int a = r / 2, comp = r % 2;
    for (int q = 0; q < 7; ++q) {
      double l0, l1, l2, w;
      radon_point(q, l0, l1, l2, w);
      const double x = l0 * g.x[0] + l1 * g.x[1] + l2 * g.x[2];
      const double y = l0 * g.y[0] + l1 * g.y[1] + l2 * g.y[2];
      double fx, fy;
      body_force(L, poro, x, y, fx, fy);
      const double lam[3] = {l0, l1, l2};
      double phi;
      if (order == 1) phi = lam[a];
      else if (a < 3) phi = lam[a] * (2 * lam[a] - 1);
      else phi = 4 * lam[a - 3] * lam[(a - 2) % 3];
      acc += w * g.area * (comp == 0 ? fx : fy) * phi;
    }
  } else if (poro && r >= nu + 6) {
    // p row: -(R eta^{n-1})_k - tau (z, lambda_k)
    const int k = r - nu - 6;
    const double* eta = eta_prev + soff[s];
    for (int b = 0; b < 3; ++b) {
      const int li = el_ldof[e * edof + nu + 3 + b];
      acc -= moment2(g, k, b) * eta[li];
    }
    double zk = 0.0;
    for (int q = 0; q < 7; ++q) {
      double l0, l1, l2, w;
      radon_point(q, l0, l1, l2, w);
      const double x = l0 * g.x[0] + l1 * g.x[1] + l2 * g.x[2];
      const double y = l0 * g.y[0] + l1 * g.y[1] + l2 * g.y[2];
      const double lam[3] = {l0, l1, l2};
      zk += w * g.area * source(L, x, y) * lam[k];
    }
    acc -= mp.tau * zk;
  }
  // Dirichlet lifting
  const int umu = order * ncell + 1;
  const double uh = 1.0 / (order * ncell), h = 1.0 / ncell;
  for (int c = 0; c < edof; ++c) {
    if (el_ldof[e * edof + c] >= 0) continue;
    const int32_t code = el_code[e * edof + c];
    if (code < 0) continue;
    const double gv = dirichlet_value(L, poro, code, umu, uh, ncell + 1, h);
    if (gv != 0.0) acc -= elem_entry(order, poro, g, mp, r, c) * gv;
  }
  f[soff[s] + lr] += acc;
}

// eta^0 at every local eta DOF (nodal interpolation of c0 p0 + alpha div u0)
__global__ void k_init_eta(const int32_t* __restrict__ code, double* __restrict__ u, int64_t n,
                           int ncell, LoadDev L) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t c = code[i];
  if ((c & 7) != 2) return;
  const int node = c >> 3;
  const double h = 1.0 / ncell;
  u[i] = initial_eta(L, (node % (ncell + 1)) * h, (node / (ncell + 1)) * h);
}

// y_s += K_e x_s over the elements of the colour (torn, sparse matrix-vector
// product with the FP64 element matrices; used for refinement residuals)
__global__ void k_elem_matvec(const int32_t* __restrict__ el_sub, const int32_t* __restrict__ el_cell,
                              const int32_t* __restrict__ el_type, const int32_t* __restrict__ el_ldof,
                              const uint8_t* __restrict__ sub_poro, const int64_t* __restrict__ soff,
                              const double* __restrict__ x, double* __restrict__ y, int nelem, int edof,
                              int order, int ncell, int colour, MatParams mpP, MatParams mpE) {
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
  const double* xs = x + soff[s];
  double acc = 0.0;
  for (int c = 0; c < edof; ++c) {
    const int lc = el_ldof[e * edof + c];
    if (lc < 0) continue;
    acc += elem_entry(order, poro, g, mp, r, c) * xs[lc];
  }
  y[soff[s] + lr] += acc;
}

// ---- launchers ---------------------------------------------------------------

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
                const LoadDev& L, hipStream_t st) {
  const int64_t nthreads = (int64_t)m.nelem * m.edof;
  const int blk = 256;
  const int grid = (int)((nthreads + blk - 1) / blk);
  for (int colour = 0; colour < 8; ++colour)
    hipLaunchKernelGGL(k_rhs, dim3(grid), dim3(blk), 0, st, m.el_sub, m.el_cell, m.el_type,
                       m.el_ldof, m.el_code, m.sub_poro, m.soff, eta_prev, f, m.nelem, m.edof,
                       m.order, m.ncell, colour, mpP, mpE, L);
}

void launch_init_eta(const DevMesh& m, double* u, const LoadDev& L, hipStream_t st) {
  const int blk = 256;
  const int grid = (int)((m.sum_ns + blk - 1) / blk);
  hipLaunchKernelGGL(k_init_eta, dim3(grid), dim3(blk), 0, st, m.code, u, m.sum_ns, m.ncell, L);
}

void launch_elem_matvec(const DevMesh& m, const double* x, double* y, MatParams mpP, MatParams mpE,
                        hipStream_t st) {
  const int64_t nthreads = (int64_t)m.nelem * m.edof;
  const int blk = 256;
  const int grid = (int)((nthreads + blk - 1) / blk);
  for (int colour = 0; colour < 8; ++colour)
    hipLaunchKernelGGL(k_elem_matvec, dim3(grid), dim3(blk), 0, st, m.el_sub, m.el_cell, m.el_type,
                       m.el_ldof, m.sub_poro, m.soff, x, y, m.nelem, m.edof, m.order, m.ncell,
                       colour, mpP, mpE);
}

}  // namespace feti
