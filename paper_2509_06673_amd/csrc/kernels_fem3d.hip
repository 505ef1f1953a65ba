// Element kernels on tetrahedra (d = 3): element matrices, assembly of the dense local
// matrices and the per-step right-hand side for nodal (RAW) data.
//
// The element matrices K_e (closed form, fem3d_device.h) are stored column-major per
// element, as in 2D, and every later use reads them: the assembly, the Dirichlet lifting
// of the right-hand side and the element-by-element residual of the refinement.  The
// assembly is deterministic without atomics: the tetrahedra are processed in 48 colours
// (cube parity in x, y and z, times the six tetrahedra of a cube), and two tetrahedra of a
// colour share no node.  The right-hand side writes one value per (element, row), which
// the 2D gather sums per DOF in a fixed element order.
#include "kernels.h"
#include "fem3d_device.h"
#include "loads_device.h"

namespace feti {

// One thread per (element, row): row r of K_e into emat (entry (r, c) at (e edof + c) edof + r).
__global__ void __launch_bounds__(256) k_elem_store3d(DevMesh m, MatParams mpP, MatParams mpE) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int edof = m.edof;
  const int64_t e = gid / edof;
  const int r = (int)(gid % edof);
  if (e >= m.nelem) return;
  const bool poro = m.sub_poro[m.el_sub[e]] != 0;
  ElemGeom3 G;
  elem_geom3(m.el_cell[e], m.el_type[e], m.ncell, G);
  const MatParams& mp = poro ? mpP : mpE;
  double* col0 = m.emat + e * edof * edof + r;
  for (int c = 0; c < edof; ++c) col0[(int64_t)c * edof] = elem_entry3(m.order, poro, G, mp, r, c);
}

__device__ inline int elem_colour3(int cell, int type, int ncell) {
  const int i = cell % ncell, j = (cell / ncell) % ncell, k = cell / (ncell * ncell);
  return ((i & 1) | ((j & 1) << 1) | ((k & 1) << 2)) * 6 + type;
}

// One thread per (element of the colour, element row): K_s += K_e (from emat).
__global__ void __launch_bounds__(256) k_assemble3d(DevMesh m, double* __restrict__ K, const int64_t* __restrict__ kofs,
                                                    const int32_t* __restrict__ ld, int colour) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int edof = m.edof;
  const int64_t e = gid / edof;
  const int r = (int)(gid % edof);
  if (e >= m.nelem) return;
  if (elem_colour3(m.el_cell[e], m.el_type[e], m.ncell) != colour) return;
  const int32_t* eld = m.el_ldof + e * edof;
  const int lr = eld[r];
  if (lr < 0) return;
  const int s = m.el_sub[e];
  double* Ks = K + kofs[s];
  const int64_t lds = ld[s];
  const double* col0 = m.emat + e * edof * edof + r;
  for (int c = 0; c < edof; ++c) {
    const int lc = eld[c];
    if (lc >= 0) Ks[(int64_t)lr * lds + lc] += col0[(int64_t)c * edof];
  }
}

// Dirichlet datum of a DOF code (RAW data on the cube lattices).
__device__ inline double dirichlet_value3(const LoadDev& L, int32_t code, int64_t nu3) {
  const int kind = code & 7;
  const int64_t node = code >> 3;
  if (kind == 0 || kind == 1 || kind == 6) {
    const int comp = kind == 6 ? 2 : kind;
    return L.g_u ? L.g_u[comp * nu3 + node] : 0.0;
  }
  if (kind == 4) return L.g_p ? L.g_p[node] : 0.0;
  return 0.0;
}

// One thread per (element, row): the row's right-hand side contribution (rows 1 and 4 of
// eq. (linalg-system)), F_u = (f_h, theta) = sum_b (phi_a, phi_b) f_b on the displacement
// rows, -R eta^{n-1} - tau Z with Z = (z_h, phi) = R z on the p rows, then minus the
// Dirichlet lifting K_e[r, D] g_D, into ebuf[e][row].
__global__ void __launch_bounds__(256) k_rhs3d(DevMesh m, const double* __restrict__ eta_prev, MatParams mpP,
                                               LoadDev L) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int edof = m.edof;
  const int64_t e = gid / edof;
  const int r = (int)(gid % edof);
  if (e >= m.nelem) return;
  const int s = m.el_sub[e];
  const bool poro = m.sub_poro[s] != 0;
  const int order = m.order;
  const int nloc = order == 2 ? 10 : 4, nu = 3 * nloc;
  const int64_t umu = (int64_t)order * m.ncell + 1, nu3 = umu * umu * umu;
  const int32_t* ec = m.el_code + e * edof;
  const int32_t* eld = m.el_ldof + e * edof;
  double acc = 0.0;
  if (eld[r] >= 0) {
    ElemGeom3 G;
    elem_geom3(m.el_cell[e], m.el_type[e], m.ncell, G);
    if (r < nu) {
      const double* fd = poro ? L.f_p : L.f_e;
      if (fd) {
        const int a = r / 3, comp = r % 3;
        for (int b = 0; b < nloc; ++b) acc += mass_p(order, G, a, b) * fd[comp * nu3 + (ec[3 * b] >> 3)];
      }
    } else if (poro && r >= nu + 8) {
      const int k = r - nu - 8;
      if (L.z)
        for (int j = 0; j < 4; ++j) acc -= mpP.tau * moment3(G, k, j) * L.z[ec[nu + 8 + j] >> 3];
      const double* eta = eta_prev + m.soff[s];
      for (int j = 0; j < 4; ++j) acc -= moment3(G, k, j) * eta[eld[nu + 4 + j]];
    }
    const double* Kr = m.emat + e * edof * edof + r;
    for (int c = 0; c < edof; ++c) {
      if (eld[c] >= 0) continue;
      const int32_t code = ec[c];
      if (code < 0) continue;
      const double gv = dirichlet_value3(L, code, nu3);
      if (gv != 0.0) acc -= Kr[(int64_t)c * edof] * gv;
    }
  }
  m.ebuf[gid] = acc;
}

void launch_elem_store3d(const DevMesh& m, MatParams mpP, MatParams mpE, hipStream_t st) {
  const int64_t n = (int64_t)m.nelem * m.edof;
  hipLaunchKernelGGL(k_elem_store3d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m, mpP, mpE);
}

void launch_assemble3d(const DevMesh& m, double* K, hipStream_t st) {
  const int64_t n = (int64_t)m.nelem * m.edof;
  for (int c = 0; c < 48; ++c)
    hipLaunchKernelGGL(k_assemble3d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m, K, m.kofs, m.ld, c);
}

void launch_rhs3d(const DevMesh& m, const double* eta_prev, double* f, MatParams mpP, const LoadDev& L,
                  hipStream_t st) {
  const int64_t n = (int64_t)m.nelem * m.edof;
  hipLaunchKernelGGL(k_rhs3d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m, eta_prev, mpP, L);
  launch_gather_elem(m, f, st);
}

}  // namespace feti
