// Device-side finite element formulas shared by the assembly, right-hand
// side and residual kernels.
//
// Element matrices of the bilinear forms of Section 2.3 on affine triangles,
//   (aD) 2 mu (eps(u), eps(v)),  (bD) -(xi, div v),  (af) (K/mu_f)(grad p, grad q),
// and the P1 mass (phi_i, phi_j), integrated exactly in closed form: every
// basis gradient is written as a linear form sum_m g[m] lambda_m in the
// barycentric coordinates, and int lambda_m lambda_n = |T| (1 + delta_mn) / 12.
//
// Element DOF order: displacement (node-major, x then y component) over the
// 3 (P1) or 6 (P2: vertices, then midpoints of edges 01, 12, 20) nodes, then
// for a poroelastic element xi_P, eta, p at the 3 vertices, for an elastic
// element xi_E at the 3 vertices.
#pragma once

#include <hip/hip_runtime.h>

namespace feti {

struct ElemGeom {
  double x[3], y[3];   // vertices (counter-clockwise)
  double gx[3], gy[3]; // grad lambda_i
  double area;
};

struct MatParams {
  double mu;      // shear modulus
  double kap1, kap2, kap3;
  double lam_inv; // 1 / lambda_E (elastic)
  double kf;      // K / mu_f
  double tau;
};

__host__ __device__ inline void elem_geom(int cell, int type, int ncell, ElemGeom& g) {
  const int i = cell % ncell, j = cell / ncell;
  const double h = 1.0 / ncell;
  const double x0 = i * h, y0 = j * h;
  if (type == 0) {
    g.x[0] = x0; g.y[0] = y0; g.x[1] = x0 + h; g.y[1] = y0; g.x[2] = x0 + h; g.y[2] = y0 + h;
  } else {
    g.x[0] = x0; g.y[0] = y0; g.x[1] = x0 + h; g.y[1] = y0 + h; g.x[2] = x0; g.y[2] = y0 + h;
  }
  const double det = (g.x[1] - g.x[0]) * (g.y[2] - g.y[0]) - (g.x[2] - g.x[0]) * (g.y[1] - g.y[0]);
  g.area = 0.5 * det;
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    // grad lambda_a = perp(x_c - x_b) / (2 |T|), perp(v) = (-v_y, v_x)
    g.gx[a] = -(g.y[c] - g.y[b]) / det;
    g.gy[a] = (g.x[c] - g.x[b]) / det;
  }
}

// coefficient of lambda_m in d/dx_d of displacement basis function a
__host__ __device__ inline double grad_coef(int order, const ElemGeom& g, int a, int m, int d) {
  const double* G = d == 0 ? g.gx : g.gy;
  if (order == 1) return G[a];
  if (a < 3) return (m == a ? 3.0 : -1.0) * G[a];  // (4 lambda_a - sum lambda) grad lambda_a
  const int p = a - 3, q = (a - 2) % 3;             // edge (p, q): 01, 12, 20
  double v = 0.0;
  if (m == q) v += 4.0 * G[p];
  if (m == p) v += 4.0 * G[q];
  return v;
}

__host__ __device__ inline double moment2(const ElemGeom& g, int m, int n) {
  return g.area * (m == n ? 2.0 : 1.0) / 12.0;
}

// int d_d phi_a d_e phi_b over the element
__host__ __device__ inline double dd_int(int order, const ElemGeom& g, int a, int d, int b, int e) {
  double s = 0.0;
  for (int m = 0; m < 3; ++m) {
    const double ca = grad_coef(order, g, a, m, d);
    if (ca == 0.0) continue;
    for (int n = 0; n < 3; ++n) s += ca * grad_coef(order, g, b, n, e) * moment2(g, m, n);
  }
  return s;
}

// int lambda_k d_e phi_b
__host__ __device__ inline double vd_int(int order, const ElemGeom& g, int k, int b, int e) {
  double s = 0.0;
  for (int n = 0; n < 3; ++n) s += grad_coef(order, g, b, n, e) * moment2(g, k, n);
  return s;
}

// Entry (r, c) of the element matrix in the element DOF order above.
__host__ __device__ inline double elem_entry(int order, bool poro, const ElemGeom& g,
                                             const MatParams& mp, int r, int c) {
  const int nu = order == 2 ? 12 : 6;  // displacement DOFs
  const bool ru = r < nu, cu = c < nu;
  if (ru && cu) {
    const int a = r / 2, ca = r % 2, b = c / 2, cb = c % 2;
    double v = dd_int(order, g, a, cb, b, ca);
    if (ca == cb) v += dd_int(order, g, a, 0, b, 0) + dd_int(order, g, a, 1, b, 1);
    return mp.mu * v;
  }
  if (ru || cu) {
    // (xi, u) coupling: B[k][(b,e)] = -int lambda_k d_e phi_b; only the xi rows/cols couple
    const int su = ru ? r : c, ss = ru ? c - nu : r - nu;
    if (ss >= 3) return 0.0;
    return -vd_int(order, g, ss, su / 2, su % 2);
  }
  const int fr = (r - nu) / 3, fc = (c - nu) / 3;  // 0 xi, 1 eta, 2 p
  const int kr = (r - nu) % 3, kc = (c - nu) % 3;
  const double mass = moment2(g, kr, kc);
  if (!poro) {
    if (fr == 0 && fc == 0) return -mp.lam_inv * mass;
    return 0.0;
  }
  if (fr == 0 && fc == 0) return -mp.kap3 * mass;
  if ((fr == 0 && fc == 1) || (fr == 1 && fc == 0)) return mp.kap1 * mass;
  if (fr == 1 && fc == 1) return mp.kap2 * mass;
  if ((fr == 1 && fc == 2) || (fr == 2 && fc == 1)) return -mass;
  if (fr == 2 && fc == 2)
    return -mp.tau * mp.kf * g.area * (g.gx[kr] * g.gx[kc] + g.gy[kr] * g.gy[kc]);
  return 0.0;
}

}  // namespace feti
