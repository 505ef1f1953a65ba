// Device-side finite element formulas on tetrahedra (the d = 3 case of Section 2).
//
// The unit cube is cut into n^3 cubes, each into the six Kuhn tetrahedra around its main
// diagonal: for the axis permutation (a, b, c) of type t the vertices are v0 = the cube's
// lower corner, v1 = v0 + h e_a, v2 = v1 + h e_b, v3 = v0 + h (1, 1, 1).  The element
// matrices of the forms of Section 2.3 are integrated exactly in closed form: every basis
// gradient is a linear form sum_m c_m lambda_m in the barycentric coordinates, and
// int lambda^alpha = 6 |T| alpha! / (|alpha| + 3)!  (|T| the volume), so
// int lambda_m lambda_n = |T| (1 + delta_mn) / 20.
//
// Element DOF order: displacement (node-major, x, y, z components) over the 4 (P1) or 10
// (P2: vertices, then the midpoints of edges 01, 02, 03, 12, 13, 23) nodes, then for a
// poroelastic element xi_P, eta, p at the 4 vertices, for an elastic element xi_E at the 4
// vertices.
#pragma once

#include <hip/hip_runtime.h>

#include "fem_device.h"

namespace feti {

struct ElemGeom3 {
  double g[4][3];  // grad lambda_i
  double vol;
};

__host__ __device__ inline void tet_perm(int type, int& a, int& b) {
  // axis permutations (a, b, c) in the order (0,1,2) (0,2,1) (1,0,2) (1,2,0) (2,0,1) (2,1,0)
  a = type / 2;
  const int r = type % 2;
  b = a == 0 ? 1 + r : (a == 1 ? 2 * r : r);
}

__host__ __device__ inline void elem_geom3(int cell, int type, int ncell, ElemGeom3& G) {
  const int i = cell % ncell, j = (cell / ncell) % ncell, k = cell / (ncell * ncell);
  (void)i; (void)j; (void)k;  // the gradients do not depend on the cube's position
  const double h = 1.0 / ncell;
  int a, b;
  tet_perm(type, a, b);
  // edge vectors from v0: e1 = h e_a, e2 = h (e_a + e_b), e3 = h (1, 1, 1)
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // J[row = coordinate][col = edge]
  J[a][0] = h;
  J[a][1] = h; J[b][1] = h;
  J[0][2] = h; J[1][2] = h; J[2][2] = h;
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  // rows of J^{-1} are the gradients of lambda_1..3 (cofactors / det)
  double inv[3][3];
  inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  for (int d = 0; d < 3; ++d) {
    G.g[1][d] = inv[0][d];
    G.g[2][d] = inv[1][d];
    G.g[3][d] = inv[2][d];
    G.g[0][d] = -(inv[0][d] + inv[1][d] + inv[2][d]);
  }
  G.vol = (det < 0 ? -det : det) / 6.0;
}

// edge e of the P2 tetrahedron: vertices (p, q)
__host__ __device__ inline void tet_edge(int e, int& p, int& q) {
  const int P[6] = {0, 0, 0, 1, 1, 2}, Q[6] = {1, 2, 3, 2, 3, 3};
  p = P[e];
  q = Q[e];
}

// coefficient of lambda_m in d/dx_d of displacement basis function a
__host__ __device__ inline double grad_coef3(int order, const ElemGeom3& G, int a, int m, int d) {
  if (order == 1) return G.g[a][d];
  if (a < 4) return (m == a ? 3.0 : -1.0) * G.g[a][d];  // (4 lambda_a - sum lambda) grad lambda_a
  int p, q;
  tet_edge(a - 4, p, q);
  double v = 0.0;
  if (m == q) v += 4.0 * G.g[p][d];
  if (m == p) v += 4.0 * G.g[q][d];
  return v;
}

__host__ __device__ inline double moment3(const ElemGeom3& G, int m, int n) {
  return G.vol * (m == n ? 2.0 : 1.0) / 20.0;
}

__host__ __device__ inline double dd_int3(int order, const ElemGeom3& G, int a, int d, int b, int e) {
  double s = 0.0;
  for (int m = 0; m < 4; ++m) {
    const double ca = grad_coef3(order, G, a, m, d);
    if (ca == 0.0) continue;
    for (int n = 0; n < 4; ++n) s += ca * grad_coef3(order, G, b, n, e) * moment3(G, m, n);
  }
  return s;
}

// int lambda_k d_e phi_b
__host__ __device__ inline double vd_int3(int order, const ElemGeom3& G, int k, int b, int e) {
  double s = 0.0;
  for (int n = 0; n < 4; ++n) s += grad_coef3(order, G, b, n, e) * moment3(G, k, n);
  return s;
}

// Entry (r, c) of the element matrix in the element DOF order above.
__host__ __device__ inline double elem_entry3(int order, bool poro, const ElemGeom3& G, const MatParams& mp, int r,
                                              int c) {
  const int nu = order == 2 ? 30 : 12;
  const bool ru = r < nu, cu = c < nu;
  if (ru && cu) {
    const int a = r / 3, ca = r % 3, b = c / 3, cb = c % 3;
    double v = dd_int3(order, G, a, cb, b, ca);
    if (ca == cb) v += dd_int3(order, G, a, 0, b, 0) + dd_int3(order, G, a, 1, b, 1) + dd_int3(order, G, a, 2, b, 2);
    return mp.mu * v;
  }
  if (ru || cu) {
    const int su = ru ? r : c, ss = ru ? c - nu : r - nu;
    if (ss >= 4) return 0.0;  // only xi couples with u
    return -vd_int3(order, G, ss, su / 3, su % 3);
  }
  const int fr = (r - nu) / 4, fc = (c - nu) / 4;  // 0 xi, 1 eta, 2 p
  const int kr = (r - nu) % 4, kc = (c - nu) % 4;
  const double mass = moment3(G, kr, kc);
  if (!poro) return (fr == 0 && fc == 0) ? -mp.lam_inv * mass : 0.0;
  if (fr == 0 && fc == 0) return -mp.kap3 * mass;
  if ((fr == 0 && fc == 1) || (fr == 1 && fc == 0)) return mp.kap1 * mass;
  if (fr == 1 && fc == 1) return mp.kap2 * mass;
  if ((fr == 1 && fc == 2) || (fr == 2 && fc == 1)) return -mass;
  if (fr == 2 && fc == 2)
    return -mp.tau * mp.kf * G.vol * (G.g[kr][0] * G.g[kc][0] + G.g[kr][1] * G.g[kc][1] + G.g[kr][2] * G.g[kc][2]);
  return 0.0;
}

// int phi_a phi_b of the scalar P_order basis (the mass of the load interpolants): each P2
// function as a homogeneous quadratic in lambda, vertex a: lambda_a^2 - sum_{k != a}
// lambda_a lambda_k, edge (p, q): 4 lambda_p lambda_q, and int lambda^alpha = 6 |T| alpha! / 7!
// for |alpha| = 4.
__host__ __device__ inline double mass_p(int order, const ElemGeom3& G, int a, int b) {
  if (order == 1) return moment3(G, a, b);
  int ti[2][4], tj[2][4], nt[2];
  double tc[2][4];
  const int fn[2] = {a, b};
  for (int f = 0; f < 2; ++f) {
    const int x = fn[f];
    if (x < 4) {
      nt[f] = 4;
      ti[f][0] = x; tj[f][0] = x; tc[f][0] = 1.0;
      int t = 1;
      for (int k = 0; k < 4; ++k)
        if (k != x) { ti[f][t] = x; tj[f][t] = k; tc[f][t] = -1.0; ++t; }
    } else {
      nt[f] = 1;
      tet_edge(x - 4, ti[f][0], tj[f][0]);
      tc[f][0] = 4.0;
    }
  }
  const double fact[5] = {1.0, 1.0, 2.0, 6.0, 24.0};
  double s = 0.0;
  for (int u = 0; u < nt[0]; ++u)
    for (int v = 0; v < nt[1]; ++v) {
      int cnt[4] = {0, 0, 0, 0};
      ++cnt[ti[0][u]]; ++cnt[tj[0][u]]; ++cnt[ti[1][v]]; ++cnt[tj[1][v]];
      s += tc[0][u] * tc[1][v] * fact[cnt[0]] * fact[cnt[1]] * fact[cnt[2]] * fact[cnt[3]];
    }
  return s * 6.0 * G.vol / 5040.0;
}

}  // namespace feti
