// Device helpers of the interface kernels: the signed Boolean gather B_s^T, the
// jump rows of sum_s B_s (plain and (B B^T)^{-1}-weighted), the rows of the
// coarse matrix G = [B_s R_s] and the relative residual of the stopping test.
#pragma once

#include "kernels.h"
#include "iface.h"

namespace feti {

// Multiplier-space value gathered onto interface DOF gb.
__device__ inline double gather_b(const DevMesh& m, const double* __restrict__ v, int64_t gb,
                                  int mode) {
  if (mode == G_SIGNED) {
    double s = 0.0;
    const int r0 = m.bg_row[2 * gb], r1 = m.bg_row[2 * gb + 1];
    if (r0 >= 0) s += m.bg_sign[2 * gb] * v[r0];
    if (r1 >= 0) s += m.bg_sign[2 * gb + 1] * v[r1];
    return s;
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int r = m.bd_row[3 * gb + k];
    if (r >= 0) s += m.bd_wt[3 * gb + k] * v[r];
  }
  return s;
}

// Relative residual of the iteration: the largest of the dual-energy ratio
// |w|_M / ref_M and the per-kind ratios |w_k| / ref_k over the kinds whose
// reference energy is not negligible (a kind without load data, whose jump
// only carries rounding, is judged by the energy ratio alone).
// w2: per-kind |w_k|^2; etot: |w|_M^2.
__device__ inline double rel_residual_of(const double* w2, double etot, const double* sc) {
  double eref = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) eref += sc[SC_EK + k];
  const double den = sc[SC_EREF];
  double rel = den > 0.0 ? sqrt(etot) / den : (etot > 0.0 ? 1.0 : 0.0);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double rk = sc[SC_REF + k] > 0.0 ? sqrt(w2[k]) / sc[SC_REF + k] : 0.0;
    rel = sc[SC_EK + k] > 1e-24 * eref ? fmax(rel, rk) : rel;
  }
  return rel;
}
// v: reduced sums, per-kind |w_k|^2 in v[2..7], per-kind energies in v[8..13]
__device__ inline double rel_residual(const double* v, const double* sc) {
  double etot = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) etot += v[8 + k];
  return rel_residual_of(v + 2, etot, sc);
}

// Update test, used for the FP64 refinement corrections.  A correction only has to
// shrink the error of the first solve by a few orders, and the residual of such a
// noise-driven interface problem keeps wandering long after its solution has
// settled, so the iteration may also stop on the size of its updates: once, for
// every field kind k that has nonzero multipliers, the last UPD_WIN updates
// |alpha| |p|_k sum to at most utol |lambda|_k.  ring holds UPD_WIN x 6 sizes (slot
// iters mod UPD_WIN receives this update's); p2, l2: per-kind |p|^2 and |lambda|^2
// after the update.  Returns whether the test is met (never when utol <= 0 or
// before UPD_WIN updates).
__device__ inline bool update_converged(double* ring, int iters, double alpha, const double* p2,
                                        const double* l2, double utol) {
  double* slot = ring + (iters % UPD_WIN) * 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) slot[k] = fabs(alpha) * sqrt(p2[k]);
  bool ok = utol > 0.0 && iters >= UPD_WIN, any = false;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const bool has = l2[k] > 0.0;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < UPD_WIN; ++i) s += ring[i * 6 + k];
    ok = ok && (!has || s <= utol * sqrt(l2[k]));
    any = any || has;
  }
  return ok && any;
}

__device__ inline double jump_raw(const DevMesh& m, const double* __restrict__ yb, int from_torn,
                                  int64_t r) {
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int64_t gb = m.jr_b[2 * r + e];
    const int64_t idx = from_torn ? (int64_t)m.b_torn[gb] : gb;
    s += m.jr_sign[2 * r + e] * yb[idx];
  }
  return s;
}

// signed jump of row j, or its (B B^T)^{-1}-weighted version over the row's group
__device__ inline double jump_row(const DevMesh& m, const double* __restrict__ yb, int from_torn,
                                  int64_t j, int scaled) {
  if (!scaled) return jump_raw(m, yb, from_torn, j);
  const int gs = m.grp_start[j], gz = m.grp_size[j];
  double s = 0.0;
  for (int k = 0; k < gz; ++k) s += m.dwt[3 * j + k] * jump_raw(m, yb, from_torn, gs + k);
  return s;
}

__device__ inline double coarse_G_row(const DevMesh& m, const double* __restrict__ a, int64_t j) {
  if (m.defl_col) {  // dual-primal coupling: the deflation vectors take the place of G
    double v = 0.0;
    for (int e = 0; e < 2; ++e) {
      const int c = m.defl_col[2 * j + e];
      if (c >= 0) v += m.defl_w[2 * j + e] * a[c];
    }
    return v;
  }
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int64_t gb = m.jr_b[2 * j + e];
    const int f = m.sub_float[m.b_sub[gb]];
    if (f < 0) continue;
    const double* R = m.rb + 3 * gb;
    s += m.jr_sign[2 * j + e] * (R[0] * a[3 * f] + R[1] * a[3 * f + 1] + R[2] * a[3 * f + 2]);
  }
  return s;
}

}  // namespace feti
