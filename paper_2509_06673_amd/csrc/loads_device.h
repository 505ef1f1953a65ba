// Analytic loads, boundary data and initial data evaluated on the device.
//
// MANUFACTURED: the smooth solution of Section 4.1,
//   u_P = sin(2 pi x) sin(2 pi y) (1, 1),   p = sin(pi x) sin(pi y),
//   u_E = u_P + beta p (x - 1/2) e_x  (x-split)  or  u_P + beta p (y - 1/2) e_y (y-split),
//   beta = -alpha / (lambda_P + 2 mu_P),
// with the body forces and the source that the governing equations (2.1)-(2.3)
// give for it (stationary, gravity off):
//   f_P = -(lambda+mu) grad div u_P - mu Lap u_P + alpha grad p,
//   f_E = -(lambda_E+mu_E) grad div u_E - mu_E Lap u_E,    z = -(K/mu_f) Lap p.
// Derivatives are written out by hand here.
// PATCH: polynomial u_P (degree <= 2) and p (degree <= 1) with the same
// interface correction, loads constant.  PERIODIC and POINT_SOURCE: the
// time-dependent loads of the learned-start and pulsed-source workloads with
// zero boundary and initial data.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/feti.h"

namespace feti {

struct LoadDev {
  int kind;
  int layout;
  double t;
  double prm[16];
  double lamP, muP, lamE, muE, alpha, c0, kf;
  // FETI_LOAD_RAW: caller data on the lattices (see feti_load) and the sides without
  // u / p Dirichlet data (traction / flux sides)
  const double *f_p, *f_e, *z, *t_side, *zw_side, *g_u, *g_p, *eta0;
  uint32_t dir_u, dir_p;
  // decoupled scheme: the fluid content eta^n of the step on the P1 lattice (the
  // prescribed eta columns of the momentum rows read it); null otherwise
  const double* eta_dec;
};

// 7-point degree-5 rule of Radon on a triangle (barycentric points, weights summing to 1):
// the centroid, and the orbits (a, a, 1 - 2a) with a = (6 -+ sqrt(15)) / 21.
__host__ __device__ inline void radon_point(int q, double& l0, double& l1, double& l2, double& w) {
  const double s15 = 3.872983346207416885;  // sqrt(15)
  if (q == 0) { l0 = l1 = l2 = 1.0 / 3.0; w = 9.0 / 40.0; return; }
  const bool first = q <= 3;
  const double a = first ? (6.0 - s15) / 21.0 : (6.0 + s15) / 21.0;
  const double b = 1.0 - 2.0 * a;
  w = first ? (155.0 - s15) / 1200.0 : (155.0 + s15) / 1200.0;
  const int r = (q - 1) % 3;
  l0 = r == 2 ? b : a;
  l1 = r == 1 ? b : a;
  l2 = r == 0 ? b : a;
}

struct Trig {
  double s2x, c2x, s2y, c2y, sx, cx, sy, cy;
};

__host__ __device__ inline Trig trig(double x, double y) {
  const double pi = 3.14159265358979323846;
  Trig t;
  t.s2x = sin(2 * pi * x); t.c2x = cos(2 * pi * x);
  t.s2y = sin(2 * pi * y); t.c2y = cos(2 * pi * y);
  t.sx = sin(pi * x); t.cx = cos(pi * x);
  t.sy = sin(pi * y); t.cy = cos(pi * y);
  return t;
}

// body force (fx, fy) in region poro/elastic at (x, y, t)
__host__ __device__ inline void body_force(const LoadDev& L, bool poro, double x, double y,
                                           double& fx, double& fy) {
  const double pi = 3.14159265358979323846;
  if (L.kind == FETI_LOAD_MANUFACTURED) {
    const Trig T = trig(x, y);
    const double a2 = 4 * pi * pi;
    const double s = T.s2x * T.s2y, cc = T.c2x * T.c2y;
    const double sxx = -a2 * s, syy = -a2 * s, sxy = a2 * cc, lap = -2 * a2 * s;
    const double lam = poro ? L.lamP : L.lamE, mu = poro ? L.muP : L.muE;
    // -div sigma(u_P) for u_P = (s, s)
    fx = -((lam + mu) * (sxx + sxy) + mu * lap);
    fy = -((lam + mu) * (sxy + syy) + mu * lap);
    const double p = T.sx * T.sy, px = pi * T.cx * T.sy, py = pi * T.sx * T.cy;
    if (poro) {
      fx += L.alpha * px;
      fy += L.alpha * py;
      return;
    }
    const double pxx = -pi * pi * p, pyy = -pi * pi * p, pxy = pi * pi * T.cx * T.cy;
    const double beta = -L.alpha / (L.lamP + 2 * L.muP);
    if (L.layout == FETI_YSPLIT) {
      const double ym = y - 0.5;
      const double qyy = pyy * ym + 2 * py, qxy = pxy * ym + px, lapq = (pxx + pyy) * ym + 2 * py;
      fx -= (lam + mu) * beta * qxy;
      fy -= (lam + mu) * beta * qyy + mu * beta * lapq;
    } else {
      const double xm = x - 0.5;
      const double qxx = pxx * xm + 2 * px, qxy = pxy * xm + py, lapq = (pxx + pyy) * xm + 2 * px;
      fx -= (lam + mu) * beta * qxx + mu * beta * lapq;
      fy -= (lam + mu) * beta * qxy;
    }
    return;
  }
  if (L.kind == FETI_LOAD_PATCH) {
    const double* a = L.prm;       // ux coefficients of 1, x, y, x^2, xy, y^2
    const double* b = L.prm + 6;   // uy coefficients
    const double c1 = L.prm[13];   // p = c0 + c1 y
    const double lam = poro ? L.lamP : L.lamE, mu = poro ? L.muP : L.muE;
    const double gdx = 2 * a[3] + b[4], gdy = a[4] + 2 * b[5];
    const double lx = 2 * a[3] + 2 * a[5], ly = 2 * b[3] + 2 * b[5];
    fx = -((lam + mu) * gdx + mu * lx);
    fy = -((lam + mu) * gdy + mu * ly);
    if (poro) {
      fy += L.alpha * c1;
      return;
    }
    const double beta = -L.alpha / (L.lamP + 2 * L.muP);
    if (L.layout == FETI_YSPLIT) {
      fy -= 2 * c1 * beta * (lam + 2 * mu);
    } else {
      fy -= (lam + mu) * beta * c1;
    }
    return;
  }
  if (L.kind == FETI_LOAD_PERIODIC) {
    const double amp = L.prm[0] * sin(L.prm[1] * L.t + L.prm[2]);
    const Trig T = trig(x, y);
    fx = amp * T.sx * T.sy;
    fy = amp * T.cx * T.sy;
    return;
  }
  fx = 0.0;
  fy = 0.0;
}

// fluid source z in the poroelastic region
__host__ __device__ inline double source(const LoadDev& L, double x, double y) {
  const double pi = 3.14159265358979323846;
  if (L.kind == FETI_LOAD_MANUFACTURED) {
    const Trig T = trig(x, y);
    return L.kf * 2 * pi * pi * T.sx * T.sy;
  }
  if (L.kind == FETI_LOAD_PERIODIC) {
    const Trig T = trig(x, y);
    return L.prm[0] * sin(L.prm[1] * L.t + L.prm[2]) * T.sx * T.sy;
  }
  if (L.kind == FETI_LOAD_POINT_SOURCE) {
    const double dx = x - L.prm[0], dy = y - L.prm[1], sg = L.prm[2];
    return sin(L.t) * exp(-(dx * dx + dy * dy) / (2 * sg * sg)) / (2 * pi * sg * sg);
  }
  return 0.0;
}

__host__ __device__ inline double exact_p(const LoadDev& L, double x, double y) {
  if (L.kind == FETI_LOAD_MANUFACTURED) {
    const double pi = 3.14159265358979323846;
    return sin(pi * x) * sin(pi * y);
  }
  if (L.kind == FETI_LOAD_PATCH) return L.prm[12] + L.prm[13] * y;
  return 0.0;
}

// exact displacement component comp in region poro/elastic (Dirichlet data, initial data)
__host__ __device__ inline double exact_u(const LoadDev& L, bool poro, int comp, double x, double y) {
  double u = 0.0;
  if (L.kind == FETI_LOAD_MANUFACTURED) {
    const double pi = 3.14159265358979323846;
    u = sin(2 * pi * x) * sin(2 * pi * y);
  } else if (L.kind == FETI_LOAD_PATCH) {
    const double* a = comp == 0 ? L.prm : L.prm + 6;
    u = a[0] + a[1] * x + a[2] * y + a[3] * x * x + a[4] * x * y + a[5] * y * y;
  } else {
    return 0.0;
  }
  if (!poro) {
    const double beta = -L.alpha / (L.lamP + 2 * L.muP);
    const double p = exact_p(L, x, y);
    if (L.layout == FETI_YSPLIT) {
      if (comp == 1) u += beta * p * (y - 0.5);
    } else {
      if (comp == 0) u += beta * p * (x - 0.5);
    }
  }
  return u;
}

// eta_0 = c0 p_0 + alpha div u_0 (eq. (mreform)) of the poroelastic initial data
__host__ __device__ inline double initial_eta(const LoadDev& L, double x, double y) {
  double divu = 0.0;
  if (L.kind == FETI_LOAD_MANUFACTURED) {
    const double pi = 3.14159265358979323846;
    const double a = 2 * pi;
    divu = a * cos(a * x) * sin(a * y) + a * sin(a * x) * cos(a * y);
  } else if (L.kind == FETI_LOAD_PATCH) {
    const double* a = L.prm;
    const double* b = L.prm + 6;
    divu = a[1] + 2 * a[3] * x + a[4] * y + b[2] + b[4] * x + 2 * b[5] * y;
  } else {
    return 0.0;
  }
  return L.c0 * exact_p(L, x, y) + L.alpha * divu;
}

}  // namespace feti
