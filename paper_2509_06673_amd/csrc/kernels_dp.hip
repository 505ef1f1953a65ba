// Dual-primal coupling: the primal coarse problem that ties the subdomains together.
//
// The shared xi / p DOFs and the shared DOFs at the corners of the subdomain grid are one
// global unknown each (primal); multipliers glue only the other shared DOFs.  Each local
// matrix is swept over every DOF but its primal ones (r), which leaves
//     N_s = [[K_rr^{-1}, -K_rr^{-1} K_rPi], [-K_Pir K_rr^{-1}, -S_s]],
//     S_s = K_PiPi - K_Pir K_rr^{-1} K_rPi,
// and the primal coarse matrix is S_PiPi = sum_s L_s^T S_s L_s (L_s: the subdomain's
// primal DOFs in the global primal order).  The kernels here move values between the
// subdomains' primal DOFs and the global primal vector, and assemble S_PiPi.
#include "kernels.h"

namespace feti {

// out[k] = sum over the owners o of primal DOF k of t1[torn(o)] + t2[torn(o)] + cy yb[o]
__global__ void __launch_bounds__(256) k_pi_gather(DevMesh m, const double* __restrict__ t1,
                                                   const double* __restrict__ t2, const double* __restrict__ yb,
                                                   double cy, double* __restrict__ out,
                                                   const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m.n_pi) return;
  double acc = 0.0;
  for (int e = 0; e < PI_SLOTS; ++e) {
    const int gb = m.pi_own[PI_SLOTS * k + e];
    if (gb < 0) break;
    const int64_t ti = m.b_torn[gb];
    double v = 0.0;
    if (t1) v += t1[ti];
    if (t2) v += t2[ti];
    if (yb) v += cy * yb[gb];
    acc += v;
  }
  out[k] = acc;
}

// u[torn(gb)] = upi[bpi[gb]] at every primal interface DOF gb
__global__ void __launch_bounds__(256) k_pi_scatter(DevMesh m, const double* __restrict__ upi,
                                                    double* __restrict__ u) {
  const int64_t gb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gb >= m.sum_nb) return;
  const int k = m.bpi[gb];
  if (k >= 0) u[m.b_torn[gb]] = upi[k];
}

// r at the owners of primal DOF k: the first owner receives the sum, the others zero
__global__ void __launch_bounds__(256) k_pi_fold(DevMesh m, double* __restrict__ r) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m.n_pi) return;
  double acc = 0.0;
  for (int e = 0; e < PI_SLOTS; ++e) {
    const int gb = m.pi_own[PI_SLOTS * k + e];
    if (gb < 0) break;
    acc += r[m.b_torn[gb]];
  }
  for (int e = 0; e < PI_SLOTS; ++e) {
    const int gb = m.pi_own[PI_SLOTS * k + e];
    if (gb < 0) break;
    r[m.b_torn[gb]] = e == 0 ? acc : 0.0;
  }
}

// S[K][L] -= A_s[a][b] over the primal pairs (a, b) of the subdomains of one colour of the
// 2 x 2 (x 2 in 3D) colouring of the subdomain grid (two subdomains of a colour share no
// node, so each launch writes every entry at most once; the colours run in a fixed order)
__global__ void __launch_bounds__(256) k_pi_assemble(DevMesh m, const double* __restrict__ A,
                                                     double* __restrict__ S, int colour) {
  const int s = blockIdx.y;
  const int sx = s % m.nsub_x, sy = (s / m.nsub_x) % m.nsub_y, sz = s / (m.nsub_x * m.nsub_y);
  if ((sx & 1) + 2 * (sy & 1) + 4 * (sz & 1) != colour) return;
  const int np = m.npi[s];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)np * np) return;
  const int a = (int)(e / np), b = (int)(e % np);
  const int nbs = m.nb[s], base = nbs - np;
  const int64_t gb0 = m.boff[s] + base;
  const int K = m.bpi[gb0 + a], L = m.bpi[gb0 + b];
  S[(int64_t)K * m.n_pi + L] -= A[m.sofs[s] + (int64_t)(base + a) * m.ldb[s] + base + b];
}

void launch_pi_gather(const DevMesh& m, const double* t1, const double* t2, const double* yb, double cy, double* out,
                      const int32_t* skip, hipStream_t st) {
  if (m.n_pi == 0) return;
  hipLaunchKernelGGL(k_pi_gather, dim3((m.n_pi + 255) / 256), dim3(256), 0, st, m, t1, t2, yb, cy, out, skip);
}

void launch_pi_scatter(const DevMesh& m, const double* upi, double* u, hipStream_t st) {
  if (m.n_pi == 0 || m.sum_nb == 0) return;
  hipLaunchKernelGGL(k_pi_scatter, dim3((unsigned)((m.sum_nb + 255) / 256)), dim3(256), 0, st, m, upi, u);
}

void launch_pi_fold(const DevMesh& m, double* r, hipStream_t st) {
  if (m.n_pi == 0) return;
  hipLaunchKernelGGL(k_pi_fold, dim3((m.n_pi + 255) / 256), dim3(256), 0, st, m, r);
}

void launch_pi_assemble(const DevMesh& m, const double* A, double* S, hipStream_t st) {
  if (m.n_pi == 0 || m.max_npi == 0) return;
  const int64_t cnt = (int64_t)m.max_npi * m.max_npi;
  const int ncol = m.nsub > m.nsub_x * m.nsub_y ? 8 : 4;
  for (int c = 0; c < ncol; ++c)
    hipLaunchKernelGGL(k_pi_assemble, dim3((unsigned)((cnt + 255) / 256), m.nsub), dim3(256), 0, st, m, A, S, c);
}

}  // namespace feti
