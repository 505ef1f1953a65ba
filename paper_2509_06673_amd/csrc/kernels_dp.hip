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

// ---- deflation by the normal-flux vectors ----------------------------------------
// The interface operator of the dual-primal coupling keeps, as nu -> 1/2, an eigenvalue
// near zero whose eigenvector is the uniform normal traction on the subdomain faces (the
// hydrostatic pressure mode).  The iteration is deflated by W = one vector per face, the
// face integrals of the normal-component basis functions (q^T B u = the integral of the
// jump of the normal displacement over the face): the start takes the W-component of the
// residual exactly, and every search direction is made F-orthogonal to W.

__global__ void __launch_bounds__(256) k_defl_column(DevMesh m, int c, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m.n_lambda) return;
  double v = 0.0;
  for (int e = 0; e < 2; ++e)
    if (m.defl_col[2 * j + e] == c) v += m.defl_w[2 * j + e];
  out[j] = v;
}

__device__ inline double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// g_c = sum over the rows j of column c of w_j v_j (one block per column, fixed order)
__global__ void __launch_bounds__(256) k_defl_wt(DevMesh m, const double* __restrict__ v, double* __restrict__ g,
                                                 const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double red[256];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int k = m.defl_ptr[c] + threadIdx.x; k < m.defl_ptr[c + 1]; k += 256) acc += m.defl_rw[k] * v[m.defl_rows[k]];
  const double s = block_sum256(acc, red);
  if (threadIdx.x == 0) g[c] = s;
}

// g_c = sum_j FW[c][j] z_j (column c of F W, contiguous): block (c, k) sums the rows of
// chunk k into part[c][k]; k_defl_apply adds the DEFL_CHUNKS partials of a column in order
__global__ void __launch_bounds__(256) k_defl_fwt(DevMesh m, const double* __restrict__ FW, const double* __restrict__ z,
                                                  double* __restrict__ part, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double red[256];
  const int c = blockIdx.x, k = blockIdx.y;
  const int64_t len = (m.n_lambda + DEFL_CHUNKS - 1) / DEFL_CHUNKS;
  const int64_t j0 = k * len, j1 = min(m.n_lambda, j0 + len);
  const double* col = FW + (int64_t)c * m.n_lambda;
  double acc = 0.0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) acc += col[j] * z[j];
  const double s = block_sum256(acc, red);
  if (threadIdx.x == 0) part[c * DEFL_CHUNKS + k] = s;
}

// a = E^{-1} g with g_d = the DEFL_CHUNKS partials of column d summed in order: one
// wavefront per row of the dense E^{-1}, each lane forming the g_d it multiplies (the
// order of both sums is that of a separate chunk sum followed by the dense coarse apply)
__global__ void __launch_bounds__(256) k_defl_apply(int n, const double* __restrict__ part,
                                                    const double* __restrict__ Einv, double* __restrict__ a,
                                                    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* Er = Einv + (int64_t)row * n;
  double s = 0.0;
  for (int d = lane; d < n; d += 64) {
    double g = 0.0;
    for (int k = 0; k < DEFL_CHUNKS; ++k) g += part[d * DEFL_CHUNKS + k];
    s += Er[d] * g;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) a[row] = s;
}

// E[c][d] = (W^T F W)_{cd} symmetrised: (sum over the rows of c of w_j FW[d][j] + the same
// with c and d exchanged) / 2 (one block per entry)
__global__ void __launch_bounds__(256) k_defl_gram(DevMesh m, const double* __restrict__ FW, double* __restrict__ E) {
  __shared__ double red[256];
  const int c = blockIdx.x, d = blockIdx.y, n = m.n_defl;
  double acc = 0.0;
  for (int k = m.defl_ptr[c] + threadIdx.x; k < m.defl_ptr[c + 1]; k += 256)
    acc += m.defl_rw[k] * FW[(int64_t)d * m.n_lambda + m.defl_rows[k]];
  for (int k = m.defl_ptr[d] + threadIdx.x; k < m.defl_ptr[d + 1]; k += 256)
    acc += m.defl_rw[k] * FW[(int64_t)c * m.n_lambda + m.defl_rows[k]];
  const double s = block_sum256(acc, red);
  if (threadIdx.x == 0) E[(int64_t)c * n + d] = 0.5 * s;
}

void launch_defl_column(const DevMesh& m, int c, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_defl_column, dim3((unsigned)((m.n_lambda + 255) / 256)), dim3(256), 0, st, m, c, out);
}

void launch_defl_wt(const DevMesh& m, const double* v, double* g, const int32_t* skip, hipStream_t st) {
  if (m.n_defl == 0) return;
  hipLaunchKernelGGL(k_defl_wt, dim3(m.n_defl), dim3(256), 0, st, m, v, g, skip);
}

void launch_defl_fwt_apply(const DevMesh& m, const double* FW, const double* z, const double* Einv, double* a,
                           double* part, const int32_t* skip, hipStream_t st) {
  if (m.n_defl == 0) return;
  hipLaunchKernelGGL(k_defl_fwt, dim3(m.n_defl, DEFL_CHUNKS), dim3(256), 0, st, m, FW, z, part, skip);
  hipLaunchKernelGGL(k_defl_apply, dim3((m.n_defl + 3) / 4), dim3(256), 0, st, m.n_defl, part, Einv, a, skip);
}

void launch_defl_gram(const DevMesh& m, const double* FW, double* E, hipStream_t st) {
  if (m.n_defl == 0) return;
  hipLaunchKernelGGL(k_defl_gram, dim3(m.n_defl, m.n_defl), dim3(256), 0, st, m, FW, E);
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
