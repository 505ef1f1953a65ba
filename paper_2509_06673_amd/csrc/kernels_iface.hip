// Interface kernels of the FETI iteration: batched symmetric GEMVs with the
// local inverses and Schur complements, the signed Boolean gather/scatter
// (B_s^T and sum_s B_s), the (B B^T)^{-1}-weighted gather/scatter of the
// Dirichlet preconditioner, the coarse space G = [B_s R_s], and the FP64
// vector updates and deterministic reductions of projected PCG.
#include <algorithm>

#include "bstep.h"
#include "kernels.h"
#include "iface.h"
#include "iface_device.h"

namespace feti {

// Scalar part of one PCG phase from the fully reduced sums v[NPART] (one thread).
__device__ void scalar_phase(const double* v, double* __restrict__ sc, int32_t* __restrict__ ist,
                             int phase) {
  switch (phase) {
    case PH_REFNORM: {
      // references from P d: per-kind norms and energies, total energy norm
      double e = 0.0;
      for (int k = 0; k < 6; ++k) {
        sc[SC_REF + k] = sqrt(v[2 + k]);
        sc[SC_EK + k] = v[8 + k];
        e += v[8 + k];
      }
      sc[SC_EREF] = sqrt(e);
      break;
    }
    case PH_INIT: {
      // rho = (w, y); the reference of each kind also covers its initial residual
      sc[SC_RHO] = v[0];
      double e = 0.0;
      for (int k = 0; k < 6; ++k) {
        sc[SC_REF + k] = fmax(sc[SC_REF + k], sqrt(v[2 + k]));
        sc[SC_EK + k] = fmax(sc[SC_EK + k], v[8 + k]);
        e += v[8 + k];
      }
      sc[SC_EREF] = fmax(sc[SC_EREF], sqrt(e));
      const double rel = rel_residual(v, sc);
      sc[SC_RES0] = rel;
      sc[SC_RES] = rel;
      ist[IS_ITERS] = 0;
      ist[IS_STATUS] = 0;
      ist[IS_DONE] = (rel <= sc[SC_TOL]) ? 1 : 0;
      if (!isfinite(v[0]) || !isfinite(rel)) { ist[IS_STATUS] = FETI_ENAN; ist[IS_DONE] = 1; }
      break;
    }
    case PH_ALPHA: {
      const double pq = v[0];
      if (!(fabs(pq) > 1e-300) || !isfinite(pq)) {
        ist[IS_STATUS] = isfinite(pq) ? FETI_EBREAKDOWN : FETI_ENAN;
        ist[IS_DONE] = 1;
        sc[SC_ALPHA] = 0.0;
        break;
      }
      sc[SC_ALPHA] = sc[SC_RHO] / pq;
      break;
    }
    case PH_CONV: {
      const double rel = rel_residual(v, sc);
      double et = 0.0;
      for (int k = 0; k < 6; ++k) {
        et += v[8 + k];
        sc[SC_KRAT + k] = sc[SC_REF + k] > 0.0 ? sqrt(v[2 + k]) / sc[SC_REF + k] : 0.0;
      }
      sc[SC_ERAT] = sc[SC_EREF] > 0.0 ? sqrt(et) / sc[SC_EREF] : 0.0;
      sc[SC_RES] = rel;
      ist[IS_ITERS] += 1;
      const bool upd = update_converged(sc + SC_URING, ist[IS_ITERS], sc[SC_ALPHA], v + 14, v + 20, sc[SC_UTOL]);
      for (int k = 0; k < 6; ++k) sc[SC_ULAM + k] = sqrt(v[20 + k]);
      if (!isfinite(rel)) { ist[IS_STATUS] = FETI_ENAN; ist[IS_DONE] = 1; }
      else if (rel <= sc[SC_TOL] || upd) ist[IS_DONE] = 1;
      else if (ist[IS_ITERS] >= ist[IS_MAXIT]) { ist[IS_STATUS] = FETI_ENOTCONV; ist[IS_DONE] = 1; }
      break;
    }
    case PH_BETA: {
      const double rho_new = v[0];
      if (!(fabs(sc[SC_RHO]) > 1e-300)) {
        ist[IS_STATUS] = FETI_EBREAKDOWN;
        ist[IS_DONE] = 1;
        break;
      }
      sc[SC_BETA] = rho_new / sc[SC_RHO];
      sc[SC_RHO] = rho_new;
      break;
    }
  }
}

// Block-wide sums of acc[0..NV) written to part[blockIdx.x] (stride NPART); the last
// block to finish sums all partials in block order (deterministic) and runs the
// phase.  counter must be zero on entry; the last block resets it.
template <int NV>
__device__ inline void block_sums(double (&v)[NPART], double (*red)[NV]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double x = v[c];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) red[wave][c] = x;
  }
  __syncthreads();
}

template <int NV>
__device__ void reduce_and_finalize(double (&acc)[NPART], double* __restrict__ part, int32_t* __restrict__ counter,
                                    double* __restrict__ sc, int32_t* __restrict__ ist, int phase, int bx, int nbx) {
  constexpr int NW = RED_BLOCK / 64;
  __shared__ double red[NW][NV];
  __shared__ int is_last;
  block_sums<NV>(acc, red);
  // the partials move between blocks through device-coherent stores and loads, and the
  // stores complete before the block is counted (no cache-wide fence needed)
  if (threadIdx.x < NV) {
    double x = 0.0;
    for (int w = 0; w < NW; ++w) x += red[w][threadIdx.x];
    __hip_atomic_store(part + bx * NPART + threadIdx.x, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x == 0)
    is_last = __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nbx - 1;
  __syncthreads();
  if (!is_last) return;
  const int nblk = nbx;
  double v[NPART];
#pragma unroll
  for (int c = 0; c < NPART; ++c) v[c] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += RED_BLOCK)
#pragma unroll
    for (int c = 0; c < NV; ++c)
      v[c] += __hip_atomic_load(part + b * NPART + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  block_sums<NV>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double x = 0.0;
      for (int w = 0; w < NW; ++w) x += red[w][c];
      v[c] = x;
    }
    scalar_phase(v, sc, ist, phase);
    *counter = 0;
  }
}

// y_s = A_s x_s for every subdomain s.  A_s is symmetric, so column k of the
// row-major block is read as row k: for a fixed k the 64 lanes of a wavefront
// read 64 consecutive entries.  Each workgroup owns 64 output rows; its four
// wavefronts split the k range and combine in LDS.  x_s is built in LDS.
// FULL = 1: the full local block (n = n_s, torn vectors); FULL = 0: the interface
// block (n = n_b, interface-space vectors).  The two are separate kernels so that
// profiles attribute the local solves and the interface iteration separately.
// MT is the stored matrix type (double, or float for the FP32 factors); vectors
// and accumulation are FP64.
template <int FULL, class MT>
__device__ __forceinline__ void sgemv_body(const DevMesh& m, const GemvArgs& a, int bx, int s) {
  if (a.skip && *a.skip) return;
  if (s >= m.nsub) return;
  const int ns = m.ns[s], nbs = m.nb[s];
  const int n = FULL ? ns : nbs;
  // row range [rlo, rhi) and column range [k0, chi)
  int rlo = 0, rhi = n, chi = n;
  if (!FULL && (a.rsel || a.csel)) {
    const int nd = nbs - m.npi[s];
    if (a.rsel == 1) rhi = nd;
    else if (a.rsel == 2) rlo = nd;
    if (a.csel == 1) chi = nd;
  }
  const int row0 = rlo + bx * 64;
  if (row0 >= rhi) return;
  extern __shared__ double smem[];
  double* xs = smem;              // n
  double* red = smem + m.max_ns;  // 4 x 64
  const int first_b = n - nbs;
  const int64_t xoff = FULL ? m.soff[s] : m.boff[s];
  for (int t = a.kb_only ? first_b + threadIdx.x : threadIdx.x; t < chi; t += blockDim.x) {
    double v = a.xbase ? a.xbase[xoff + t] : 0.0;
    if (a.gmode != G_NONE && t >= first_b) v += a.gcoef * gather_b(m, a.v, m.boff[s] + (t - first_b), a.gmode);
    if (a.pi_mode && t >= first_b) {
      const int q = m.bpi[m.boff[s] + (t - first_b)];
      if (q >= 0) v = a.pi_v ? a.pi_v[q] : 0.0;
    }
    xs[t] = v;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = row0 + lane;
  const int k0 = a.kb_only ? first_b : 0;
  const int kq = (chi - k0 + 3) / 4;
  const int kb = k0 + wave * kq, ke = min(chi, kb + kq);
  const MT* A = static_cast<const MT*>(a.A) + a.aofs[s];
  const int64_t ld = a.lda[s];
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  if (i < rhi) {
    // batches of eight independent column loads in flight before their FMAs
    const MT* col = A + (int64_t)kb * ld + i;
    int k = kb;
    for (; k + 8 <= ke; k += 8, col += 8 * ld) {
      MT v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = col[(int64_t)u * ld];
      acc0 += (double)v[0] * xs[k + 0];
      acc1 += (double)v[1] * xs[k + 1];
      acc2 += (double)v[2] * xs[k + 2];
      acc3 += (double)v[3] * xs[k + 3];
      acc0 += (double)v[4] * xs[k + 4];
      acc1 += (double)v[5] * xs[k + 5];
      acc2 += (double)v[6] * xs[k + 6];
      acc3 += (double)v[7] * xs[k + 7];
    }
    if (k < ke) {
      // the last (ke - k < 8) columns: loads together, products in order
      MT v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = k + u < ke ? col[(int64_t)u * ld] : (MT)0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k + u < ke) acc0 += (double)v[u] * xs[k + u];
    }
  }
  red[wave * 64 + lane] = (acc0 + acc1) + (acc2 + acc3);
  __syncthreads();
  if (wave == 0 && i < rhi) {
    double yv = (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
    if (a.ybase) yv += a.ybase[xoff + i];
    if (a.alpha_c) {
      const int f = m.sub_float[s];
      if (f >= 0) {
        const double* R = m.rfull + 3 * (m.soff[s] + i);
        yv += R[0] * a.alpha_c[3 * f] + R[1] * a.alpha_c[3 * f + 1] + R[2] * a.alpha_c[3 * f + 2];
      }
    }
    a.y[xoff + i] = yv;
  }
}

template <int FULL, class MT>
__global__ void __launch_bounds__(256) k_sgemv(DevMesh m, GemvArgs a) {
  sgemv_body<FULL, MT>(m, a, blockIdx.x, blockIdx.y);
}

// Blocks [0, nlb): out_j = jump_row(yb).  Blocks [nlb, nlb + n_float) (when g is
// given): g_f = R_b^T B_s^T out for the floating subdomain s = float_sub[f],
// evaluated from yb directly, so G^T out needs no second pass.
__device__ __forceinline__ void jump_body(const DevMesh& m, const double* __restrict__ yb, int from_torn,
                                          double* __restrict__ out, int scaled, double* __restrict__ g, int nlb,
                                          const int32_t* __restrict__ skip, int bx) {
  if (skip && *skip) return;
  if (bx < nlb) {
    const int64_t j = (int64_t)bx * blockDim.x + threadIdx.x;
    if (j < m.n_lambda) out[j] = jump_row(m, yb, from_torn, j, scaled);
    return;
  }
  const int f = bx - nlb;
  if (!g || f >= m.n_float) return;
  const int s = m.float_sub[f];
  const int nbs = m.nb[s];
  const int64_t b0 = m.boff[s];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nbs; i += blockDim.x) {
    const int64_t gb = b0 + i;
    double v = 0.0;
    for (int slot = 0; slot < 2; ++slot) {
      const int r = m.bg_row[2 * gb + slot];
      if (r >= 0) v += m.bg_sign[2 * gb + slot] * jump_row(m, yb, from_torn, r, scaled);
    }
    const double* R = m.rb + 3 * gb;
    acc[0] += R[0] * v;
    acc[1] += R[1] * v;
    acc[2] += R[2] * v;
  }
  __shared__ double red[3][256];
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) g[3 * f + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_jump(DevMesh m, const double* __restrict__ yb, int from_torn,
                                              double* __restrict__ out, int scaled,
                                              double* __restrict__ g, int nlb,
                                              const int32_t* __restrict__ skip) {
  jump_body(m, yb, from_torn, out, scaled, g, nlb, skip, blockIdx.x);
}

// g_f = R_s^T x_s for each floating subdomain s = float_sub[f], with
// x_s = base_s + gsign * B_s^T v (base torn and/or v multipliers).
__device__ __forceinline__ void coarse_g_body(const DevMesh& m, const double* __restrict__ v,
                                              const double* __restrict__ base, double gsign, double* __restrict__ g,
                                              const int32_t* __restrict__ skip, int f) {
  if (skip && *skip) return;
  if (f >= m.n_float) return;
  const int s = m.float_sub[f];
  const int ns = m.ns[s], nbs = m.nb[s], first_b = ns - nbs;
  const int64_t so = m.soff[s];
  double acc[3] = {0.0, 0.0, 0.0};
  // without a torn base only the interface part is nonzero
  for (int i = base ? threadIdx.x : first_b + threadIdx.x; i < ns; i += blockDim.x) {
    double x = base ? base[so + i] : 0.0;
    if (v && i >= first_b) x += gsign * gather_b(m, v, m.boff[s] + (i - first_b), G_SIGNED);
    const double* R = m.rfull + 3 * (so + i);
    acc[0] += R[0] * x;
    acc[1] += R[1] * x;
    acc[2] += R[2] * x;
  }
  __shared__ double red[3][256];
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) g[3 * f + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_coarse_g(DevMesh m, const double* __restrict__ v,
                                                  const double* __restrict__ base, double gsign,
                                                  double* __restrict__ g,
                                                  const int32_t* __restrict__ skip) {
  coarse_g_body(m, v, base, gsign, g, skip, blockIdx.x);
}

// a = scale * Cinv g (Cinv symmetric n_c x n_c): one wavefront per row
__device__ __forceinline__ void coarse_apply_body(int nc, const double* __restrict__ C, const double* __restrict__ g,
                                                  double* __restrict__ a, double scale,
                                                  const int32_t* __restrict__ skip, int bx) {
  if (skip && *skip) return;
  const int row = bx * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nc) return;
  const double* Cr = C + (int64_t)row * nc;
  double s = 0.0;
  // eight row entries per lane in flight, summed in the order of the plain loop
  int k = lane;
  for (; k + 7 * 64 < nc; k += 8 * 64) {
    double c[8], x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c[u] = Cr[k + u * 64];
      x[u] = g[k + u * 64];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += c[u] * x[u];
  }
  for (; k < nc; k += 64) s += Cr[k] * g[k];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) a[row] = scale * s;
}

__global__ void __launch_bounds__(256) k_coarse_apply(int nc, const double* __restrict__ C,
                                                      const double* __restrict__ g,
                                                      double* __restrict__ a, double scale,
                                                      const int32_t* __restrict__ skip) {
  coarse_apply_body(nc, C, g, a, scale, skip, blockIdx.x);
}

// v_j = vin_j + scale * (G a)_j, (G a)_j = sum_e sign_e R_b(gb_e) . a_{float(sub(gb_e))}
__device__ __forceinline__ void coarse_correct_body(const DevMesh& m, const double* __restrict__ a, double scale,
                                                    const double* __restrict__ vin, double* __restrict__ v,
                                                    const int32_t* __restrict__ skip, int bx) {
  if (skip && *skip) return;
  const int64_t j = (int64_t)bx * blockDim.x + threadIdx.x;
  if (j >= m.n_lambda) return;
  v[j] = (vin ? vin[j] : 0.0) + scale * coarse_G_row(m, a, j);
}

__global__ void k_coarse_correct(DevMesh m, const double* __restrict__ a, double scale,
                                 const double* __restrict__ vin, double* __restrict__ v,
                                 const int32_t* __restrict__ skip) {
  coarse_correct_body(m, a, scale, vin, v, skip, blockIdx.x);
}

// v = vin - G a (a may be null: v = vin), then (x, v) reduced; the last block runs phase
__global__ void __launch_bounds__(RED_BLOCK) k_correct_dot(DevMesh m, const double* __restrict__ a,
                                                           const double* __restrict__ vin,
                                                           double* __restrict__ v,
                                                           const double* __restrict__ x,
                                                           double* __restrict__ part,
                                                           int32_t* __restrict__ counter,
                                                           double* __restrict__ sc,
                                                           int32_t* __restrict__ ist, int phase) {
  if (ist[IS_DONE]) return;
  double acc[NPART];
#pragma unroll
  for (int c = 0; c < NPART; ++c) acc[c] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RED_BLOCK;
  for (int64_t j = (int64_t)blockIdx.x * RED_BLOCK + threadIdx.x; j < m.n_lambda; j += stride) {
    const double vj = vin[j] - (a ? coarse_G_row(m, a, j) : 0.0);
    v[j] = vj;
    acc[0] += x[j] * vj;
  }
  reduce_and_finalize<1>(acc, part, counter, sc, ist, phase, blockIdx.x, gridDim.x);
}

// G^T G, one thread per entry (r, c): sum over the jump rows of subdomain float_sub[r/3]
__global__ void k_gtg(DevMesh m, double* __restrict__ C, int nc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nc * nc) return;
  const int r = (int)(t / nc), c = (int)(t % nc);
  const int s = m.float_sub[r / 3], ca = r % 3;
  const int st = m.float_sub[c / 3], cb = c % 3;
  const int nbs = m.nb[s];
  const int64_t b0 = m.boff[s];
  double acc = 0.0;
  for (int bl = 0; bl < nbs; ++bl) {
    const int64_t gb = b0 + bl;
    for (int slot = 0; slot < 2; ++slot) {
      const int j = m.bg_row[2 * gb + slot];
      if (j < 0) continue;
      const double gs = m.bg_sign[2 * gb + slot] * m.rb[3 * gb + ca];
      for (int e = 0; e < 2; ++e) {
        const int64_t gb2 = m.jr_b[2 * (int64_t)j + e];
        if (m.b_sub[gb2] != st) continue;
        acc += gs * m.jr_sign[2 * (int64_t)j + e] * m.rb[3 * gb2 + cb];
      }
    }
  }
  C[t] = acc;
}

// ---- PCG vector kernels with deterministic two-level reductions ---------------

// Reductions over the multipliers: slot 0: (x, y); slots 2..7: per-kind |nrm|^2;
// slots 8..13: per-kind sum_j |mdiag_j| nrm_j^2 (any pointer may be null); the
// last block runs the scalar phase.
__device__ __forceinline__ void reduce_body(const DevMesh& m, const double* __restrict__ x,
                                            const double* __restrict__ y, const double* __restrict__ nrm,
                                            const double* __restrict__ mdiag, double* __restrict__ part,
                                            int32_t* __restrict__ counter, double* __restrict__ sc,
                                            int32_t* __restrict__ ist, int phase, int bx, int nbx) {
  if (ist[IS_DONE] && phase != PH_INIT && phase != PH_REFNORM) return;
  double acc[NPART];
#pragma unroll
  for (int c = 0; c < NPART; ++c) acc[c] = 0.0;
  const int64_t n = m.n_lambda;
  const int64_t stride = (int64_t)nbx * RED_BLOCK;
  for (int64_t j = (int64_t)bx * RED_BLOCK + threadIdx.x; j < n; j += stride) {
    if (x) acc[0] += x[j] * y[j];
    if (nrm) {
      const double v2 = nrm[j] * nrm[j], e2 = fabs(mdiag[j]) * v2;
      const int k = m.row_kind[j];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        acc[2 + c] += c == k ? v2 : 0.0;
        acc[8 + c] += c == k ? e2 : 0.0;
      }
    }
  }
  reduce_and_finalize<14>(acc, part, counter, sc, ist, phase, bx, nbx);
}

__global__ void __launch_bounds__(RED_BLOCK) k_reduce(DevMesh m, const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ nrm,
                                                      const double* __restrict__ mdiag,
                                                      double* __restrict__ part,
                                                      int32_t* __restrict__ counter,
                                                      double* __restrict__ sc,
                                                      int32_t* __restrict__ ist, int phase) {
  reduce_body(m, x, y, nrm, mdiag, part, counter, sc, ist, phase, blockIdx.x, gridDim.x);
}

// M_jj = sum over the interface DOFs b of row j's group of (B^T D)[b, j]^2 S_bb[b, b]
template <class MT>
__global__ void k_precond_diag(DevMesh m, const MT* __restrict__ S, double* __restrict__ md) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m.n_lambda) return;
  const int gs = m.grp_start[j], gz = m.grp_size[j];
  const int slot = (int)(j - gs);
  double acc = 0.0;
  for (int k = 0; k < gz; ++k) {
    const int64_t r = gs + k;
    for (int e = 0; e < 2; ++e) {
      if (e == 1 && k + 1 < gz) continue;  // shared with the next row of the chain
      const int64_t gb = m.jr_b[2 * r + e];
      const int s = m.b_sub[gb];
      const int bl = (int)(gb - m.boff[s]);
      const double wgt = m.bd_wt[3 * gb + slot];
      acc += wgt * wgt * (double)S[m.sofs[s] + (int64_t)bl * m.ldb[s] + bl];
    }
  }
  md[j] = acc;
}


// lam += alpha p; r -= alpha q_raw; w -= alpha q; then the convergence norms of w
__global__ void __launch_bounds__(RED_BLOCK) k_cg_lam(DevMesh m, const double* __restrict__ p,
                                                      const double* __restrict__ qraw,
                                                      const double* __restrict__ q,
                                                      double* __restrict__ lam,
                                                      double* __restrict__ r,
                                                      double* __restrict__ w,
                                                      const double* __restrict__ mdiag,
                                                      double* __restrict__ part,
                                                      int32_t* __restrict__ counter,
                                                      double* __restrict__ sc,
                                                      int32_t* __restrict__ ist) {
  if (ist[IS_DONE]) return;
  const double al = sc[SC_ALPHA];
  double acc[NPART];
#pragma unroll
  for (int c = 0; c < NPART; ++c) acc[c] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RED_BLOCK;
  for (int64_t j = (int64_t)blockIdx.x * RED_BLOCK + threadIdx.x; j < m.n_lambda; j += stride) {
    const double pj = p[j];
    const double lj = lam[j] + al * pj;
    lam[j] = lj;
    r[j] -= al * qraw[j];
    const double wn = w[j] - al * q[j];
    w[j] = wn;
    const double v2 = wn * wn, e2 = fabs(mdiag[j]) * v2;
    const int k = m.row_kind[j];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      acc[2 + c] += c == k ? v2 : 0.0;
      acc[8 + c] += c == k ? e2 : 0.0;
      acc[14 + c] += c == k ? pj * pj : 0.0;
      acc[20 + c] += c == k ? lj * lj : 0.0;
    }
  }
  reduce_and_finalize<26>(acc, part, counter, sc, ist, PH_CONV, blockIdx.x, gridDim.x);
}

// p = y + beta p
__global__ void k_cg_p(int64_t n, const double* __restrict__ sc, const int32_t* __restrict__ ist,
                       const double* __restrict__ y, double* __restrict__ p) {
  if (ist[IS_DONE]) return;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  p[j] = y[j] + sc[SC_BETA] * p[j];
}

// z = a x + b y (plain vector combination)
__device__ __forceinline__ void axpby_body(int64_t n, double a, const double* __restrict__ x, double b,
                                           const double* __restrict__ y, double* __restrict__ z, int bx) {
  const int64_t j = (int64_t)bx * blockDim.x + threadIdx.x;
  if (j >= n) return;
  z[j] = (x ? a * x[j] : 0.0) + (y ? b * y[j] : 0.0);
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b,
                        const double* __restrict__ y, double* __restrict__ z) {
  axpby_body(n, a, x, b, y, z, blockIdx.x);
}

// copy a dense block (rows x cols) between leading dimensions, batched
template <class TS, class TD>
__global__ void k_copy_block(const int64_t* __restrict__ src_ofs, const int32_t* __restrict__ src_ld,
                             const int32_t* __restrict__ src_at, const int64_t* __restrict__ dst_ofs,
                             const int32_t* __restrict__ dst_ld, const int32_t* __restrict__ cnt,
                             const TS* __restrict__ src, TD* __restrict__ dst) {
  const int s = blockIdx.y;
  const int nbs = cnt[s], at = src_at[s];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nbs * nbs) return;
  const int i = (int)(t / nbs), j = (int)(t % nbs);
  dst[dst_ofs[s] + (int64_t)i * dst_ld[s] + j] = (TD)src[src_ofs[s] + (int64_t)(at + i) * src_ld[s] + at + j];
}

// r_b -= B_s^T lam on every interface DOF (torn vector r)
__device__ __forceinline__ void sub_gather_body(const DevMesh& m, const double* __restrict__ lam,
                                                double* __restrict__ r, int bx) {
  const int64_t gb = (int64_t)bx * blockDim.x + threadIdx.x;
  if (gb >= m.sum_nb) return;
  r[m.b_torn[gb]] -= gather_b(m, lam, gb, G_SIGNED);
}

__global__ void k_sub_gather(DevMesh m, const double* __restrict__ lam, double* __restrict__ r) {
  sub_gather_body(m, lam, r, blockIdx.x);
}

// per-block, per-kind max |x| and max |y| over a torn vector (kinds from the DOF codes)
__global__ void __launch_bounds__(256) k_kind_maxabs(DevMesh m, const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     double* __restrict__ part) {
  __shared__ double red[12][256];
  double acc[12];
  for (int c = 0; c < 12; ++c) acc[c] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m.sum_ns; i += stride) {
    const int k = m.code[i] & 7;
    acc[k] = fmax(acc[k], fabs(x[i]));
    acc[6 + k] = fmax(acc[6 + k], fabs(y[i]));
  }
  for (int c = 0; c < 12; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 12; ++c) red[c][threadIdx.x] = fmax(red[c][threadIdx.x], red[c][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 12) part[blockIdx.x * 12 + threadIdx.x] = red[threadIdx.x][0];
}

// scalar state of a solve: every slot cleared, the tolerances and the iteration cap set
__global__ void k_init_scalars(double* __restrict__ sc, int32_t* __restrict__ ist, double tol, double utol,
                               int maxit) {
  const int t = threadIdx.x;
  if (t < SC_COUNT) sc[t] = t == SC_TOL ? tol : (t == SC_UTOL ? utol : 0.0);
  if (t < IS_COUNT) ist[t] = t == IS_MAXIT ? maxit : 0;
}

// z = 0 (a kernel, so that graph captures hold no memset nodes)
__global__ void k_zero(int64_t n, double* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = 0.0;
}

__global__ void k_copy_scalar(double* __restrict__ sc, int src, int dst) {
  if (threadIdx.x == 0) sc[dst] = sc[src];
}

__device__ __forceinline__ void pick_start_body(int64_t n, const double* __restrict__ sc, const double* __restrict__ alt,
                                                double* __restrict__ lam, int32_t* __restrict__ flag,
                                                const double* __restrict__ alt2, double* __restrict__ dst2,
                                                const double* __restrict__ alt3, double* __restrict__ dst3, bool allow,
                                                int bx) {
  const int64_t j = (int64_t)bx * blockDim.x + threadIdx.x;
  const bool take = allow && sc[SC_SEL1] < sc[SC_SEL0];
  if (j == 0 && flag) *flag = take ? 1 : 0;
  if (j >= n || !take) return;
  lam[j] = alt[j];
  if (alt2) dst2[j] = alt2[j];
  if (alt3) dst3[j] = alt3[j];
}

__global__ void k_pick_start(int64_t n, const double* __restrict__ sc, const double* __restrict__ alt,
                             double* __restrict__ lam, int32_t* __restrict__ flag, const double* __restrict__ alt2,
                             double* __restrict__ dst2, const double* __restrict__ alt3, double* __restrict__ dst3) {
  pick_start_body(n, sc, alt, lam, flag, alt2, dst2, alt3, dst3, true, blockIdx.x);
}

// 64 rows per block; the four wavefronts split the coarse index, wavefront 0 finishes
__device__ __forceinline__ void h_project_body(int64_t n, int nc, const double* __restrict__ H,
                                               const double* __restrict__ a, const double* __restrict__ b,
                                               const double* __restrict__ g1, const double* __restrict__ g2,
                                               double* __restrict__ out, double* __restrict__ r_out,
                                               double* __restrict__ out2, int bx) {
  __shared__ double gl[HPROJ_NC_MAX];
  __shared__ double red[4][64];
  for (int k = threadIdx.x; k < nc; k += blockDim.x) gl[k] = g1[k] - (g2 ? g2[k] : 0.0);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t j = (int64_t)bx * 64 + lane;
  const int cq = (nc + 3) / 4, cb = wave * cq, ce = min(nc, cb + cq);
  double acc = 0.0;
  if (j < n)
    for (int c = cb; c < ce; c += 16) {
      double h[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) h[u] = H[(int64_t)min(c + u, ce - 1) * n + j];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (c + u < ce) acc += h[u] * gl[c + u];
    }
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && j < n) {
    const double corr = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    const double v = a[j] - (b ? b[j] : 0.0);
    if (r_out) r_out[j] = v;
    const double o = v - corr;
    out[j] = o;
    if (out2) out2[j] = o;
  }
}

__global__ void __launch_bounds__(256) k_h_project(int64_t n, int nc, const double* __restrict__ H,
                                                   const double* __restrict__ a, const double* __restrict__ b,
                                                   const double* __restrict__ g1, const double* __restrict__ g2,
                                                   double* __restrict__ out, double* __restrict__ r_out,
                                                   double* __restrict__ out2) {
  h_project_body(n, nc, H, a, b, g1, g2, out, r_out, out2, blockIdx.x);
}

// ---- launchers ---------------------------------------------------------------

void launch_copy_scalar(double* sc, int src, int dst, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(64), 0, st, sc, src, dst);
}

void launch_pick_start(int64_t n, const double* sc, const double* alt, double* lam, int32_t* flag, hipStream_t st,
                       const double* alt2, double* dst2, const double* alt3, double* dst3) {
  hipLaunchKernelGGL(k_pick_start, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, sc, alt, lam, flag, alt2,
                     dst2, alt3, dst3);
}

void launch_h_project(int64_t n, int nc, const double* H, const double* a, const double* b, const double* g1,
                      const double* g2, double* out, double* r_out, double* out2, hipStream_t st) {
  hipLaunchKernelGGL(k_h_project, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, st, n, nc, H, a, b, g1, g2, out,
                     r_out, out2);
}

void launch_init_scalars(double* sc, int32_t* ist, double tol, double utol, int maxit, hipStream_t st) {
  static_assert(SC_COUNT <= 64 && IS_COUNT <= 64, "one 64-thread block clears the scalars");
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, st, sc, ist, tol, utol, maxit);
}

void launch_zero(int64_t n, double* z, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, z);
}


void launch_sub_gather(const DevMesh& m, const double* lam, double* r, hipStream_t st) {
  const int blk = 256;
  hipLaunchKernelGGL(k_sub_gather, dim3((unsigned)((m.sum_nb + blk - 1) / blk)), dim3(blk), 0, st, m,
                     lam, r);
}

void launch_kind_maxabs(const DevMesh& m, const double* x, const double* y, double* part, int nblk,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_kind_maxabs, dim3(nblk), dim3(256), 0, st, m, x, y, part);
}

// per-block sums of x_i^2 (fixed grid-stride order and tree, so the same inputs give the
// same partials)
__global__ void __launch_bounds__(256) k_sumsq(int64_t n, const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) acc += x[i] * x[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

void launch_sumsq(int64_t n, const double* x, double* part, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq, dim3(nblk), dim3(256), 0, st, n, x, part);
}

void launch_sgemv(const DevMesh& m, const GemvArgs& a, hipStream_t st) {
  const size_t shm = sizeof(double) * ((size_t)m.max_ns + 4 * 64);
  if (a.which_n == 0) {
    const dim3 grid((m.max_ns + 63) / 64, m.nsub);
    if (a.a_f32) hipLaunchKernelGGL((k_sgemv<1, float>), grid, dim3(256), shm, st, m, a);
    else hipLaunchKernelGGL((k_sgemv<1, double>), grid, dim3(256), shm, st, m, a);
  } else {
    const dim3 grid((m.max_nb + 63) / 64, m.nsub);
    if (a.a_f32) hipLaunchKernelGGL((k_sgemv<0, float>), grid, dim3(256), shm, st, m, a);
    else hipLaunchKernelGGL((k_sgemv<0, double>), grid, dim3(256), shm, st, m, a);
  }
}

void launch_jump(const DevMesh& m, const double* yb, int from_torn, double* out, int scaled,
                 double* g, const int32_t* skip, hipStream_t st) {
  const int blk = 256;
  const int nlb = (int)((m.n_lambda + blk - 1) / blk);
  const int extra = g ? m.n_float : 0;
  hipLaunchKernelGGL(k_jump, dim3(nlb + extra), dim3(blk), 0, st, m, yb, from_torn, out, scaled, g, nlb,
                     skip);
}

void launch_coarse_g(const DevMesh& m, const double* v, const double* base, double gsign, double* g,
                     const int32_t* skip, hipStream_t st) {
  if (m.n_float == 0) return;
  hipLaunchKernelGGL(k_coarse_g, dim3(m.n_float), dim3(256), 0, st, m, v, base, gsign, g, skip);
}

void launch_coarse_apply(int nc, const double* Cinv, const double* g, double* a, double scale,
                         const int32_t* skip, hipStream_t st) {
  if (nc == 0) return;
  hipLaunchKernelGGL(k_coarse_apply, dim3((nc + 3) / 4), dim3(256), 0, st, nc, Cinv, g, a, scale, skip);
}

void launch_coarse_correct(const DevMesh& m, const double* a, double scale, const double* vin,
                           double* v, const int32_t* skip, hipStream_t st) {
  const int blk = 256;
  hipLaunchKernelGGL(k_coarse_correct, dim3((unsigned)((m.n_lambda + blk - 1) / blk)), dim3(blk), 0,
                     st, m, a, scale, vin, v, skip);
}

static int red_grid(const DevMesh& m) {
  const int64_t b = (m.n_lambda + RED_BLOCK - 1) / RED_BLOCK;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, RED_NBLK));
}

void launch_correct_dot(const DevMesh& m, const double* a, const double* vin, double* v,
                        const double* x, double* part, int32_t* counter, double* sc, int32_t* ist,
                        int phase, hipStream_t st) {
  hipLaunchKernelGGL(k_correct_dot, dim3(red_grid(m)), dim3(RED_BLOCK), 0, st, m, a, vin, v, x, part,
                     counter, sc, ist, phase);
}

void launch_gtg(const DevMesh& m, double* C, int nc, hipStream_t st) {
  if (nc == 0) return;
  const int64_t cnt = (int64_t)nc * nc;
  hipLaunchKernelGGL(k_gtg, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, m, C, nc);
}

void launch_reduce(const DevMesh& m, const double* x, const double* y, const double* nrm,
                   const double* mdiag, double* part, int32_t* counter, double* sc, int32_t* ist,
                   int phase, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(red_grid(m)), dim3(RED_BLOCK), 0, st, m, x, y, nrm, mdiag, part,
                     counter, sc, ist, phase);
}

template <class MT>
void launch_precond_diag(const DevMesh& m, const MT* S, double* mdiag, hipStream_t st) {
  const int blk = 256;
  hipLaunchKernelGGL(k_precond_diag<MT>, dim3((unsigned)((m.n_lambda + blk - 1) / blk)), dim3(blk), 0,
                     st, m, S, mdiag);
}
template void launch_precond_diag<double>(const DevMesh&, const double*, double*, hipStream_t);
template void launch_precond_diag<float>(const DevMesh&, const float*, double*, hipStream_t);

void launch_cg_lam(const DevMesh& m, const double* p, const double* qraw, const double* q,
                   double* lam, double* r, double* w, const double* mdiag, double* part,
                   int32_t* counter, double* sc, int32_t* ist, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_lam, dim3(red_grid(m)), dim3(RED_BLOCK), 0, st, m, p, qraw, q, lam, r, w, mdiag,
                     part, counter, sc, ist);
}

void launch_cg_p(int64_t n, const double* sc, const int32_t* ist, const double* y, double* p,
                 hipStream_t st) {
  const int blk = 256;
  hipLaunchKernelGGL(k_cg_p, dim3((unsigned)((n + blk - 1) / blk)), dim3(blk), 0, st, n, sc, ist, y, p);
}

void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z,
                  hipStream_t st) {
  const int blk = 256;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + blk - 1) / blk)), dim3(blk), 0, st, n, a, x, b, y, z);
}

template <class TS, class TD>
void launch_copy_block(int nsub, int maxn, const int64_t* src_ofs, const int32_t* src_ld,
                       const int32_t* src_at, const int64_t* dst_ofs, const int32_t* dst_ld,
                       const int32_t* cnt, const TS* src, TD* dst, hipStream_t st) {
  const int64_t c = (int64_t)maxn * maxn;
  hipLaunchKernelGGL((k_copy_block<TS, TD>), dim3((unsigned)((c + 255) / 256), nsub), dim3(256), 0, st,
                     src_ofs, src_ld, src_at, dst_ofs, dst_ld, cnt, src, dst);
}
template void launch_copy_block<double, double>(int, int, const int64_t*, const int32_t*, const int32_t*,
                                                const int64_t*, const int32_t*, const int32_t*,
                                                const double*, double*, hipStream_t);
template void launch_copy_block<float, float>(int, int, const int64_t*, const int32_t*, const int32_t*,
                                              const int64_t*, const int32_t*, const int32_t*,
                                              const float*, float*, hipStream_t);

// dst = (float) src, n elements
// out[node] = x at the first torn DOF (lowest subdomain) of each code of kind `kind`
__global__ void k_field_scatter(int64_t n, const int32_t* __restrict__ code, const uint8_t* __restrict__ first,
                                const double* __restrict__ x, int kind, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !first[i]) return;
  const int32_t c = code[i];
  if ((c & 7) == kind) out[c >> 3] = x[i];
}

void launch_field_scatter(const DevMesh& m, const double* x, int kind, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_field_scatter, dim3((unsigned)((m.sum_ns + 255) / 256)), dim3(256), 0, st, m.sum_ns, m.code,
                     m.first, x, kind, out);
}

__global__ void k_to_f32(int64_t n, const double* __restrict__ src, float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

void launch_to_f32(int64_t n, const double* src, float* dst, hipStream_t st) {
  const int blk = 256;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + blk - 1) / blk)), dim3(blk), 0, st, n, src, dst);
}

__global__ void k_to_f64(int64_t n, const float* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

void launch_to_f64(int64_t n, const float* src, double* dst, hipStream_t st) {
  const int blk = 256;
  hipLaunchKernelGGL(k_to_f64, dim3((unsigned)((n + blk - 1) / blk)), dim3(blk), 0, st, n, src, dst);
}

// ---- batched launches: the same operation on every problem of a batch --------
// The problem is the last grid dimension; each problem's blocks beyond its own need
// return at once.  Vectors are named by role (BVec), so that one launch reaches the
// same vector of every problem.

__device__ inline int64_t blen(const BProb& p, int len) { return len == BL_TORN ? p.m.sum_ns : p.m.n_lambda; }
__device__ inline double* bvec(const BProb& p, int r) { return r >= 0 ? p.v[r] : nullptr; }

__global__ void __launch_bounds__(256) kb_axpby(const BProb* __restrict__ P, int len, double a, int x, double b, int y,
                                                int z) {
  const BProb& p = P[blockIdx.y];
  axpby_body(blen(p, len), a, bvec(p, x), b, bvec(p, y), p.v[z], blockIdx.x);
}

// start of the first solve: lam = a lam_prev + b lam_prev2 (terms with a zero
// coefficient are not read)
__global__ void __launch_bounds__(256) kb_start(const BProb* __restrict__ P, const BStepVals* __restrict__ V) {
  const BProb& p = P[blockIdx.y];
  const BStepVals& v = V[blockIdx.y];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= p.m.n_lambda) return;
  const double* lp = p.v[BV_LAMP];
  const double* lp2 = p.v[BV_LAMP2];
  double x = 0.0;
  if (v.a_prev != 0.0) x = v.a_prev * lp[j] + (v.b_prev2 != 0.0 ? v.b_prev2 * lp2[j] : 0.0);
  p.v[BV_LAM][j] = x;
}

template <int FULL, class MT>
__global__ void __launch_bounds__(256) kb_sgemv(const BProb* __restrict__ P, BGemv g, const int32_t* __restrict__ items) {
  // work item blockIdx.x: (problem, subdomain, 64-row tile)
  const int32_t* it = items + 3 * (int64_t)blockIdx.x;
  const BProb& p = P[it[0]];
  GemvArgs a;
  a.A = g.mat == BM_KINV ? p.kinv : (g.mat == BM_SPLUS ? p.splus : p.sbb);
  a.a_f32 = p.f32;
  a.aofs = FULL ? p.m.kofs : p.m.sofs;
  a.lda = FULL ? p.m.ld : p.m.ldb;
  a.which_n = FULL ? 0 : 1;
  a.xbase = bvec(p, g.xbase);
  a.v = bvec(p, g.v);
  a.gmode = g.gmode;
  a.gcoef = g.gcoef;
  a.y = p.v[g.y];
  a.alpha_c = p.nc > 0 ? bvec(p, g.alpha_c) : nullptr;
  a.kb_only = g.kb_only;
  a.ybase = bvec(p, g.ybase);
  sgemv_body<FULL, MT>(p.m, a, it[2], it[1]);
}

__global__ void __launch_bounds__(256) kb_jump(const BProb* __restrict__ P, int yb, int from_torn, int out, int scaled,
                                               int g) {
  const BProb& p = P[blockIdx.y];
  const int nlb = (int)((p.m.n_lambda + 255) / 256);
  jump_body(p.m, p.v[yb], from_torn, p.v[out], scaled, p.nc > 0 ? bvec(p, g) : nullptr, nlb, nullptr, blockIdx.x);
}

__global__ void __launch_bounds__(256) kb_coarse_g(const BProb* __restrict__ P, int v, int base, double gsign, int g) {
  const BProb& p = P[blockIdx.y];
  if (p.nc == 0) return;
  coarse_g_body(p.m, bvec(p, v), bvec(p, base), gsign, p.v[g], nullptr, blockIdx.x);
}

__global__ void __launch_bounds__(256) kb_coarse_apply(const BProb* __restrict__ P, int g, int a, double scale) {
  const BProb& p = P[blockIdx.y];
  if (p.nc == 0) return;
  coarse_apply_body(p.nc, p.Cinv, p.v[g], p.v[a], scale, nullptr, blockIdx.x);
}

__global__ void __launch_bounds__(256) kb_coarse_correct(const BProb* __restrict__ P, int a, double scale, int vin,
                                                         int v) {
  const BProb& p = P[blockIdx.y];
  if (p.nc == 0 && vin == v) return;  // no coarse space: v = vin
  coarse_correct_body(p.m, p.v[a], p.nc > 0 ? scale : 0.0, bvec(p, vin), p.v[v], nullptr, blockIdx.x);
}

__global__ void __launch_bounds__(256) kb_h_project(const BProb* __restrict__ P, int a, int b, int g1, int g2, int out,
                                                    int r_out, int out2) {
  const BProb& p = P[blockIdx.y];
  h_project_body(p.m.n_lambda, p.nc, p.H, p.v[a], bvec(p, b), p.v[g1], bvec(p, g2), p.v[out], bvec(p, r_out),
                 bvec(p, out2), blockIdx.x);
}

__global__ void __launch_bounds__(RED_BLOCK) kb_reduce(const BProb* __restrict__ P, int x, int y, int nrm, int phase) {
  const BProb& p = P[blockIdx.y];
  reduce_body(p.m, bvec(p, x), bvec(p, y), bvec(p, nrm), p.mdiag, p.part, p.ist + IS_CNT0 + phase, p.sc, p.ist, phase,
              blockIdx.x, gridDim.x);
}

__global__ void kb_init_scalars(const BProb* __restrict__ P, double tol, double utol, int maxit) {
  const BProb& p = P[blockIdx.y];
  const int t = threadIdx.x;
  if (t < SC_COUNT) p.sc[t] = t == SC_TOL ? tol : (t == SC_UTOL ? utol : 0.0);
  if (t < IS_COUNT) p.ist[t] = t == IS_MAXIT ? maxit : 0;
}

__global__ void kb_copy_scalar(const BProb* __restrict__ P, int src, int dst) {
  const BProb& p = P[blockIdx.y];
  if (threadIdx.x == 0) p.sc[dst] = p.sc[src];
}

__global__ void __launch_bounds__(256) kb_pick_start(const BProb* __restrict__ P, const BStepVals* __restrict__ V,
                                                     int alt, int lam, int alt2, int dst2, int alt3, int dst3) {
  const BProb& p = P[blockIdx.y];
  pick_start_body(p.m.n_lambda, p.sc, p.v[alt], p.v[lam], nullptr, bvec(p, alt2), bvec(p, dst2), bvec(p, alt3),
                  bvec(p, dst3), V[blockIdx.y].cand != 0, blockIdx.x);
}

__global__ void __launch_bounds__(256) kb_sub_gather(const BProb* __restrict__ P, int lam, int r) {
  const BProb& p = P[blockIdx.y];
  sub_gather_body(p.m, p.v[lam], p.v[r], blockIdx.x);
}

void launchb_axpby(const BProb* P, const BDims& d, int len, double a, int x, double b, int y, int z, hipStream_t st) {
  hipLaunchKernelGGL(kb_axpby, dim3(len == BL_TORN ? d.ns_blk : d.nl_blk, d.P), dim3(256), 0, st, P, len, a, x, b, y,
                     z);
}

void launchb_start(const BProb* P, const BStepVals* V, const BDims& d, hipStream_t st) {
  hipLaunchKernelGGL(kb_start, dim3(d.nl_blk, d.P), dim3(256), 0, st, P, V);
}

void launchb_sgemv(const BProb* P, const BDims& d, const BGemv& g, int f32, hipStream_t st) {
  const size_t shm = sizeof(double) * ((size_t)d.max_ns + 4 * 64);
  if (g.full) {
    if (d.n_full_items == 0) return;
    const dim3 grid(d.n_full_items);
    if (f32) hipLaunchKernelGGL((kb_sgemv<1, float>), grid, dim3(256), shm, st, P, g, d.full_items);
    else hipLaunchKernelGGL((kb_sgemv<1, double>), grid, dim3(256), shm, st, P, g, d.full_items);
  } else {
    if (d.n_iface_items == 0) return;
    const dim3 grid(d.n_iface_items);
    if (f32) hipLaunchKernelGGL((kb_sgemv<0, float>), grid, dim3(256), shm, st, P, g, d.iface_items);
    else hipLaunchKernelGGL((kb_sgemv<0, double>), grid, dim3(256), shm, st, P, g, d.iface_items);
  }
}

void launchb_jump(const BProb* P, const BDims& d, int yb, int from_torn, int out, int scaled, int g, hipStream_t st) {
  hipLaunchKernelGGL(kb_jump, dim3(d.nl_blk + (g >= 0 ? d.nflt : 0), d.P), dim3(256), 0, st, P, yb, from_torn, out,
                     scaled, g);
}

void launchb_coarse_g(const BProb* P, const BDims& d, int v, int base, double gsign, int g, hipStream_t st) {
  if (d.nflt == 0) return;
  hipLaunchKernelGGL(kb_coarse_g, dim3(d.nflt, d.P), dim3(256), 0, st, P, v, base, gsign, g);
}

void launchb_coarse_apply(const BProb* P, const BDims& d, int g, int a, double scale, hipStream_t st) {
  if (d.nc_blk == 0) return;
  hipLaunchKernelGGL(kb_coarse_apply, dim3(d.nc_blk, d.P), dim3(256), 0, st, P, g, a, scale);
}

void launchb_coarse_correct(const BProb* P, const BDims& d, int a, double scale, int vin, int v, hipStream_t st) {
  hipLaunchKernelGGL(kb_coarse_correct, dim3(d.nl_blk, d.P), dim3(256), 0, st, P, a, scale, vin, v);
}

void launchb_h_project(const BProb* P, const BDims& d, int a, int b, int g1, int g2, int out, int r_out, int out2,
                       hipStream_t st) {
  hipLaunchKernelGGL(kb_h_project, dim3(d.nl64_blk, d.P), dim3(256), 0, st, P, a, b, g1, g2, out, r_out, out2);
}

void launchb_reduce(const BProb* P, const BDims& d, int x, int y, int nrm, int phase, hipStream_t st) {
  hipLaunchKernelGGL(kb_reduce, dim3(d.red_blk, d.P), dim3(RED_BLOCK), 0, st, P, x, y, nrm, phase);
}

void launchb_init_scalars(const BProb* P, const BDims& d, double tol, double utol, int maxit, hipStream_t st) {
  hipLaunchKernelGGL(kb_init_scalars, dim3(1, d.P), dim3(64), 0, st, P, tol, utol, maxit);
}

void launchb_copy_scalar(const BProb* P, const BDims& d, int src, int dst, hipStream_t st) {
  hipLaunchKernelGGL(kb_copy_scalar, dim3(1, d.P), dim3(64), 0, st, P, src, dst);
}

void launchb_pick_start(const BProb* P, const BStepVals* V, const BDims& d, int alt, int lam, int alt2, int dst2,
                        int alt3, int dst3, hipStream_t st) {
  hipLaunchKernelGGL(kb_pick_start, dim3(d.nl_blk, d.P), dim3(256), 0, st, P, V, alt, lam, alt2, dst2, alt3, dst3);
}

void launchb_sub_gather(const BProb* P, const BDims& d, int lam, int r, hipStream_t st) {
  hipLaunchKernelGGL(kb_sub_gather, dim3(d.nb_blk, d.P), dim3(256), 0, st, P, lam, r);
}

}  // namespace feti
