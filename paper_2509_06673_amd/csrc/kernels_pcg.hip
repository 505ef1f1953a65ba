// Persistent projected PCG on F lambda = d (Section 3, Algorithms 1 and 2, with the
// FETI-1 projection and the Dirichlet preconditioner of eq.
// (feti_dirichlet_preconditioner)).
//
// One cooperative launch runs every iteration of a solve (instead of a chain of
// about ten dependent kernels per iteration).  An iteration is six grid-wide
// phases separated by barriers:
//   A  y_b = (K_s^+)_bb B_s^T p      per 64-row tile, p = y + beta p_old formed on the fly
//   B  q_raw = sum_s B_s y_b, g = G^T q_raw, partial sums of (p, q_raw)
//                                                                 -> alpha in every block
//   D  q = q_raw - G (G^T G)^{-1} g, lam += alpha p, r -= alpha q_raw, w -= alpha q,
//      p_old = p, residual norms                                  -> stopping test in every block
//   E  z_b = S_bb (B_s^T D w)
//   F  z = D sum_s B_s z_b, g = G^T z
//   G  y = z - G (G^T G)^{-1} g, partial sums of (w, y)          -> beta in every block
// p stays in the range of the projection P (it is built from projected vectors), and
// P is orthogonal, so (p, P q_raw) = (p, q_raw): alpha needs no projected q, and the
// projection of q is applied row by row inside the updates.
// The scalars of a phase are reduced by every block from the same per-block
// partials in the same order, so all blocks take identical decisions and leave
// the loop together.  Consecutive reductions alternate between two partial
// buffers: a buffer is rewritten only after a further barrier, which every
// block passes only once it has read the buffer.  The coarse solve
// (G^T G)^{-1} g is applied redundantly by each block that owns multiplier rows
// (n_c is small).  Reductions are deterministic: fixed wave and block order.
//
// The barrier spins with a bound: a block that waits too long raises the abort
// flag, every block leaves at its next barrier, and the host reports an error.
#include <algorithm>

#include "pcg_device.h"

namespace feti {

// sum over c in [cb, ce) of H[c][j] g[c] into c0 (even offsets) and c1 (odd offsets):
// the loads of up to 16 coarse indices are in flight together (indices past ce read
// row ce - 1 and are not used), so a lane's share costs one round trip
__device__ inline void h_rows(const double* __restrict__ H, int64_t NL, int64_t j, int cb, int ce,
                              const double* gl, double& c0, double& c1) {
  for (int c = cb; c < ce; c += 16) {
    double h[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) h[u] = H[(int64_t)min(c + u, ce - 1) * NL + j];
#pragma unroll
    for (int u = 0; u < 16; u += 2) {
      if (c + u < ce) c0 += h[u] * gl[c + u];
      if (c + u + 1 < ce) c1 += h[u + 1] * gl[c + u + 1];
    }
  }
}

// Phases A and E: every 64-row tile of every interface block, two tiles per block
// at a time (one per half).
template <class MT, int SCALED>
__device__ __forceinline__ void gemv_phase(const PcgArgs& a, const MT* A, const double* src, const double* src2,
                                           double beta, double* yout, double* xs2, double* red8) {
  const DevMesh& m = a.m;
  const int half = threadIdx.x / 256, ht = threadIdx.x % 256;
  for (int t2 = blockIdx.x; 2 * t2 < a.ntile; t2 += gridDim.x) {
    const int t = 2 * t2 + half;
    const bool valid = t < a.ntile;
    gemv_tile<MT, SCALED, GEMV_BATCH, GEMV_PF>(m, A, valid ? a.tile_sub[t] : 0, valid ? a.tile_row0[t] : 0, valid,
                                               src, src2, beta, yout, xs2 + half * m.max_nb, red8 + half * 256, ht);
  }
}

// Phase A when beta is still to be formed from the partials bpart of phase G (each
// thread loads the partials of blocks threadIdx.x + k PB, then a block sum): the partial loads are issued with those of the first
// gather pass (y and p_old at the entries' rows), the block sum follows, and then
// p = y + beta p_old is formed and the products run as in gemv_phase.  Returns the sum
// (the caller forms beta = sum / rho).
template <class MT>
__device__ __forceinline__ double gemv_phase_a(const PcgArgs& a, const MT* A, const double* bpart, int nblk,
                                               double rho, double& beta, double* yout, double* xs2, double* red8,
                                               double* red) {
  const DevMesh& m = a.m;
  const int half = threadIdx.x / 256, ht = threadIdx.x % 256;
  const int wave = ht >> 6, lane = ht & 63;
  double bs[1] = {0.0};
  for (int b = threadIdx.x; b < nblk; b += PB) bs[0] += ald(bpart + b * PCG_NPART);
  bool have = false;
  auto finish_beta = [&]() {
    block_sum<1>(bs, red);
    beta = bs[0] / rho;
    have = true;
  };
  for (int t2 = blockIdx.x; 2 * t2 < a.ntile; t2 += gridDim.x) {
    const int t = 2 * t2 + half;
    const bool valid = t < a.ntile;
    const int s = valid ? a.tile_sub[t] : 0, row0 = valid ? a.tile_row0[t] : 0;
    const int nbs = valid ? m.nb[s] : 0;
    const int64_t b0 = valid ? m.boff[s] : 0;
    double* xs = xs2 + half * m.max_nb;
    double* red4 = red8 + half * 256;
    const int i = row0 + lane;
    const int kq = (nbs + 3) / 4;
    const int kb = wave * kq, ke = min(nbs, kb + kq);
    MT pre[GEMV_BATCH];
    const MT* col = nullptr;
    if (GEMV_PF) {
      // the first column batch is loaded before the gather (its latency overlaps it)
      const int64_t ld = valid ? m.ldb[s] : 0;
      col = valid ? A + m.sofs[s] + (int64_t)kb * ld + i : A;
#pragma unroll
      for (int u = 0; u < GEMV_BATCH; ++u) pre[u] = (i < nbs && kb + u < ke) ? col[(int64_t)u * ld] : (MT)0;
    }
    __syncthreads();  // xs and red4 of the previous tiles are consumed
    if (!have) {
      // first pass of the gather (entries ht and ht + 256) with beta pending
      double s0[2], s1[2], y0[2], p0[2], y1[2], p1[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool in = ht + 256 * h < nbs;
        const int64_t gb = b0 + (in ? ht + 256 * h : 0);
        const int q0 = in ? m.bg_row[2 * gb] : -1, q1 = in ? m.bg_row[2 * gb + 1] : -1;
        const int r0 = q0 >= 0 ? q0 : 0, r1 = q1 >= 0 ? q1 : 0;
        s0[h] = q0 >= 0 ? m.bg_sign[2 * gb] : 0.0;
        s1[h] = q1 >= 0 ? m.bg_sign[2 * gb + 1] : 0.0;
        y0[h] = ald(a.y + r0);
        p0[h] = ald(a.p + r0);
        y1[h] = ald(a.y + r1);
        p1[h] = ald(a.p + r1);
      }
      finish_beta();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double v = s0[h] * (y0[h] + beta * p0[h]);
        v += s1[h] * (y1[h] + beta * p1[h]);
        if (ht + 256 * h < nbs) xs[ht + 256 * h] = v;
      }
      // later passes (n_b > 512)
      if (nbs > 512) gather_x<0>(m, nbs - 512, b0 + 512, a.y, a.p, beta, xs + 512, ht);
    } else {
      gather_x<0>(m, nbs, b0, a.y, a.p, beta, xs, ht);
    }
    __syncthreads();
    double v = 0.0;
    if (GEMV_PF) {
      if (i < nbs) v = tile_cols_pf<MT, GEMV_BATCH>(col, m.ldb[s], kb, ke, xs, pre);
    } else {
      if (i < nbs) v = tile_cols<MT>(A + m.sofs[s], m.ldb[s], i, kb, ke, xs);
    }
    red4[wave * 64 + lane] = v;
    __syncthreads();
    if (wave == 0 && i < nbs)
      ast(yout + b0 + i, (red4[lane] + red4[64 + lane]) + (red4[128 + lane] + red4[192 + lane]));
  }
  if (!have) finish_beta();
  return bs[0];
}

// Phases B and F: out_j = (scaled) jump of yb; g_f = R_s^T B_s^T out for the
// floating subdomains (when there is a coarse space).
// With part: also this block's partial of (x, out), x = x1 + xbeta x2.
__device__ void jump_phase(const PcgArgs& a, const double* yb, double* out, int scaled, double* red,
                           const double* x1 = nullptr, const double* x2 = nullptr, double xbeta = 0.0,
                           double* part = nullptr) {
  const DevMesh& m = a.m;
  const int64_t NL = m.n_lambda;
  const int nlb = (int)((NL + PB - 1) / PB);
  const int nitems = nlb + (a.nc > 0 ? m.n_float : 0);
  double dot[1] = {0.0};
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    if (it < nlb) {
      const int64_t j = (int64_t)it * PB + threadIdx.x;
      if (j < NL) {
        const double v = pjump_row(m, yb, j, scaled);
        ast(out + j, v);
        if (part) dot[0] += (ald(x1 + j) + xbeta * ald(x2 + j)) * v;
      }
      continue;
    }
    const int f = it - nlb;
    const int s = m.float_sub[f];
    const int nbs = m.nb[s];
    const int64_t b0 = m.boff[s];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nbs; i += PB) {
      const int64_t gb = b0 + i;
      double v = 0.0;
      for (int slot = 0; slot < 2; ++slot) {
        const int r = m.bg_row[2 * gb + slot];
        if (r >= 0) v += m.bg_sign[2 * gb + slot] * pjump_row(m, yb, r, scaled);
      }
      const double* R = m.rb + 3 * gb;
      acc[0] += R[0] * v;
      acc[1] += R[1] * v;
      acc[2] += R[2] * v;
    }
    block_sum<3>(acc, red);
    if (threadIdx.x < 3) ast(a.g + 3 * f + threadIdx.x, acc[threadIdx.x]);
  }
  if (part) {
    block_sum<1>(dot, red);
    if (threadIdx.x == 0) ast(part + blockIdx.x * PCG_NPART, dot[0]);
  }
}

// Phases C and G: vout = vin - G (G^T G)^{-1} g and this block's partial of (x, vout),
// x_j = x1_j + xbeta x2_j (x2 may be null).  With H = G (G^T G)^{-1} precomputed the
// correction is one coalesced pass; otherwise (G^T G)^{-1} g is formed in LDS and
// the rows of G are evaluated from the index tables.
__device__ void correct_dot_phase(const PcgArgs& a, const double* vin, double* vout, const double* x1, const double* x2, double xbeta, double* part, double* acl,
                                  double* red4, double* red) {
  const DevMesh& m = a.m;
  const int64_t NL = m.n_lambda;
  const int64_t first = (int64_t)blockIdx.x * PB;
  double acc[1] = {0.0};
  if (a.H) {
    // q_j = vin_j - sum_c H[c][j] g_c, H = G (G^T G)^{-1} (coarse-index major): each
    // block takes 64-row chunks, its four wavefronts split the coarse index
    if ((int64_t)blockIdx.x * 64 < NL) {
      double* gl = acl + PCG_NC_LOCAL;
      for (int k = threadIdx.x; k < a.nc; k += PB) gl[k] = ald(a.g + k);
      __syncthreads();
      constexpr int NW = PB / 64;
      const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
      const int cq = (a.nc + NW - 1) / NW, cb = wave * cq, ce = min(a.nc, cb + cq);
      for (int64_t j0 = (int64_t)blockIdx.x * 64; j0 < NL; j0 += (int64_t)gridDim.x * 64) {
        const int64_t j = j0 + lane;
        // wavefront 0's row operands first: their loads overlap those of the sums
        const bool row = wave == 0 && j < NL;
        const double vin_j = row ? ald(vin + j) : 0.0;
        const double x1_j = row ? ald(x1 + j) : 0.0, x2_j = row && x2 ? ald(x2 + j) : 0.0;
        double c0 = 0.0, c1 = 0.0;
        if (j < NL) h_rows(a.H, NL, j, cb, ce, gl, c0, c1);
        red4[wave * 64 + lane] = c0 + c1;
        __syncthreads();
        if (row) {
          double corr = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) corr += red4[w * 64 + lane];
          const double vj = vin_j - corr;
          ast(vout + j, vj);
          const double xj = x2 ? x1_j + xbeta * x2_j : x1_j;
          acc[0] += xj * vj;
        }
        __syncthreads();
      }
    }
  } else if (first < NL) {
    if (a.nc > 0) {
      // ac = Cinv g: g staged in LDS, one thread per row; Cinv is symmetric, so row t
      // is read as column t (consecutive threads, consecutive addresses)
      double* gl = acl + PCG_NC_LOCAL;
      for (int k = threadIdx.x; k < a.nc; k += PB) gl[k] = ald(a.g + k);
      __syncthreads();
      for (int t = threadIdx.x; t < a.nc; t += PB) {
        double s0 = 0.0, s1 = 0.0;
        int k = 0;
        for (; k + 2 <= a.nc; k += 2) {
          s0 += a.Cinv[(int64_t)k * a.nc + t] * gl[k];
          s1 += a.Cinv[(int64_t)(k + 1) * a.nc + t] * gl[k + 1];
        }
        if (k < a.nc) s0 += a.Cinv[(int64_t)k * a.nc + t] * gl[k];
        acl[t] = s0 + s1;
      }
      __syncthreads();
    }
    for (int64_t j = first + threadIdx.x; j < NL; j += (int64_t)gridDim.x * PB) {
      const double vj = ald(vin + j) - (a.nc > 0 ? coarse_G_row(m, acl, j) : 0.0);
      ast(vout + j, vj);
      const double xj = x2 ? ald(x1 + j) + xbeta * ald(x2 + j) : ald(x1 + j);
      acc[0] += xj * vj;
    }
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) ast(part + blockIdx.x * PCG_NPART, acc[0]);
}

// alpha = rho / (p, q_raw) from the block sum pq of the partials; false (with status
// set) on a breakdown.  Every block sees the same sum, so all take the same branch.
__device__ inline bool alpha_of(double pq, double rho, double& alpha, int& status) {
  if (!(fabs(pq) > 1e-300) || !isfinite(pq)) {
    status = isfinite(pq) ? FETI_EBREAKDOWN : FETI_ENAN;
    alpha = 0.0;
    return false;
  }
  alpha = rho / pq;
  return true;
}

// Phase D: alpha = rho / (p, q_raw) from the partials apart of phase B, q = q_raw - H g
// (H = G (G^T G)^{-1}, coarse-index major; 64-row chunks, the wavefronts of the block
// split the coarse index), then lam += alpha p, r -= alpha q_raw, w -= alpha q,
// p_old = p, and this block's partial sums: per-kind |w|^2 (0..5), the dual energy (6)
// and, with the update test (NV = 19), per-kind |p|^2 (7..12) and |lambda|^2 (13..18).
// The partials of (p, q_raw) are loaded with g and summed after the projection sums
// of the first chunk, so that their latency overlaps the H loads.  Returns false on a
// breakdown of alpha (before any update).
template <int NV>
__device__ inline bool update_phase(const PcgArgs& a, const double* apart, int nblk, double rho, double& alpha,
                                    int& status, double beta, double* part, double* acl, double* red4,
                                    double* red) {
  const DevMesh& m = a.m;
  const int64_t NL = m.n_lambda;
  double pq[1] = {0.0};
  for (int b = threadIdx.x; b < nblk; b += PB) pq[0] += ald(apart + b * PCG_NPART);
  bool have_alpha = false;
  double acc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) acc[c] = 0.0;
  if ((int64_t)blockIdx.x * 64 < NL) {
    double* gl = acl + PCG_NC_LOCAL;
    for (int k = threadIdx.x; k < a.nc; k += PB) gl[k] = ald(a.g + k);
    __syncthreads();
    constexpr int NW = PB / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cq = (a.nc + NW - 1) / NW, cb = wave * cq, ce = min(a.nc, cb + cq);
    for (int64_t j0 = (int64_t)blockIdx.x * 64; j0 < NL; j0 += (int64_t)gridDim.x * 64) {
      const int64_t j = j0 + lane;
      // wavefront 0's update operands first: their loads overlap those of the sums
      const bool row = wave == 0 && j < NL;
      const double qr = row ? ald(a.qraw + j) : 0.0, yj = row ? ald(a.y + j) : 0.0;
      const double pold = row ? ald(a.p + j) : 0.0, wj = row ? ald(a.w + j) : 0.0;
      const double lam_j = row ? a.lam[j] : 0.0, r_j = row ? a.r[j] : 0.0, md = row ? a.mdiag[j] : 0.0;
      const int kind = row ? m.row_kind[j] : 0;
      double c0 = 0.0, c1 = 0.0;
      if (j < NL) h_rows(a.H, NL, j, cb, ce, gl, c0, c1);
      red4[wave * 64 + lane] = c0 + c1;
      if (!have_alpha) {
        block_sum<1>(pq, red);  // its barriers also publish red4
        have_alpha = true;
        if (!alpha_of(pq[0], rho, alpha, status)) return false;
      }
      __syncthreads();
      if (row) {
        double corr = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) corr += red4[w * 64 + lane];
        const double pj = yj + beta * pold;
        const double lj = lam_j + alpha * pj;
        a.lam[j] = lj;
        a.r[j] = r_j - alpha * qr;
        const double wn = wj - alpha * (qr - corr);
        ast(a.w + j, wn);
        ast(a.p + j, pj);
        const double v2 = wn * wn;
        const int k = kind;
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += (c == k) ? v2 : 0.0;
        acc[6] += fabs(md) * v2;
        if (NV > 7) {
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            acc[7 + c] += (c == k) ? pj * pj : 0.0;
            acc[13 + c] += (c == k) ? lj * lj : 0.0;
          }
        }
      }
      __syncthreads();
    }
  }
  if (!have_alpha) {
    block_sum<1>(pq, red);
    if (!alpha_of(pq[0], rho, alpha, status)) return false;
  }
  // only wavefront 0 holds row sums: a shuffle reduction there, lane 0 stores
  if (threadIdx.x < 64) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double x = acc[c];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      acc[c] = x;
    }
    if (threadIdx.x == 0)
#pragma unroll
      for (int c = 0; c < NV; ++c) ast(part + blockIdx.x * PCG_NPART + c, acc[c]);
  }
  return true;
}

static_assert(PCG_MAX_GRID * 19 <= GT_LOADS * PB, "the stopping test stages every partial sum once");

__global__ void __launch_bounds__(PCG_BLOCK) k_pcg_persistent(PcgArgs a) {
  extern __shared__ double lds[];
  __shared__ int s_ok, s_upd;
  __shared__ double s_res;
  __shared__ double s_ring[UPD_WIN * 6];
  __shared__ double s_kc[14];  // references of the stopping test (see stop_test_wave0)
  const DevMesh& m = a.m;
  double* xs = lds;                          // 2 x max_nb gathered vectors (one per tile)
  double* red4 = xs + 2 * m.max_nb;          // PB partial rows
  double* acl = red4 + PB;                   // coarse coefficients, then g (2 x PCG_NC_LOCAL)
  double* red = acl + 2 * PCG_NC_LOCAL;
  double* stage = red + (PB / 64) * PCG_NPART;  // nblk x 19 staged partial sums
  const int nblk = gridDim.x;
  uint32_t gen = 0;  // the host clears the barrier before the launch

  const double tol = a.sc[SC_TOL];
  const double utol = a.sc[SC_UTOL];
  const bool upd = utol > 0.0;  // the same in every block
  double rho = a.sc[SC_RHO], beta = a.sc[SC_BETA], alpha = a.sc[SC_ALPHA], res = a.sc[SC_RES];
  int iters = a.ist[IS_ITERS];
  const int maxit = a.ist[IS_MAXIT];
  int status = a.ist[IS_STATUS];
  bool ok = true;
  const bool start_done = a.ist[IS_DONE] != 0 || iters >= maxit;  // the same in every block
  int rk = 0;  // reductions so far: partial buffer rk & 1
  auto partbuf = [&](int k) { return a.part + (size_t)(k & 1) * nblk * PCG_NPART; };
  __shared__ double conv[19];  // totals of the last stopping test
  if (threadIdx.x < 19) conv[threadIdx.x] = 0.0;
  if (threadIdx.x < 6) {
    s_kc[threadIdx.x] = a.sc[SC_REF + threadIdx.x];
    s_kc[6 + threadIdx.x] = a.sc[SC_EK + threadIdx.x];
  }
  if (threadIdx.x == 0) {
    s_kc[12] = a.sc[SC_EREF];
    double eref = 0.0;
    for (int k = 0; k < 6; ++k) eref += a.sc[SC_EK + k];
    s_kc[13] = eref;
  }
  __syncthreads();
  int it_local = 0, ph = 0;
  auto stamp = [&]() {
    if (a.tstamp && blockIdx.x == 0 && threadIdx.x == 0 && it_local < a.tstamp_iters)
      a.tstamp[it_local * 10 + ph] = (long long)wall_clock64();
    ++ph;
  };
  stamp();
  for (; !start_done; ++it_local, ph = 1) {  // stamp 0 of a later iteration is stamp 6 of the one before
    // (A) y_b = (K^+)_bb B^T p,  p = y + beta p_old (beta from the partials of phase G,
    // except in the first iteration of a launch)
    if (it_local == 0) {
      if (a.fm32) gemv_phase<float, 0>(a, (const float*)a.fm, a.y, a.p, beta, a.yb, xs, red4);
      else gemv_phase<double, 0>(a, (const double*)a.fm, a.y, a.p, beta, a.yb, xs, red4);
    } else {
      const double t0 = a.fm32 ? gemv_phase_a<float>(a, (const float*)a.fm, partbuf(rk), nblk, rho, beta, a.yb, xs, red4, red)
                               : gemv_phase_a<double>(a, (const double*)a.fm, partbuf(rk), nblk, rho, beta, a.yb, xs, red4, red);
      ++rk;
      rho = t0;
    }
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // (B) q_raw = B y_b, g = G^T q_raw, partial (p, q_raw)
    jump_phase(a, a.yb, a.qraw, 0, red, a.y, a.p, beta, partbuf(rk));
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // (D) alpha, q = P q_raw, updates and the norms of w (and of p and lambda for the
    // update test)
    {
      const double* apart = partbuf(rk++);
      const bool good = upd ? update_phase<19>(a, apart, nblk, rho, alpha, status, beta, partbuf(rk), acl, red4, red)
                            : update_phase<7>(a, apart, nblk, rho, alpha, status, beta, partbuf(rk), acl, red4, red);
      if (!good) break;
    }
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // (E) z_b = S_bb (B^T D w), then the stopping test.  Its partial sums are loaded
    // before the products, which do not depend on its outcome, so that their latency
    // overlaps the gather; the products of the last iteration are not used.
    {
      double tl[GT_LOADS];
      if (upd) gt_issue<19>(partbuf(rk), nblk, tl);
      else gt_issue<7>(partbuf(rk), nblk, tl);
      if (a.mm32) gemv_phase<float, 1>(a, (const float*)a.mm, a.w, nullptr, 0.0, a.zb, xs, red4);
      else gemv_phase<double, 1>(a, (const double*)a.mm, a.w, nullptr, 0.0, a.zb, xs, red4);
      if (upd) gt_finish<19>(tl, nblk, conv, stage);
      else gt_finish<7>(tl, nblk, conv, stage);
      ++rk;
      // counted within this launch, so that the ring holds only this launch's updates
      if (threadIdx.x < 64) stop_test_wave0(conv, s_kc, s_ring, it_local + 1, alpha, utol, upd, &s_res, &s_upd);
      __syncthreads();
      res = s_res;
      iters += 1;
      if (!isfinite(res)) { status = FETI_ENAN; break; }
      if (res <= tol || s_upd) break;
      if (iters >= maxit) { status = FETI_ENOTCONV; break; }
    }
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // (F) z = D B z_b, g = G^T z
    jump_phase(a, a.zb, a.z, 1, red);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // (G) y = P z, partial (w, y)
    correct_dot_phase(a, a.z, a.y, a.w, nullptr, 0.0, partbuf(rk), acl, red4, red);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // beta = (w, y) / rho is formed at the start of the next phase A
    if (!(fabs(rho) > 1e-300)) { status = FETI_EBREAKDOWN; break; }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.sc[SC_RHO] = rho;
    a.sc[SC_ALPHA] = alpha;
    a.sc[SC_BETA] = beta;
    a.sc[SC_RES] = res;
    double et = 0.0;
    for (int k = 0; k < 6; ++k) {
      a.sc[SC_KRAT + k] = a.sc[SC_REF + k] > 0.0 ? sqrt(conv[k]) / a.sc[SC_REF + k] : 0.0;
    }
    et = conv[6];
    a.sc[SC_ERAT] = a.sc[SC_EREF] > 0.0 ? sqrt(et) / a.sc[SC_EREF] : 0.0;
    a.ist[IS_ITERS] = iters;
    a.ist[IS_STATUS] = ok ? status : FETI_EHIP;
    a.ist[IS_DONE] = 1;
  }
}

// H[c][j] = (G (G^T G)^{-1})_{j c}: row c of the symmetric Cinv is its column c
__global__ void k_build_h(DevMesh m, const double* __restrict__ Cinv, int nc, double* __restrict__ H) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (j >= m.n_lambda) return;
  H[(int64_t)c * m.n_lambda + j] = coarse_G_row(m, Cinv + (int64_t)c * nc, j);
}

void launch_build_h(const DevMesh& m, const double* Cinv, int nc, double* H, hipStream_t st) {
  if (nc == 0) return;
  hipLaunchKernelGGL(k_build_h, dim3((unsigned)((m.n_lambda + 255) / 256), nc), dim3(256), 0, st, m, Cinv, nc, H);
}

size_t pcg_shmem(const DevMesh& m) {
  return sizeof(double) * (2 * (size_t)m.max_nb + PB + 2 * PCG_NC_LOCAL + (PB / 64) * PCG_NPART +
                           (size_t)PCG_MAX_GRID * 19);
}

int pcg_max_grid(const DevMesh& m) {
  int dev = 0, coop = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pcg_persistent, PB, pcg_shmem(m)) != hipSuccess)
    return 0;
  return std::max(0, per_cu) * cus;
}

hipError_t launch_pcg_persistent(const PcgArgs& a, int grid, hipStream_t st) {
  PcgArgs arg = a;
  void* params[] = {&arg};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_pcg_persistent), dim3(grid), dim3(PB),
                                    params, (unsigned)pcg_shmem(a.m), st);
}

}  // namespace feti
