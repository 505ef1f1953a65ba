// Projected PCG (Section 3, Algorithms 1 and 2, with the FETI-1 projection and the
// Dirichlet preconditioner of eq. (feti_dirichlet_preconditioner)) for a batch of
// independent problems in one cooperative launch.
//
// The phases of an iteration are those of the single-problem launch
// (kernels_pcg.hip), over work lists that span every problem: 64-row tiles of
// the interface blocks, chunks of PCG_BLOCK multiplier rows and the floating
// subdomains.  Each problem keeps its own scalars.  After each reduction the block
// with blockIdx = problem mod grid sums that problem's chunk partials (in chunk
// order) and publishes alpha, the stopping decision or beta before the next
// barrier, so an iteration has ten barriers: A | B | C | C' | D | D' | E | F | G | G'.
// A finished problem drops out of the work lists; the launch ends when every
// problem has finished.
#include <cstdio>

#include "pcg_device.h"

namespace feti {

// column loads in flight per lane in the GEMV phases (the batch's interface blocks stream
// from HBM, so more bytes in flight pay than for one problem's cache-resident blocks)
#ifndef FETI_BATCH_GEMV_NB
#define FETI_BATCH_GEMV_NB 8
#endif
constexpr int BATCH_GEMV_NB = FETI_BATCH_GEMV_NB;
// waves per SIMD the register allocation must allow (4: two blocks of PCG_BLOCK threads
// per compute unit)
#ifndef FETI_BATCH_MIN_WAVES
#define FETI_BATCH_MIN_WAVES 4
#endif
constexpr int BATCH_MIN_WAVES = FETI_BATCH_MIN_WAVES;
// 1: the column loads of the GEMV phases run one batch ahead of the products
#ifndef FETI_BATCH_GEMV_PF
#define FETI_BATCH_GEMV_PF 0
#endif
constexpr int BATCH_GEMV_PF = FETI_BATCH_GEMV_PF;

__device__ inline int iload(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void istore(int32_t* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// a problem finishes with a status: published for every block, counted once
__device__ inline void finish(const BatchArgs& a, int p, int status) {
  const ProbArgs& pr = a.probs[p];
  pr.ist[IS_STATUS] = status;
  pr.ist[IS_DONE] = 1;
  a.status[p] = status;
  istore(a.done + p, 1);
  __hip_atomic_fetch_add(a.ndone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class MT>
__device__ void batch_gemv(const BatchArgs& a, int precond_phase, double* xs2, double* red8) {
  const int half = threadIdx.x / 256, ht = threadIdx.x % 256;
  for (int t2 = blockIdx.x; 2 * t2 < a.ntile; t2 += gridDim.x) {
    const int t = 2 * t2 + half;
    int p = t < a.ntile ? a.tile_prob[t] : 0;
    const bool valid = t < a.ntile && !iload(a.done + p);
    const ProbArgs& pr = a.probs[p];
    double* xs = xs2 + half * a.max_nb;
    double* red4 = red8 + half * 256;
    const int s = valid ? a.tile_sub[t] : 0, row0 = valid ? a.tile_row0[t] : 0;
    if (!precond_phase)
      gemv_tile<MT, 0, BATCH_GEMV_NB, BATCH_GEMV_PF>(pr.m, (const MT*)pr.fm, s, row0, valid, pr.y, pr.p,
                                                     valid ? ald(a.beta + p) : 0.0, pr.yb, xs, red4, ht);
    else
      gemv_tile<MT, 1, BATCH_GEMV_NB, BATCH_GEMV_PF>(pr.m, (const MT*)pr.mm, s, row0, valid, pr.w, nullptr, 0.0,
                                                     pr.zb, xs, red4, ht);
  }
}

// Phases B and F: jump rows of every chunk, G^T of every floating subdomain
__device__ void batch_jump(const BatchArgs& a, int scaled, double* red) {
  const int nitems = a.nrow + a.nflt;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    if (it < a.nrow) {
      const int p = a.row_prob[it];
      if (iload(a.done + p)) continue;
      const ProbArgs& pr = a.probs[p];
      const double* yb = scaled ? pr.zb : pr.yb;
      double* out = scaled ? pr.z : pr.qraw;
      const int64_t j = (int64_t)a.row_chunk[it] * PB + threadIdx.x;
      if (j < pr.m.n_lambda) ast(out + j, pjump_row(pr.m, yb, j, scaled));
      continue;
    }
    const int k = it - a.nrow;
    const int p = a.flt_prob[k];
    if (iload(a.done + p)) continue;
    const ProbArgs& pr = a.probs[p];
    const DevMesh& m = pr.m;
    const double* yb = scaled ? pr.zb : pr.yb;
    const int f = a.flt_f[k];
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
    if (threadIdx.x < 3) ast(pr.g + 3 * f + threadIdx.x, acc[threadIdx.x]);
  }
}

// Phases C and G: vout = vin - G (G^T G)^{-1} g per chunk, partial of (x, vout) with
// x = x1 + beta x2 (C: p = y + beta p_old against q; G: w against y)
__device__ void batch_correct_dot(const BatchArgs& a, int second, double* acl, double* red) {
  for (int it = blockIdx.x; it < a.nrow; it += gridDim.x) {
    const int p = a.row_prob[it];
    if (iload(a.done + p)) continue;
    const ProbArgs& pr = a.probs[p];
    const DevMesh& m = pr.m;
    if (pr.nc > 0) {
      double* gl = acl + PCG_NC_LOCAL;
      for (int k = threadIdx.x; k < pr.nc; k += PB) gl[k] = ald(pr.g + k);
      __syncthreads();
      for (int t = threadIdx.x; t < pr.nc; t += PB) {
        double s0 = 0.0;
        for (int k = 0; k < pr.nc; ++k) s0 += pr.Cinv[(int64_t)k * pr.nc + t] * gl[k];
        acl[t] = s0;
      }
      __syncthreads();
    }
    const double* vin = second ? pr.z : pr.qraw;
    double* vout = second ? pr.y : pr.q;
    const double bt = second ? 0.0 : ald(a.beta + p);
    double acc[1] = {0.0};
    const int64_t j = (int64_t)a.row_chunk[it] * PB + threadIdx.x;
    if (j < m.n_lambda) {
      const double vj = ald(vin + j) - (pr.nc > 0 ? coarse_G_row(m, acl, j) : 0.0);
      ast(vout + j, vj);
      const double xj = second ? ald(pr.w + j) : ald(pr.y + j) + bt * ald(pr.p + j);
      acc[0] = xj * vj;
    }
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) ast(pr.part + (int64_t)a.row_chunk[it] * PCG_NPART, acc[0]);
  }
}

// sum of problem p's chunk partials, slot c, in chunk order (one thread)
__device__ inline double chunk_total(const ProbArgs& pr, int c) {
  double s = 0.0;
  for (int k = 0; k < pr.nrow_items; ++k) s += ald(pr.part + (int64_t)k * PCG_NPART + c);
  return s;
}

// Phase D on one chunk of problem p's multiplier rows: the updates and the chunk's
// partial sums: per-kind |w|^2 (0..5), the dual energy (6) and, with the update
// test (NV = 19), per-kind |p|^2 (7..12) and |lambda|^2 (13..18).
template <int NV>
__device__ inline void batch_update(const BatchArgs& a, const ProbArgs& pr, int p, int it, double* red) {
  const double al = ald(a.alpha + p), bt = ald(a.beta + p);
  double acc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) acc[c] = 0.0;
  const int64_t j = (int64_t)a.row_chunk[it] * PB + threadIdx.x;
  if (j < pr.m.n_lambda) {
    const double pj = ald(pr.y + j) + bt * ald(pr.p + j);
    const double lj = pr.lam[j] + al * pj;
    pr.lam[j] = lj;
    pr.r[j] -= al * ald(pr.qraw + j);
    const double wn = ald(pr.w + j) - al * ald(pr.q + j);
    ast(pr.w + j, wn);
    ast(pr.p + j, pj);
    const double v2 = wn * wn;
    const int k = pr.m.row_kind[j];
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += (c == k) ? v2 : 0.0;
    acc[6] = fabs(pr.mdiag[j]) * v2;
    if (NV > 7) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        acc[7 + c] = (c == k) ? pj * pj : 0.0;
        acc[13 + c] = (c == k) ? lj * lj : 0.0;
      }
    }
  }
  block_store<NV>(acc, red, pr.part + (int64_t)a.row_chunk[it] * PCG_NPART);
}

__global__ void __launch_bounds__(PCG_BLOCK, BATCH_MIN_WAVES) k_pcg_batch(BatchArgs a) {
  extern __shared__ double lds[];
  __shared__ int s_ok;
  double* xs = lds;                 // 2 x max_nb
  double* red8 = xs + 2 * a.max_nb; // PB
  double* acl = red8 + PB;          // 2 x PCG_NC_LOCAL
  double* red = acl + 2 * PCG_NC_LOCAL;
  const int nblk = gridDim.x;
  uint32_t gen = 0;  // the host clears the barrier and the finished count before the launch
  bool ok = true;
  // prologue: each designated block loads its problems' state
  if (threadIdx.x == 0)
    for (int p = blockIdx.x; p < a.P; p += nblk) {
      const ProbArgs& pr = a.probs[p];
      ast(a.rho + p, pr.sc[SC_RHO]);
      ast(a.beta + p, 0.0);
      a.iters[p] = 0;
      a.status[p] = pr.ist[IS_STATUS];
      const int d = pr.ist[IS_DONE] || pr.ist[IS_MAXIT] <= 0;
      istore(a.done + p, d);
      if (d) __hip_atomic_fetch_add(a.ndone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  ok = grid_sync(a.bar, nblk, gen, &s_ok);
  while (ok) {
    if (iload(a.ndone) >= a.P) break;  // read after a barrier: the same in every block
    // (A) y_b = (K^+)_bb B^T p, p = y + beta p_old
    if (a.f32) batch_gemv<float>(a, 0, xs, red8);
    else batch_gemv<double>(a, 0, xs, red8);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    // (B) q_raw = B y_b, g = G^T q_raw
    batch_jump(a, 0, red);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    // (C) q = P q_raw, partials of (p, q)
    batch_correct_dot(a, 0, acl, red);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    // (C') alpha = rho / (p, q)
    if (threadIdx.x == 0)
      for (int p = blockIdx.x; p < a.P; p += nblk) {
        if (iload(a.done + p)) continue;
        const double pq = chunk_total(a.probs[p], 0);
        if (!(fabs(pq) > 1e-300) || !isfinite(pq)) finish(a, p, isfinite(pq) ? FETI_EBREAKDOWN : FETI_ENAN);
        else ast(a.alpha + p, ald(a.rho + p) / pq);
      }
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    // (D) lam += alpha p, r -= alpha q_raw, w -= alpha q, p_old = p; partial norms of w
    // (and of p and lambda for a problem with the update test)
    for (int it = blockIdx.x; it < a.nrow; it += nblk) {
      const int p = a.row_prob[it];
      if (iload(a.done + p)) continue;
      const ProbArgs& pr = a.probs[p];
      if (pr.sc[SC_UTOL] > 0.0) batch_update<19>(a, pr, p, it, red);
      else batch_update<7>(a, pr, p, it, red);
    }
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    // (D') stopping test
    if (threadIdx.x == 0)
      for (int p = blockIdx.x; p < a.P; p += nblk) {
        if (iload(a.done + p)) continue;
        const ProbArgs& pr = a.probs[p];
        double w2[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) w2[k] = chunk_total(pr, k);
        const double rel = rel_residual_of(w2, chunk_total(pr, 6), pr.sc);
        const int its = a.iters[p] + 1;
        a.iters[p] = its;
        pr.ist[IS_ITERS] += 1;
        pr.sc[SC_RES] = rel;
        bool upd = false;
        if (pr.sc[SC_UTOL] > 0.0) {
          double p2[6], l2[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            p2[k] = chunk_total(pr, 7 + k);
            l2[k] = chunk_total(pr, 13 + k);
          }
          upd = update_converged(pr.sc + SC_URING, its, ald(a.alpha + p), p2, l2, pr.sc[SC_UTOL]);
        }
        if (!isfinite(rel)) finish(a, p, FETI_ENAN);
        else if (rel <= pr.sc[SC_TOL] || upd) finish(a, p, 0);
        else if (pr.ist[IS_ITERS] >= pr.ist[IS_MAXIT]) finish(a, p, FETI_ENOTCONV);
      }
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    // (E) z_b = S_bb B^T D w
    if (a.f32) batch_gemv<float>(a, 1, xs, red8);
    else batch_gemv<double>(a, 1, xs, red8);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    // (F) z = D B z_b, g = G^T z
    batch_jump(a, 1, red);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    // (G) y = P z, partials of (w, y)
    batch_correct_dot(a, 1, acl, red);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    // (G') beta = rho_new / rho
    if (threadIdx.x == 0)
      for (int p = blockIdx.x; p < a.P; p += nblk) {
        if (iload(a.done + p)) continue;
        const double rn = chunk_total(a.probs[p], 0), ro = ald(a.rho + p);
        if (!(fabs(ro) > 1e-300)) { finish(a, p, FETI_EBREAKDOWN); continue; }
        ast(a.beta + p, rn / ro);
        ast(a.rho + p, rn);
      }
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
  }
  if (!ok && threadIdx.x == 0)
    for (int p = blockIdx.x; p < a.P; p += nblk) {
      const ProbArgs& pr = a.probs[p];
      if (!pr.ist[IS_DONE]) { pr.ist[IS_STATUS] = FETI_EHIP; pr.ist[IS_DONE] = 1; a.status[p] = FETI_EHIP; }
    }
}

size_t pcg_batch_shmem(int max_nb) {
  return sizeof(double) * (2 * (size_t)max_nb + PB + 2 * PCG_NC_LOCAL + (PB / 64) * PCG_NPART);
}

int pcg_batch_max_grid(int max_nb) {
  int dev = 0, coop = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pcg_batch, PB, pcg_batch_shmem(max_nb)) != hipSuccess)
    return 0;
  return std::max(0, per_cu) * cus;
}

void pcg_batch_describe(int max_nb, char* buf, size_t n) {
  hipFuncAttributes fa{};
  (void)hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k_pcg_batch));
  int per_cu = 0, per_cu256 = 0;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pcg_batch, PB, pcg_batch_shmem(max_nb));
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu256, k_pcg_batch, 256, pcg_batch_shmem(max_nb));
  std::snprintf(buf, n, "regs %d, max threads %d, static LDS %zu, local %zu; blocks per CU %d (of 256 threads: %d)",
                fa.numRegs, fa.maxThreadsPerBlock, fa.sharedSizeBytes, fa.localSizeBytes, per_cu, per_cu256);
}

hipError_t launch_pcg_batch(const BatchArgs& a, int grid, hipStream_t st) {
  BatchArgs arg = a;
  void* params[] = {&arg};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_pcg_batch), dim3(grid), dim3(PB), params,
                                    (unsigned)pcg_batch_shmem(a.max_nb), st);
}

}  // namespace feti
