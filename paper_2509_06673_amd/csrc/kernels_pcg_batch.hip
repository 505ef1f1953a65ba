// Projected PCG (Section 3, Algorithms 1 and 2, with the FETI-1 projection and the
// Dirichlet preconditioner of eq. (feti_dirichlet_preconditioner)) for a batch of
// independent problems in one cooperative launch.
//
// The phases of an iteration are those of the single-problem launch
// (kernels_pcg.hip), over work lists that span every problem: 64-row tiles of
// the interface blocks, chunks of PCG_BLOCK multiplier rows and the floating
// subdomains.  Each problem keeps its own scalars: a block that stores a chunk
// partial of a reduction counts it on the problem's counter, and the block that
// completes the count sums that problem's chunk partials (a fixed tree) and
// publishes alpha, the stopping decision or beta before the next barrier.  An
// iteration has seven barriers: A | B | C (alpha) | D (stopping test) | E | F |
// G (beta).  A finished problem drops out of the work lists; the launch ends when
// every problem has finished.
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

// a problem finishes with a status: published for every block, counted once.  The
// per-problem state is written by whichever block completes a reduction, so every
// access to it that another block may repeat is device-coherent.
__device__ inline void finish(const BatchArgs& a, int p, int status) {
  const ProbArgs& pr = a.probs[p];
  istore(pr.ist + IS_STATUS, status);
  istore(pr.ist + IS_DONE, 1);
  istore(a.status + p, status);
  istore(a.done + p, 1);
  __hip_atomic_fetch_add(a.ndone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// After this block stored a chunk partial of problem p: counts it, and returns true in
// the block that completes the count (which then resets the counter).  The partial
// stores are device-coherent and complete before the count.
__device__ inline bool last_chunk(int32_t* cnt, int total, int* s_flag) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x == 0) {
    const bool last = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == total - 1;
    if (last) __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *s_flag = last ? 1 : 0;
  }
  __syncthreads();
  return *s_flag != 0;
}

// Sums over problem p's chunk partials of the slots [0, NV), in chunk order, into tot
// (LDS; lane c of the first wavefront sums slot c).
template <int NV>
__device__ inline void chunk_totals(const ProbArgs& pr, double* tot) {
  if (threadIdx.x < NV) {
    // eight chunk loads in flight at a time, added in chunk order
    const int n = pr.nrow_items;
    const double* src = pr.part + threadIdx.x;
    double s = 0.0;
    for (int k = 0; k < n; k += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = k + u < n ? ald(src + (int64_t)(k + u) * PCG_NPART) : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k + u < n) s += v[u];
    }
    tot[threadIdx.x] = s;
  }
  __syncthreads();
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
__device__ void batch_correct_dot(const BatchArgs& a, int second, double* acl, double* red, int* s_flag) {
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
    if (!last_chunk(a.cnt + 3 * p + (second ? 2 : 0), pr.nrow_items, s_flag)) continue;
    chunk_totals<1>(pr, red);
    if (threadIdx.x == 0) {
      if (!second) {
        // alpha = rho / (p, q)
        const double pq = red[0];
        if (!(fabs(pq) > 1e-300) || !isfinite(pq)) finish(a, p, isfinite(pq) ? FETI_EBREAKDOWN : FETI_ENAN);
        else ast(a.alpha + p, ald(a.rho + p) / pq);
      } else {
        // beta = rho_new / rho
        const double rn = red[0], ro = ald(a.rho + p);
        if (!(fabs(ro) > 1e-300)) {
          finish(a, p, FETI_EBREAKDOWN);
        } else {
          ast(a.beta + p, rn / ro);
          ast(a.rho + p, rn);
        }
      }
    }
  }
}

// Phase D on one chunk of problem p's multiplier rows: the updates and the chunk's
// partial sums: per-kind |w|^2 (0..5), the dual energy (6) and, with the update
// test (NV = 19), per-kind |p|^2 (7..12) and |lambda|^2 (13..18).
template <int NV>
__device__ inline void batch_update(const BatchArgs& a, const ProbArgs& pr, int p, int it, double* red,
                                    int* s_flag) {
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
  if (!last_chunk(a.cnt + 3 * p + 1, pr.nrow_items, s_flag)) return;
  // stopping test of problem p
  chunk_totals<NV>(pr, red);
  const double* t = red;
  if (threadIdx.x == 0) {
    // the tolerances and references are constant during the launch; the counters and
    // the update ring are read and written device-coherently
    const double rel = rel_residual_of(t, t[6], pr.sc);
    const int its = iload(a.iters + p) + 1;
    istore(a.iters + p, its);
    const int total = iload(pr.ist + IS_ITERS) + 1;
    istore(pr.ist + IS_ITERS, total);
    ast(pr.sc + SC_RES, rel);
    bool upd = false;
    if (NV > 7) {
      double* ring = red + 32;  // LDS, past the totals
      static_assert(32 + UPD_WIN * 6 <= (PB / 64) * PCG_NPART, "the update ring fits the reduction scratch");
#pragma unroll
      for (int k = 0; k < UPD_WIN * 6; ++k) ring[k] = ald(pr.sc + SC_URING + k);
      upd = update_converged(ring, its, ald(a.alpha + p), t + 7, t + 13, pr.sc[SC_UTOL]);
#pragma unroll
      for (int k = 0; k < UPD_WIN * 6; ++k) ast(pr.sc + SC_URING + k, ring[k]);
    }
    if (!isfinite(rel)) finish(a, p, FETI_ENAN);
    else if (rel <= pr.sc[SC_TOL] || upd) finish(a, p, 0);
    else if (total >= pr.ist[IS_MAXIT]) finish(a, p, FETI_ENOTCONV);
  }
}

__global__ void __launch_bounds__(PCG_BLOCK, BATCH_MIN_WAVES) k_pcg_batch(BatchArgs a) {
  extern __shared__ double lds[];
  __shared__ int s_ok, s_flag;
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
      for (int c = 0; c < 3; ++c) istore(a.cnt + 3 * p + c, 0);
      istore(a.iters + p, 0);
      istore(a.status + p, pr.ist[IS_STATUS]);
      const int d = pr.ist[IS_DONE] || pr.ist[IS_MAXIT] <= 0;
      istore(a.done + p, d);
      if (d) __hip_atomic_fetch_add(a.ndone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  ok = grid_sync(a.bar, nblk, gen, &s_ok);
  int it_local = 0, ph = 0;
  auto stamp = [&]() {
    if (a.tstamp && blockIdx.x == 0 && threadIdx.x == 0 && it_local < a.tstamp_iters)
      a.tstamp[it_local * 12 + ph] = (long long)wall_clock64();
    ++ph;
  };
  stamp();
  for (; ok; ++it_local, ph = 1) {  // stamp 0 of a later iteration is stamp 7 of the one before
    if (iload(a.ndone) >= a.P) break;  // read after a barrier: the same in every block
    // (A) y_b = (K^+)_bb B^T p, p = y + beta p_old
    if (a.f32) batch_gemv<float>(a, 0, xs, red8);
    else batch_gemv<double>(a, 0, xs, red8);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // (B) q_raw = B y_b, g = G^T q_raw
    batch_jump(a, 0, red);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // (C) q = P q_raw, partials of (p, q); alpha = rho / (p, q) by the last chunk's block
    batch_correct_dot(a, 0, acl, red, &s_flag);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // (D) lam += alpha p, r -= alpha q_raw, w -= alpha q, p_old = p; partial norms of w
    // (and of p and lambda for a problem with the update test); the stopping test by
    // the last chunk's block
    for (int it = blockIdx.x; it < a.nrow; it += nblk) {
      const int p = a.row_prob[it];
      if (iload(a.done + p)) continue;
      const ProbArgs& pr = a.probs[p];
      if (pr.sc[SC_UTOL] > 0.0) batch_update<19>(a, pr, p, it, red, &s_flag);
      else batch_update<7>(a, pr, p, it, red, &s_flag);
    }
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // (E) z_b = S_bb B^T D w
    if (a.f32) batch_gemv<float>(a, 1, xs, red8);
    else batch_gemv<double>(a, 1, xs, red8);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // (F) z = D B z_b, g = G^T z
    batch_jump(a, 1, red);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
    // (G) y = P z, partials of (w, y); beta = rho_new / rho by the last chunk's block
    batch_correct_dot(a, 1, acl, red, &s_flag);
    if (!(ok = grid_sync(a.bar, nblk, gen, &s_ok))) break;
    stamp();
  }
  if (!ok && threadIdx.x == 0)
    for (int p = blockIdx.x; p < a.P; p += nblk) {
      const ProbArgs& pr = a.probs[p];
      if (!iload(pr.ist + IS_DONE)) {
        istore(pr.ist + IS_STATUS, FETI_EHIP);
        istore(pr.ist + IS_DONE, 1);
        istore(a.status + p, FETI_EHIP);
      }
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
