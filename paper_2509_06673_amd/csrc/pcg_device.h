// Device helpers shared by the persistent PCG kernels (single problem and batch):
// device-coherent loads and stores, the bounded grid barrier, deterministic block
// sums, the jump rows read coherently and one interface GEMV tile.
#pragma once

#include "iface.h"
#include "iface_device.h"
#include "kernels.h"
#include "pcg.h"

namespace feti {

constexpr int PB = PCG_BLOCK;
#ifndef FETI_GEMV_BATCH
#define FETI_GEMV_BATCH 8
#endif
constexpr int GEMV_BATCH = FETI_GEMV_BATCH;  // column loads in flight per lane (multiple of 4)
// 1: the GEMV phases of the single-problem launch load one column batch ahead of the
// products (and the first batch before the gather)
#ifndef FETI_GEMV_PF
#define FETI_GEMV_PF 0
#endif
constexpr int GEMV_PF = FETI_GEMV_PF;
static_assert(GEMV_BATCH % 4 == 0, "GEMV batches are consumed four at a time");
constexpr long long PCG_SPIN_LIMIT = 1ll << 21;

// Data that one block writes and another reads within the launch (the multiplier
// vectors p, y, w, q, q_raw, z, the interface-space vectors, g and the partial
// sums) moves through device-coherent
// loads and stores (agent-scope relaxed atomics: no cache flush is needed);
// everything a thread reads back only itself, and the read-only matrices, use
// plain accesses.
__device__ inline double ald(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void ast(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier; returns false when the launch is being aborted.  Arrival
// counters only grow (the host clears them before a launch): a group's counter
// reaches (k + 1) * group size at barrier k, its last block then counts the group
// at the top level, and the last group publishes gen = k + 1.
// Every thread waits for its own stores to complete before its block arrives.
__device__ inline bool grid_sync(GridBarrier* b, uint32_t nblk, uint32_t& gen, int* s_ok) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x == 0) {
    // two levels: groups of PCG_BAR_GROUP blocks, then the groups
    const uint32_t grp = blockIdx.x / PCG_BAR_GROUP;
    const uint32_t ngrp = (nblk + PCG_BAR_GROUP - 1) / PCG_BAR_GROUP;
    const uint32_t gsize = min((uint32_t)PCG_BAR_GROUP, nblk - grp * PCG_BAR_GROUP);
    int ok = 1;
    bool last = false;
    const uint32_t p1 =
        __hip_atomic_fetch_add(&b->grp[grp * PCG_BAR_STRIDE], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p1 == (gen + 1) * gsize - 1) {
      if (ngrp == 1) {
        last = true;  // one group: its last block publishes at once
      } else {
        const uint32_t p2 = __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = p2 == (gen + 1) * ngrp - 1;
      }
    }
    if (last) {
      __hip_atomic_store(&b->gen, gen + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long long spins = 0;
      while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= gen) {
        if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
        if (++spins > PCG_SPIN_LIMIT) {
          __hip_atomic_store(&b->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    gen += 1;
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// jump of row j of the interface-space vector yb (signed sum of its two entries)
__device__ inline double pjump_raw(const DevMesh& m, const double* yb, int64_t r) {
  return m.jr_sign[2 * r] * ald(yb + m.jr_b[2 * r]) + m.jr_sign[2 * r + 1] * ald(yb + m.jr_b[2 * r + 1]);
}
__device__ inline double pjump_row(const DevMesh& m, const double* yb, int64_t j, int scaled) {
  if (!scaled) return pjump_raw(m, yb, j);
  const int gs = m.grp_start[j], gz = m.grp_size[j];
  double s = 0.0;
  for (int k = 0; k < gz; ++k) s += m.dwt[3 * j + k] * pjump_raw(m, yb, gs + k);
  return s;
}

// Deterministic block-wide sums of v[0..NV); the result is valid in every thread.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double x = v[c];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    v[c] = x;
  }
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < NV; ++c) red[wave * NV + c] = v[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double s = 0.0;
    for (int wv = 0; wv < PB / 64; ++wv) s += red[wv * NV + c];
    v[c] = s;
  }
  __syncthreads();
}

// Block-wide sums of v[0..NV) stored to dst[0..NV) (device-coherent), in the order of
// block_sum; the per-wave partials go through LDS so that no register array is
// indexed by the thread.
template <int NV>
__device__ inline void block_store(double (&v)[NV], double* red, double* dst) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double x = v[c];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    v[c] = x;
  }
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < NV; ++c) red[wave * NV + c] = v[c];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int wv = 0; wv < PB / 64; ++wv) s += red[wv * NV + threadIdx.x];
    ast(dst + threadIdx.x, s);
  }
  __syncthreads();
}

// Sum of the per-block partials part[b][0..NV) over all blocks into
// v[0..NV) (LDS), in two parts so that the loads overlap other work: gt_issue spreads
// the nblk x NV device-coherent loads over the threads (at most GT_LOADS each, issued
// together) into registers; gt_finish stages them in LDS (stage: nblk x NV doubles)
// and adds them in a fixed order.  v is valid in every thread after gt_finish.
constexpr int GT_LOADS = 10;
template <int NV>
__device__ inline void gt_issue(const double* part, int nblk, double (&t)[GT_LOADS]) {
  const int total = nblk * NV;  // <= GT_LOADS * PB (checked on the host)
#pragma unroll
  for (int k = 0; k < GT_LOADS; ++k) {
    const int idx = threadIdx.x + k * PB;
    t[k] = idx < total ? ald(part + (idx / NV) * PCG_NPART + idx % NV) : 0.0;
  }
}
template <int NV>
__device__ inline void gt_finish(const double (&t)[GT_LOADS], int nblk, double* v, double* stage) {
  const int total = nblk * NV;
#pragma unroll
  for (int k = 0; k < GT_LOADS; ++k) {
    const int idx = threadIdx.x + k * PB;
    if (idx < total) stage[idx] = t[k];
  }
  __syncthreads();
  // value c is summed by the 16 lanes 16 c .. 16 c + 15 (lane q: blocks q, q + 16, ...,
  // in order), then by a fixed shuffle tree over the 16 lanes
  static_assert(NV * 16 <= PB, "16 lanes per summed value");
  const int c = threadIdx.x >> 4, q = threadIdx.x & 15;
  if (c < NV) {
    double x = 0.0;
    int b = q;
    for (; b + 48 < nblk; b += 64) {
      const double u0 = stage[b * NV + c], u1 = stage[(b + 16) * NV + c];
      const double u2 = stage[(b + 32) * NV + c], u3 = stage[(b + 48) * NV + c];
      x += u0;
      x += u1;
      x += u2;
      x += u3;
    }
    for (; b < nblk; b += 16) x += stage[b * NV + c];
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) x += __shfl_xor(x, off, 16);
    if (q == 0) v[c] = x;
  }
  __syncthreads();  // v complete; stage free again
}

// The stopping decisions of an iteration from the totals conv (LDS; per-kind |w_k|^2
// in 0..5, |w|_M^2 in 6, per-kind |p|^2 in 7..12 and |lambda|^2 in 13..18), evaluated
// by wavefront 0 with kind k in lane k: the relative residual of rel_residual_of and,
// with upd, the update test of update_converged (the same operations on the same
// values, so the same results).  kc (LDS): the references sc[SC_REF..+6) in 0..5,
// sc[SC_EK..+6) in 6..11, sc[SC_EREF] in 12 and the sum of the six reference
// energies in 13.  Lane 0 stores the residual in *res and the update-test result in
// *upd_ok.
__device__ inline void stop_test_wave0(const double* conv, const double* kc, double* ring, int iters,
                                       double alpha, double utol, bool upd, double* res, int* upd_ok) {
  const int lane = threadIdx.x & 63;
  const bool kl = lane < 6;
  const int k = kl ? lane : 0;
  const double nan = __builtin_nan("");
  // residual: the largest of the energy ratio and the ratios of the included kinds
  // (fmax ignores NaN operands, so NaN stands for an excluded kind)
  const double rk = kc[k] > 0.0 ? sqrt(conv[k]) / kc[k] : 0.0;
  double rel = kl && kc[6 + k] > 1e-24 * kc[13] ? rk : nan;
  if (lane == 0) {
    const double den = kc[12], et = conv[6];
    rel = fmax(den > 0.0 ? sqrt(et) / den : (et > 0.0 ? 1.0 : 0.0), rel);
  }
  for (int off = 4; off > 0; off >>= 1) rel = fmax(rel, __shfl_xor(rel, off, 64));
  // update test
  bool ok = true, has = false;
  if (upd && kl) {
    double* slot = ring + (iters % UPD_WIN) * 6;
    slot[k] = fabs(alpha) * sqrt(conv[7 + k]);
    const double l2 = conv[13 + k];
    has = l2 > 0.0;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < UPD_WIN; ++i) s += ring[i * 6 + k];
    ok = !has || s <= utol * sqrt(l2);
  }
  const bool all_ok = __ballot(!ok) == 0ull;
  const bool any_has = __ballot(has) != 0ull;
  if (lane == 0) {
    *res = rel;
    *upd_ok = upd && utol > 0.0 && iters >= UPD_WIN && all_ok && any_has;
  }
}

// x_b of subdomain block (nbs entries from b0) gathered into xs by the threads
// ht = 0..255: SCALED = 0: x_b = B_s^T p with p = src + beta src2; SCALED = 1:
// x_b = B_s^T D src.
template <int SCALED>
__device__ inline void gather_x(const DevMesh& m, int nbs, int64_t b0, const double* src, const double* src2,
                                double beta, double* xs, int ht) {
  // two entries per thread and pass, their loads issued together; branch-free: an
  // absent entry (or one past nbs) reads row 0 with weight 0
  for (int i0 = ht; i0 < nbs; i0 += 512) {
    double v[2] = {0.0, 0.0};
    if (SCALED) {
      int r[2][3];
      double wt[2][3], x[2][3];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool in = i0 + 256 * h < nbs;
        const int64_t gb = b0 + (in ? i0 + 256 * h : 0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int rk = in ? m.bd_row[3 * gb + k] : -1;
          r[h][k] = rk >= 0 ? rk : 0;
          wt[h][k] = rk >= 0 ? m.bd_wt[3 * gb + k] : 0.0;
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < 3; ++k) x[h][k] = ald(src + r[h][k]);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < 3; ++k) v[h] += wt[h][k] * x[h][k];
    } else {
      int r0[2], r1[2];
      double s0[2], s1[2], y0[2], p0[2], y1[2], p1[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool in = i0 + 256 * h < nbs;
        const int64_t gb = b0 + (in ? i0 + 256 * h : 0);
        const int q0 = in ? m.bg_row[2 * gb] : -1, q1 = in ? m.bg_row[2 * gb + 1] : -1;
        r0[h] = q0 >= 0 ? q0 : 0;
        r1[h] = q1 >= 0 ? q1 : 0;
        s0[h] = q0 >= 0 ? m.bg_sign[2 * gb] : 0.0;
        s1[h] = q1 >= 0 ? m.bg_sign[2 * gb + 1] : 0.0;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        y0[h] = ald(src + r0[h]);
        p0[h] = ald(src2 + r0[h]);
        y1[h] = ald(src + r1[h]);
        p1[h] = ald(src2 + r1[h]);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        v[h] = s0[h] * (y0[h] + beta * p0[h]);
        v[h] += s1[h] * (y1[h] + beta * p1[h]);
      }
    }
    xs[i0] = v[0];
    if (i0 + 256 < nbs) xs[i0 + 256] = v[1];
  }
}

// sum over the columns k in [kb, ke) of A_s[i][k] xs[k] (A_s column-major with leading
// dimension ld): batches of GEMV_BATCH independent column loads in flight before their
// FMAs (a lane's column range is a chain of dependent round trips to HBM, so the
// batch size sets the bytes in flight), the last columns as one batch
template <class MT, int NB = GEMV_BATCH>
__device__ inline double tile_cols(const MT* As, int64_t ld, int i, int kb, int ke, const double* xs) {
  static_assert(NB % 4 == 0, "GEMV batches are consumed four at a time");
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  const MT* col = As + (int64_t)kb * ld + i;
  int k = kb;
  for (; k + NB <= ke; k += NB, col += NB * ld) {
    MT v[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) v[u] = col[(int64_t)u * ld];
#pragma unroll
    for (int u = 0; u < NB; u += 4) {
      acc0 += (double)v[u + 0] * xs[k + u + 0];
      acc1 += (double)v[u + 1] * xs[k + u + 1];
      acc2 += (double)v[u + 2] * xs[k + u + 2];
      acc3 += (double)v[u + 3] * xs[k + u + 3];
    }
  }
  if (k < ke) {
    // the last (ke - k < NB) columns: loads together, products in order
    MT v[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) v[u] = k + u < ke ? col[(int64_t)u * ld] : (MT)0;
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (k + u < ke) acc0 += (double)v[u] * xs[k + u];
  }
  return (acc0 + acc1) + (acc2 + acc3);
}

// The same sum with the loads of the next batch issued before the products of the
// current one (two batches in flight), and the first batch (v) loaded by the caller
// before x_b is gathered, so that its latency overlaps the gather.  The products are
// those of tile_cols in the same order.
template <class MT, int NB>
__device__ inline double tile_cols_pf(const MT* col, int64_t ld, int kb, int ke, const double* xs, MT (&v)[NB]) {
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  for (int k = kb; k < ke; k += NB) {
    const int kn = k + NB;
    MT w[NB];
    if (kn < ke) {
#pragma unroll
      for (int u = 0; u < NB; ++u) w[u] = kn + u < ke ? col[(int64_t)(kn - kb + u) * ld] : (MT)0;
    }
    if (kn <= ke) {
#pragma unroll
      for (int u = 0; u < NB; u += 4) {
        acc0 += (double)v[u + 0] * xs[k + u + 0];
        acc1 += (double)v[u + 1] * xs[k + u + 1];
        acc2 += (double)v[u + 2] * xs[k + u + 2];
        acc3 += (double)v[u + 3] * xs[k + u + 3];
      }
    } else {
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (k + u < ke) acc0 += (double)v[u] * xs[k + u];
    }
    if (kn < ke) {
#pragma unroll
      for (int u = 0; u < NB; ++u) v[u] = w[u];
    }
  }
  return (acc0 + acc1) + (acc2 + acc3);
}

// One 64-row tile of y_b = A_s x_b (interface block of subdomain s) by one half of
// the block (four wavefronts, threads ht = 0..255): x_b gathered into xs, the
// wavefronts split the column range and combine in red4.  SCALED as in gather_x.
// valid = false: the half only takes part in the block's barriers.  PF: the column
// loads run ahead of the products (tile_cols_pf).
template <class MT, int SCALED, int NB = GEMV_BATCH, int PF = 0>
__device__ inline void gemv_tile(const DevMesh& m, const MT* A, int s, int row0, bool valid, const double* src,
                          const double* src2, double beta, double* yout, double* xs, double* red4, int ht) {
  const int wave = ht >> 6, lane = ht & 63;
  const int nbs = valid ? m.nb[s] : 0;
  const int64_t b0 = valid ? m.boff[s] : 0;
  const int i = row0 + lane;
  const int kq = (nbs + 3) / 4;
  const int kb = wave * kq, ke = min(nbs, kb + kq);
  MT pre[NB];
  const MT* col = nullptr;
  if (PF) {
    const int64_t ld = valid ? m.ldb[s] : 0;
    col = valid ? A + m.sofs[s] + (int64_t)kb * ld + i : A;
#pragma unroll
    for (int u = 0; u < NB; ++u) pre[u] = (i < nbs && kb + u < ke) ? col[(int64_t)u * ld] : (MT)0;
  }
  __syncthreads();  // xs and red4 of the previous tiles are consumed
  gather_x<SCALED>(m, nbs, b0, src, src2, beta, xs, ht);
  __syncthreads();
  double v = 0.0;
  if (PF) {
    if (i < nbs) v = tile_cols_pf<MT, NB>(col, m.ldb[s], kb, ke, xs, pre);
  } else {
    if (i < nbs) v = tile_cols<MT, NB>(A + m.sofs[s], m.ldb[s], i, kb, ke, xs);
  }
  red4[wave * 64 + lane] = v;
  __syncthreads();
  if (wave == 0 && i < nbs)
    ast(yout + b0 + i, (red4[lane] + red4[64 + lane]) + (red4[128 + lane] + red4[192 + lane]));
}

}  // namespace feti
