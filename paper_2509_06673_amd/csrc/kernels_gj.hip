// Batched pivot-free symmetric Gauss-Jordan elimination on MFMA, in FP64 or FP32.
//
// Each local matrix K_s is swept pivot block by pivot block in its
// [interior | interface] order.  Sweeping a pivot block P of
//     [[P, C], [C^T, D]]  gives  [[-P^{-1}, P^{-1} C], [C^T P^{-1}, D - C^T P^{-1} C]],
// so after the interior blocks the trailing block holds the interface Schur
// complement S_bb = K_bb - K_bI K_II^{-1} K_Ib of eq. (reduced-system) (it is
// copied out at that point), and after every non-fixed pivot the swept block
// holds -K_ss^{-1}.  The pivots are the D of the LDL^T factorisation in the
// same order: the order [I_U | I_P | b_U | b_P] makes K_s quasi-definite (the
// U block is positive definite, the P Schur complement negative definite),
// so no pivoting is needed (Theorem 3.1's reduction).
//
// The O(n^3) part is the rank-kw update D -= C^T W with W = P^{-1} C, done on
// v_mfma_f64_16x16x4 (FP64) or v_mfma_f32_16x16x4 (FP32) tiles: each 64x64
// output tile is owned by one workgroup of four wavefronts, each computing a
// 32x32 quarter as 2x2 MFMA blocks.  The swept matrix stays symmetric, so only the
// tiles on and below the diagonal are updated: every entry is read from the lower
// triangle (row max(i, j), column min(i, j)), the panel rows and columns are written
// on both sides, and the end result is mirrored once.  In the FP32 variant the small pivot
// blocks are inverted and W is accumulated in FP64 before rounding to FP32;
// the update runs in FP32 on the matrix cores.
#include "kernels.h"

namespace feti {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// One 16x16x4 MFMA per element type.  Operands: lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16].  Result register r of lane l holds column l % 16 and the
// row given by row() (the two instructions differ; both checked by a lane probe).
template <class T> struct Mfma;
template <> struct Mfma<double> {
  typedef dbl4 acc4;
  __device__ static acc4 run(double a, double b, acc4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int r) { return (lane / 16) + 4 * r; }
};
template <> struct Mfma<float> {
  typedef flt4 acc4;
  __device__ static acc4 run(float a, float b, acc4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int r) { return 4 * (lane / 16) + r; }
};

constexpr int GJ_NB = 128;  // maximum panel width (the plan may use less)
constexpr int GJ_KC = 32;   // pivots per chunk of the update's inner products

// (1) invert the pivot block in LDS (in FP64) by a blocked in-place Gauss-Jordan sweep:
// for each sub-panel S of 32 pivots (R = the other indices of the block),
//   M_SS <- M_SS^{-1} (32 element steps),  M_SR <- M_SS^{-1} M_SR,
//   M_RR <- M_RR - M_RS M_SR,               M_RS <- -M_RS M_SS^{-1},
// which is the element sweep (pivot 1/p, row / p, column -c/p, rest - c r / p) applied to
// the 32 pivots in turn.  512 threads; products formed in registers, then written.
template <class T>
__global__ void __launch_bounds__(512) k_gj_pivot(const int32_t* __restrict__ pstart,
                                                  const int32_t* __restrict__ pwidth,
                                                  const int64_t* __restrict__ aofs,
                                                  const int32_t* __restrict__ lda,
                                                  const T* __restrict__ A,
                                                  double* __restrict__ pinv,
                                                  int32_t* __restrict__ status, int nmat, int step,
                                                  int nb) {
  const int m = blockIdx.x;
  const int kw = pwidth[step * nmat + m];
  if (kw == 0) return;
  const int k0 = pstart[step * nmat + m];
  const T* Am = A + aofs[m];
  const int64_t ld = lda[m];
  constexpr int SB = 32;  // sub-panel
  __shared__ double M[GJ_NB][GJ_NB + 1];
  const int tid = threadIdx.x;
  for (int t = tid; t < GJ_NB * GJ_NB; t += 512) {
    const int i = t >> 7, j = t & (GJ_NB - 1);
    if (i < kw && j < kw) M[i][j] = (double)Am[(k0 + max(i, j)) * ld + k0 + min(i, j)];
  }
  __syncthreads();
  bool bad = false;
  for (int s0 = 0; s0 < kw; s0 += SB) {
    const int sw = min(SB, kw - s0);
    // M_SS <- M_SS^{-1}: element steps on the sub-panel block (thread: entries t, t + 512)
    for (int k = s0; k < s0 + sw; ++k) {
      const double piv = M[k][k];
      if (!(fabs(piv) > 0.0) || !isfinite(piv)) bad = true;
      const double pinvk = 1.0 / piv;
      double nv[2];
      int ii[2], jj[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = tid + 512 * h;
        const int i = s0 + (t >> 5), j = s0 + (t & 31);
        ii[h] = i;
        jj[h] = j;
        nv[h] = 0.0;
        if ((t >> 5) < sw && (t & 31) < sw) {
          if (i == k) nv[h] = j == k ? pinvk : M[k][j] * pinvk;
          else nv[h] = j == k ? -M[i][k] * pinvk : M[i][j] - M[i][k] * (M[k][j] * pinvk);
        }
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = tid + 512 * h;
        if ((t >> 5) < sw && (t & 31) < sw) M[ii[h]][jj[h]] = nv[h];
      }
      __syncthreads();
    }
    if (sw == kw) break;  // the whole block was one sub-panel
    // M_SR <- M_SS^{-1} M_SR: thread (row a = tid / 16, columns tid % 16 + 16 c)
    {
      const int a = tid >> 4, cb = tid & 15;
      double acc[GJ_NB / 16];
#pragma unroll
      for (int c = 0; c < GJ_NB / 16; ++c) acc[c] = 0.0;
      if (a < sw)
        for (int bq = 0; bq < sw; ++bq) {
          const double pab = M[s0 + a][s0 + bq];
#pragma unroll
          for (int c = 0; c < GJ_NB / 16; ++c) {
            const int j = cb + 16 * c;
            if (j < kw && (j < s0 || j >= s0 + sw)) acc[c] += pab * M[s0 + bq][j];
          }
        }
      __syncthreads();
      if (a < sw)
#pragma unroll
        for (int c = 0; c < GJ_NB / 16; ++c) {
          const int j = cb + 16 * c;
          if (j < kw && (j < s0 || j >= s0 + sw)) M[s0 + a][j] = acc[c];
        }
      __syncthreads();
    }
    // M_RR <- M_RR - M_RS M_SR and the new column block M_RS <- -M_RS M_SS^{-1}: thread
    // (rows 4 (tid / 16) .. + 3, columns tid % 16 + 16 c); the column block is formed in
    // registers from the old M_RS before anything is written
    {
      const int rb = (tid >> 4) * 4, cb = tid & 15;
      double acc[4][GJ_NB / 16];
      double col[4][2];  // new M_RS entries of this thread: rows rb..rb+3, columns s0 + cb, s0 + cb + 16
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int c = 0; c < GJ_NB / 16; ++c) acc[r][c] = 0.0;
        col[r][0] = col[r][1] = 0.0;
      }
      for (int bq = 0; bq < sw; ++bq) {
        double mrs[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) mrs[r] = rb + r < kw ? M[rb + r][s0 + bq] : 0.0;
#pragma unroll
        for (int c = 0; c < GJ_NB / 16; ++c) {
          const int j = cb + 16 * c;
          const double msr = j < kw ? M[s0 + bq][j] : 0.0;
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[r][c] += mrs[r] * msr;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int ac = cb + 16 * h;  // column of M_SS^{-1}
          const double pinv_ba = ac < sw ? M[s0 + bq][s0 + ac] : 0.0;
#pragma unroll
          for (int r = 0; r < 4; ++r) col[r][h] -= mrs[r] * pinv_ba;
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = rb + r;
        if (i >= kw || (i >= s0 && i < s0 + sw)) continue;
#pragma unroll
        for (int c = 0; c < GJ_NB / 16; ++c) {
          const int j = cb + 16 * c;
          if (j < kw && (j < s0 || j >= s0 + sw)) M[i][j] -= acc[r][c];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int ac = cb + 16 * h;
          if (ac < sw) M[i][s0 + ac] = col[r][h];
        }
      }
      __syncthreads();
    }
  }
  if (bad && tid == 0) status[m] = 1;
  double* Pm = pinv + (int64_t)m * nb * nb;
  for (int t = tid; t < GJ_NB * GJ_NB; t += 512) {
    const int i = t >> 7, j = t & (GJ_NB - 1);
    if (i < kw && j < kw) Pm[i * nb + j] = M[i][j];
  }
}

// (2) W = P^{-1} C over all columns outside the panel, in FP64 on the matrix cores, stored
// in T.  One workgroup per 64 columns j0 .. j0 + 63 of a matrix: C[k][j0 + x] is staged in
// LDS (in FP64), and the product W^T = C^T P^{-1} (P^{-1} is symmetric) is formed from
// chunks of 32 rows of P^{-1} staged in turn; each of the four wavefronts computes 64
// columns x 32 rows of W as 4 x 2 blocks of 16 x 16.
template <class T>
__global__ void __launch_bounds__(256) k_gj_row(const int32_t* __restrict__ pstart,
                                                const int32_t* __restrict__ pwidth,
                                                const int64_t* __restrict__ aofs,
                                                const int32_t* __restrict__ lda,
                                                const int32_t* __restrict__ nn,
                                                const T* __restrict__ A,
                                                const double* __restrict__ pinv,
                                                T* __restrict__ wrow, int nmat, int step,
                                                int nb, int max_n) {
  const int m = blockIdx.y;
  const int kw = pwidth[step * nmat + m];
  if (kw == 0) return;
  const int k0 = pstart[step * nmat + m];
  const int n = nn[m];
  const int j0 = blockIdx.x * 64;
  if (j0 >= n) return;
  // column blocks fully inside the panel have nothing to form
  if (j0 >= k0 && j0 + 64 <= k0 + kw) return;
  __shared__ double Ct[GJ_NB][64];        // C[k][j0 + x]
  __shared__ double Pc[GJ_KC][GJ_NB + 4];  // rows kc .. kc + 31 of P^{-1}
  const T* Am = A + aofs[m];
  const int64_t ld = lda[m];
  const int kp = (kw + 3) & ~3;
  for (int t = threadIdx.x; t < kp * 64; t += blockDim.x) {
    const int k = t / 64, x = t % 64;
    const int j = j0 + x;
    Ct[k][x] = (k < kw && j < n && !(j >= k0 && j < k0 + kw)) ? (double)Am[max(k0 + k, j) * ld + min(k0 + k, j)]
                                                                : 0.0;
  }
  const double* Pm = pinv + (int64_t)m * nb * nb;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int lr = lane % 16, lk = lane / 16;
  const int ib = wave * 32;  // rows i of W (columns of the product) of this wavefront
  Mfma<double>::acc4 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<double>::acc4{0.0, 0.0, 0.0, 0.0};
  for (int kc = 0; kc < kp; kc += GJ_KC) {
    const int kn = min(GJ_KC, kp - kc);
    __syncthreads();  // Ct staged, or the previous chunk consumed
    for (int t = threadIdx.x; t < kn * GJ_NB; t += blockDim.x) {
      const int k = t / GJ_NB, i = t % GJ_NB;
      Pc[k][i] = (kc + k < kw && i < kw) ? Pm[(kc + k) * nb + i] : 0.0;
    }
    __syncthreads();
    if (ib < kw)
      for (int k = 0; k < kn; k += 4) {
        double av[4], bv[2];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = Ct[kc + k + lk][a * 16 + lr];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Pc[k + lk][ib + b * 16 + lr];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<double>::run(av[a], bv[b], acc[a][b]);
      }
  }
  if (ib >= kw) return;
  T* W = wrow + (int64_t)m * nb * max_n;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = j0 + a * 16 + Mfma<double>::row(lane, r);
        const int i = ib + b * 16 + lr;
        if (i < kw && j < n && !(j >= k0 && j < k0 + kw)) W[(int64_t)i * max_n + j] = (T)acc[a][b][r];
      }
}

// (3) D -= C^T W outside the panel rows and columns (MFMA), on the tiles on and
// below the diagonal.  One workgroup per 64-row strip of a matrix: the strip's panel
// block C[k][i0 + i] is staged in LDS once, and the workgroup walks the 64-column
// tiles j0 <= i0 of the row, staging W[k][j0 + j] and updating the 64x64 tile of A
// (four wavefronts, a 32x32 quarter each as 2x2 MFMA blocks).
template <class T>
__global__ void __launch_bounds__(256) k_gj_update(const int32_t* __restrict__ pstart,
                                                   const int32_t* __restrict__ pwidth,
                                                   const int64_t* __restrict__ aofs,
                                                   const int32_t* __restrict__ lda,
                                                   const int32_t* __restrict__ nn,
                                                   T* __restrict__ A,
                                                   const T* __restrict__ wrow, int nmat,
                                                   int step, int nb, int max_n) {
  const int m = blockIdx.y;
  const int kw = pwidth[step * nmat + m];
  if (kw == 0) return;
  const int n = nn[m];
  const int i0 = blockIdx.x * 64;
  if (i0 >= n) return;
  const int k0 = pstart[step * nmat + m];
  // strips fully inside the panel rows have nothing to update
  if (i0 >= k0 && i0 + 64 <= k0 + kw) return;
  T* Am = A + aofs[m];
  const int ld = lda[m];
  const T* W = wrow + (int64_t)m * nb * max_n;
  __shared__ T Ct[GJ_NB][64];  // C[k][i0 + i]
  __shared__ T Wt[GJ_KC][64];  // W[k][j0 + j] for one chunk of GJ_KC pivots
  const int kp = (kw + 3) & ~3;     // padded to the MFMA depth
  for (int t = threadIdx.x; t < kp * 64; t += blockDim.x) {
    const int k = t / 64, x = t % 64;
    const int i = i0 + x;
    Ct[k][x] = (k < kw && i < n) ? Am[(int64_t)max(k0 + k, i) * ld + min(k0 + k, i)] : T(0);
  }
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const int lr = lane % 16, lk = lane / 16;
  for (int j0 = 0; j0 <= i0; j0 += 64) {
    // column tiles fully inside the panel columns have nothing to update
    if (j0 >= k0 && j0 + 64 <= k0 + kw) continue;
    // the lane's 16 entries of the A tile are loaded before the products, so that their
    // latency overlaps the matrix-core work (entries outside the update read as 0)
    T old[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + wi + a * 16 + Mfma<T>::row(lane, r);
          const int j = j0 + wj + b * 16 + (lane % 16);
          const bool upd = i < n && j < n && !(i >= k0 && i < k0 + kw) && !(j >= k0 && j < k0 + kw);
          old[a][b][r] = upd ? Am[(int64_t)i * ld + j] : T(0);
        }
    typename Mfma<T>::acc4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = typename Mfma<T>::acc4{T(0), T(0), T(0), T(0)};
    // the panel's pivots in chunks of GJ_KC: W[k][j0 + j] of the chunk staged in LDS, then
    // the rank-4 MFMA steps over it; the next chunk's W entries are loaded into registers
    // while the current chunk's products run
    constexpr int WPT = GJ_KC * 64 / 256;  // staged W entries per thread and chunk
    T wr[WPT];
    auto load_chunk = [&](int kc) {
#pragma unroll
      for (int q = 0; q < WPT; ++q) {
        const int t = threadIdx.x + q * 256;
        const int k = t / 64, x = t % 64;
        const int j = j0 + x;
        wr[q] = (kc + k < kw && j < n && !(j >= k0 && j < k0 + kw)) ? W[(int64_t)(kc + k) * max_n + j] : T(0);
      }
    };
    load_chunk(0);
    for (int kc = 0; kc < kp; kc += GJ_KC) {
      const int kn = min(GJ_KC, kp - kc);
      __syncthreads();  // Ct staged, or the previous chunk consumed
#pragma unroll
      for (int q = 0; q < WPT; ++q) {
        const int t = threadIdx.x + q * 256;
        Wt[t / 64][t % 64] = wr[q];
      }
      __syncthreads();
      if (kc + GJ_KC < kp) load_chunk(kc + GJ_KC);
      for (int k = 0; k < kn; k += 4) {
        T av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = Ct[kc + k + lk][wi + a * 16 + lr];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Wt[k + lk][wj + b * 16 + lr];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = Mfma<T>::run(av[a], bv[b], acc[a][b]);
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + wi + a * 16 + Mfma<T>::row(lane, r);
          const int j = j0 + wj + b * 16 + (lane % 16);
          if (i >= n || j >= n) continue;
          if ((i >= k0 && i < k0 + kw) || (j >= k0 && j < k0 + kw)) continue;
          Am[(int64_t)i * ld + j] = old[a][b][r] - acc[a][b][r];
        }
  }
}

// (4) write the swept panel into the lower triangle: the panel rows W left of the panel,
// the panel columns W^T below it, the pivot block -P^{-1}.  One workgroup per 64 columns
// j0 .. j0 + 63 of a matrix: W[k][j0 + x] is staged in LDS (coalesced reads), then the
// rows are written along j and the columns along k (32 consecutive entries of a row of
// A per 32 threads).  The upper triangle is never read again.
template <class T>
__global__ void __launch_bounds__(256) k_gj_write(const int32_t* __restrict__ pstart,
                                                  const int32_t* __restrict__ pwidth,
                                                  const int64_t* __restrict__ aofs,
                                                  const int32_t* __restrict__ lda,
                                                  const int32_t* __restrict__ nn,
                                                  T* __restrict__ A,
                                                  const double* __restrict__ pinv,
                                                  const T* __restrict__ wrow, int nmat,
                                                  int step, int nb, int max_n) {
  const int m = blockIdx.y;
  const int kw = pwidth[step * nmat + m];
  if (kw == 0) return;
  const int k0 = pstart[step * nmat + m];
  const int n = nn[m];
  const int j0 = blockIdx.x * 64;
  if (j0 >= n) return;
  T* Am = A + aofs[m];
  const int64_t ld = lda[m];
  const T* W = wrow + (int64_t)m * nb * max_n;
  const double* Pm = pinv + (int64_t)m * nb * nb;
  __shared__ T Ws[GJ_NB][65];
  for (int t = threadIdx.x; t < kw * 64; t += blockDim.x) {
    const int k = t / 64, x = t % 64;
    const int j = j0 + x;
    Ws[k][x] = (j < n && !(j >= k0 && j < k0 + kw)) ? W[(int64_t)k * max_n + j] : T(0);
  }
  __syncthreads();
  // rows k0 + k, columns j < k0 (lower triangle): along j
  for (int t = threadIdx.x; t < kw * 64; t += blockDim.x) {
    const int k = t / 64, x = t % 64;
    const int j = j0 + x;
    if (j < n && j < k0) Am[(int64_t)(k0 + k) * ld + j] = Ws[k][x];
  }
  // columns k0 + k, rows j >= k0 + kw (lower triangle), and the pivot block: along k
  for (int t = threadIdx.x; t < kw * 64; t += blockDim.x) {
    const int x = t / kw, k = t % kw;
    const int j = j0 + x;
    if (j >= n) continue;
    if (j >= k0 + kw) Am[(int64_t)j * ld + k0 + k] = Ws[k][x];
    else if (j >= k0) Am[(int64_t)j * ld + k0 + k] = (T)(-Pm[(j - k0) * nb + k]);
  }
}

template <class T>
__global__ void k_gj_snapshot(const int32_t* __restrict__ pflag, const int64_t* __restrict__ aofs,
                              const int32_t* __restrict__ lda, const int32_t* __restrict__ nn,
                              const int64_t* __restrict__ snap_ofs,
                              const int32_t* __restrict__ snap_at,
                              const int32_t* __restrict__ snap_ld, const T* __restrict__ A,
                              T* __restrict__ snap, int nmat, int step) {
  const int m = blockIdx.y;
  if (!(pflag[step * nmat + m] & 1) || snap_ofs[m] < 0) return;
  const int n = nn[m], at = snap_at[m], nbm = n - at;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nbm * nbm) return;
  const int i = (int)(t / nbm), j = (int)(t % nbm);
  snap[snap_ofs[m] + (int64_t)i * snap_ld[m] + j] = A[aofs[m] + (int64_t)(at + max(i, j)) * lda[m] + at + min(i, j)];
}

// K^+ = -(swept block), zero on the rows and columns that were not swept: the thread
// of a lower entry (i >= j) writes it and its mirror
template <class T>
__global__ void k_gj_finalize(const int64_t* __restrict__ aofs, const int32_t* __restrict__ lda,
                              const int32_t* __restrict__ nn, const int32_t* __restrict__ nswept,
                              T* __restrict__ A) {
  const int m = blockIdx.z;
  const int n = nn[m], ns = nswept[m];
  const int i = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || j > i) return;
  T* a = A + aofs[m];
  const int64_t ld = lda[m];
  const T v = (i < ns && j < ns) ? -a[(int64_t)i * ld + j] : T(0);
  a[(int64_t)i * ld + j] = v;
  if (j != i) a[(int64_t)j * ld + i] = v;
}

template <class T>
void launch_gj_step(const GJPlan& p, T* A, T* snap, int step, bool snap_now, hipStream_t st) {
  T* wrow = static_cast<T*>(p.wrow);
  hipLaunchKernelGGL(k_gj_pivot<T>, dim3(p.nmat), dim3(512), 0, st, p.pstart, p.pwidth, p.aofs, p.lda,
                     A, p.pinv, p.status, p.nmat, step, p.nb);
  hipLaunchKernelGGL(k_gj_row<T>, dim3((p.max_n + 63) / 64, p.nmat), dim3(256), 0, st, p.pstart,
                     p.pwidth, p.aofs, p.lda, p.n, A, p.pinv, wrow, p.nmat, step, p.nb, p.max_n);
  const int nt = (p.max_n + 63) / 64;
  hipLaunchKernelGGL(k_gj_update<T>, dim3(nt, p.nmat), dim3(256), 0, st, p.pstart, p.pwidth,
                     p.aofs, p.lda, p.n, A, wrow, p.nmat, step, p.nb, p.max_n);
  hipLaunchKernelGGL(k_gj_write<T>, dim3((p.max_n + 63) / 64, p.nmat), dim3(256), 0, st, p.pstart,
                     p.pwidth, p.aofs, p.lda, p.n, A, p.pinv, wrow, p.nmat, step, p.nb, p.max_n);
  if (snap != nullptr && snap_now) {
    const int64_t cnt = (int64_t)p.max_n * p.max_n;
    hipLaunchKernelGGL(k_gj_snapshot<T>, dim3((unsigned)((cnt + 255) / 256), p.nmat), dim3(256), 0, st,
                       p.pflag, p.aofs, p.lda, p.n, p.snap_ofs, p.snap_at, p.snap_ld, A, snap,
                       p.nmat, step);
  }
}

template <class T>
void launch_gj_finalize(const GJPlan& p, T* A, const int32_t* nswept, hipStream_t st) {
  hipLaunchKernelGGL(k_gj_finalize<T>, dim3((p.max_n + 255) / 256, p.max_n, p.nmat), dim3(256), 0, st,
                     p.aofs, p.lda, p.n, nswept, A);
}

template void launch_gj_step<double>(const GJPlan&, double*, double*, int, bool, hipStream_t);
template void launch_gj_step<float>(const GJPlan&, float*, float*, int, bool, hipStream_t);
template void launch_gj_finalize<double>(const GJPlan&, double*, const int32_t*, hipStream_t);
template void launch_gj_finalize<float>(const GJPlan&, float*, const int32_t*, hipStream_t);

}  // namespace feti
