// Local solves y_s = K_s^+ x_s of every subdomain from the lower triangle of the
// symmetric K_s^+ (the generalised inverse of the symmetric local matrix, proof of
// Theorem 3.1), stored as packed 64 x 64 tiles: about half the bytes of the dense
// blocks, and the product is bound by HBM bandwidth.
//
// One wavefront per stored tile (I, J), J <= I: the row part A_IJ x_J comes from the
// coalesced column loads of the tile, which are also staged in LDS (16 columns at a
// time, so that four blocks fit a CU) for the transposed part A_IJ^T x_I (off-diagonal
// tiles only).  Both parts go
// to a partial buffer; a second kernel sums, for every row, the partials of its
// tile row and tile column in a fixed order (deterministic, no atomics).
#include "kernels.h"

namespace feti {

constexpr int SYM_TS = 64;                 // tile size
constexpr int SYM_TE = SYM_TS * SYM_TS;    // elements per tile
constexpr int SYM_WAVES = 4;               // tiles per block
constexpr int SYM_Q = 16;                  // tile columns staged in LDS at a time
constexpr int SYM_LD = 65;                 // LDS row stride of the staged columns

// Tile t of the packed storage: column-major 64 x 64, element (i, k) of tile (I, J)
// at t * 4096 + k * 64 + i = K_s[I * 64 + i][J * 64 + k] (zero outside n_s).
template <class T>
__global__ void __launch_bounds__(256) k_sym_pack(SymArgs a, const T* __restrict__ K, const int64_t* __restrict__ kofs,
                                                  const int32_t* __restrict__ ld, const int32_t* __restrict__ ns,
                                                  T* __restrict__ P) {
  const int t = blockIdx.x;
  const int s = a.t_sub[t], I = a.t_I[t], J = a.t_J[t], n = ns[s];
  const T* Ks = K + kofs[s];
  const int64_t lds = ld[s];
  for (int e = threadIdx.x; e < SYM_TE; e += blockDim.x) {
    const int i = e / SYM_TS, k = e % SYM_TS;  // consecutive threads read along a row of K_s
    const int r = I * SYM_TS + i, c = J * SYM_TS + k;
    P[(int64_t)t * SYM_TE + k * SYM_TS + i] = (r < n && c < n) ? Ks[(int64_t)r * lds + c] : (T)0;
  }
}

template <class T>
__global__ void __launch_bounds__(256) k_sym_tiles(SymArgs a, const T* __restrict__ P, const int64_t* __restrict__ soff,
                                                   const int32_t* __restrict__ ns, const double* __restrict__ x) {
  __shared__ double L[SYM_WAVES][SYM_Q * SYM_LD];
  __shared__ double xv[SYM_WAVES][2][SYM_TS];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.x * SYM_WAVES + wave;
  const bool valid = t < a.ntile;  // an idle wavefront still takes part in the block barriers
  const int s = valid ? a.t_sub[t] : 0, I = valid ? a.t_I[t] : 0, J = valid ? a.t_J[t] : 0;
  const int n = valid ? ns[s] : 0;
  const double* xs = x + (valid ? soff[s] : 0);
  double* xJ = xv[wave][0];
  double* xI = xv[wave][1];
  xJ[lane] = (J * SYM_TS + lane < n) ? xs[J * SYM_TS + lane] : 0.0;
  xI[lane] = (I * SYM_TS + lane < n) ? xs[I * SYM_TS + lane] : 0.0;
  const T* tile = P + (int64_t)(valid ? t : 0) * SYM_TE;
  double* Lw = L[wave];
  double u = 0.0;
  for (int h = 0; h < SYM_TS / SYM_Q; ++h) {
    __syncthreads();  // xv written, or the previous columns consumed
    if (valid) {
#pragma unroll
      for (int kk = 0; kk < SYM_Q; ++kk) {
        const int k = h * SYM_Q + kk;
        const double v = (double)tile[k * SYM_TS + lane];
        u += v * xJ[k];
        Lw[kk * SYM_LD + lane] = v;
      }
    }
    __syncthreads();
    if (valid && I != J && (lane & 16) == 0) {
      // (A^T x_I)_k for the SYM_Q columns k of this step: lanes l and l + 32 (l < 16) take
      // the two halves of the i range of column h * SYM_Q + l (the shuffle pairs only
      // lanes of this branch)
      const int kk = lane & (SYM_Q - 1), i0 = (lane >> 5) * 32;
      double v = 0.0;
#pragma unroll 8
      for (int i = 0; i < 32; ++i) v += Lw[kk * SYM_LD + i0 + i] * xI[i0 + i];
      v += __shfl_xor(v, 32, 64);
      if (lane < 32) a.part[(int64_t)t * 2 * SYM_TS + SYM_TS + h * SYM_Q + kk] = v;
    }
  }
  if (valid) a.part[(int64_t)t * 2 * SYM_TS + lane] = u;
}

// y_s[r] = sum over J <= I of row parts of tiles (I, J) + sum over I' > I of the
// transposed parts of tiles (I', I), I = r / 64 (tile order: fixed)
__global__ void __launch_bounds__(256) k_sym_sum(SymArgs a, const int64_t* __restrict__ soff,
                                                 const int32_t* __restrict__ ns, double* __restrict__ y) {
  const int s = blockIdx.y;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ns[s]) return;
  const int I = r / SYM_TS, i = r % SYM_TS, T = a.nt[s];
  const int64_t base = a.tbase[s];
  double acc = 0.0;
  const int64_t row0 = base + (int64_t)I * (I + 1) / 2;
  for (int J = 0; J <= I; ++J) acc += a.part[(row0 + J) * 2 * SYM_TS + i];
  for (int I2 = I + 1; I2 < T; ++I2)
    acc += a.part[(base + (int64_t)I2 * (I2 + 1) / 2 + I) * 2 * SYM_TS + SYM_TS + i];
  y[soff[s] + r] = acc;
}

template <class T>
void launch_sym_pack(const SymArgs& a, const T* K, const int64_t* kofs, const int32_t* ld, const int32_t* ns, T* P,
                     hipStream_t st) {
  if (a.ntile == 0) return;
  hipLaunchKernelGGL((k_sym_pack<T>), dim3(a.ntile), dim3(256), 0, st, a, K, kofs, ld, ns, P);
}

void launch_sym_gemv(const DevMesh& m, const SymArgs& a, const double* x, double* y, hipStream_t st) {
  if (a.ntile == 0) return;
  const unsigned nb = (unsigned)((a.ntile + SYM_WAVES - 1) / SYM_WAVES);
  if (a.f32)
    hipLaunchKernelGGL((k_sym_tiles<float>), dim3(nb), dim3(SYM_WAVES * 64), 0, st, a, (const float*)a.P, m.soff,
                       m.ns, x);
  else
    hipLaunchKernelGGL((k_sym_tiles<double>), dim3(nb), dim3(SYM_WAVES * 64), 0, st, a, (const double*)a.P, m.soff,
                       m.ns, x);
  hipLaunchKernelGGL(k_sym_sum, dim3((unsigned)((m.max_ns + 255) / 256), m.nsub), dim3(256), 0, st, a, m.soff, m.ns,
                     y);
}

template void launch_sym_pack<double>(const SymArgs&, const double*, const int64_t*, const int32_t*, const int32_t*,
                                      double*, hipStream_t);
template void launch_sym_pack<float>(const SymArgs&, const float*, const int64_t*, const int32_t*, const int32_t*,
                                     float*, hipStream_t);

}  // namespace feti
