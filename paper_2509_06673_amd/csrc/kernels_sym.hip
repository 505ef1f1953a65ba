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
//
// The recovery product K_s^+ [0; B_s^T v] (x zero on the interior DOFs) needs only the
// tiles whose tile row reaches the interface block: their row parts carry every
// interface column and their transposed parts every interface row.
#include "bstep.h"
#include "iface_device.h"
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

// entry k of x_s: the torn vector (KB = 0), or [0; gcoef B_s^T v] (KB = 1, v may be null);
// with a.pi_mode the primal DOFs take a.pi_v[primal index] (0 if null) instead
template <int KB>
__device__ inline double sym_x(const DevMesh& m, const SymArgs& a, int s, int n, int k, const double* xs,
                               const double* v, double gcoef) {
  if (k >= n) return 0.0;
  const int first_b = n - m.nb[s];
  if (a.pi_mode && k >= first_b) {
    const int q = m.bpi[m.boff[s] + (k - first_b)];
    if (q >= 0) return a.pi_v ? a.pi_v[q] : 0.0;
  }
  if (!KB) return xs[k];
  return (k >= first_b && v) ? gcoef * gather_b(m, v, m.boff[s] + (k - first_b), G_SIGNED) : 0.0;
}

// The row and transposed parts of stored tile t by this wavefront (valid = false: the
// wavefront only takes part in the block's barriers).
template <class T, int KB>
__device__ __forceinline__ void sym_tile_body(const DevMesh& m, const SymArgs& a, const T* __restrict__ P,
                                              const double* x, const double* v, double gcoef, int t, bool valid) {
  __shared__ double L[SYM_WAVES][SYM_Q * SYM_LD];
  __shared__ double xv[SYM_WAVES][2][SYM_TS];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = valid ? a.t_sub[t] : 0, I = valid ? a.t_I[t] : 0, J = valid ? a.t_J[t] : 0;
  const int n = valid ? m.ns[s] : 0;
  const double* xs = (valid && x) ? x + m.soff[s] : nullptr;
  double* xJ = xv[wave][0];
  double* xI = xv[wave][1];
  xJ[lane] = valid ? sym_x<KB>(m, a, s, n, J * SYM_TS + lane, xs, v, gcoef) : 0.0;
  xI[lane] = valid ? sym_x<KB>(m, a, s, n, I * SYM_TS + lane, xs, v, gcoef) : 0.0;
  const T* tile = P + (int64_t)(valid ? t : 0) * SYM_TE;
  double* Lw = L[wave];
  double u = 0.0;
  for (int h = 0; h < SYM_TS / SYM_Q; ++h) {
    __syncthreads();  // xv written, or the previous columns consumed
    if (valid) {
#pragma unroll
      for (int kk = 0; kk < SYM_Q; ++kk) {
        const int k = h * SYM_Q + kk;
        const double w = (double)tile[k * SYM_TS + lane];
        u += w * xJ[k];
        Lw[kk * SYM_LD + lane] = w;
      }
    }
    __syncthreads();
    if (valid && I != J && (lane & 16) == 0) {
      // (A^T x_I)_k for the SYM_Q columns k of this step: lanes l and l + 32 (l < 16) take
      // the two halves of the i range of column h * SYM_Q + l (the shuffle pairs only
      // lanes of this branch)
      const int kk = lane & (SYM_Q - 1), i0 = (lane >> 5) * 32;
      double w = 0.0;
#pragma unroll 8
      for (int i = 0; i < 32; ++i) w += Lw[kk * SYM_LD + i0 + i] * xI[i0 + i];
      w += __shfl_xor(w, 32, 64);
      if (lane < 32) a.part[(int64_t)t * 2 * SYM_TS + SYM_TS + h * SYM_Q + kk] = w;
    }
  }
  if (valid) a.part[(int64_t)t * 2 * SYM_TS + lane] = u;
}

template <class T>
__global__ void __launch_bounds__(256) k_sym_tiles(SymArgs a, const T* __restrict__ P, DevMesh m,
                                                   const double* __restrict__ x) {
  const int t = blockIdx.x * SYM_WAVES + (threadIdx.x >> 6);
  sym_tile_body<T, 0>(m, a, P, x, nullptr, 0.0, t, t < a.ntile);
}

template <class T>
__global__ void __launch_bounds__(256) k_sym_tiles_kb(SymArgs a, const T* __restrict__ P, DevMesh m,
                                                      const double* __restrict__ v, double gcoef) {
  const int k = blockIdx.x * SYM_WAVES + (threadIdx.x >> 6);
  const bool valid = k < a.n_kb_tiles;
  sym_tile_body<T, 1>(m, a, P, nullptr, v, gcoef, valid ? a.kb_tiles[k] : 0, valid);
}

// y_s[r] = sum over J <= I of row parts of tiles (I, J) + sum over I' > I of the
// transposed parts of tiles (I', I), I = r / 64 (tile order: fixed); KB: only the
// tiles of tile rows >= tb[s] were computed.  Then y += ybase and y += R alpha_c on
// floating subdomains (either may be null).
template <int KB>
__device__ __forceinline__ void sym_sum_body(const SymArgs& a, const DevMesh& m, int s, int r, double* y,
                                             const double* ybase, const double* alpha_c) {
  if (r >= m.ns[s]) return;
  const int I = r / SYM_TS, i = r % SYM_TS, T = a.nt[s];
  const int64_t base = a.tbase[s];
  const int tb = KB ? a.tb[s] : 0;
  double acc = 0.0;
  if (I >= tb) {
    const int64_t row0 = base + (int64_t)I * (I + 1) / 2;
    for (int J = 0; J <= I; ++J) acc += a.part[(row0 + J) * 2 * SYM_TS + i];
  }
  for (int I2 = max(I + 1, tb); I2 < T; ++I2)
    acc += a.part[(base + (int64_t)I2 * (I2 + 1) / 2 + I) * 2 * SYM_TS + SYM_TS + i];
  const int64_t so = m.soff[s];
  double yv = acc;
  if (ybase) yv += ybase[so + r];
  if (alpha_c) {
    const int f = m.sub_float[s];
    if (f >= 0) {
      const double* R = m.rfull + 3 * (so + r);
      yv += R[0] * alpha_c[3 * f] + R[1] * alpha_c[3 * f + 1] + R[2] * alpha_c[3 * f + 2];
    }
  }
  y[so + r] = yv;
}

template <int KB>
__global__ void __launch_bounds__(256) k_sym_sum(SymArgs a, DevMesh m, double* __restrict__ y,
                                                 const double* __restrict__ ybase,
                                                 const double* __restrict__ alpha_c) {
  sym_sum_body<KB>(a, m, blockIdx.y, blockIdx.x * blockDim.x + threadIdx.x, y, ybase, alpha_c);
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
    hipLaunchKernelGGL((k_sym_tiles<float>), dim3(nb), dim3(SYM_WAVES * 64), 0, st, a, (const float*)a.P, m, x);
  else
    hipLaunchKernelGGL((k_sym_tiles<double>), dim3(nb), dim3(SYM_WAVES * 64), 0, st, a, (const double*)a.P, m, x);
  hipLaunchKernelGGL((k_sym_sum<0>), dim3((unsigned)((m.max_ns + 255) / 256), m.nsub), dim3(256), 0, st, a, m, y,
                     (const double*)nullptr, (const double*)nullptr);
}

void launch_sym_gemv_kb(const DevMesh& m, const SymArgs& a, const double* v, double gcoef, const double* ybase,
                        const double* alpha_c, double* y, hipStream_t st) {
  if (a.n_kb_tiles > 0) {
    const unsigned nb = (unsigned)((a.n_kb_tiles + SYM_WAVES - 1) / SYM_WAVES);
    if (a.f32)
      hipLaunchKernelGGL((k_sym_tiles_kb<float>), dim3(nb), dim3(SYM_WAVES * 64), 0, st, a, (const float*)a.P, m, v,
                         gcoef);
    else
      hipLaunchKernelGGL((k_sym_tiles_kb<double>), dim3(nb), dim3(SYM_WAVES * 64), 0, st, a, (const double*)a.P, m,
                         v, gcoef);
  }
  hipLaunchKernelGGL((k_sym_sum<1>), dim3((unsigned)((m.max_ns + 255) / 256), m.nsub), dim3(256), 0, st, a, m, y,
                     ybase, alpha_c);
}

template void launch_sym_pack<double>(const SymArgs&, const double*, const int64_t*, const int32_t*, const int32_t*,
                                      double*, hipStream_t);
template void launch_sym_pack<float>(const SymArgs&, const float*, const int64_t*, const int32_t*, const int32_t*,
                                     float*, hipStream_t);

// ---- batched launches ---------------------------------------------------------
// Tile work items are (problem, stored tile) pairs, one per wavefront; sum items are
// (problem, subdomain, block of 256 rows).

template <class T, int KB>
__global__ void __launch_bounds__(256) kb_sym_tiles(const BProb* __restrict__ P, const int32_t* __restrict__ items,
                                                    int nitems, int x, int v, double gcoef) {
  const int k = blockIdx.x * SYM_WAVES + (threadIdx.x >> 6);
  const bool valid = k < nitems;
  const BProb& p = P[valid ? items[2 * k] : items[0]];
  sym_tile_body<T, KB>(p.m, p.sym, (const T*)p.sym.P, x >= 0 ? p.v[x] : nullptr, v >= 0 ? p.v[v] : nullptr, gcoef,
                       valid ? items[2 * k + 1] : 0, valid);
}

template <int KB>
__global__ void __launch_bounds__(256) kb_sym_sum(const BProb* __restrict__ P, const int32_t* __restrict__ items,
                                                  int y, int ybase, int alpha_c) {
  const int32_t* it = items + 3 * (int64_t)blockIdx.x;
  const BProb& p = P[it[0]];
  sym_sum_body<KB>(p.sym, p.m, it[1], it[2] * 256 + threadIdx.x, p.v[y], ybase >= 0 ? p.v[ybase] : nullptr,
                   (alpha_c >= 0 && p.nc > 0) ? p.v[alpha_c] : nullptr);
}

void launchb_sym_gemv(const BProb* P, const BDims& d, int kb, int x, int v, double gcoef, int ybase, int alpha_c,
                      int y, int f32, hipStream_t st) {
  const int n = kb ? d.n_sym_kb_items : d.n_sym_items;
  const int32_t* items = kb ? d.sym_kb_items : d.sym_items;
  if (n > 0) {
    const unsigned nb = (unsigned)((n + SYM_WAVES - 1) / SYM_WAVES);
    if (kb) {
      if (f32) hipLaunchKernelGGL((kb_sym_tiles<float, 1>), dim3(nb), dim3(256), 0, st, P, items, n, x, v, gcoef);
      else hipLaunchKernelGGL((kb_sym_tiles<double, 1>), dim3(nb), dim3(256), 0, st, P, items, n, x, v, gcoef);
    } else {
      if (f32) hipLaunchKernelGGL((kb_sym_tiles<float, 0>), dim3(nb), dim3(256), 0, st, P, items, n, x, v, gcoef);
      else hipLaunchKernelGGL((kb_sym_tiles<double, 0>), dim3(nb), dim3(256), 0, st, P, items, n, x, v, gcoef);
    }
  }
  if (d.n_sum_items == 0) return;
  if (kb)
    hipLaunchKernelGGL((kb_sym_sum<1>), dim3(d.n_sum_items), dim3(256), 0, st, P, d.sum_items, y, ybase, alpha_c);
  else
    hipLaunchKernelGGL((kb_sym_sum<0>), dim3(d.n_sum_items), dim3(256), 0, st, P, d.sum_items, y, ybase, alpha_c);
}

}  // namespace feti
