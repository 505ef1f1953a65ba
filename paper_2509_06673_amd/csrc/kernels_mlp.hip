// Kernels of the learned warm-start network: a three-layer perceptron with BF16
// weights and activations and FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x16_bf16), GELU activations, mean squared error and Adam with
// FP32 master weights.
//
// Products run as 64 x 64 output tiles, four wavefronts of 32 x 32 (2 x 2 MFMA
// blocks) per tile, k in steps of 16 staged through LDS; a long k range is split
// over blockIdx.z into FP32 partials that the epilogue sums in split order, so
// every result is deterministic.
#include <algorithm>
#include <cmath>

#include "mlp.h"

namespace feti {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;  // output tile
constexpr int GK = 16;  // k step (one MFMA depth)

// FP32 -> BF16, round to nearest, ties to even (NaN kept quiet)
__device__ inline uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// MFMA operands (checked by a lane probe): lane l holds A[l % 16][4 (l / 16) + v] and
// B[4 (l / 16) + v][l % 16], v = 0..3; result register r holds row 4 (l / 16) + r,
// column l % 16.
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT, z = blockIdx.z;
  const int kb = z * g.kchunk, ke = min(g.K, kb + g.kchunk);
  __shared__ uint16_t As[GT][GK + 4];  // As[m][k]
  __shared__ uint16_t Bs[GT][GK + 4];  // Bs[n][k]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const int lr = lane % 16, lk = 4 * (lane / 16);
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool a_kfast = g.sak == 1, b_kfast = g.sbk == 1;
  for (int k0 = kb; k0 < ke; k0 += GK) {
    for (int e = tid; e < GT * GK; e += 256) {
      const int mm = a_kfast ? e / GK : e % GT, kk = a_kfast ? e % GK : e / GT;
      const int m = m0 + mm, k = k0 + kk;
      As[mm][kk] = (m < g.M && k < ke) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : (uint16_t)0;
      const int nn = b_kfast ? e / GK : e % GT, k2i = b_kfast ? e % GK : e / GT;
      const int n = n0 + nn, k2 = k0 + k2i;
      Bs[nn][k2i] = (n < g.N && k2 < ke) ? g.B[(int64_t)k2 * g.sbk + (int64_t)n * g.sbn] : (uint16_t)0;
    }
    __syncthreads();
    bf16x4 av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        av[a][v] = (short)As[wi + a * 16 + lr][lk + v];
        bv[a][v] = (short)Bs[wj + a * 16 + lr][lk + v];
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
  float* P = g.P + (int64_t)z * g.M * g.N;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wi + a * 16 + 4 * (lane / 16) + r;
        const int n = n0 + wj + b * 16 + lr;
        if (m < g.M && n < g.N) P[(int64_t)m * g.N + n] = acc[a][b][r];
      }
}

void gemm_plan(GemmArgs& g, int target_blocks) {
  const int tiles = ((g.M + GT - 1) / GT) * ((g.N + GT - 1) / GT);
  const int ksteps = std::max(1, (g.K + GK - 1) / GK);
  int split = std::max(1, std::min(ksteps, target_blocks / std::max(tiles, 1)));
  const int steps_per = (ksteps + split - 1) / split;
  g.kchunk = steps_per * GK;
  g.nsplit = std::max(1, (g.K + g.kchunk - 1) / g.kchunk);
}

size_t gemm_partial_floats(const GemmArgs& g) { return (size_t)g.nsplit * g.M * g.N; }

void launch_gemm_bf16(const GemmArgs& g, hipStream_t st) {
  const dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT, g.nsplit);
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, g);
}

__global__ void k_epilogue(const float* __restrict__ P, int nsplit, int M, int N, int mode,
                           const float* __restrict__ bias, const float* __restrict__ zsrc, float* __restrict__ out,
                           uint16_t* __restrict__ out_bf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t MN = (int64_t)M * N;
  if (i >= MN) return;
  float s = 0.f;
  for (int zz = 0; zz < nsplit; ++zz) s += P[zz * MN + i];
  const int n = (int)(i % N);
  if (mode == EP_STORE) {
    out[i] = s;
  } else if (mode == EP_BIAS) {
    out[i] = s + bias[n];
  } else if (mode == EP_BIAS_GELU) {
    const float zv = s + bias[n];
    out[i] = zv;
    out_bf[i] = f2bf(gelu_f(zv));
  } else {
    const float d = s * gelu_grad_f(zsrc[i]);
    out[i] = d;
    out_bf[i] = f2bf(d);
  }
}

void launch_epilogue(const float* P, int nsplit, int M, int N, int mode, const float* bias, const float* z,
                     float* out, uint16_t* out_bf, hipStream_t st) {
  const int64_t n = (int64_t)M * N;
  hipLaunchKernelGGL(k_epilogue, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, nsplit, M, N, mode, bias,
                     z, out, out_bf);
}

__global__ void k_standardize(const float* __restrict__ x, int64_t rows, int cols, const float* __restrict__ mean,
                              const float* __restrict__ inv_std, uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int c = (int)(i % cols);
  out[i] = f2bf((x[i] - mean[c]) * inv_std[c]);
}

void launch_standardize(const float* x, int64_t rows, int cols, const float* mean, const float* inv_std,
                        uint16_t* out, hipStream_t st) {
  const int64_t n = rows * cols;
  hipLaunchKernelGGL(k_standardize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, rows, cols, mean,
                     inv_std, out);
}

__global__ void k_colsum(const float* __restrict__ x, int rows, int cols, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int r = 0; r < rows; ++r) s += x[(int64_t)r * cols + c];
  out[c] = (float)s;
}

void launch_colsum(const float* x, int rows, int cols, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3((cols + 255) / 256), dim3(256), 0, st, x, rows, cols, out);
}

__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             const float* __restrict__ out_scale, int rows, int cols,
                                             float* __restrict__ dy, uint16_t* __restrict__ dy_bf,
                                             double* __restrict__ part) {
  const int64_t n = (int64_t)rows * cols;
  const float c2 = 2.0f / (float)n;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % cols);
    const float d = y[i] - t[i] / out_scale[c];
    acc += (double)d * (double)d;
    const float g = c2 * d;
    dy[i] = g;
    dy_bf[i] = f2bf(g);
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_mse_final(const double* __restrict__ part, int nb, int64_t n, double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b];
  loss[0] = s / (double)n;
}

void launch_mse(const float* y, const float* t, const float* out_scale, int rows, int cols, float* dy,
                uint16_t* dy_bf, double* part, double* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_mse, dim3(MLP_LOSS_BLOCKS), dim3(256), 0, st, y, t, out_scale, rows, cols, dy, dy_bf, part);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, st, part, MLP_LOSS_BLOCKS, (int64_t)rows * cols, loss);
}

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float beta1, float beta2, float eps, float c1, float c2,
                       uint16_t* __restrict__ pbf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  pbf[i] = f2bf(pi);
}

void launch_adam(int64_t n, float* p, const float* g, float* m, float* v, int step, float lr, float beta1,
                 float beta2, float eps, uint16_t* pbf, hipStream_t st) {
  const float c1 = 1.0f - (float)std::pow((double)beta1, step);
  const float c2 = 1.0f - (float)std::pow((double)beta2, step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, g, m, v, lr, beta1, beta2,
                     eps, c1, c2, pbf);
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(x[i]);
}

void launch_to_bf16(int64_t n, const float* x, uint16_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, out);
}

__global__ void k_column_stats(const float* __restrict__ x, int64_t rows, int cols, float* __restrict__ mean,
                               float* __restrict__ inv_std) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0, s2 = 0.0;
  for (int64_t r = 0; r < rows; ++r) {
    const double v = x[r * cols + c];
    s += v;
    s2 += v * v;
  }
  const double mu = s / (double)rows;
  const double var = fmax(s2 / (double)rows - mu * mu, 0.0);
  const double sd = sqrt(var), rms = sqrt(s2 / (double)rows);
  mean[c] = (float)mu;
  inv_std[c] = (sd > 1e-6 * rms && sd > 0.0) ? (float)(1.0 / sd) : 0.0f;
}

void launch_column_stats(const float* x, int64_t rows, int cols, float* mean, float* inv_std, hipStream_t st) {
  hipLaunchKernelGGL(k_column_stats, dim3((cols + 255) / 256), dim3(256), 0, st, x, rows, cols, mean, inv_std);
}

__global__ void k_column_rms(const float* __restrict__ x, int64_t rows, int cols, float* __restrict__ rms) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s2 = 0.0;
  for (int64_t r = 0; r < rows; ++r) {
    const double v = x[r * cols + c];
    s2 += v * v;
  }
  const double q = sqrt(s2 / (double)rows);
  rms[c] = q > 0.0 ? (float)q : 1.0f;
}

void launch_column_rms(const float* x, int64_t rows, int cols, float* rms, hipStream_t st) {
  hipLaunchKernelGGL(k_column_rms, dim3((cols + 255) / 256), dim3(256), 0, st, x, rows, cols, rms);
}

// rho = root mean square of v (1 for a zero vector), one block, fixed summation order
__device__ double block_rms(int64_t n, const double* __restrict__ v) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += v[i] * v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sqrt(red[0] / (double)n);
  __syncthreads();
  return r > 0.0 ? r : 1.0;
}

// One block: x = [lam_n, lam_nm1, load] / rho, rho = rms(lam_n)
__global__ void __launch_bounds__(256) k_ws_features(int64_t n, const double* __restrict__ lam_n,
                                                     const double* __restrict__ lam_nm1,
                                                     const double* __restrict__ load, float* __restrict__ x) {
  const double inv = 1.0 / block_rms(n, lam_n);
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    x[i] = (float)(lam_n[i] * inv);
    x[n + i] = (float)(lam_nm1[i] * inv);
    x[2 * n + i] = (float)(load[i] * inv);
  }
}

void launch_ws_features(int64_t n, const double* lam_n, const double* lam_nm1, const double* load, float* x_row,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_ws_features, dim3(1), dim3(256), 0, st, n, lam_n, lam_nm1, load, x_row);
}

// One block: t = (lam_np1 - 2 lam_n + lam_nm1) / rho, rho = rms(lam_n)
__global__ void __launch_bounds__(256) k_ws_target(int64_t n, const double* __restrict__ lam_np1,
                                                   const double* __restrict__ lam_n,
                                                   const double* __restrict__ lam_nm1, float* __restrict__ t) {
  const double inv = 1.0 / block_rms(n, lam_n);
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
    t[i] = (float)((lam_np1[i] - 2.0 * lam_n[i] + lam_nm1[i]) * inv);
}

void launch_ws_target(int64_t n, const double* lam_np1, const double* lam_n, const double* lam_nm1, float* t_row,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_ws_target, dim3(1), dim3(256), 0, st, n, lam_np1, lam_n, lam_nm1, t_row);
}

// One block: lam = 2 lam_n - lam_nm1 + rho y out_scale, rho = rms(lam_n)
__global__ void __launch_bounds__(256) k_ws_apply(int64_t n, const double* __restrict__ lam_n,
                                                  const double* __restrict__ lam_nm1, const float* __restrict__ y,
                                                  const float* __restrict__ out_scale, double* __restrict__ lam) {
  const double rho = block_rms(n, lam_n);
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
    lam[i] = 2.0 * lam_n[i] - lam_nm1[i] + rho * (double)y[i] * (double)out_scale[i];
}

void launch_ws_apply(int64_t n, const double* lam_n, const double* lam_nm1, const float* y, const float* out_scale,
                     double* lam, hipStream_t st) {
  hipLaunchKernelGGL(k_ws_apply, dim3(1), dim3(256), 0, st, n, lam_n, lam_nm1, y, out_scale, lam);
}

}  // namespace feti
