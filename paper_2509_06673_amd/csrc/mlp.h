// Kernels of the learned warm-start network (kernels_mlp.hip): BF16 matrix products
// on the matrix cores with FP32 accumulation, their epilogues, the loss, Adam and the
// feature scaling.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace feti {

// C(m, n) = sum_k A(m, k) B(k, n) over split z's k range, A(m, k) = A[m sam + k sak],
// B(k, n) = B[k sbk + n sbn] (BF16 bit patterns); FP32 partials P[z][m][n].
struct GemmArgs {
  const uint16_t* A = nullptr;
  int64_t sam = 0, sak = 0;
  const uint16_t* B = nullptr;
  int64_t sbk = 0, sbn = 0;
  float* P = nullptr;
  int M = 0, N = 0, K = 0;
  int kchunk = 0;  // k range of a split (multiple of the k step)
  int nsplit = 1;
};
// choose the split of the k range for an M x N x K product (fills kchunk, nsplit)
void gemm_plan(GemmArgs& g, int target_blocks = 512);
size_t gemm_partial_floats(const GemmArgs& g);
void launch_gemm_bf16(const GemmArgs& g, hipStream_t st);

// epilogue of a product: sum the partials in split order, then
enum { EP_STORE = 0, EP_BIAS = 1, EP_BIAS_GELU = 2, EP_GELU_BACK = 3 };
//   EP_STORE:      out = s
//   EP_BIAS:       out = s + bias
//   EP_BIAS_GELU:  out = s + bias (pre-activation), out_bf = bf16(gelu(out))
//   EP_GELU_BACK:  out = s * gelu'(z), out_bf = bf16(out)
void launch_epilogue(const float* P, int nsplit, int M, int N, int mode, const float* bias, const float* z,
                     float* out, uint16_t* out_bf, hipStream_t st);

// out[b][i] = bf16((x[b][i] - mean[i]) inv_std[i])
void launch_standardize(const float* x, int64_t rows, int cols, const float* mean, const float* inv_std,
                        uint16_t* out, hipStream_t st);
// out[j] = sum_b x[b][j] (column sums, in row order)
void launch_colsum(const float* x, int rows, int cols, float* out, hipStream_t st);
// loss = sum((y - t inv_scale)^2) / (rows cols) into loss[0] (FP64); dy = 2 (y - t inv_scale) / (rows cols)
// and its BF16 copy; part: workspace of MLP_LOSS_BLOCKS doubles
constexpr int MLP_LOSS_BLOCKS = 256;
void launch_mse(const float* y, const float* t, const float* out_scale, int rows, int cols, float* dy,
                uint16_t* dy_bf, double* part, double* loss, hipStream_t st);
// Adam on n parameters at step t (bias-corrected), and the BF16 copy of the parameters
void launch_adam(int64_t n, float* p, const float* g, float* m, float* v, int step, float lr, float beta1,
                 float beta2, float eps, uint16_t* pbf, hipStream_t st);
void launch_to_bf16(int64_t n, const float* x, uint16_t* out, hipStream_t st);
// per-column mean and 1/std (0 for a column without spread) of a rows x cols matrix
void launch_column_stats(const float* x, int64_t rows, int cols, float* mean, float* inv_std, hipStream_t st);
// per-column root mean square (1 for an all-zero column)
void launch_column_rms(const float* x, int64_t rows, int cols, float* rms, hipStream_t st);
// x_row = [lam_n, lam_nm1, load] / rho (FP32); t_row = (lam_np1 - 2 lam_n + lam_nm1) / rho;
// rho = root mean square of lam_n (1 if it is zero)
void launch_ws_features(int64_t n, const double* lam_n, const double* lam_nm1, const double* load, float* x_row,
                        hipStream_t st);
void launch_ws_target(int64_t n, const double* lam_np1, const double* lam_n, const double* lam_nm1, float* t_row,
                      hipStream_t st);
// lam = 2 lam_n - lam_nm1 + rho y out_scale
void launch_ws_apply(int64_t n, const double* lam_n, const double* lam_nm1, const float* y, const float* out_scale,
                     double* lam, hipStream_t st);

}  // namespace feti
