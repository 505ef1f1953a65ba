/* Learned warm start of the interface iteration: C ABI.
 *
 * The interface problem F lambda = d is solved at every backward-Euler step
 * (Section 2.5, Section 3); Algorithms 1 and 2 start each step from the previous
 * multipliers.  This library adds a small network that predicts the multipliers
 * of the next step from the last two steps and the next step's load:
 *
 *   x   = [lambda^n, lambda^{n-1}, load^{n+1}] / rho      (3 N_lambda features, FP32)
 *   lambda^{n+1} ~ 2 lambda^n - lambda^{n-1} + rho s * MLP(std(x))
 *
 * with rho the root mean square of lambda^n: the discrete problem is linear, so
 * dividing a sample by its own magnitude removes the load amplitude from what the
 * network has to learn.
 * with std(x) = (x - mean) * inv_std per feature, s a per-output scale, and MLP a
 * three-layer perceptron  n_in -> h -> h -> n_out  with GELU activations (the erf
 * form).  Weights are kept as FP32 master copies and BF16 copies; every product
 * takes BF16 operands and accumulates in FP32 on the matrix cores; biases are FP32.
 * Training minimises the mean squared error of the scaled target
 * (lambda^{n+1} - 2 lambda^n + lambda^{n-1}) / (rho s) with Adam.  The solver keeps the
 * prediction only when its projected residual beats the previous-step start
 * (FETI_START_BEST in feti.h).
 *
 * Parameter layout (flat FP32): W1 [h][n_in], b1 [h], W2 [h][h], b2 [h],
 * W3 [n_out][h], b3 [n_out].
 *
 * Pointers named *_dev are device memory (caller-owned); all work is ordered on
 * the stream given at creation; calls that return host values synchronise.
 * Errors: FETI_EINVAL (bad argument), FETI_ENOMEM, FETI_EHIP, with the message in
 * feti_ws_last_error; no call retains caller memory.
 */
#ifndef FETI_WS_H
#define FETI_WS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct feti_ws_s* feti_ws;

/* max_batch: the largest batch of train or forward calls. */
int feti_ws_create(feti_ws* out, void* hip_stream, int32_t n_in, int32_t n_hidden, int32_t n_out,
                   int32_t max_batch);
int feti_ws_destroy(feti_ws ws);
const char* feti_ws_last_error(feti_ws ws);

/* sizes: [0] parameters, [1] n_in, [2] n_hidden, [3] n_out, [4] max_batch */
int feti_ws_sizes(feti_ws ws, int64_t* sizes_host);

/* FP32 master parameters in and out (the BF16 copies follow; Adam state is reset). */
int feti_ws_set_params(feti_ws ws, const float* params_dev);
int feti_ws_get_params(feti_ws ws, float* params_dev);

/* Feature and target scaling: per-feature mean and inverse standard deviation
 * (n_in each) and per-output scale (n_out).  feti_ws_fit_scaling computes them
 * from raw samples X [nsamples][n_in] and targets T [nsamples][n_out] (a feature
 * without spread gets inv_std 0; the output scale is the root mean square of the
 * target column, 1 for an all-zero column). */
int feti_ws_set_scaling(feti_ws ws, const float* mean_dev, const float* inv_std_dev, const float* out_scale_dev);
int feti_ws_fit_scaling(feti_ws ws, const float* x_dev, const float* t_dev, int64_t nsamples);

/* y [batch][n_out] = MLP(std(x)) for raw features x [batch][n_in] (scaled units). */
int feti_ws_forward(feti_ws ws, const float* x_dev, int32_t batch, float* y_dev);

/* Loss (mean squared error against t / s, t raw [batch][n_out]) and its gradient
 * with respect to the FP32 parameters (flat, the parameter layout). */
int feti_ws_loss_grad(feti_ws ws, const float* x_dev, const float* t_dev, int32_t batch, double* loss_host,
                      float* grad_dev);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on a batch; loss_host may be NULL. */
int feti_ws_train_step(feti_ws ws, const float* x_dev, const float* t_dev, int32_t batch, float lr,
                       double* loss_host);

/* Raw feature row [lam_n, lam_nm1, load] / rho (3 n FP32) and target row
 * (lam_np1 - 2 lam_n + lam_nm1) / rho (n FP32) from FP64 multiplier vectors,
 * rho = rms(lam_n) (1 if lam_n = 0). */
int feti_ws_make_features(feti_ws ws, int64_t n, const double* lam_n_dev, const double* lam_nm1_dev,
                          const double* load_dev, float* x_row_dev);
int feti_ws_make_target(feti_ws ws, int64_t n, const double* lam_np1_dev, const double* lam_n_dev,
                        const double* lam_nm1_dev, float* t_row_dev);

/* Predicted multipliers lam_out = 2 lam_n - lam_nm1 + rho s * MLP(std(x)) (FP64, n_out). */
int feti_ws_predict(feti_ws ws, const double* lam_n_dev, const double* lam_nm1_dev, const double* load_dev,
                    double* lam_out_dev);

#ifdef __cplusplus
}
#endif

#endif /* FETI_WS_H */
