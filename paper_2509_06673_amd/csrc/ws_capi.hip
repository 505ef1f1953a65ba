// C ABI of the learned warm start (include/feti_ws.h): the network's buffers and the
// order of its products, forward and backward.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/feti.h"
#include "../../include/feti_ws.h"
#include "mlp.h"

using namespace feti;

struct feti_ws_s {
  hipStream_t stream = nullptr;
  std::string err;
  int n_in = 0, h = 0, n_out = 0, max_batch = 0;
  int64_t np = 0;
  int64_t off[6] = {0, 0, 0, 0, 0, 0};  // W1, b1, W2, b2, W3, b3
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* pbf = nullptr;
  float *mean = nullptr, *inv_std = nullptr, *out_scale = nullptr;
  uint16_t *A0 = nullptr, *A1 = nullptr, *A2 = nullptr, *G1 = nullptr, *G2 = nullptr, *G3 = nullptr;
  float *Z1 = nullptr, *Z2 = nullptr, *Y = nullptr, *dY = nullptr, *dZ1 = nullptr, *dZ2 = nullptr;
  float* P = nullptr;
  size_t pcap = 0;
  double *lpart = nullptr, *loss = nullptr;
  float* x1 = nullptr;
  int step = 0;
  std::vector<void*> allocs;
};

namespace {

int wfail(feti_ws w, int code, const std::string& msg) {
  if (w) w->err = msg;
  return code;
}

#define WCHK(expr)                                                                         \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess) return wfail(w, FETI_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)
#define WRC(expr)            \
  do {                       \
    int _rc = (expr);        \
    if (_rc != FETI_OK) return _rc; \
  } while (0)

template <class T>
int walloc(feti_ws w, T** p, size_t count) {
  *p = nullptr;
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return wfail(w, FETI_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  w->allocs.push_back(*p);
  return FETI_OK;
}

// the products of one training step for a batch (forward 0..2, backward 3..7)
std::vector<GemmArgs> products(const feti_ws_s* w, int b) {
  const uint16_t* W1 = w->pbf + w->off[0];
  const uint16_t* W2 = w->pbf + w->off[2];
  const uint16_t* W3 = w->pbf + w->off[4];
  const int ni = w->n_in, h = w->h, no = w->n_out;
  std::vector<GemmArgs> v(8);
  auto set = [](GemmArgs& g, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                int64_t sbn, int M, int N, int K) {
    g.A = A; g.sam = sam; g.sak = sak; g.B = B; g.sbk = sbk; g.sbn = sbn; g.M = M; g.N = N; g.K = K;
  };
  set(v[0], w->A0, ni, 1, W1, 1, ni, b, h, ni);   // Z1 = A0 W1^T
  set(v[1], w->A1, h, 1, W2, 1, h, b, h, h);      // Z2 = A1 W2^T
  set(v[2], w->A2, h, 1, W3, 1, h, b, no, h);     // Y = A2 W3^T
  set(v[3], w->G3, 1, no, w->A2, h, 1, no, h, b); // dW3 = G3^T A2
  set(v[4], w->G3, no, 1, W3, h, 1, b, h, no);    // dA2 = G3 W3
  set(v[5], w->G2, 1, h, w->A1, h, 1, h, h, b);   // dW2 = G2^T A1
  set(v[6], w->G2, h, 1, W2, h, 1, b, h, h);      // dA1 = G2 W2
  set(v[7], w->G1, 1, h, w->A0, ni, 1, h, ni, b); // dW1 = G1^T A0
  return v;
}

// split plan whose partials fit the workspace
void plan(GemmArgs& g, size_t cap) {
  int target = 512;
  for (;;) {
    gemm_plan(g, target);
    if (gemm_partial_floats(g) <= cap || target <= 1) return;
    target /= 2;
  }
}

int run_gemm(feti_ws w, GemmArgs g, float* out, int mode, const float* bias, const float* z, uint16_t* out_bf) {
  plan(g, w->pcap);
  if (gemm_partial_floats(g) > w->pcap) return wfail(w, FETI_EINVAL, "product exceeds the workspace");
  g.P = w->P;
  launch_gemm_bf16(g, w->stream);
  launch_epilogue(w->P, g.nsplit, g.M, g.N, mode, bias, z, out, out_bf, w->stream);
  return FETI_OK;
}

int forward_impl(feti_ws w, const float* x, int b) {
  auto pr = products(w, b);
  launch_standardize(x, b, w->n_in, w->mean, w->inv_std, w->A0, w->stream);
  WRC(run_gemm(w, pr[0], w->Z1, EP_BIAS_GELU, w->p + w->off[1], nullptr, w->A1));
  WRC(run_gemm(w, pr[1], w->Z2, EP_BIAS_GELU, w->p + w->off[3], nullptr, w->A2));
  WRC(run_gemm(w, pr[2], w->Y, EP_BIAS, w->p + w->off[5], nullptr, nullptr));
  return FETI_OK;
}

int backward_impl(feti_ws w, const float* t, int b) {
  auto pr = products(w, b);
  launch_mse(w->Y, t, w->out_scale, b, w->n_out, w->dY, w->G3, w->lpart, w->loss, w->stream);
  WRC(run_gemm(w, pr[3], w->g + w->off[4], EP_STORE, nullptr, nullptr, nullptr));
  launch_colsum(w->dY, b, w->n_out, w->g + w->off[5], w->stream);
  WRC(run_gemm(w, pr[4], w->dZ2, EP_GELU_BACK, nullptr, w->Z2, w->G2));
  launch_colsum(w->dZ2, b, w->h, w->g + w->off[3], w->stream);
  WRC(run_gemm(w, pr[5], w->g + w->off[2], EP_STORE, nullptr, nullptr, nullptr));
  WRC(run_gemm(w, pr[6], w->dZ1, EP_GELU_BACK, nullptr, w->Z1, w->G1));
  launch_colsum(w->dZ1, b, w->h, w->g + w->off[1], w->stream);
  WRC(run_gemm(w, pr[7], w->g + w->off[0], EP_STORE, nullptr, nullptr, nullptr));
  return FETI_OK;
}

int check_batch(feti_ws w, int b) {
  if (b < 1 || b > w->max_batch) return wfail(w, FETI_EINVAL, "batch outside 1..max_batch");
  return FETI_OK;
}

}  // namespace

extern "C" {

int feti_ws_create(feti_ws* out, void* hip_stream, int32_t n_in, int32_t n_hidden, int32_t n_out,
                   int32_t max_batch) {
  if (!out) return FETI_EINVAL;
  *out = nullptr;
  if (n_in < 1 || n_hidden < 1 || n_out < 1 || max_batch < 1) return FETI_EINVAL;
  feti_ws w = new feti_ws_s();
  w->stream = (hipStream_t)hip_stream;
  w->n_in = n_in; w->h = n_hidden; w->n_out = n_out; w->max_batch = max_batch;
  const int64_t sz[6] = {(int64_t)n_hidden * n_in, n_hidden, (int64_t)n_hidden * n_hidden, n_hidden,
                         (int64_t)n_out * n_hidden, n_out};
  int64_t o = 0;
  for (int i = 0; i < 6; ++i) { w->off[i] = o; o += sz[i]; }
  w->np = o;
  auto fail_all = [&](int rc) {
    for (void* p : w->allocs) (void)hipFree(p);
    delete w;
    return rc;
  };
  int rc = FETI_OK;
  const int64_t B = max_batch;
  if ((rc = walloc(w, &w->p, w->np)) || (rc = walloc(w, &w->g, w->np)) || (rc = walloc(w, &w->m, w->np)) ||
      (rc = walloc(w, &w->v, w->np)) || (rc = walloc(w, &w->pbf, w->np)) || (rc = walloc(w, &w->mean, n_in)) ||
      (rc = walloc(w, &w->inv_std, n_in)) || (rc = walloc(w, &w->out_scale, n_out)) ||
      (rc = walloc(w, &w->A0, B * n_in)) || (rc = walloc(w, &w->A1, B * n_hidden)) ||
      (rc = walloc(w, &w->A2, B * n_hidden)) || (rc = walloc(w, &w->G1, B * n_hidden)) ||
      (rc = walloc(w, &w->G2, B * n_hidden)) || (rc = walloc(w, &w->G3, B * n_out)) ||
      (rc = walloc(w, &w->Z1, B * n_hidden)) || (rc = walloc(w, &w->Z2, B * n_hidden)) ||
      (rc = walloc(w, &w->Y, B * n_out)) || (rc = walloc(w, &w->dY, B * n_out)) ||
      (rc = walloc(w, &w->dZ1, B * n_hidden)) || (rc = walloc(w, &w->dZ2, B * n_hidden)) ||
      (rc = walloc(w, &w->lpart, MLP_LOSS_BLOCKS)) || (rc = walloc(w, &w->loss, 1)) ||
      (rc = walloc(w, &w->x1, n_in)))
    return fail_all(rc);
  // workspace for the partial sums: the largest product at the smallest and largest batch
  size_t cap = 0;
  for (int b : {1, max_batch})
    for (GemmArgs g : products(w, b)) {
      gemm_plan(g);
      cap = std::max(cap, gemm_partial_floats(g));
    }
  w->pcap = cap;
  if ((rc = walloc(w, &w->P, cap))) return fail_all(rc);
  // identity scaling until set or fitted
  std::vector<float> zeros(std::max(n_in, n_out), 0.0f), ones(std::max(n_in, n_out), 1.0f);
  if (hipMemcpy(w->mean, zeros.data(), n_in * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(w->inv_std, ones.data(), n_in * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(w->out_scale, ones.data(), n_out * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(w->p, 0, w->np * sizeof(float)) != hipSuccess || hipMemset(w->pbf, 0, w->np * 2) != hipSuccess ||
      hipMemset(w->m, 0, w->np * sizeof(float)) != hipSuccess || hipMemset(w->v, 0, w->np * sizeof(float)) != hipSuccess)
    return fail_all(FETI_EHIP);
  *out = w;
  return FETI_OK;
}

int feti_ws_destroy(feti_ws w) {
  if (!w) return FETI_EINVAL;
  if (w->stream) (void)hipStreamSynchronize(w->stream);
  else (void)hipDeviceSynchronize();
  for (void* p : w->allocs) (void)hipFree(p);
  delete w;
  return FETI_OK;
}

const char* feti_ws_last_error(feti_ws w) { return w ? w->err.c_str() : "null warm-start handle"; }

int feti_ws_sizes(feti_ws w, int64_t* s) {
  if (!w || !s) return FETI_EINVAL;
  s[0] = w->np; s[1] = w->n_in; s[2] = w->h; s[3] = w->n_out; s[4] = w->max_batch;
  return FETI_OK;
}

int feti_ws_set_params(feti_ws w, const float* params) {
  if (!w || !params) return FETI_EINVAL;
  WCHK(hipMemcpyAsync(w->p, params, w->np * sizeof(float), hipMemcpyDeviceToDevice, w->stream));
  WCHK(hipMemsetAsync(w->m, 0, w->np * sizeof(float), w->stream));
  WCHK(hipMemsetAsync(w->v, 0, w->np * sizeof(float), w->stream));
  launch_to_bf16(w->np, w->p, w->pbf, w->stream);
  w->step = 0;
  WCHK(hipGetLastError());
  WCHK(hipStreamSynchronize(w->stream));
  return FETI_OK;
}

int feti_ws_get_params(feti_ws w, float* params) {
  if (!w || !params) return FETI_EINVAL;
  WCHK(hipMemcpyAsync(params, w->p, w->np * sizeof(float), hipMemcpyDeviceToDevice, w->stream));
  WCHK(hipStreamSynchronize(w->stream));
  return FETI_OK;
}

int feti_ws_set_scaling(feti_ws w, const float* mean, const float* inv_std, const float* out_scale) {
  if (!w || !mean || !inv_std || !out_scale) return FETI_EINVAL;
  WCHK(hipMemcpyAsync(w->mean, mean, w->n_in * sizeof(float), hipMemcpyDeviceToDevice, w->stream));
  WCHK(hipMemcpyAsync(w->inv_std, inv_std, w->n_in * sizeof(float), hipMemcpyDeviceToDevice, w->stream));
  WCHK(hipMemcpyAsync(w->out_scale, out_scale, w->n_out * sizeof(float), hipMemcpyDeviceToDevice, w->stream));
  WCHK(hipStreamSynchronize(w->stream));
  return FETI_OK;
}

int feti_ws_fit_scaling(feti_ws w, const float* x, const float* t, int64_t ns) {
  if (!w || !x || !t || ns < 1) return FETI_EINVAL;
  launch_column_stats(x, ns, w->n_in, w->mean, w->inv_std, w->stream);
  launch_column_rms(t, ns, w->n_out, w->out_scale, w->stream);
  WCHK(hipGetLastError());
  WCHK(hipStreamSynchronize(w->stream));
  return FETI_OK;
}

int feti_ws_forward(feti_ws w, const float* x, int32_t batch, float* y) {
  if (!w || !x || !y) return FETI_EINVAL;
  WRC(check_batch(w, batch));
  WRC(forward_impl(w, x, batch));
  WCHK(hipMemcpyAsync(y, w->Y, (size_t)batch * w->n_out * sizeof(float), hipMemcpyDeviceToDevice, w->stream));
  WCHK(hipGetLastError());
  WCHK(hipStreamSynchronize(w->stream));
  return FETI_OK;
}

int feti_ws_loss_grad(feti_ws w, const float* x, const float* t, int32_t batch, double* loss, float* grad) {
  if (!w || !x || !t || !grad) return FETI_EINVAL;
  WRC(check_batch(w, batch));
  WRC(forward_impl(w, x, batch));
  WRC(backward_impl(w, t, batch));
  WCHK(hipMemcpyAsync(grad, w->g, w->np * sizeof(float), hipMemcpyDeviceToDevice, w->stream));
  if (loss) WCHK(hipMemcpyAsync(loss, w->loss, sizeof(double), hipMemcpyDeviceToHost, w->stream));
  WCHK(hipGetLastError());
  WCHK(hipStreamSynchronize(w->stream));
  return FETI_OK;
}

int feti_ws_train_step(feti_ws w, const float* x, const float* t, int32_t batch, float lr, double* loss) {
  if (!w || !x || !t || !(lr > 0.0f)) return FETI_EINVAL;
  WRC(check_batch(w, batch));
  WRC(forward_impl(w, x, batch));
  WRC(backward_impl(w, t, batch));
  w->step += 1;
  launch_adam(w->np, w->p, w->g, w->m, w->v, w->step, lr, 0.9f, 0.999f, 1e-8f, w->pbf, w->stream);
  if (loss) {
    WCHK(hipMemcpyAsync(loss, w->loss, sizeof(double), hipMemcpyDeviceToHost, w->stream));
    WCHK(hipStreamSynchronize(w->stream));
  }
  WCHK(hipGetLastError());
  return FETI_OK;
}

int feti_ws_make_features(feti_ws w, int64_t n, const double* lam_n, const double* lam_nm1, const double* load,
                          float* x_row) {
  if (!w || !lam_n || !lam_nm1 || !load || !x_row || n < 1) return FETI_EINVAL;
  launch_ws_features(n, lam_n, lam_nm1, load, x_row, w->stream);
  WCHK(hipGetLastError());
  return FETI_OK;
}

int feti_ws_make_target(feti_ws w, int64_t n, const double* lam_np1, const double* lam_n, const double* lam_nm1,
                        float* t_row) {
  if (!w || !lam_np1 || !lam_n || !lam_nm1 || !t_row || n < 1) return FETI_EINVAL;
  launch_ws_target(n, lam_np1, lam_n, lam_nm1, t_row, w->stream);
  WCHK(hipGetLastError());
  return FETI_OK;
}

int feti_ws_predict(feti_ws w, const double* lam_n, const double* lam_nm1, const double* load, double* lam_out) {
  if (!w || !lam_n || !lam_nm1 || !load || !lam_out) return FETI_EINVAL;
  if (w->n_in != 3 * w->n_out) return wfail(w, FETI_EINVAL, "predict needs n_in = 3 n_out");
  launch_ws_features(w->n_out, lam_n, lam_nm1, load, w->x1, w->stream);
  WRC(forward_impl(w, w->x1, 1));
  launch_ws_apply(w->n_out, lam_n, lam_nm1, w->Y, w->out_scale, lam_out, w->stream);
  WCHK(hipGetLastError());
  return FETI_OK;
}

}  // extern "C"
