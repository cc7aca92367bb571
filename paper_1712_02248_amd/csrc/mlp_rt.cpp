// Host runtime of the learned warm start (declared in nmfrp.h): a
// k' -> hidden -> hidden -> r multilayer perceptron trained with Adam on pairs
// (compressed column, converged H row).  Every buffer lives in the caller's
// workspace; all kernels run on the stream given at creation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/nmfrp.h"
#include "common.h"

namespace {

constexpr int kMaxEpochs = 1024;

size_t take(size_t* off, size_t bytes) {
  const size_t o = *off;
  *off += (bytes + 255) / 256 * 256;
  return o;
}

struct MlpLayout {
  int64_t np;                 // parameter count
  size_t P, Gr, M1, M2;       // flat params, grads, Adam moments (np floats each)
  size_t Xs, Ts, nrm, A1, A2, Z3, D3, D2, D1;
  size_t lpart, loss, hist;
  size_t total;
};

int64_t param_count(int64_t k, int64_t h, int64_t r) { return k * h + h + h * h + h + h * r + r; }

MlpLayout mlp_layout(int k, int h, int r, int mb) {
  MlpLayout L;
  size_t off = 0;
  const size_t f = sizeof(float);
  L.np = param_count(k, h, r);
  L.P = take(&off, L.np * f);
  L.Gr = take(&off, L.np * f);
  L.M1 = take(&off, L.np * f);
  L.M2 = take(&off, L.np * f);
  L.Xs = take(&off, (size_t)mb * k * f);
  L.Ts = take(&off, (size_t)mb * r * f);
  L.nrm = take(&off, (size_t)mb * f);
  L.A1 = take(&off, (size_t)mb * h * f);
  L.A2 = take(&off, (size_t)mb * h * f);
  L.Z3 = take(&off, (size_t)mb * r * f);
  L.D3 = take(&off, (size_t)mb * r * f);
  L.D2 = take(&off, (size_t)mb * h * f);
  L.D1 = take(&off, (size_t)mb * h * f);
  L.lpart = take(&off, 256 * sizeof(double));
  L.loss = take(&off, sizeof(double));
  L.hist = take(&off, kMaxEpochs * sizeof(double));
  L.total = off;
  return L;
}

bool valid_dims(int k, int h, int r, int mb) {
  return k >= 1 && k <= 1024 && h >= 1 && h <= 4096 && r >= 1 && r <= 256 && mb >= 1 && mb <= 65536;
}

}  // namespace

struct nmf_mlp {
  int k, h, r, mb;
  MlpLayout L;
  char* ws;
  hipStream_t st;
  int64_t t = 0;  // Adam step count
  std::string err;
  template <class T> T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
  // parameter tensors inside the flat vector (order W1, b1, W2, b2, W3, b3)
  float* W1() { return at<float>(L.P); }
  float* b1() { return W1() + (int64_t)k * h; }
  float* W2() { return b1() + h; }
  float* b2() { return W2() + (int64_t)h * h; }
  float* W3() { return b2() + h; }
  float* b3() { return W3() + (int64_t)h * r; }
  float* g(float* p) { return at<float>(L.Gr) + (p - at<float>(L.P)); }
};

namespace {

nmf_status mfail(nmf_mlp* n, nmf_status s, const std::string& msg) {
  if (n) n->err = msg;
  nmf_set_thread_error(msg.c_str());
  return s;
}

#define MCHK(n, expr)                                                                \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return mfail((n), NMF_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// forward on Bn scaled rows already in Xs; leaves A1, A2, Z3
hipError_t forward(nmf_mlp* n, int Bn, hipStream_t st) {
  const MlpLayout& L = n->L;
  hipError_t e;
  if ((e = launch_mlp_gemm(0, 0, 1, n->at<float>(L.Xs), n->k, n->W1(), n->h, n->at<float>(L.A1), n->h, Bn,
                           n->h, n->k, n->b1(), nullptr, 0, st)))
    return e;
  if ((e = launch_mlp_gemm(0, 0, 1, n->at<float>(L.A1), n->h, n->W2(), n->h, n->at<float>(L.A2), n->h, Bn,
                           n->h, n->h, n->b2(), nullptr, 0, st)))
    return e;
  return launch_mlp_gemm(0, 0, 0, n->at<float>(L.A2), n->h, n->W3(), n->r, n->at<float>(L.Z3), n->r, Bn, n->r,
                         n->h, n->b3(), nullptr, 0, st);
}

// loss and gradients of one batch (rows idx of X/T, or the first Bn rows)
hipError_t loss_grad(nmf_mlp* n, const float* X, int64_t ldx, const float* T, int64_t ldt, const int* idx,
                     int64_t nsrc, int Bn, double* loss_acc) {
  const MlpLayout& L = n->L;
  hipStream_t st = n->st;
  hipError_t e;
  const int k = n->k, h = n->h, r = n->r;
  float *Xs = n->at<float>(L.Xs), *A1 = n->at<float>(L.A1), *A2 = n->at<float>(L.A2);
  float *D3 = n->at<float>(L.D3), *D2 = n->at<float>(L.D2), *D1 = n->at<float>(L.D1);
  if ((e = launch_scale_rows(X, ldx, idx, nsrc, Bn, k, T, ldt, r, Xs, n->at<float>(L.Ts), n->at<float>(L.nrm),
                             st)))
    return e;
  if ((e = forward(n, Bn, st))) return e;
  if ((e = launch_loss_grad(n->at<float>(L.Z3), n->at<float>(L.Ts), Bn, r, D3, n->at<double>(L.lpart),
                            n->at<double>(L.loss), loss_acc, st)))
    return e;
  // layer 3: gW3 = A2^T dZ3, gb3 = colsum dZ3, dZ2 = (dZ3 W3^T) * [A2 > 0]
  if ((e = launch_mlp_gemm(1, 0, 0, A2, h, D3, r, n->g(n->W3()), r, h, r, Bn, nullptr, nullptr, 0, st))) return e;
  if ((e = launch_colsum(D3, Bn, r, n->g(n->b3()), st))) return e;
  if ((e = launch_mlp_gemm(0, 1, 2, D3, r, n->W3(), r, D2, h, Bn, h, r, nullptr, A2, h, st))) return e;
  // layer 2
  if ((e = launch_mlp_gemm(1, 0, 0, A1, h, D2, h, n->g(n->W2()), h, h, h, Bn, nullptr, nullptr, 0, st))) return e;
  if ((e = launch_colsum(D2, Bn, h, n->g(n->b2()), st))) return e;
  if ((e = launch_mlp_gemm(0, 1, 2, D2, h, n->W2(), h, D1, h, Bn, h, h, nullptr, A1, h, st))) return e;
  // layer 1
  if ((e = launch_mlp_gemm(1, 0, 0, Xs, k, D1, h, n->g(n->W1()), h, k, h, Bn, nullptr, nullptr, 0, st))) return e;
  return launch_colsum(D1, Bn, h, n->g(n->b1()), st);
}

}  // namespace

// Inference on n rows: out = ||x|| softplus(net(x / ||x||)), in chunks of the
// workspace batch size.  Shared with nmf_init_learned.
hipError_t mlp_infer_rows(nmf_mlp* net, const float* in, int64_t ld_in, int64_t n, float* out, int64_t ldo,
                          hipStream_t st) {
  const MlpLayout& L = net->L;
  hipError_t e;
  for (int64_t b0 = 0; b0 < n; b0 += net->mb) {
    const int Bn = (int)((n - b0) < net->mb ? (n - b0) : net->mb);
    if ((e = launch_scale_rows(in + b0 * ld_in, ld_in, nullptr, Bn, Bn, net->k, nullptr, 0, net->r,
                               net->at<float>(L.Xs), nullptr, net->at<float>(L.nrm), st)))
      return e;
    if ((e = forward(net, Bn, st))) return e;
    if ((e = launch_infer_out(net->at<float>(L.Z3), net->at<float>(L.nrm), Bn, net->r, out + b0 * ldo, ldo, st)))
      return e;
  }
  return hipSuccess;
}

void mlp_dims(const nmf_mlp* net, int* k, int* h, int* r) {
  *k = net->k;
  *h = net->h;
  *r = net->r;
}

extern "C" {

int64_t nmf_mlp_n_params(int32_t k_in, int32_t hidden, int32_t r_out) {
  if (k_in < 1 || hidden < 1 || r_out < 1) return 0;
  return param_count(k_in, hidden, r_out);
}

size_t nmf_mlp_workspace_bytes(int32_t k_in, int32_t hidden, int32_t r_out, int32_t max_batch) {
  if (!valid_dims(k_in, hidden, r_out, max_batch)) return 0;
  return mlp_layout(k_in, hidden, r_out, max_batch).total;
}

nmf_status nmf_mlp_create(int32_t k_in, int32_t hidden, int32_t r_out, int32_t max_batch, const float* params,
                          void* workspace, size_t ws_bytes, void* hip_stream, nmf_mlp** out) {
  if (!out) return mfail(nullptr, NMF_EINVAL, "null output pointer");
  *out = nullptr;
  if (!valid_dims(k_in, hidden, r_out, max_batch))
    return mfail(nullptr, NMF_EINVAL, "need 1<=k_in<=1024, 1<=hidden<=4096, 1<=r_out<=256, 1<=max_batch<=65536");
  if (!params) return mfail(nullptr, NMF_EINVAL, "initial parameters required");
  const MlpLayout L = mlp_layout(k_in, hidden, r_out, max_batch);
  if (!workspace || ((uintptr_t)workspace & 255)) return mfail(nullptr, NMF_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return mfail(nullptr, NMF_ENOMEM, "workspace too small");
  nmf_mlp* n = new nmf_mlp();
  n->k = k_in;
  n->h = hidden;
  n->r = r_out;
  n->mb = max_batch;
  n->L = L;
  n->ws = (char*)workspace;
  n->st = (hipStream_t)hip_stream;
  nmf_status s = nmf_mlp_set_params(n, params);
  if (s != NMF_OK) {
    delete n;
    return s;
  }
  *out = n;
  return NMF_OK;
}

void nmf_mlp_destroy(nmf_mlp* n) { delete n; }

const char* nmf_mlp_last_error(const nmf_mlp* n) { return n ? n->err.c_str() : nmf_last_error(nullptr); }

nmf_status nmf_mlp_set_params(nmf_mlp* n, const float* flat) {
  if (!n || !flat) return mfail(n, NMF_EINVAL, "null argument");
  const MlpLayout& L = n->L;
  MCHK(n, hipMemcpyAsync(n->at<float>(L.P), flat, L.np * sizeof(float), hipMemcpyDeviceToDevice, n->st));
  MCHK(n, launch_fill_f32(n->at<float>(L.M1), L.np, 0.f, n->st));
  MCHK(n, launch_fill_f32(n->at<float>(L.M2), L.np, 0.f, n->st));
  n->t = 0;
  return NMF_OK;
}

nmf_status nmf_mlp_get_params(nmf_mlp* n, float* flat) {
  if (!n || !flat) return mfail(n, NMF_EINVAL, "null argument");
  MCHK(n, hipMemcpyAsync(flat, n->at<float>(n->L.P), n->L.np * sizeof(float), hipMemcpyDeviceToDevice, n->st));
  return NMF_OK;
}

nmf_status nmf_mlp_loss_grad(nmf_mlp* n, const float* in_rows, int64_t ld_in, const float* tgt_rows,
                             int64_t ld_tgt, int32_t batch, double* loss, float* grads_flat) {
  if (!n || !in_rows || !tgt_rows) return mfail(n, NMF_EINVAL, "null argument");
  if (batch < 1 || batch > n->mb) return mfail(n, NMF_EINVAL, "batch must be in [1, max_batch]");
  if (ld_in < n->k || ld_tgt < n->r) return mfail(n, NMF_EINVAL, "leading dimension too small");
  MCHK(n, loss_grad(n, in_rows, ld_in, tgt_rows, ld_tgt, nullptr, batch, batch, nullptr));
  if (grads_flat)
    MCHK(n, hipMemcpyAsync(grads_flat, n->at<float>(n->L.Gr), n->L.np * sizeof(float), hipMemcpyDeviceToDevice,
                           n->st));
  if (loss) {
    MCHK(n, hipMemcpyAsync(loss, n->at<double>(n->L.loss), sizeof(double), hipMemcpyDeviceToHost, n->st));
    MCHK(n, hipStreamSynchronize(n->st));
  }
  return NMF_OK;
}

nmf_status nmf_mlp_train(nmf_mlp* n, const float* in_rows, int64_t ld_in, const float* tgt_rows, int64_t ld_tgt,
                         int64_t npairs, const int32_t* order, int32_t epochs, int32_t batch, float lr,
                         double* epoch_loss) {
  if (!n || !in_rows || !tgt_rows) return mfail(n, NMF_EINVAL, "null argument");
  if (npairs < 1 || npairs > INT32_MAX) return mfail(n, NMF_EINVAL, "npairs must be in [1, 2^31)");
  if (epochs < 0 || epochs > kMaxEpochs) return mfail(n, NMF_EINVAL, "epochs must be in [0, 1024]");
  if (batch < 1 || batch > n->mb) return mfail(n, NMF_EINVAL, "batch must be in [1, max_batch]");
  if (ld_in < n->k || ld_tgt < n->r) return mfail(n, NMF_EINVAL, "leading dimension too small");
  if (!(lr > 0.f) || !std::isfinite(lr)) return mfail(n, NMF_EINVAL, "lr must be positive and finite");
  const MlpLayout& L = n->L;
  double* hist = n->at<double>(L.hist);
  if (epochs) MCHK(n, launch_fill_i32((int*)hist, 2 * (int64_t)epochs, 0, n->st));  // 0.0 doubles
  const int64_t nb = (npairs + batch - 1) / batch;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t b0 = b * batch;
      const int Bn = (int)((npairs - b0) < batch ? (npairs - b0) : batch);
      const float* X = in_rows;
      const float* T = tgt_rows;
      const int* idx = nullptr;
      if (order) idx = order + (int64_t)ep * npairs + b0;
      else {
        X += b0 * ld_in;
        T += b0 * ld_tgt;
      }
      MCHK(n, loss_grad(n, X, ld_in, T, ld_tgt, idx, order ? npairs : Bn, Bn, hist + ep));
      ++n->t;
      MCHK(n, launch_adam(n->at<float>(L.P), n->at<float>(L.Gr), n->at<float>(L.M1), n->at<float>(L.M2), L.np, lr,
                          (int)(n->t < INT32_MAX ? n->t : INT32_MAX), n->st));
    }
  }
  if (epoch_loss && epochs) {
    MCHK(n, hipMemcpyAsync(epoch_loss, hist, epochs * sizeof(double), hipMemcpyDeviceToHost, n->st));
    MCHK(n, hipStreamSynchronize(n->st));
    for (int ep = 0; ep < epochs; ++ep) epoch_loss[ep] /= (double)nb;
  }
  return NMF_OK;
}

nmf_status nmf_mlp_infer(nmf_mlp* n, const float* in_rows, int64_t ld_in, int64_t rows, float* out_rows,
                         int64_t ld_out) {
  if (!n) return mfail(n, NMF_EINVAL, "null network");
  if (rows < 0) return mfail(n, NMF_EINVAL, "rows must be >= 0");
  if (rows == 0) return NMF_OK;
  if (!in_rows || !out_rows) return mfail(n, NMF_EINVAL, "null argument");
  if (ld_in < n->k || ld_out < n->r) return mfail(n, NMF_EINVAL, "leading dimension too small");
  MCHK(n, mlp_infer_rows(n, in_rows, ld_in, rows, out_rows, ld_out, n->st));
  return NMF_OK;
}

nmf_status nmf_nnls_rows(const float* Xr, int64_t ldx, int64_t rows, int32_t k, const float* Wh, int32_t r,
                         int32_t sweeps, int32_t warm_start, float* Ht, int64_t ldh, void* hip_stream) {
  if (rows < 0 || k < 1 || r < 1 || sweeps < 0) return mfail(nullptr, NMF_EINVAL, "bad sizes");
  if (warm_start != 0 && warm_start != 1) return mfail(nullptr, NMF_EINVAL, "warm_start must be 0 or 1");
  if (r > 128) return mfail(nullptr, NMF_EINVAL, "r > 128 is not supported by this build");
  if (r > 64 && k > 256) return mfail(nullptr, NMF_EINVAL, "k > 256 is not supported with r > 64");
  if (k > 1024 || nnls_rows_lds_bytes(k, r) > 64 * 1024) return mfail(nullptr, NMF_EINVAL, "k too large for r");
  if (rows > INT32_MAX) return mfail(nullptr, NMF_EINVAL, "too many rows");
  if (rows == 0) return NMF_OK;
  if (!Xr || !Wh || !Ht) return mfail(nullptr, NMF_EINVAL, "null pointer");
  if (ldx < k || ldh < r) return mfail(nullptr, NMF_EINVAL, "leading dimension too small");
  hipError_t e = launch_nnls_rows(Xr, ldx, (int)rows, k, Wh, r, sweeps, warm_start, Ht, ldh, (hipStream_t)hip_stream);
  return e ? mfail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

}  // extern "C"
