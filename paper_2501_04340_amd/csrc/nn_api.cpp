// C ABI of the warm-start network: parameters, training data, Adam training
// and inference, all on the GPU in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <string>
#include <vector>

#include "common.hpp"
#include "device/nn.hpp"
#include "ietidp.h"
#include "nn_model.hpp"

using ieti::rt::DBuf;
using ieti::rt::dalloc;
using ieti::rt::dupload;
using ieti::rt::fail;

namespace ieti {
namespace nn {

int Mlp::init(const ieti_nn_arch* a) {
  if (!a) return fail(IETI_ERR_INVALID_ARG, "architecture is NULL");
  if (a->n_in < 1 || a->n_hidden < 1 || a->n_layers < 1 || a->n_comb < 1 || a->n_out < 1)
    return fail(IETI_ERR_INVALID_ARG, "network sizes must be >= 1");
  if (int64_t(a->n_comb) * a->n_out > (int64_t(1) << 24) || a->n_hidden > (1 << 16) || a->n_in > (1 << 20))
    return fail(IETI_ERR_INVALID_ARG, "network too large");
  arch = *a;
  dims.assign(1, a->n_in);
  for (int l = 0; l < a->n_layers; ++l) dims.push_back(a->n_hidden);
  dims.push_back(int64_t(a->n_comb) * a->n_out);
  woff.clear();
  n_params = 0;
  for (int l = 1; l < int(dims.size()); ++l) {
    woff.push_back(n_params);
    n_params += dims[l] * (dims[l - 1] + 1);
  }
  return IETI_OK;
}

void Work::release() {
  for (auto& b : H) b.release();
  H.clear();
  for (auto* b : {&Y, &dY, &dZ0, &dZ1, &pred}) b->release();
  part.release();
  cap = 0;
}

int Work::reserve(const Mlp& m, int64_t n, hipStream_t s) {
  if (n <= cap) return IETI_OK;
  release();
  int rc = 0;
  const int L = m.layers();
  H.resize(L);
  int64_t dmax = 0;
  for (int l = 0; l < L; ++l) {
    if ((rc = dalloc(H[l], n * (m.dims[l] + 1)))) return rc;
    fill_column(H[l].ptr, n, m.dims[l] + 1, m.dims[l], 1.f, s);
    dmax = std::max(dmax, m.dims[l]);
  }
  const int64_t dout = m.dims[L];
  dmax = std::max(dmax, dout);
  if ((rc = dalloc(Y, n * dout))) return rc;
  if ((rc = dalloc(dY, n * dout))) return rc;
  if ((rc = dalloc(dZ0, n * dmax))) return rc;
  if ((rc = dalloc(dZ1, n * dmax))) return rc;
  if ((rc = dalloc(pred, n * m.arch.n_out))) return rc;
  if ((rc = dalloc(part, std::max(1, loss_blocks(n, m.arch.n_out))))) return rc;
  cap = n;
  return IETI_OK;
}

void forward(const Mlp& m, const float* theta, int64_t n, Work& w, hipStream_t s) {
  const int L = m.layers();
  for (int l = 1; l <= L; ++l) {
    const int64_t din = m.dims[l - 1] + 1, dout = m.dims[l];
    const float* W = theta + m.woff[l - 1];
    // z = h' W'^T: A(i,k) = H[i*din + k], B(k,j) = W'[j*din + k]
    float* out = (l < L) ? w.H[l].ptr : w.Y.ptr;
    const int64_t ldc = (l < L) ? dout + 1 : dout;
    gemm(n, dout, din, w.H[l - 1].ptr, din, 1, W, 1, din, out, ldc, l < L ? EPI_TANH : EPI_NONE, nullptr, 0, s);
  }
}

void backward(const Mlp& m, const float* theta, int64_t n, Work& w, float* grad, hipStream_t s) {
  const int L = m.layers();
  const float* dZ = w.dY.ptr;
  int64_t ldz = m.dims[L];
  float* bufs[2] = {w.dZ0.ptr, w.dZ1.ptr};
  int nb = 0;
  for (int l = L; l >= 1; --l) {
    const int64_t din = m.dims[l - 1] + 1, dout = m.dims[l];
    // dW'_l = dZ^T H_{l-1}: A(i,k) = dZ[k*ldz + i], B(k,j) = H[k*din + j]
    gemm(dout, din, n, dZ, 1, ldz, w.H[l - 1].ptr, din, 1, grad + m.woff[l - 1], din, EPI_NONE, nullptr, 0, s);
    if (l > 1) {
      // dZ_{l-1} = (dZ W_l)[:, :d_{l-1}] * (1 - H_{l-1}^2): B(k,j) = W'[k*din + j]
      const int64_t dprev = m.dims[l - 1];
      float* out = bufs[nb];
      gemm(n, dprev, dout, dZ, ldz, 1, theta + m.woff[l - 1], din, 1, out, dprev, EPI_DTANH, w.H[l - 1].ptr, din, s);
      dZ = out;
      ldz = dprev;
      nb ^= 1;
    }
  }
}

}  // namespace nn
}  // namespace ieti

struct ieti_nn {
  ieti::nn::Mlp mlp;
  hipStream_t stream = nullptr;
  DBuf<float> theta, grad, m, v;
  int64_t adam_t = 0;
  DBuf<float> X, C, T;  // training data; X with the trailing ones column
  int64_t n_data = 0;
  DBuf<float> Cb, Tb;
  DBuf<int32_t> idx;
  DBuf<double> loss;
  ieti::nn::Work work;
  // input normalisation x' = (x - shift) * scale and output scale: the
  // network computes on normalised rows, predictions are out_scale * output
  std::vector<float> shift, scale;
  double out_scale = 1.0;
  ~ieti_nn() {
    for (auto* b : {&theta, &grad, &m, &v, &X, &C, &T, &Cb, &Tb}) b->release();
    idx.release();
    loss.release();
    work.release();
    if (stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

namespace N = ieti::nn;

// rows [n][n_in] -> normalised rows [n][n_in + 1] with the trailing 1 of the bias column
std::vector<float> normalised_inputs(const ieti_nn* nn, const float* X, int64_t n) {
  const int64_t d = nn->mlp.arch.n_in;
  std::vector<float> xo(size_t(n) * (d + 1));
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < d; ++j) xo[i * (d + 1) + j] = (X[i * d + j] - nn->shift[j]) * nn->scale[j];
    xo[i * (d + 1) + d] = 1.f;
  }
  return xo;
}

// SplitMix64 (Steele, Lea & Flood 2014): the shuffling generator.
uint64_t splitmix64(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int check_rows(ieti_nn* nn, int64_t n) {
  int rc = nn->work.reserve(nn->mlp, n, nn->stream);
  if (rc) return rc;
  if (nn->Cb.n < n * nn->mlp.arch.n_comb) {
    if ((rc = dalloc(nn->Cb, n * nn->mlp.arch.n_comb))) return rc;
    if ((rc = dalloc(nn->Tb, n * nn->mlp.arch.n_out))) return rc;
  }
  return IETI_OK;
}

// forward + loss (+ backward) on the data rows idx[0..n) already on the device
int step_rows(ieti_nn* nn, const int32_t* d_idx, int64_t n, bool grad, double* d_loss, int accumulate) {
  const auto& a = nn->mlp.arch;
  hipStream_t s = nn->stream;
  auto& w = nn->work;
  N::gather_rows(nn->X.ptr, a.n_in + 1, d_idx, n, a.n_in + 1, w.H[0].ptr, a.n_in + 1, s);
  N::gather_rows(nn->C.ptr, a.n_comb, d_idx, n, a.n_comb, nn->Cb.ptr, a.n_comb, s);
  N::gather_rows(nn->T.ptr, a.n_out, d_idx, n, a.n_out, nn->Tb.ptr, a.n_out, s);
  N::forward(nn->mlp, nn->theta.ptr, n, w, s);
  N::combine_loss(w.Y.ptr, nn->Cb.ptr, nn->Tb.ptr, n, a.n_comb, a.n_out, nullptr, w.dY.ptr, w.part.ptr, s);
  N::sum_partials(w.part.ptr, N::loss_blocks(n, a.n_out), d_loss, accumulate, s);
  if (grad) N::backward(nn->mlp, nn->theta.ptr, n, w, nn->grad.ptr, s);
  return IETI_OK;
}

}  // namespace

extern "C" {

int ieti_nn_create(const ieti_nn_arch* arch, ieti_nn** out) {
  if (!out) return fail(IETI_ERR_INVALID_ARG, "output pointer is NULL");
  *out = nullptr;
  ieti_nn* nn = new ieti_nn();
  int rc = nn->mlp.init(arch);
  if (!rc) {
    nn->shift.assign(size_t(arch->n_in), 0.f);
    nn->scale.assign(size_t(arch->n_in), 1.f);
  }
  if (!rc) {
    hipError_t e = hipStreamCreateWithFlags(&nn->stream, hipStreamNonBlocking);
    if (e != hipSuccess) rc = fail(IETI_ERR_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
  }
  for (auto* b : {&nn->theta, &nn->grad, &nn->m, &nn->v})
    if (!rc) rc = dalloc(*b, nn->mlp.n_params);
  if (!rc) rc = dalloc(nn->loss, 4);
  if (!rc) {
    for (auto* b : {&nn->theta, &nn->grad, &nn->m, &nn->v})
      if (hipMemset(b->ptr, 0, b->n * sizeof(float)) != hipSuccess) rc = fail(IETI_ERR_HIP, "hipMemset failed");
    if (!rc && hipDeviceSynchronize() != hipSuccess) rc = fail(IETI_ERR_HIP, "hipDeviceSynchronize failed");
  }
  if (rc) {
    delete nn;
    return rc;
  }
  *out = nn;
  return IETI_OK;
}

int ieti_nn_num_params(const ieti_nn* nn, int64_t* n_params) {
  if (!nn || !n_params) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  *n_params = nn->mlp.n_params;
  return IETI_OK;
}

int ieti_nn_set_params(ieti_nn* nn, const float* params) {
  if (!nn || !params) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  for (int64_t i = 0; i < nn->mlp.n_params; ++i)
    if (!std::isfinite(params[i])) return fail(IETI_ERR_INVALID_ARG, "parameters must be finite");
  HIP_TRY(hipMemcpy(nn->theta.ptr, params, nn->mlp.n_params * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(nn->m.ptr, 0, nn->m.n * sizeof(float)));
  HIP_TRY(hipMemset(nn->v.ptr, 0, nn->v.n * sizeof(float)));
  HIP_TRY(hipDeviceSynchronize());
  nn->adam_t = 0;
  return IETI_OK;
}

int ieti_nn_get_params(const ieti_nn* nn, float* params) {
  if (!nn || !params) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  HIP_TRY(hipStreamSynchronize(nn->stream));
  HIP_TRY(hipMemcpy(params, nn->theta.ptr, nn->mlp.n_params * sizeof(float), hipMemcpyDeviceToHost));
  return IETI_OK;
}

int ieti_nn_set_data(ieti_nn* nn, const float* X, const float* C, const float* Y, int64_t n) {
  if (!nn || !X || !C || !Y || n < 1) return fail(IETI_ERR_INVALID_ARG, "NULL data or n < 1");
  if (n > (int64_t(1) << 30)) return fail(IETI_ERR_INVALID_ARG, "too many rows");
  const auto& a = nn->mlp.arch;
  std::vector<float> xo = normalised_inputs(nn, X, n);
  std::vector<float> yo(size_t(n) * a.n_out);
  const double inv = 1.0 / nn->out_scale;
  for (size_t i = 0; i < yo.size(); ++i) yo[i] = float(double(Y[i]) * inv);
  int rc = dupload(nn->X, xo);
  if (!rc) rc = dupload(nn->C, C, n * a.n_comb);
  if (!rc) rc = dupload(nn->T, yo);
  if (rc) return rc;
  nn->n_data = n;
  return IETI_OK;
}

int ieti_nn_loss_grad(ieti_nn* nn, int64_t row0, int64_t nrows, double* loss, float* grad) {
  if (!nn) return fail(IETI_ERR_INVALID_ARG, "network is NULL");
  if (row0 < 0 || nrows < 1 || row0 + nrows > nn->n_data) return fail(IETI_ERR_INVALID_ARG, "rows out of range");
  int rc = check_rows(nn, nrows);
  if (rc) return rc;
  std::vector<int32_t> idx(nrows);
  std::iota(idx.begin(), idx.end(), int32_t(row0));
  if ((rc = dupload(nn->idx, idx))) return rc;
  step_rows(nn, nn->idx.ptr, nrows, grad != nullptr, nn->loss.ptr, 0);
  double sq = 0.0;
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(&sq, nn->loss.ptr, sizeof(double), hipMemcpyDeviceToHost, nn->stream));
  if (grad)
    HIP_TRY(hipMemcpyAsync(grad, nn->grad.ptr, nn->mlp.n_params * sizeof(float), hipMemcpyDeviceToHost, nn->stream));
  HIP_TRY(hipStreamSynchronize(nn->stream));
  if (loss) *loss = sq / (double(nrows) * nn->mlp.arch.n_out);
  return IETI_OK;
}

int ieti_nn_train(ieti_nn* nn, const ieti_nn_train_opts* opts, double* epoch_loss) {
  if (!nn || !opts) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  if (nn->n_data < 1) return fail(IETI_ERR_STATE, "no training data");
  if (opts->epochs < 0 || opts->batch < 0 || !(opts->lr > 0.f)) return fail(IETI_ERR_INVALID_ARG, "bad options");
  const int64_t n = nn->n_data;
  const int64_t batch = std::min<int64_t>(opts->batch > 0 ? opts->batch : 256, n);
  const float b1 = opts->beta1 > 0.f ? opts->beta1 : 0.9f;
  const float b2 = opts->beta2 > 0.f ? opts->beta2 : 0.999f;
  const float eps = opts->eps > 0.f ? opts->eps : 1e-8f;
  int rc = check_rows(nn, batch);
  if (rc) return rc;
  DBuf<double> eloss;
  if ((rc = dalloc(eloss, std::max(1, opts->epochs)))) return rc;
  hipStream_t s = nn->stream;
  std::vector<int32_t> perm(n);
  uint64_t state = opts->seed;
  for (int ep = 0; ep < opts->epochs; ++ep) {
    std::iota(perm.begin(), perm.end(), 0);
    for (int64_t i = n - 1; i > 0; --i) {
      const int64_t j = int64_t(splitmix64(state) % uint64_t(i + 1));
      std::swap(perm[i], perm[j]);
    }
    if ((rc = dupload(nn->idx, perm))) break;
    for (int64_t b0 = 0; b0 < n; b0 += batch) {
      const int64_t nb = std::min(batch, n - b0);
      step_rows(nn, nn->idx.ptr + b0, nb, true, eloss.ptr + ep, b0 > 0);
      ++nn->adam_t;
      const float c1 = float(1.0 / (1.0 - std::pow(double(b1), double(nn->adam_t))));
      const float c2 = float(1.0 / (1.0 - std::pow(double(b2), double(nn->adam_t))));
      N::adam(nn->theta.ptr, nn->grad.ptr, nn->m.ptr, nn->v.ptr, nn->mlp.n_params, opts->lr, b1, b2, eps, c1, c2, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      rc = fail(IETI_ERR_HIP, std::string("training launch: ") + hipGetErrorString(e));
      break;
    }
    // the permutation buffer is reused by the next epoch
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      rc = fail(IETI_ERR_HIP, std::string("training: ") + hipGetErrorString(e));
      break;
    }
  }
  if (!rc && epoch_loss && opts->epochs > 0) {
    std::vector<double> h(opts->epochs);
    hipError_t e = hipMemcpy(h.data(), eloss.ptr, h.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = fail(IETI_ERR_HIP, "copy of the epoch losses failed");
    for (int ep = 0; ep < opts->epochs && !rc; ++ep) epoch_loss[ep] = h[ep] / (double(n) * nn->mlp.arch.n_out);
  }
  eloss.release();
  return rc;
}

int ieti_nn_predict(ieti_nn* nn, const float* X, const float* C, int64_t n, float* pred) {
  if (!nn || !X || !C || !pred || n < 1) return fail(IETI_ERR_INVALID_ARG, "NULL argument or n < 1");
  const auto& a = nn->mlp.arch;
  int rc = check_rows(nn, n);
  if (rc) return rc;
  hipStream_t s = nn->stream;
  auto& w = nn->work;
  std::vector<float> xo = normalised_inputs(nn, X, n);
  HIP_TRY(hipMemcpyAsync(w.H[0].ptr, xo.data(), xo.size() * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(nn->Cb.ptr, C, size_t(n) * a.n_comb * sizeof(float), hipMemcpyHostToDevice, s));
  N::forward(nn->mlp, nn->theta.ptr, n, w, s);
  N::combine_loss(w.Y.ptr, nn->Cb.ptr, nullptr, n, a.n_comb, a.n_out, w.pred.ptr, nullptr, nullptr, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(pred, w.pred.ptr, size_t(n) * a.n_out * sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (nn->out_scale != 1.0)
    for (int64_t i = 0; i < n * a.n_out; ++i) pred[i] = float(double(pred[i]) * nn->out_scale);
  return IETI_OK;
}

int ieti_nn_init_params(ieti_nn* nn, uint64_t seed) {
  if (!nn) return fail(IETI_ERR_INVALID_ARG, "network is NULL");
  const auto& m = nn->mlp;
  std::vector<float> theta(size_t(m.n_params), 0.f);
  uint64_t state = seed;
  for (int l = 1; l < int(m.dims.size()); ++l) {
    const int64_t din = m.dims[l - 1], dout = m.dims[l];
    const double lim = std::sqrt(6.0 / double(din + dout));
    for (int64_t i = 0; i < dout; ++i)
      for (int64_t j = 0; j < din; ++j) {
        const double u = double(splitmix64(state) >> 11) * (1.0 / 9007199254740992.0);  // [0, 1), 53 bits
        theta[size_t(m.woff[l - 1] + i * (din + 1) + j)] = float((2.0 * u - 1.0) * lim);
      }
  }
  return ieti_nn_set_params(nn, theta.data());
}

int ieti_nn_set_normalisation(ieti_nn* nn, const float* shift, const float* scale, double out_scale) {
  if (!nn) return fail(IETI_ERR_INVALID_ARG, "network is NULL");
  const int64_t d = nn->mlp.arch.n_in;
  if (!(out_scale > 0.0) || !std::isfinite(out_scale)) return fail(IETI_ERR_INVALID_ARG, "output scale must be > 0");
  for (int64_t j = 0; j < d; ++j)
    if ((shift && !std::isfinite(shift[j])) || (scale && !std::isfinite(scale[j])))
      return fail(IETI_ERR_INVALID_ARG, "normalisation must be finite");
  for (int64_t j = 0; j < d; ++j) {
    nn->shift[j] = shift ? shift[j] : 0.f;
    nn->scale[j] = scale ? scale[j] : 1.f;
  }
  nn->out_scale = out_scale;
  return IETI_OK;
}

int ieti_nn_fit_normalisation(ieti_nn* nn, const float* X, const float* Y, int64_t n) {
  if (!nn || !X || !Y || n < 1) return fail(IETI_ERR_INVALID_ARG, "NULL data or n < 1");
  const int64_t d = nn->mlp.arch.n_in, no = nn->mlp.arch.n_out;
  std::vector<float> sh(d), sc(d);
  for (int64_t j = 0; j < d; ++j) {
    double mean = 0.0, var = 0.0;
    for (int64_t i = 0; i < n; ++i) mean += X[i * d + j];
    mean /= double(n);
    for (int64_t i = 0; i < n; ++i) var += (X[i * d + j] - mean) * (X[i * d + j] - mean);
    const double sd = std::sqrt(var / double(n));
    sh[j] = float(mean);
    sc[j] = float(sd > 1e-12 ? 1.0 / sd : 1.0);
  }
  double sq = 0.0;
  for (int64_t i = 0; i < n * no; ++i) sq += double(Y[i]) * double(Y[i]);
  const double rms = std::sqrt(sq / double(n * no));
  return ieti_nn_set_normalisation(nn, sh.data(), sc.data(), rms > 0.0 && std::isfinite(rms) ? rms : 1.0);
}

int ieti_nn_get_normalisation(const ieti_nn* nn, float* shift, float* scale, double* out_scale) {
  if (!nn) return fail(IETI_ERR_INVALID_ARG, "network is NULL");
  if (shift) std::copy(nn->shift.begin(), nn->shift.end(), shift);
  if (scale) std::copy(nn->scale.begin(), nn->scale.end(), scale);
  if (out_scale) *out_scale = nn->out_scale;
  return IETI_OK;
}

void ieti_nn_destroy(ieti_nn* nn) { delete nn; }

// File: 8-byte tag, the five int32 sizes of ieti_nn_arch, the int64
// parameter count, the parameters as FP32, then (version 02) the n_in
// feature shifts and scales as FP32 and the output scale as FP64 (host byte
// order).  Version 01 files (no normalisation) load with the identity.
static const char kNNTag[8] = {'I', 'E', 'T', 'I', 'N', 'N', '0', '2'};
static const char kNNTag1[8] = {'I', 'E', 'T', 'I', 'N', 'N', '0', '1'};

int ieti_nn_save(const ieti_nn* nn, const char* path) {
  if (!nn || !path) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  std::vector<float> theta(size_t(nn->mlp.n_params));
  int rc = ieti_nn_get_params(nn, theta.data());
  if (rc) return rc;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(IETI_ERR_INVALID_ARG, std::string("cannot open ") + path + " for writing");
  const ieti_nn_arch& a = nn->mlp.arch;
  const int32_t sizes[5] = {a.n_in, a.n_hidden, a.n_layers, a.n_comb, a.n_out};
  const int64_t n = nn->mlp.n_params;
  bool ok = std::fwrite(kNNTag, 1, 8, f) == 8 && std::fwrite(sizes, sizeof(int32_t), 5, f) == 5 &&
            std::fwrite(&n, sizeof(int64_t), 1, f) == 1 &&
            std::fwrite(theta.data(), sizeof(float), theta.size(), f) == theta.size() &&
            std::fwrite(nn->shift.data(), sizeof(float), nn->shift.size(), f) == nn->shift.size() &&
            std::fwrite(nn->scale.data(), sizeof(float), nn->scale.size(), f) == nn->scale.size() &&
            std::fwrite(&nn->out_scale, sizeof(double), 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(IETI_ERR_INVALID_ARG, std::string("writing ") + path + " failed");
  return IETI_OK;
}

int ieti_nn_load(const char* path, ieti_nn** out) {
  if (!path || !out) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(IETI_ERR_INVALID_ARG, std::string("cannot open ") + path);
  char tag[8];
  int32_t sizes[5];
  int64_t n = -1;
  bool ok = std::fread(tag, 1, 8, f) == 8 && (std::equal(tag, tag + 8, kNNTag) || std::equal(tag, tag + 8, kNNTag1)) &&
            std::fread(sizes, sizeof(int32_t), 5, f) == 5 && std::fread(&n, sizeof(int64_t), 1, f) == 1;
  const bool v2 = ok && std::equal(tag, tag + 8, kNNTag);
  ieti_nn_arch a{sizes[0], sizes[1], sizes[2], sizes[3], sizes[4]};
  ieti::nn::Mlp check;
  if (!ok || check.init(&a) != IETI_OK || check.n_params != n) {
    std::fclose(f);
    return fail(IETI_ERR_INVALID_ARG, std::string(path) + " is not a network file of this library");
  }
  std::vector<float> theta(static_cast<size_t>(n)), sh(size_t(a.n_in), 0.f), sc(size_t(a.n_in), 1.f);
  double osc = 1.0;
  ok = std::fread(theta.data(), sizeof(float), theta.size(), f) == theta.size();
  if (ok && v2)
    ok = std::fread(sh.data(), sizeof(float), sh.size(), f) == sh.size() &&
         std::fread(sc.data(), sizeof(float), sc.size(), f) == sc.size() && std::fread(&osc, sizeof(double), 1, f) == 1;
  std::fclose(f);
  if (!ok) return fail(IETI_ERR_INVALID_ARG, std::string(path) + " is truncated");
  ieti_nn* nn = nullptr;
  int rc = ieti_nn_create(&a, &nn);
  if (!rc) rc = ieti_nn_set_params(nn, theta.data());
  if (!rc) rc = ieti_nn_set_normalisation(nn, sh.data(), sc.data(), osc);
  if (rc) {
    ieti_nn_destroy(nn);
    return rc;
  }
  *out = nn;
  return IETI_OK;
}

// Dataset file: 8-byte tag, int32 n_in, n_comb, n_out, then rows of
// n_in + n_comb + n_out FP32 values (features, coefficients, targets).
static const char kDSTag[8] = {'I', 'E', 'T', 'I', 'D', 'S', '0', '1'};

int ieti_nn_dataset_append(const char* path, const float* X, const float* C, const float* Y, int64_t n, int32_t n_in,
                           int32_t n_comb, int32_t n_out) {
  if (!path || !X || !C || !Y || n < 1 || n_in < 1 || n_comb < 1 || n_out < 1)
    return fail(IETI_ERR_INVALID_ARG, "NULL argument or empty rows");
  int32_t sz[3] = {0, 0, 0};
  FILE* f = std::fopen(path, "rb");
  bool fresh = f == nullptr;
  if (f) {
    char tag[8];
    const bool ok = std::fread(tag, 1, 8, f) == 8 && std::equal(tag, tag + 8, kDSTag) &&
                    std::fread(sz, sizeof(int32_t), 3, f) == 3;
    std::fclose(f);
    if (!ok) return fail(IETI_ERR_INVALID_ARG, std::string(path) + " is not a dataset file of this library");
    if (sz[0] != n_in || sz[1] != n_comb || sz[2] != n_out)
      return fail(IETI_ERR_INVALID_ARG, std::string(path) + " holds rows of other sizes");
  }
  f = std::fopen(path, fresh ? "wb" : "ab");
  if (!f) return fail(IETI_ERR_INVALID_ARG, std::string("cannot open ") + path + " for writing");
  bool ok = true;
  if (fresh) {
    const int32_t h[3] = {n_in, n_comb, n_out};
    ok = std::fwrite(kDSTag, 1, 8, f) == 8 && std::fwrite(h, sizeof(int32_t), 3, f) == 3;
  }
  for (int64_t i = 0; i < n && ok; ++i)
    ok = std::fwrite(X + i * n_in, sizeof(float), size_t(n_in), f) == size_t(n_in) &&
         std::fwrite(C + i * n_comb, sizeof(float), size_t(n_comb), f) == size_t(n_comb) &&
         std::fwrite(Y + i * n_out, sizeof(float), size_t(n_out), f) == size_t(n_out);
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(IETI_ERR_INVALID_ARG, std::string("writing ") + path + " failed");
  return IETI_OK;
}

int ieti_nn_train_file(const char* dataset_path, const ieti_nn_arch* arch, const ieti_nn_train_opts* opts,
                       const char* model_out, double* epoch_loss) {
  if (!dataset_path || !arch || !opts || !model_out) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  FILE* f = std::fopen(dataset_path, "rb");
  if (!f) return fail(IETI_ERR_INVALID_ARG, std::string("cannot open ") + dataset_path);
  char tag[8];
  int32_t sz[3];
  bool ok = std::fread(tag, 1, 8, f) == 8 && std::equal(tag, tag + 8, kDSTag) && std::fread(sz, sizeof(int32_t), 3, f) == 3;
  if (!ok || sz[0] != arch->n_in || sz[1] != arch->n_comb || sz[2] != arch->n_out) {
    std::fclose(f);
    return fail(IETI_ERR_INVALID_ARG, std::string(dataset_path) + " is not a dataset for this architecture");
  }
  const size_t w = size_t(sz[0]) + size_t(sz[1]) + size_t(sz[2]);
  std::vector<float> rows;
  std::vector<float> buf(w);
  while (std::fread(buf.data(), sizeof(float), w, f) == w) rows.insert(rows.end(), buf.begin(), buf.end());
  std::fclose(f);
  const int64_t n = int64_t(rows.size() / w);
  if (n < 1) return fail(IETI_ERR_INVALID_ARG, std::string(dataset_path) + " holds no rows");
  std::vector<float> X(size_t(n) * sz[0]), C(size_t(n) * sz[1]), Y(size_t(n) * sz[2]);
  for (int64_t i = 0; i < n; ++i) {
    const float* r = rows.data() + size_t(i) * w;
    std::copy(r, r + sz[0], X.begin() + i * sz[0]);
    std::copy(r + sz[0], r + sz[0] + sz[1], C.begin() + i * sz[1]);
    std::copy(r + sz[0] + sz[1], r + w, Y.begin() + i * sz[2]);
  }
  ieti_nn* nn = nullptr;
  int rc = ieti_nn_create(arch, &nn);
  if (!rc) rc = ieti_nn_init_params(nn, opts->seed);
  if (!rc) rc = ieti_nn_fit_normalisation(nn, X.data(), Y.data(), n);
  if (!rc) rc = ieti_nn_set_data(nn, X.data(), C.data(), Y.data(), n);
  if (!rc) rc = ieti_nn_train(nn, opts, epoch_loss);
  if (!rc) rc = ieti_nn_save(nn, model_out);
  ieti_nn_destroy(nn);
  return rc;
}

}  // extern "C"

// used by the solver to copy a network's parameters
namespace ieti {
namespace nn {
const Mlp& mlp_of(const ieti_nn* nn) { return nn->mlp; }
const std::vector<float>& shift_of(const ieti_nn* nn) { return nn->shift; }
const std::vector<float>& scale_of(const ieti_nn* nn) { return nn->scale; }
double out_scale_of(const ieti_nn* nn) { return nn->out_scale; }
const float* params_of(const ieti_nn* nn) { return nn->theta.ptr; }
hipStream_t stream_of(const ieti_nn* nn) { return nn->stream; }
}  // namespace nn
}  // namespace ieti
