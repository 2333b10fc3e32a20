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
  std::vector<float> xo(size_t(n) * (a.n_in + 1));
  for (int64_t i = 0; i < n; ++i) {
    std::copy(X + i * a.n_in, X + (i + 1) * a.n_in, xo.begin() + i * (a.n_in + 1));
    xo[i * (a.n_in + 1) + a.n_in] = 1.f;
  }
  int rc = dupload(nn->X, xo);
  if (!rc) rc = dupload(nn->C, C, n * a.n_comb);
  if (!rc) rc = dupload(nn->T, Y, n * a.n_out);
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
  std::vector<float> xo(size_t(n) * (a.n_in + 1));
  for (int64_t i = 0; i < n; ++i) {
    std::copy(X + i * a.n_in, X + (i + 1) * a.n_in, xo.begin() + i * (a.n_in + 1));
    xo[i * (a.n_in + 1) + a.n_in] = 1.f;
  }
  HIP_TRY(hipMemcpyAsync(w.H[0].ptr, xo.data(), xo.size() * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(nn->Cb.ptr, C, size_t(n) * a.n_comb * sizeof(float), hipMemcpyHostToDevice, s));
  N::forward(nn->mlp, nn->theta.ptr, n, w, s);
  N::combine_loss(w.Y.ptr, nn->Cb.ptr, nullptr, n, a.n_comb, a.n_out, w.pred.ptr, nullptr, nullptr, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(pred, w.pred.ptr, size_t(n) * a.n_out * sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return IETI_OK;
}

void ieti_nn_destroy(ieti_nn* nn) { delete nn; }

// File: 8-byte tag, the five int32 sizes of ieti_nn_arch, the int64
// parameter count, the parameters as FP32 (host byte order).
static const char kNNTag[8] = {'I', 'E', 'T', 'I', 'N', 'N', '0', '1'};

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
            std::fwrite(theta.data(), sizeof(float), theta.size(), f) == theta.size();
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
  bool ok = std::fread(tag, 1, 8, f) == 8 && std::equal(tag, tag + 8, kNNTag) &&
            std::fread(sizes, sizeof(int32_t), 5, f) == 5 && std::fread(&n, sizeof(int64_t), 1, f) == 1;
  ieti_nn_arch a{sizes[0], sizes[1], sizes[2], sizes[3], sizes[4]};
  ieti::nn::Mlp check;
  if (!ok || check.init(&a) != IETI_OK || check.n_params != n) {
    std::fclose(f);
    return fail(IETI_ERR_INVALID_ARG, std::string(path) + " is not a network file of this library");
  }
  std::vector<float> theta(static_cast<size_t>(n));
  ok = std::fread(theta.data(), sizeof(float), theta.size(), f) == theta.size();
  std::fclose(f);
  if (!ok) return fail(IETI_ERR_INVALID_ARG, std::string(path) + " is truncated");
  ieti_nn* nn = nullptr;
  int rc = ieti_nn_create(&a, &nn);
  if (!rc) rc = ieti_nn_set_params(nn, theta.data());
  if (rc) {
    ieti_nn_destroy(nn);
    return rc;
  }
  *out = nn;
  return IETI_OK;
}

}  // extern "C"

// used by the solver to copy a network's parameters
namespace ieti {
namespace nn {
const Mlp& mlp_of(const ieti_nn* nn) { return nn->mlp; }
const float* params_of(const ieti_nn* nn) { return nn->theta.ptr; }
hipStream_t stream_of(const ieti_nn* nn) { return nn->stream; }
}  // namespace nn
}  // namespace ieti
