// Host-side driver of the warm-start network: shapes, parameter layout and
// the forward and backward passes built from the kernels in device/nn.hpp.
#pragma once

#include <cstdint>
#include <vector>

#include "common.hpp"
#include "device/nn.hpp"
#include "ietidp.h"

namespace ieti {
namespace nn {

struct Mlp {
  ieti_nn_arch arch{};
  std::vector<int64_t> dims;  // d_0 = n_in, d_1..d_L = n_hidden, d_{L+1} = n_comb * n_out
  std::vector<int64_t> woff;  // offset of W'_l (d_l x (d_{l-1}+1), row-major), index l-1
  int64_t n_params = 0;
  int init(const ieti_nn_arch* a);
  int layers() const { return int(dims.size()) - 1; }
};

// activations and gradients for up to cap rows
struct Work {
  int64_t cap = 0;
  std::vector<rt::DBuf<float>> H;  // H[l]: cap x (d_l + 1), last column 1, l = 0..L
  rt::DBuf<float> Y, dY, dZ0, dZ1, pred;
  rt::DBuf<double> part;
  int reserve(const Mlp& m, int64_t n, hipStream_t s);
  void release();
};

// Y = network output for the n rows whose inputs are in w.H[0]
void forward(const Mlp& m, const float* theta, int64_t n, Work& w, hipStream_t s);
// grad = d loss / d theta from w.dY (after forward on the same rows)
void backward(const Mlp& m, const float* theta, int64_t n, Work& w, float* grad, hipStream_t s);

}  // namespace nn
}  // namespace ieti

namespace ieti {
namespace nn {
// accessors of a network object (defined with it)
const Mlp& mlp_of(const ieti_nn* nn);
const std::vector<float>& shift_of(const ieti_nn* nn);
const std::vector<float>& scale_of(const ieti_nn* nn);
double out_scale_of(const ieti_nn* nn);
const float* params_of(const ieti_nn* nn);
hipStream_t stream_of(const ieti_nn* nn);
}  // namespace nn
}  // namespace ieti
