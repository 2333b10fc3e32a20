// FP32 kernels of the warm-start network: a multilayer perceptron with tanh
// hidden layers whose linear output is split into n_comb groups of n_out
// values; the prediction of a row is the sum of the groups weighted by the
// row's n_comb coefficients (the solution of the linear problem is linear in
// the source, so the coefficients carry the source amplitudes).
//
// Layout.  Activations are row-major with one extra trailing column that
// holds 1, so that a layer with weights W (d_out x d_in) and bias b is one
// product with W' = [W b] (d_out x (d_in+1), row-major): z = h' W'^T.  The
// parameters are the W' of every layer, concatenated.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ieti {
namespace nn {

enum Epilogue { EPI_NONE = 0, EPI_TANH = 1, EPI_DTANH = 2 };

// C[i*ldc + j] = epi(sum_k A[i*sai + k*sak] * B[k*sbk + j*sbj]) for i < M,
// j < N on the FP32 matrix cores.  EPI_DTANH multiplies by
// (1 - aux[i*ldaux + j]^2), the derivative of tanh at the stored output aux.
void gemm(int64_t M, int64_t N, int64_t K, const float* A, int64_t sai, int64_t sak, const float* B, int64_t sbk,
          int64_t sbj, float* C, int64_t ldc, int epi, const float* aux, int64_t ldaux, hipStream_t s);

// column c of an n x ld row-major matrix set to v
void fill_column(float* X, int64_t n, int64_t ld, int64_t c, float v, hipStream_t s);
// dst row r = src row idx[r] (ncols floats each; row strides lds, ldd)
void gather_rows(const float* src, int64_t lds, const int32_t* idx, int64_t n, int64_t ncols, float* dst, int64_t ldd,
                 hipStream_t s);
// pred[i][o] = sum_r C[i][r] Y[i][r*n_out + o]; with T != null also
// dY[i][r*n_out+o] = C[i][r] * 2 (pred - T) / (n n_out) and per-block partial
// sums of (pred - T)^2 in part (FP64), count returned by loss_blocks.
void combine_loss(const float* Y, const float* C, const float* T, int64_t n, int n_comb, int n_out, float* pred,
                  float* dY, double* part, hipStream_t s);
int loss_blocks(int64_t n, int n_out);
// out[0] += sum part[0..nblk) (fixed order), or out[0] = ... when accumulate == 0
void sum_partials(const double* part, int nblk, double* out, int accumulate, hipStream_t s);
// Adam (Kingma & Ba, Algorithm 1) on n parameters; c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
void adam(float* theta, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2, float eps,
          float c1, float c2, hipStream_t s);
// warm-start features: X[f][j] = (log(nu[feat_patch[f][j]]) - shift[j]) * scale[j], X[f][n_feat] = 1,
// Cf[f][r] = load_scale[comb_patch[f][r]]
void features(const double* nu, const double* load_scale, const int32_t* feat_patch, const float* shift,
              const float* scale, int n_facets, int n_feat, const int32_t* comb_patch, int n_comb, float* X,
              float* Cf, hipStream_t s);
// lam[out_row[f][o]] = out_scale * out_sign[f][o] * pred[f][o] (rows not covered stay as filled)
void scatter_prediction(const float* pred, const int32_t* out_row, const int8_t* out_sign, int64_t n, double out_scale,
                        double* lam, hipStream_t s);

}  // namespace nn
}  // namespace ieti
