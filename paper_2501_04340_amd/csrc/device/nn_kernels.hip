// gfx950 kernels of the warm-start network (FP32).  The products run on the
// FP32 matrix cores (v_mfma_f32_16x16x4f32) from LDS-staged 64x64x16 tiles;
// everything else is elementwise or a fixed-order reduction, so a training
// step is deterministic for a given launch configuration.
#include <hip/hip_runtime.h>

#include <cmath>

#include "nn.hpp"

namespace ieti {
namespace nn {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

// One 64x64 output tile per workgroup of 4 waves; wave w owns the 32x32
// quadrant (w/2, w%2) as 2x2 MFMA blocks.  Operand layout of
// v_mfma_f32_16x16x4f32 (lane l): A row l%16, k l/16; B k l/16, col l%16;
// accumulator element r: row 4(l/16) + r, col l%16.  The global loads are
// laid out so that consecutive lanes touch consecutive addresses whichever
// operand stride is 1.
__global__ __launch_bounds__(NT) void k_gemm(int64_t M, int64_t N, int64_t K, const float* __restrict__ A,
                                             int64_t sai, int64_t sak, const float* __restrict__ B, int64_t sbk,
                                             int64_t sbj, float* __restrict__ C, int64_t ldc, int epi,
                                             const float* __restrict__ aux, int64_t ldaux) {
  __shared__ float As[BK][BM + 1];
  __shared__ float Bs[BK][BN + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t i0 = int64_t(blockIdx.y) * BM, j0 = int64_t(blockIdx.x) * BN;
  const bool a_krow = (sak == 1);
  const bool b_jrow = (sbj == 1);
  v4f acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) acc[m][n] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    float ra[4], rb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + NT * u;
      const int ii = a_krow ? e / BK : e % BM;
      const int ka = a_krow ? e % BK : e / BM;
      const int64_t gi = i0 + ii, gka = k0 + ka;
      ra[u] = (gi < M && gka < K) ? A[gi * sai + gka * sak] : 0.f;
      const int jj = b_jrow ? e % BN : e / BK;
      const int kb = b_jrow ? e / BN : e % BK;
      const int64_t gj = j0 + jj, gkb = k0 + kb;
      rb[u] = (gj < N && gkb < K) ? B[gkb * sbk + gj * sbj] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + NT * u;
      if (a_krow) As[e % BK][e / BK] = ra[u];
      else As[e / BM][e % BM] = ra[u];
      if (b_jrow) Bs[e / BN][e % BN] = rb[u];
      else Bs[e % BK][e / BK] = rb[u];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + (lane >> 4);
      float a[2], b[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) a[m] = As[kk][32 * (w >> 1) + 16 * m + (lane & 15)];
#pragma unroll
      for (int n = 0; n < 2; ++n) b[n] = Bs[kk][32 * (w & 1) + 16 * n + (lane & 15)];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], b[n], acc[m][n], 0, 0, 0);
    }
  }
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + 32 * (w >> 1) + 16 * m + 4 * (lane >> 4) + r;
        const int64_t gj = j0 + 32 * (w & 1) + 16 * n + (lane & 15);
        if (gi < M && gj < N) {
          float v = acc[m][n][r];
          if (epi == EPI_TANH) {
            v = tanhf(v);
          } else if (epi == EPI_DTANH) {
            const float h = aux[gi * ldaux + gj];
            v *= (1.f - h * h);
          }
          C[gi * ldc + gj] = v;
        }
      }
}

__global__ void k_fill_column(float* X, int64_t n, int64_t ld, int64_t c, float v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) X[i * ld + c] = v;
}

__global__ void k_gather_rows(const float* __restrict__ src, int64_t lds, const int32_t* __restrict__ idx, int64_t n,
                              int64_t ncols, float* __restrict__ dst, int64_t ldd) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t r = e / ncols, c = e % ncols;
  dst[r * ldd + c] = src[int64_t(idx[r]) * lds + c];
}

constexpr int LOSS_THREADS = 256;

__global__ __launch_bounds__(LOSS_THREADS) void k_combine_loss(const float* __restrict__ Y, const float* __restrict__ Cc,
                                                               const float* __restrict__ T, int64_t n, int n_comb,
                                                               int n_out, float* __restrict__ pred,
                                                               float* __restrict__ dY, double* __restrict__ part) {
  __shared__ double red[LOSS_THREADS];
  const int64_t e = int64_t(blockIdx.x) * LOSS_THREADS + threadIdx.x;
  double sq = 0.0;
  if (e < n * n_out) {
    const int64_t i = e / n_out;
    const int o = int(e % n_out);
    const int64_t ldy = int64_t(n_comb) * n_out;
    float acc = 0.f;
    for (int r = 0; r < n_comb; ++r) acc += Cc[i * n_comb + r] * Y[i * ldy + int64_t(r) * n_out + o];
    if (pred) pred[e] = acc;
    if (T) {
      const float diff = acc - T[e];
      sq = double(diff) * double(diff);
      const float g = 2.f * diff / float(double(n) * double(n_out));
      for (int r = 0; r < n_comb; ++r) dY[i * ldy + int64_t(r) * n_out + o] = Cc[i * n_comb + r] * g;
    }
  }
  if (!part) return;
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int h = LOSS_THREADS / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int nblk, double* out,
                                                      int accumulate) {
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += part[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = accumulate ? out[0] + red[0] : red[0];
}

__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void k_features(const double* __restrict__ nu, const double* __restrict__ load_scale,
                           const int32_t* __restrict__ feat_patch, const float* __restrict__ shift,
                           const float* __restrict__ scale, int n_facets, int n_feat,
                           const int32_t* __restrict__ comb_patch, int n_comb, float* __restrict__ X,
                           float* __restrict__ Cf) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t wx = n_feat + 1;
  const int64_t nx = int64_t(n_facets) * wx;
  if (e < nx) {
    const int64_t f = e / wx, j = e % wx;
    X[e] = (j == n_feat) ? 1.f
                         : float((log(nu[feat_patch[f * n_feat + j]]) - double(shift[j])) * double(scale[j]));
  } else if (e < nx + int64_t(n_facets) * n_comb) {
    const int64_t c = e - nx;
    Cf[c] = float(load_scale[comb_patch[c]]);
  }
}

__global__ void k_scatter_prediction(const float* __restrict__ pred, const int32_t* __restrict__ out_row,
                                     const int8_t* __restrict__ out_sign, int64_t n, double out_scale,
                                     double* __restrict__ lam) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int32_t row = out_row[e];
  if (row >= 0) lam[row] = out_scale * double(out_sign[e]) * double(pred[e]);
}

inline unsigned nblocks(int64_t n, int b) { return unsigned((n + b - 1) / b); }

}  // namespace

void gemm(int64_t M, int64_t N, int64_t K, const float* A, int64_t sai, int64_t sak, const float* B, int64_t sbk,
          int64_t sbj, float* C, int64_t ldc, int epi, const float* aux, int64_t ldaux, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  dim3 grid(nblocks(N, BN), nblocks(M, BM));
  hipLaunchKernelGGL(k_gemm, grid, dim3(NT), 0, s, M, N, K, A, sai, sak, B, sbk, sbj, C, ldc, epi, aux, ldaux);
}

void fill_column(float* X, int64_t n, int64_t ld, int64_t c, float v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_column, dim3(nblocks(n, 256)), dim3(256), 0, s, X, n, ld, c, v);
}

void gather_rows(const float* src, int64_t lds, const int32_t* idx, int64_t n, int64_t ncols, float* dst, int64_t ldd,
                 hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3(nblocks(n * ncols, 256)), dim3(256), 0, s, src, lds, idx, n, ncols, dst,
                     ldd);
}

int loss_blocks(int64_t n, int n_out) { return int(nblocks(n * n_out, LOSS_THREADS)); }

void combine_loss(const float* Y, const float* C, const float* T, int64_t n, int n_comb, int n_out, float* pred,
                  float* dY, double* part, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_combine_loss, dim3(loss_blocks(n, n_out)), dim3(LOSS_THREADS), 0, s, Y, C, T, n, n_comb,
                     n_out, pred, dY, part);
}

void sum_partials(const double* part, int nblk, double* out, int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, nblk, out, accumulate);
}

void adam(float* theta, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2, float eps,
          float c1, float c2, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_adam, dim3(nblocks(n, 256)), dim3(256), 0, s, theta, g, m, v, n, lr, beta1, beta2, eps, c1, c2);
}

void features(const double* nu, const double* load_scale, const int32_t* feat_patch, const float* shift,
              const float* scale, int n_facets, int n_feat, const int32_t* comb_patch, int n_comb, float* X,
              float* Cf, hipStream_t s) {
  const int64_t n = int64_t(n_facets) * (n_feat + 1 + n_comb);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_features, dim3(nblocks(n, 256)), dim3(256), 0, s, nu, load_scale, feat_patch, shift, scale,
                     n_facets, n_feat, comb_patch, n_comb, X, Cf);
}

void scatter_prediction(const float* pred, const int32_t* out_row, const int8_t* out_sign, int64_t n, double out_scale,
                        double* lam, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scatter_prediction, dim3(nblocks(n, 256)), dim3(256), 0, s, pred, out_row, out_sign, n,
                     out_scale, lam);
}

}  // namespace nn
}  // namespace ieti
