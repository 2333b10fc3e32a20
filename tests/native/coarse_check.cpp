// Host-side check of the coarse problem's tile plan (test program, CPU only).
//
// For a few problems with random symmetric positive definite S_c (n x n) and
// random G (m x n), build_coarse_plan's task lists are run in plain loops as
// the GPU kernels define them (tile fill, per level the diagonal-tile
// Cholesky with the inverse of its factor, the panel products X L_cc^{-T},
// the updates C -= A B^T, then the extraction), and the results are compared
// with the definitions: L_c L_c^T = S_c, H = G L_c^{-T} (H L_c^T = G), and
// U = L_c^{-T} (L_c^T U = I).  Prints one line, exit 0 when the residuals are
// at rounding level.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "host/plan.hpp"

using namespace ieti;

int main() {
  const int T = 64;
  const int64_t TT = int64_t(T) * T;
  const int64_t ms[] = {0, 1, 130, 64, 700, 257};
  const int64_t ns[] = {0, 3, 64, 65, 150, 1};
  const int NP = 6;
  std::vector<CoarseDims> dims(NP);
  int64_t spi = 0, goff = 0;
  for (int p = 0; p < NP; ++p) {
    dims[p].m = ms[p];
    dims[p].n = ns[p];
    dims[p].spi_off = spi;
    dims[p].g_off = goff;
    spi += ns[p] * ns[p];
    goff += ms[p] * ns[p];
  }
  std::mt19937_64 rng(11);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> S(spi, 0.0), G(goff, 0.0);
  for (int p = 0; p < NP; ++p) {
    const int64_t n = ns[p], m = ms[p];
    std::vector<double> A(n * n);
    for (auto& v : A) v = nd(rng);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) {
        double s = (i == j) ? double(n) : 0.0;
        for (int64_t k = 0; k < n; ++k) s += A[i * n + k] * A[j * n + k];
        S[dims[p].spi_off + i * n + j] = s;
      }
    for (int64_t i = 0; i < m * n; ++i) G[dims[p].g_off + i] = nd(rng);
  }
  CoarsePlan cp;
  build_coarse_plan(dims, T, cp);
  std::vector<double> pool(cp.pool_elems, 0.0), inv(cp.inv_elems, 0.0);
  // fill
  for (size_t t = 0; t < cp.fill_task.size(); t += 7) {
    const int64_t* k = &cp.fill_task[t];
    const double* src = k[1] == 0 ? S.data() : (k[1] == 1 ? G.data() : nullptr);
    for (int a = 0; a < T; ++a)
      for (int b = 0; b < T; ++b) {
        double v = (k[6] && a == b) ? 1.0 : 0.0;
        if (src && a < k[4] && b < k[5]) v = src[k[2] + a * k[3] + b];
        pool[k[0] + b * T + a] = v;
      }
  }
  int bad_pivot = 0;
  for (int64_t c = 0; c < cp.n_levels; ++c) {
    for (int64_t q = cp.potrf_ptr[c]; q < cp.potrf_ptr[c + 1]; ++q) {
      double* A = &pool[cp.potrf_task[3 * q]];
      double* Li = &inv[cp.potrf_task[3 * q + 2]];
      for (int k = 0; k < T; ++k) {  // column-major: A[col * T + row]
        double d = A[k * T + k];
        for (int j = 0; j < k; ++j) d -= A[j * T + k] * A[j * T + k];
        if (!(d > 0.0)) bad_pivot = 1;
        const double l = std::sqrt(d);
        A[k * T + k] = l;
        for (int i = k + 1; i < T; ++i) {
          double s = A[k * T + i];
          for (int j = 0; j < k; ++j) s -= A[j * T + i] * A[j * T + k];
          A[k * T + i] = s / l;
        }
      }
      for (int j = 0; j < T; ++j)
        for (int i = 0; i < j; ++i) A[j * T + i] = 0.0;
      for (int j = 0; j < T; ++j)  // inverse of the lower factor, column j
        for (int i = 0; i < T; ++i) {
          double s = (i == j) ? 1.0 : 0.0;
          for (int k = j; k < i; ++k) s -= A[k * T + i] * Li[j * T + k];
          Li[j * T + i] = i < j ? 0.0 : s / A[i * T + i];
        }
    }
    for (int64_t q = cp.trsm_ptr[c]; q < cp.trsm_ptr[c + 1]; ++q) {
      double* X = &pool[cp.trsm_task[2 * q]];
      const double* Li = &inv[cp.trsm_task[2 * q + 1]];
      std::vector<double> out(TT, 0.0);
      for (int i = 0; i < T; ++i)
        for (int j = 0; j < T; ++j) {  // (X L^{-T})[i][j] = sum_k X[i][k] Li[j][k]
          double s = 0.0;
          for (int k = 0; k < T; ++k) s += X[k * T + i] * Li[k * T + j];
          out[j * T + i] = s;
        }
      for (int64_t e = 0; e < TT; ++e) X[e] = out[e];
    }
    for (int64_t q = cp.upd_ptr[c]; q < cp.upd_ptr[c + 1]; ++q) {
      double* C = &pool[cp.upd_task[3 * q]];
      for (int64_t pi = 0; pi < cp.upd_task[3 * q + 2]; ++pi) {
        const int64_t pr = cp.upd_task[3 * q + 1] + pi;
        const double* A = &pool[cp.upd_pair[2 * pr]];
        const double* B = &pool[cp.upd_pair[2 * pr + 1]];
        for (int i = 0; i < T; ++i)
          for (int j = 0; j < T; ++j) {
            double s = 0.0;
            for (int k = 0; k < T; ++k) s += A[k * T + i] * B[k * T + j];
            C[j * T + i] -= s;
          }
      }
    }
  }
  std::vector<double> H(goff, 0.0), Ht(goff, 0.0), U(spi, 0.0);
  auto extract = [&](const std::vector<int64_t>& tk, double* dst, double* dstt) {
    for (size_t t = 0; t < tk.size(); t += 7) {
      const int64_t* k = &tk[t];
      for (int a = 0; a < k[5]; ++a)
        for (int b = 0; b < k[6]; ++b) {
          const double v = pool[k[0] + b * T + a];
          dst[k[1] + a * k[3] + b] = v;
          if (k[2] >= 0) dstt[k[2] + b * k[4] + a] = v;
        }
    }
  };
  extract(cp.out_h_task, H.data(), Ht.data());
  extract(cp.out_l_task, U.data(), nullptr);
  // residuals against the definitions, with L from a plain Cholesky of S_c
  double rh = 0.0, ru = 0.0, rt = 0.0;
  for (int p = 0; p < NP; ++p) {
    const int64_t n = ns[p], m = ms[p];
    if (n == 0) continue;
    std::vector<double> L(n * n, 0.0);
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = j; i < n; ++i) {
        double s = S[dims[p].spi_off + i * n + j];
        for (int64_t k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
        L[i * n + j] = i == j ? std::sqrt(s) : s / L[j * n + j];
      }
    double gmax = 0.0;
    for (int64_t r = 0; r < m; ++r)
      for (int64_t c = 0; c < n; ++c) {  // (H L^T)[r][c] = sum_k H[r][k] L[c][k] = G[r][c]
        double s = 0.0;
        for (int64_t k = 0; k <= c; ++k) s += H[dims[p].g_off + r * n + k] * L[c * n + k];
        const double g = G[dims[p].g_off + r * n + c];
        gmax = std::max(gmax, std::fabs(g));
        rh = std::max(rh, std::fabs(s - g));
        rt = std::max(rt, std::fabs(Ht[dims[p].g_off + c * m + r] - H[dims[p].g_off + r * n + c]));
      }
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) {  // (L^T U)[i][j] = sum_k L[k][i] U[k][j] = delta_ij
        double s = 0.0;
        for (int64_t k = i; k < n; ++k) s += L[k * n + i] * U[dims[p].spi_off + k * n + j];
        ru = std::max(ru, std::fabs(s - (i == j ? 1.0 : 0.0)));
        if (i > j && U[dims[p].spi_off + i * n + j] != 0.0) ru = 1.0;  // U is upper triangular
      }
  }
  std::printf("coarse tiles: levels %lld pool %lld H residual %.3e U residual %.3e Ht %.3e pivots %s\n",
              (long long)cp.n_levels, (long long)cp.pool_elems, rh, ru, rt, bad_pivot ? "bad" : "ok");
  return (rh < 1e-10 && ru < 1e-10 && rt == 0.0 && !bad_pivot) ? 0 : 1;
}
