// Launch wrappers of the gfx950 kernels of the IETI-DP hot path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ieti {
namespace dev {

constexpr int TILE = 64;

// ---- factorisation (tile pool, column-major 64x64 tiles)
void fill(double* p, int64_t n, double v, hipStream_t s);
void scatter(double* pool, const int64_t* dst, const double* val, int64_t n, hipStream_t s);
// potrf task [off_jj, subdomain, off of the inverse]; writes L_jj and L_jj^{-1}
void potrf_tiles(double* pool, double* inv, const int64_t* task, int64_t ntask, int* err, hipStream_t s);
// trsm task [off_ij, off of L_jj^{-1}]: L_ij = A_ij L_jj^{-T}
void trsm_tiles(double* pool, const double* inv, const int64_t* task, int64_t ntask, hipStream_t s);
// update task [off_C, first pair, pair count], pairs [off_A, off_B]: C -= sum A B^T;
// at most UPDATE_WGS workgroups, each walking its share of the tasks
constexpr int64_t UPDATE_WGS = 1024;
void update_tiles(double* pool, const int64_t* task, const int64_t* pair, int64_t ntask, hipStream_t s);
void copy_tiles(const double* pool, const int64_t* task, int64_t ntask, double scale, double* dst, hipStream_t s);

// ---- triangular solves with the tile factor (augmented vectors)
// diag task [off of L_jj^{-1}, vec_j]: y_j <- L_jj^{-1} y_j (or ^{-T})
void trsv_diag(const double* inv, const int64_t* task, int64_t ntask, double* y, bool transposed, hipStream_t s);
// update task [vec_dst, first pair, count], pairs [off_tile, vec_src]: y_dst -= sum L x (or L^T x)
void trsv_update(const double* pool, const int64_t* task, const int64_t* pair, int64_t ntask, double* y,
                 bool transposed, hipStream_t s);

// ---- coarse problem
void sum_sources(const double* src, const int64_t* ptr, const int64_t* idx, int64_t nout, double* out, hipStream_t s);
void build_G(const double* Phi, const int64_t* row_src, const int64_t* slot_phi_row, const int32_t* I_sub,
             const int32_t* glob2loc, int64_t m_r, int64_t n_gp, double* G, hipStream_t s);
void chol_small(double* A, int64_t n, int* err, hipStream_t s);
void solve_rows_LT(const double* L, int64_t n, const double* G, int64_t m, double* H, double* Ht, hipStream_t s);
void tri_small(const double* L, int64_t n, const double* in, double* out, bool transposed, hipStream_t s);

// ---- interface operators and PCG (FP64 recurrences)
// xg[slot(+1)] = x[row], xg[slot(-1)] = -x[row]
void gather_rows(const double* x, const int64_t* row_src, int64_t m_r, double* xg, hipStream_t s);
// v[slot] = (M_k xg_k)[slot] for every interface slot; part[block] = sum xg.v over the block's rows.
// task [matrix row start, first slot, nrows, ld, first slot of the subdomain]; ev_* may be null.
// Launch shapes: 4 waves, each owning rpw rows at a time (4 rpw rows per
// workgroup = per task), unroll vectors in flight per lane and row, nt =
// non-temporal loads.  Variant index = 4 * (rpw index in {2,4,8}) + 2 * (unroll - 1) + nt.
struct GemvShape {
  int rpw, unroll, nt;
};
constexpr int GEMV_VARIANTS = 12;
constexpr int GEMV_DEFAULT = 4;  // rpw 4, unroll 1, cached loads
GemvShape gemv_shape(int variant);
inline int gemv_rows(int variant) { return 4 * gemv_shape(variant).rpw; }
// Matrix entries stored in FP64 or FP32; vectors and accumulation in FP64.
void gemv(const double* M, const int64_t* task, int64_t ntask, int64_t max_ld, const double* xg, double* v,
          double* part, const int* done, hipStream_t s, int variant, hipEvent_t ev_start = nullptr,
          hipEvent_t ev_stop = nullptr);
void gemv(const float* M, const int64_t* task, int64_t ntask, int64_t max_ld, const double* xg, double* v,
          double* part, const int* done, hipStream_t s, int variant, hipEvent_t ev_start = nullptr,
          hipEvent_t ev_stop = nullptr);
void to_float(const double* in, float* out, int64_t n, hipStream_t s);
// out[c] = sum_row Ht[c][row] * x[row]
void coarse_project(const double* Ht, int64_t n_gp, int64_t m_r, const double* x, double* out, hipStream_t s);
// q[row] = v[src0] - v[src1] + sum_c H[row][c] t[c]  (H may be null)
void combine(const double* v, const int64_t* row_src, int64_t m_r, const double* H, const double* t, int64_t n_gp,
             double* q, hipStream_t s);
int combine_blocks(int64_t m_r);
// scal: [0..1] rz (ping-pong by iteration parity par), [2] alpha, [3] beta, [4] rtol^2 ||b||^2, [5] ||r||^2
void pcg_F(const double* v, const int64_t* row_src, int64_t m_r, const double* H, const double* part_t,
           int64_t n_gp, int nblk, const double* part_g, int ngemv, const double* p, double* lam, double* r,
           double* xg_r, double* part_rr, double* scal, int par, int* done, int* err, hipStream_t s);
void pcg_M(const double* w, const int64_t* row_src, int64_t m_r, const double* H, int64_t n_gp, const double* part_g,
           int ngemv, const double* part_rr, int nblk, double* p, double* z, double* xg_p, double* part_t,
           double* scal, int par, int* done, int* iters, int init, hipStream_t s);

// ---- recovery / rhs helpers
void gather_add(const double* y, const int64_t* idx, double sgn, int64_t n, double* out, hipStream_t s);
void rhs_assemble(const double* y, const int64_t* A_aug, const int64_t* row_src, int64_t m_r, double* e, hipStream_t s);
void recovery_rhs(double* y, const int64_t* krp_ptr, const int64_t* krp_pos, const int32_t* krp_col,
                  const double* krp_val, int64_t nrows, const double* pglob, const int64_t* I_aug,
                  const int32_t* I_row, const double* I_sign, int64_t nslots, const double* lam, hipStream_t s);
void write_output(const double* y, const int64_t* src, const int64_t* edge, int64_t n, const double* pglob,
                  const int64_t* primal_edges, int64_t n_gp, double* a, hipStream_t s);
void axpy_rows(const double* H, const double* w, int64_t m, int64_t n, const double* e, double* b, hipStream_t s);
void vec_copy(const double* x, double* y, int64_t n, hipStream_t s);
// out = a x + b y
void axpby(const double* x, const double* y, double* out, double a, double b, int64_t n, hipStream_t s);
void dot_partial(const double* x, const double* y, int64_t n, double* part, hipStream_t s);

}  // namespace dev
}  // namespace ieti
