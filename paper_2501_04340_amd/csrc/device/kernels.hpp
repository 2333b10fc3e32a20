// Launch wrappers of the gfx950 kernels of the IETI-DP hot path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ieti {
namespace dev {

constexpr int TILE = 64;

// ---- factorisation (tile pool, column-major 64x64 tiles)
void fill(double* p, int64_t n, double v, hipStream_t s);
// out[dst[i]] = val[i], i < n (distinct destinations)
void scatter(double* out, const int64_t* dst, const double* val, int64_t n, hipStream_t s);
// the tile pool from the assembled entries (destination-ordered, tile t's in
// tile_ptr[t] .. tile_ptr[t + 1] - 1), every tile written whole
void assemble_tiles(double* pool, const int64_t* dst, const double* val, const int64_t* tile_ptr, int64_t ntile,
                    hipStream_t s);
// potrf task [off_jj, subdomain, off of the inverse]; writes L_jj and L_jj^{-1}; a pivot not
// above piv_tol[subdomain] flags the subdomain in err
void potrf_tiles(double* pool, double* inv, const int64_t* task, int64_t ntask, const double* piv_tol, int* err,
                 hipStream_t s);
// trsm task [off_ij, off of L_jj^{-1}]: L_ij = A_ij L_jj^{-T}
void trsm_tiles(double* pool, const double* inv, const int64_t* task, int64_t ntask, hipStream_t s);
// update task [off_C, first pair, pair count], pairs [off_A, off_B]: C -= sum A B^T;
// at most max_wgs workgroups (persistent), each walking its share of the tasks
constexpr int64_t UPDATE_WGS = 2048;
void update_tiles(double* pool, const int64_t* task, const int64_t* pair, int64_t ntask, hipStream_t s,
                  int64_t max_wgs = UPDATE_WGS);
// dst32 (optional): the same entries rounded to FP32, same layout
void copy_tiles(const double* pool, const int64_t* task, int64_t ntask, double scale, double* dst, hipStream_t s,
                float* dst32 = nullptr);

// ---- triangular solves with the tile factor (augmented vectors)
// diag task [off of L_jj^{-1}, vec_j]: y_j <- L_jj^{-1} y_j (or ^{-T})
void trsv_diag(const double* inv, const int64_t* task, int64_t ntask, double* y, bool transposed, hipStream_t s);
// update task [vec_dst, first pair, count], pairs [off_tile, vec_src]: y_dst -= sum L x (or L^T x)
void trsv_update(const double* pool, const int64_t* task, const int64_t* pair, int64_t ntask, double* y,
                 bool transposed, hipStream_t s);

// ---- problems of a batch (a single problem is a batch of one)
// Per-problem descriptor, PD_N int64 fields per problem: multiplier rows
// [MR0, MR1), global primal indices [GP0, GP0 + NGP), offsets of its blocks
// of H / G (row-major (MR1-MR0) x NGP), Ht (NGP x (MR1-MR0)) and of its dense
// coarse matrix (NGP x NGP), its row blocks [B0, B1), the offset of its
// H^T p block partials (NGP per row block), and its ranges of GEMV partials
// for the three row-streaming task lists (8, 16, 32 rows per workgroup) and
// the symmetric GEMV's output blocks: [T0 + 2i, T0 + 2i + 1), i < 4.
enum {
  PD_MR0 = 0, PD_MR1, PD_GP0, PD_NGP, PD_H, PD_HT, PD_SPI, PD_B0, PD_B1, PD_PT, PD_T0, PD_N = PD_T0 + 8
};
// Row blocks: blk[2b] = first multiplier row, blk[2b+1] = problem; at most 256 rows of one problem each.
struct Batch {
  const int64_t* pd = nullptr;
  const int64_t* blk = nullptr;
  int n_prob = 0;
  int n_blk = 0;
  int64_t n_gp_total = 0;
  int64_t max_gp = 0;
  // optional PCG coefficient record: hist[(p * hcap + i) * 2 + {0, 1}] = (alpha_i, beta_i)
  double* hist = nullptr;
  int hcap = 0;
};

// ---- coarse problem (per-problem dense blocks)
void sum_sources(const double* src, const int64_t* ptr, const int64_t* idx, int64_t nout, double* out, hipStream_t s);
// g2l[g2l_off[k] + c]: local primal slot of the c-th primal of subdomain k's problem, or -1
void build_G(const double* Phi, const int64_t* row_src, const int64_t* slot_phi_row, const int32_t* I_sub,
             const int32_t* g2l, const int64_t* g2l_off, double* G, const Batch& B, hipStream_t s);
// coarse tile factorisation helpers (tasks of CoarsePlan): dense row-major
// S_c / G blocks into tiles, tiles back into dense H, H^T and U = L_c^{-T}
void dense_to_tiles(double* pool, const int64_t* task, int64_t ntask, const double* S, const double* G,
                    hipStream_t s);
void tiles_to_dense(const double* pool, const int64_t* task, int64_t ntask, double* dst, double* dst_t, hipStream_t s);
// out_p = L_p^{-1} in_p (transposed = false) or L_p^{-T} in_p through U_p = L_p^{-T}
void tri_small_inv(const double* U, const double* in, double* out, bool transposed, const Batch& B, hipStream_t s);

// ---- interface operators and PCG (FP64 recurrences)
// xg[slot(+1)] = x[row], xg[slot(-1)] = -x[row]; with ds (per slot, may be null) the
// scaled jump operator of the preconditioner: xg[slot] = +-ds[slot] x[row]
void gather_rows(const double* x, const int64_t* row_src, int64_t m_r, double* xg, hipStream_t s,
                 const double* ds = nullptr);
// v[slot] = (M_k xg_k)[slot] for every interface slot; part[block] = sum xg.v over the block's rows.
// task [matrix row start, first slot, nrows, ld, first slot of the subdomain]; done (per problem,
// may be null) with task_prob skips the tasks of finished problems; ev_* may be null.
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
          double* part, const int* done, const int32_t* task_prob, hipStream_t s, int variant,
          hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
void gemv(const float* M, const int64_t* task, int64_t ntask, int64_t max_ld, const double* xg, double* v,
          double* part, const int* done, const int32_t* task_prob, hipStream_t s, int variant,
          hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// Symmetric variant: reads each lower 64x64 tile of the dense blocks once (the
// diagonal tile whole), SYM_TILES tiles of one tile row per task, writing a row
// partial for y_I and a column partial per tile for y_t (t < I) into the output
// blocks' contiguous partial lists; the reduction sums each 64-slot block's
// partials in list order and forms part_g per block.  Variant index GEMV_SYM
// (after the row-streaming shapes).
constexpr int SYM_TILES = 8;
constexpr int SYM_WAVES = 8;  // waves per task (64 / SYM_WAVES rows each)
constexpr int GEMV_SYM = GEMV_VARIANTS;
constexpr int GEMV_SHAPES = GEMV_VARIANTS + 1;
constexpr int SYM_TASK = 8 + SYM_TILES;  // int64 per task
struct SymGemv {
  // task: [matrix offset of tile (I, t0), ld, ncols, slot of tile row I, slot of tile column t0,
  //        destination of the row partial, rows of tile row I inside n_I, columns from t0 inside
  //        n_I, destinations of the SYM_TILES column partials (-1: none)]; the entries outside
  //        n_I (the padding of the last tile row and column) are not read
  const int64_t* task = nullptr;
  const int32_t* task_prob = nullptr;
  int64_t ntask = 0;
  const int64_t* blk = nullptr;       // [first slot, first partial, partial count] per output block of 64 slots
  const int32_t* blk_prob = nullptr;
  int64_t nblk = 0;
  double* part = nullptr;             // each block's partials contiguous: 64 entries apiece
};
// Reduction of the PCG's coarse block partials, t_p = H_p^T p = sum over the
// problem's row blocks of part_t, one task [problem, first column] per 64
// columns of a problem's n_gp; run by extra workgroups of the symmetric
// GEMV's block reduction (cr) or on its own (coarse_reduce).
struct CoarseReduce {
  const double* part_t = nullptr;
  const int64_t* task = nullptr;
  int64_t ntask = 0;
  double* t = nullptr;
};
void gemv_sym(const double* M, const SymGemv& g, const double* xg, double* v, double* part_g, const int* done,
              hipStream_t s, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr,
              const CoarseReduce* cr = nullptr, const Batch* B = nullptr);
void gemv_sym(const float* M, const SymGemv& g, const double* xg, double* v, double* part_g, const int* done,
              hipStream_t s, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr,
              const CoarseReduce* cr = nullptr, const Batch* B = nullptr);
void coarse_reduce(const CoarseReduce& c, const int* done, const Batch& B, hipStream_t s);
void to_float(const double* in, float* out, int64_t n, hipStream_t s);
// out[c] = sum over problem(c)'s rows of Ht[c][row] x[row]; cprob[c] = problem of global primal c
void coarse_project(const double* Ht, const double* x, double* out, const int32_t* cprob, const Batch& B,
                    hipStream_t s);
// q[row] = v[src0] - v[src1] + sum_c H_p[row][c] t_p[c], H_p read from its transpose Ht (may be null); with ds:
// ds[src0] v[src0] - ds[src1] v[src1]
void combine(const double* v, const int64_t* row_src, const double* Ht, const double* t, double* q, const Batch& B,
             hipStream_t s, const double* ds = nullptr);
// scal + 8 p: [0..1] rz (ping-pong by iteration parity par), [2] alpha, [3] beta, [4] tol^2, [5] ||r||^2;
// done / iters per problem; gt = index of the GEMV task list in use (part_g ranges);
// ds = per-slot scaling of the preconditioner's jump operator, or null (D_s = I)
// Ht: the transposed coarse rows (n_gp x m per problem); tvec: t = H^T p reduced by coarse_reduce
void pcg_F(const double* v, const int64_t* row_src, const double* Ht, const double* tvec, const double* part_g,
           const double* p, double* lam, double* r, double* xg_r, double* part_rr, double* scal, int par, int* done,
           int* err, const Batch& B, int gt, hipStream_t s, const double* ds);
// the same with FP32-stored coarse rows (inner PCG of the mixed path)
void pcg_F(const double* v, const int64_t* row_src, const float* Ht, const double* tvec, const double* part_g,
           const double* p, double* lam, double* r, double* xg_r, double* part_rr, double* scal, int par, int* done,
           int* err, const Batch& B, int gt, hipStream_t s, const double* ds);
void pcg_M(const double* w, const int64_t* row_src, const double* H, const double* part_g, const double* part_rr,
           double* p, double* z, double* xg_p, double* part_t, double* scal, int par, int* done, int* iters, int init,
           const Batch& B, int gt, hipStream_t s, const double* ds);
void pcg_M(const double* w, const int64_t* row_src, const float* H, const double* part_g, const double* part_rr,
           double* p, double* z, double* xg_p, double* part_t, double* scal, int par, int* done, int* iters, int init,
           const Batch& B, int gt, hipStream_t s, const double* ds);

// ---- recovery / rhs helpers
void gather_add(const double* y, const int64_t* idx, double sgn, int64_t n, double* out, hipStream_t s);
void rhs_assemble(const double* y, const int64_t* A_aug, const int64_t* row_src, int64_t m_r, double* e, hipStream_t s);
// y[p_pos[i]] = pglob[p_glob[i]] (0 where p_glob < 0), y[A_aug[t]] = I_sign[t] lam[I_row[t]] (0 where I_row < 0)
void recovery_sources(double* y, const int64_t* p_pos, const int64_t* p_glob, int64_t np, const double* pglob,
                      const int64_t* A_aug, const int32_t* I_row, const double* I_sign, int64_t nslots,
                      const double* lam, hipStream_t s);
void write_output(const double* y, const int64_t* src, const int64_t* edge, int64_t n, const double* pglob,
                  const int64_t* primal_edges, int64_t n_gp, double* a, hipStream_t s);
// b[row] = e[row] - sum_c H_p[row][c] w_p[c] (H_p read from its transpose Ht)
void axpy_rows(const double* Ht, const double* w, const double* e, double* b, const Batch& B, hipStream_t s);
void vec_copy(const double* x, double* y, int64_t n, hipStream_t s);
// out = a x + b y
void axpby(const double* x, const double* y, double* out, double a, double b, int64_t n, hipStream_t s);
// part[b] = sum over row block b of x y
void dot_blocks(const double* x, const double* y, double* part, const Batch& B, hipStream_t s);

}  // namespace dev
}  // namespace ieti
