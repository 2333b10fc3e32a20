// Factorisation plan: ordering, tile structure and task lists of the batched
// partial Cholesky factorisation of every subdomain's augmented matrix
//
//     [ K_rr   K_rp   E_I ]      r = [r_V (nested dissection), r_I]
//     [ K_pr   K_pp   0   ]      p = local primal DOFs
//     [ E_I^T  0      0   ]      E_I selects the interface DOFs r_I
//
// Eliminating the r block leaves the trailing block
//
//     [ K_pp - K_pr K_rr^{-1} K_rp     -(K_rr^{-1} K_rp)_I^T ]
//     [ -(K_rr^{-1} K_rp)_I            -(K_rr^{-1})_II        ]
//
// i.e. the local coarse contribution (minus the paper's F, Section 2.1), the
// primal coupling of G and the local inverse block that W needs; after the
// r_V columns are eliminated the r_I block holds the Schur complement
// S_rIrI of the Dirichlet preconditioner (Eq. DirPrec).
#pragma once

#include <cstdint>
#include <vector>

#include "model.hpp"

namespace ieti {

struct SubPlan {
  int64_t nV = 0, nI = 0, nP = 0;      // true sizes
  int64_t nVp = 0, nIp = 0, nPp = 0;   // padded to the tile size
  int64_t nt = 0, ntV = 0, ntr = 0;    // tiles: total, r_V, r (= r_V + r_I)
  std::vector<int32_t> pos_of_local;   // local [r,p] index -> augmented position
  std::vector<int64_t> vdummy;         // augmented positions of identity dummies in the r_V block
  std::vector<int64_t> tile_off;       // nt*nt, lower tiles: pool offset or -1
  int64_t S_off = 0;                   // offset of the dense nIp x nIp S / Sinv blocks
  int64_t I_off = 0;                   // offset into the concatenated interface vectors
  int64_t P_off = 0;                   // offset into the concatenated local primal vectors
  int64_t r_off = 0;                   // offset into concatenated augmented vectors (nt*T each)
  int64_t Phi_off = 0;                 // dense nIp x nPp block (K_rr^{-1} K_rp)_I
  int64_t SPi_off = 0;                 // dense nPp x nPp local coarse block
  int32_t levS = 0;                    // level at whose start S_rIrI is complete
  int32_t nlev = 0;                    // number of levels of this subdomain
};

// Deferred tile updates: a target's pending contributions are issued once
// `defer` of them are pending (`defer_tail` inside a subdomain's dense r_I
// tail) or at the target's deadline.
struct PlanParams {
  int defer = 8;
  int defer_tail = 4;
};
struct Plan {
  int T = 64;
  int64_t pool_elems = 0;
  int64_t n_steps = 0;   // number of levels of the schedule
  int64_t inv_elems = 0;  // inverses of the factored diagonal tiles
  std::vector<SubPlan> sub;
  // per step, ranges into flat task arrays
  std::vector<int64_t> potrf_ptr, trsm_ptr, upd_ptr, copy_ptr;
  std::vector<int64_t> potrf_task;   // [off_jj, sub, off of L_jj^{-1}]
  std::vector<int64_t> trsm_task;    // [off_ij, off of L_jj^{-1}]
  std::vector<int64_t> upd_task;     // [off_il, first pair, pair count]
  std::vector<int64_t> upd_pair;     // [off_ij, off_lj]
  std::vector<int64_t> copy_task;    // [off_tile, dst_offset_in_S, ld (= nIp), transpose-needed]
  // scatter of the assembled entries into the tile pool
  std::vector<int64_t> scatter_dst;  // in destination order
  std::vector<double> scatter_val;
  std::vector<int64_t> tile_ptr;     // pool tile t (offset T*T*t): entries tile_ptr[t] .. tile_ptr[t + 1] - 1
  std::vector<int64_t> scatter_src;  // per entry: index into the concatenated CSR values, -1 = constant 1
                                     // (E_I), -2 - k = identity dummy of subdomain k
  // dense S / Sinv storage
  int64_t S_elems = 0;
  int64_t I_total = 0;   // sum nIp
  int64_t P_total = 0;   // sum nP
  int64_t r_total = 0;   // sum (nVp + nIp + nPp + nIp): augmented vectors
  int64_t Phi_elems = 0, SPi_elems = 0;
  // extraction after the factorisation: [off_tile, dst, dst_transposed or -1, ld, is_diag]
  std::vector<int64_t> xsinv_task, xphi_task, xspi_task;
  // triangular solves with the factor, per level: diag [off of L_jj^{-1}, vec_j],
  // update targets [vec_dst, first pair, pair count] with pairs [off_tile, vec_src]
  std::vector<int64_t> fdiag_ptr, fdiag_task, ffull_ptr, ffull_task, ffull_pair;
  std::vector<int64_t> bdiag_ptr, bdiag_task, bupd_ptr, bupd_task, bupd_pair;
  // interface gather/scatter: per padded interface slot, multiplier row (-1 = pad) and sign
  std::vector<int32_t> I_row;
  std::vector<double> I_sign;
  std::vector<int64_t> row_src;        // 2 per multiplier row: slots in the +1 and -1 subdomain
  std::vector<int64_t> I_aug;          // per padded interface slot: index into augmented vectors (I block)
  std::vector<int64_t> A_aug;          // per padded interface slot: index into augmented vectors (E_I block)
  // primal maps
  std::vector<int32_t> P_glob;         // per local primal slot: global primal index
  std::vector<int64_t> P_aug;          // per local primal slot: index into augmented vectors
  std::vector<int32_t> P_sub;          // per local primal slot: subdomain
  std::vector<int32_t> glob2loc;       // ragged: [g2l_off[k] + c] local primal slot of the c-th primal DOF of
                                       // subdomain k's problem within the subdomain, or -1
  std::vector<int64_t> g2l_off;        // N_sub + 1
  std::vector<int64_t> spi_off;        // per problem: offset of its dense coarse block (n_problems + 1)
  std::vector<int32_t> I_sub;          // per padded interface slot: subdomain
  // coarse matrix assembly: CSR over the entries of the per-problem blocks, sources in the SPi array
  std::vector<int64_t> spi_ptr, spi_src;
  // recovery without a forward sweep (one transposed update launch): target r column tile c,
  // pairs [tile (i, c) of a primal or E_I row tile i, vec of row tile i]
  std::vector<int64_t> rec_task, rec_pair;
  // every padded primal position of the augmented vectors and its global primal index (-1: padding)
  std::vector<int64_t> recP_pos, recP_glob;
  // output: augmented index and edge id of every owned r DOF
  std::vector<int64_t> out_src, out_edge;
  // initial augmented right-hand side [j_r; j_p; 0]
  std::vector<double> b_aug0;
  // per subdomain: pivot threshold of the factorisation, PIVOT_REL times the
  // largest diagonal entry of K_rr (also the value of its identity dummies,
  // which keeps them above the threshold at any scale)
  std::vector<double> piv_tol;
  static constexpr double PIVOT_REL = 1e-13;
  // per subdomain: level of each r column tile (the schedule's step), and the
  // parameters the update task lists were built with
  std::vector<std::vector<int32_t>> col_level;
  PlanParams params;
  double flops = 0.0;    // algorithmic flops of the tile factorisation
  // scalar-level work in the same elimination order, sum_j c_j^2 (no tiles,
  // no padding): of K_rr alone, and with the augmented trailing rows
  double flops_scalar_rr = 0.0, flops_scalar_aug = 0.0;
  double dense_flops = 0.0;
  int64_t n_update_tasks = 0;
};

// The coarse problem of every problem of a batch as a tile factorisation
// run by the same kernels as the local ones: the column block
//
//     [ S_c ]   n_gp x n_gp, symmetric positive definite (lower tiles)
//     [ G   ]   m_r  x n_gp
//     [ I   ]   n_gp x n_gp
//
// in 64x64 tiles; eliminating its n_gp columns (Cholesky of S_c, panel solves
// of the rows below, updates of the later columns) leaves L_c in the S_c
// tiles, H = G L_c^{-T} in the G tiles and L_c^{-T} in the identity tiles.
struct CoarseDims {
  int64_t m = 0, n = 0;       // multiplier rows and primal DOFs of the problem
  int64_t spi_off = 0;        // its dense row-major S_c (n x n) in the assembled coarse array
  int64_t g_off = 0;          // its dense row-major G / H (m x n); H^T (n x m) at the same offset
};
struct CoarsePlan {
  int64_t pool_elems = 0, inv_elems = 0;
  int64_t n_levels = 0;
  // tile fill: [off_tile, source (0: S_c, 1: G, -1: none), source offset, ld, rows, cols, identity]
  //   entry (a, b) = source[off + a ld + b] for a < rows, b < cols, else (identity && a == b)
  std::vector<int64_t> fill_task;
  // per level: ranges into the task arrays (formats of the local factorisation)
  std::vector<int64_t> potrf_ptr, trsm_ptr, upd_ptr;
  std::vector<int64_t> potrf_task;  // [off_cc, problem, off of L_cc^{-1}]
  std::vector<int64_t> trsm_task;   // [off_xc, off of L_cc^{-1}]
  std::vector<int64_t> upd_task;    // [off_target, first pair, pair count]
  std::vector<int64_t> upd_pair;    // [off_A, off_B]
  // extraction: [off_tile, dst offset, transposed dst offset or -1, ld, transposed ld, rows, cols]
  //   H and H^T from the G tiles (into the H / Ht arrays), L_c^{-T} (row-major n x n at
  //   spi_off) from the identity tiles
  std::vector<int64_t> out_h_task, out_l_task;
};
void build_coarse_plan(const std::vector<CoarseDims>& dims, int T, CoarsePlan& cp);

// ordering: 0 = nested dissection, 1 = natural
int build_plan(const Model& m, int T, int ordering, Plan& plan, Error& err, const PlanParams& pp = PlanParams());
// rebuild only the deferred-update task lists of a plan for new parameters
int build_update_tasks(Plan& plan, const PlanParams& pp, Error& err);
// recompute the value arrays (scatter_val, krp_val, b_aug0) from the model's
// current matrix values and loads; the structure is unchanged
void refill_values(const Model& m, Plan& plan);

}  // namespace ieti
