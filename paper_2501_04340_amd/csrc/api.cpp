// C ABI of the IETI-DP library: host assembly, device factorisation and
// the PCG solve of the interface problem (Section 2.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "common.hpp"
#include "device/kernels.hpp"
#include "device/nn.hpp"
#include "host/model.hpp"
#include "host/plan.hpp"
#include "ietidp.h"
#include "nn_model.hpp"

namespace {

using ieti::rt::DBuf;
using ieti::rt::dalloc;
using ieti::rt::dupload;
using ieti::rt::fail;

// Named phase range for rocprofv3's marker trace (--marker-trace): pushed on
// construction, popped when the scope ends.
struct Phase {
  explicit Phase(const char* name) { roctxRangePushA(name); }
  ~Phase() { roctxRangePop(); }
  Phase(const Phase&) = delete;
  Phase& operator=(const Phase&) = delete;
};

}  // namespace

struct ieti_handle {
  ieti::Model model;
  ieti::Plan plan;
  int plan_T = 0, plan_ordering = -1;
  // factorisation parameters (deferral thresholds of the plan, persistent
  // update workgroups): in use, those the current plan was built with, and
  // the autotuner's record [defer, defer_tail, update workgroups, ms]
  ieti::PlanParams pparams, plan_pp;
  int64_t upd_wgs = ieti::dev::UPDATE_WGS;
  bool ftuned = false;
  std::vector<double> ftune_log;
  bool uploaded = false, factored = false;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  int device = -1;
  int64_t max_ld = 0;
  int nblk = 0;
  std::vector<int64_t> gemv_task_h[3];  // GEMV task lists for 8, 16 and 32 rows per workgroup
  // device buffers
  DBuf<double> piv_tol;  // per subdomain: pivot threshold of the factorisation
  DBuf<double> pool, inv, scatter_val, S, Sinv, Phi, SPi, Spi_glob, G, H, Ht, I_sign, b_aug0, y;
  // coarse problem as a tile factorisation: its tile pool, diagonal-tile
  // inverses, pivot thresholds (per problem), U = L_c^{-T} (dense per problem,
  // at the offsets of Spi_glob) and the task lists of CoarsePlan
  ieti::CoarsePlan cplan;
  DBuf<double> cpool, cinv, ctol, Lti;
  DBuf<int64_t> cfill, cpotrf, ctrsm, cupd, cupd_pair, cout_h, cout_l;
  DBuf<int64_t> scatter_dst, tile_ptr, potrf, trsm, upd, upd_pair, copyS, xsinv, xphi, xspi, fdiag, ffull, ffull_pair, rec_task, rec_pair;
  DBuf<int64_t> bdiag, bupd, bupd_pair;
  DBuf<int64_t> spi_ptr, spi_src, row_src, I_aug, A_aug, slot_phi_row, dsrc_ptr, dsrc_idx, recP_pos, recP_glob;
  DBuf<int64_t> out_src, out_edge, primal_edges, d_edges;  // d_edges: prescribed boundary coefficients
  DBuf<double> d_vals;
  DBuf<int64_t> gemv_tasks[3];
  int ngemv_r[3] = {0, 0, 0};
  int gvar[2] = {-1, -1};                              // GEMV launch shape for FP64 / FP32 blocks (-1 = untuned)
  float gtime[2][ieti::dev::GEMV_SHAPES] = {};        // autotuner: ms per launch of each shape
  // symmetric GEMV: tasks over lower tiles, output blocks, partial lists and buffer
  DBuf<int64_t> sym_task, sym_blk;
  DBuf<int32_t> sym_tprob, sym_bprob;
  DBuf<double> sym_part;
  ieti::dev::SymGemv symg;
  double sym_elems = 0.0;  // matrix entries read per symmetric application (lower tiles inside n_I)
  DBuf<int32_t> I_row, I_sub, glob2loc;
  DBuf<double> yj;  // L_rr^{-1} j_r of the right-hand side's forward solve (augmented layout)
  DBuf<double> lam, r, z, p, q, v, b, e, dtil, w, t, pglob, part, scal, aout, tmp;
  DBuf<double> xgp, xgr, part_g, part_t;  // gathered B^T p and B^T r, GEMV and coarse partials
  // reduction of the coarse partials into t = H^T p once per iteration: 64-column chunks per problem
  DBuf<int64_t> ctask_red;
  DBuf<double> tvec;
  ieti::dev::CoarseReduce cred;
  DBuf<double> lam_acc, rtrue;            // outer multipliers and FP64 residual (mixed precision)
  DBuf<float> S32, Sinv32;                // FP32 copies of S_rIrI and (K_rr^{-1})_II (mixed precision)
  DBuf<float> H32, Ht32;                  // FP32 copies of the coarse rows H and H^T (mixed precision)
  bool mixed = false;
  hipGraph_t graph = nullptr, graph32 = nullptr;
  hipGraphExec_t graph_exec = nullptr, graph_exec32 = nullptr;
  // launch sequences replayed every solve: [0] right-hand side, [1] recovery
  hipGraph_t seq_graph[2] = {nullptr, nullptr};
  hipGraphExec_t seq_exec[2] = {nullptr, nullptr};

  // learned warm start: a copy of the network, its row layout and work space
  struct Warm {
    bool on = false;
    ieti::nn::Mlp mlp;
    DBuf<float> theta, shift, scale, Cf;
    DBuf<int32_t> feat_patch, comb_patch, out_row;
    DBuf<int8_t> out_sign;
    ieti::nn::Work work;
    int n_facets = 0, n_feat = 0, n_comb = 0, n_out = 0;
    double out_scale = 1.0;
    void release() {
      for (auto* b : {&theta, &shift, &scale, &Cf}) b->release();
      for (auto* b : {&feat_patch, &comb_patch, &out_row}) b->release();
      out_sign.release();
      work.release();
      on = false;
    }
  } warm;
  DBuf<double> nu_d, lscale_d;  // per-patch reluctivity and load scale (warm-start features)

  // batch structure on the device (a single problem is a batch of one)
  DBuf<int64_t> pd, blk, g2l_off;
  DBuf<int32_t> cprob, task_prob[3];
  ieti::dev::Batch B;
  DBuf<double> hist;               // PCG coefficient record (B.hist), 2 * B.hcap per problem
  std::vector<int> hist_n;         // iterations of each problem's last PCG run
  std::vector<int64_t> pd_h, blk_h;
  DBuf<int> pdone, piters;                 // per problem: PCG finished (1 ok, 3 breakdown), iterations
  DBuf<double> dscale;                     // per interface slot: scaling of the preconditioner's jump operator
  int scaling = IETI_SCALE_IDENTITY;
  int* pflags_h = nullptr;                 // pinned host copy: done[n_prob], iters[n_prob]
  int* pchk_h = nullptr;                   // pinned: two slots of done[n_prob] for the convergence checks
  hipEvent_t ev_chk[2] = {nullptr, nullptr};
  // per-problem results of the last solve
  std::vector<int> p_iters, p_outer, p_status, p_warm;
  std::vector<double> p_relres, p_relres0;

  DBuf<int> flags;  // [0] err (factor), [3] pcg err, [4] coarse err
  int* flags_h = nullptr;
  double factor_ms = 0.0;
  double bnorm = 0.0;
  std::vector<double> lambda_h;
  bool rhs_ready = false;
  // kernel timing (event pairs around launches); kind 0 = FP64 GEMV, 1 = update, 2 = FP32 GEMV
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;  // (kind, index of start event)
  double k_count[3] = {0, 0, 0}, k_ms[3] = {0, 0, 0}, upd_tasks = 0;
  // per problem: sizes of the algorithmic byte model of one interface operator
  // application (entries of the lower triangles of the interface blocks,
  // sum n_I, sum n_I n_p) and the applications of the last solve by block
  // precision ([0] FP64, [1] FP32)
  std::vector<double> pb_entries, pb_sumI, pb_sumInp;
  std::vector<int> cntF[2], cntM[2];

  ~ieti_handle() {
    DBuf<double>* ds[] = {&piv_tol, &pool, &inv, &scatter_val, &S, &Sinv, &Phi, &SPi, &Spi_glob, &G, &H, &Ht, &I_sign, &b_aug0, &y,
                          &yj, &lam, &r, &z, &p, &q, &v, &b, &e, &dtil, &w, &t, &pglob, &part, &scal, &aout,
                          &tmp, &xgp, &xgr, &part_g, &part_t, &lam_acc, &rtrue, &cpool, &cinv, &ctol, &Lti, &tvec};
    for (auto* d : ds) d->release();
    DBuf<int64_t>* is[] = {&scatter_dst, &tile_ptr, &potrf, &trsm, &upd, &upd_pair, &copyS, &xsinv, &xphi, &xspi, &fdiag,
                           &ffull, &ffull_pair, &rec_task, &rec_pair, &bdiag, &bupd, &bupd_pair, &spi_ptr, &spi_src, &row_src, &I_aug, &A_aug, &slot_phi_row, &dsrc_ptr,
                           &dsrc_idx, &recP_pos, &recP_glob, &out_src, &out_edge, &primal_edges,
                           &gemv_tasks[0], &gemv_tasks[1], &gemv_tasks[2], &cfill, &cpotrf, &ctrsm, &cupd,
                           &cupd_pair, &cout_h, &cout_l, &ctask_red};
    for (auto* d : is) d->release();
    I_row.release();
    I_sub.release();
    d_edges.release();
    d_vals.release();
    hist.release();
    sym_task.release();
    sym_blk.release();
    sym_tprob.release();
    sym_bprob.release();
    sym_part.release();
    pd.release();
    blk.release();
    g2l_off.release();
    cprob.release();
    for (auto& t : task_prob) t.release();
    pdone.release();
    piters.release();
    dscale.release();
    if (pflags_h) (void)hipHostFree(pflags_h);
    if (pchk_h) (void)hipHostFree(pchk_h);
    for (auto e : ev_chk)
      if (e) (void)hipEventDestroy(e);
    glob2loc.release();
    flags.release();
    if (flags_h) (void)hipHostFree(flags_h);
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (ev2) (void)hipEventDestroy(ev2);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (graph_exec32) (void)hipGraphExecDestroy(graph_exec32);
    if (graph32) (void)hipGraphDestroy(graph32);
    for (int i = 0; i < 2; ++i) {
      if (seq_exec[i]) (void)hipGraphExecDestroy(seq_exec[i]);
      if (seq_graph[i]) (void)hipGraphDestroy(seq_graph[i]);
    }
    S32.release();
    Sinv32.release();
    H32.release();
    Ht32.release();
    warm.release();
    nu_d.release();
    lscale_d.release();
    if (own_stream) (void)hipStreamDestroy(own_stream);
  }
};

namespace {

int validate(const ieti_problem* pr) {
  if (!pr) return fail(IETI_ERR_INVALID_ARG, "problem is NULL");
  if (pr->version != IETI_ABI_VERSION) return fail(IETI_ERR_INVALID_ARG, "ABI version mismatch");
  if (pr->geom_kind != IETI_GEOM_BOX && pr->geom_kind != IETI_GEOM_ANNULUS)
    return fail(IETI_ERR_INVALID_ARG, "unknown geometry kind");
  for (int d = 0; d < 3; ++d)
    if (pr->patches[d] < 1) return fail(IETI_ERR_INVALID_ARG, "patch counts must be >= 1");
  if (pr->degree_p < 1 || pr->degree_p > 6) return fail(IETI_ERR_INVALID_ARG, "degree must be in 1..6");
  if (pr->n_el < 1) return fail(IETI_ERR_INVALID_ARG, "n_el must be >= 1");
  if (!pr->patch_to_subdomain || !pr->nu_per_patch || !pr->J)
    return fail(IETI_ERR_INVALID_ARG, "partition, reluctivity and source are required");
  if (pr->geom_kind == IETI_GEOM_ANNULUS) {
    if (!pr->periodic[0] || pr->periodic[1] || pr->periodic[2] || pr->patches[1] + 3 > 16)
      return fail(IETI_ERR_INVALID_ARG, "annulus needs periodic azimuth and at most 13 radial patches");
  } else {
    for (int d = 0; d < 3; ++d)
      if (pr->periodic[d]) return fail(IETI_ERR_INVALID_ARG, "box geometry cannot be periodic");
  }
  for (int d = 0; d < 3; ++d)
    if (pr->periodic[d] && pr->patches[d] < 3) return fail(IETI_ERR_INVALID_ARG, "periodic direction needs >= 3 patches");
  return IETI_OK;
}

int build_plan_if_needed(ieti_handle* h, int T, int ordering) {
  const bool same_structure = h->plan_T == T && h->plan_ordering == ordering;
  const bool same_params = h->plan_pp.defer == h->pparams.defer && h->plan_pp.defer_tail == h->pparams.defer_tail;
  if (same_structure && same_params) return IETI_OK;
  ieti::Error err{0, ""};
  if (same_structure) {
    // new deferral thresholds: only the update task lists change
    int rc = ieti::build_update_tasks(h->plan, h->pparams, err);
    if (rc) return fail(rc, err.msg);
    h->plan_pp = h->pparams;
    h->factored = false;
    if (h->uploaded) {
      if ((rc = dupload(h->upd, h->plan.upd_task))) return rc;
      if ((rc = dupload(h->upd_pair, h->plan.upd_pair))) return rc;
    }
    return IETI_OK;
  }
  int rc = ieti::build_plan(h->model, T, ordering, h->plan, err, h->pparams);
  if (rc) return fail(rc, err.msg);
  h->plan_T = T;
  h->plan_ordering = ordering;
  h->plan_pp = h->pparams;
  h->uploaded = false;
  h->factored = false;
  return IETI_OK;
}

void drop_graphs(ieti_handle* h) {
  for (hipGraphExec_t* g : {&h->graph_exec, &h->graph_exec32, &h->seq_exec[0], &h->seq_exec[1]})
    if (*g) {
      (void)hipGraphExecDestroy(*g);
      *g = nullptr;
    }
  for (hipGraph_t* g : {&h->graph, &h->graph32, &h->seq_graph[0], &h->seq_graph[1]})
    if (*g) {
      (void)hipGraphDestroy(*g);
      *g = nullptr;
    }
}

// Runs a launch sequence that is identical in every solve: captured into a
// graph on first use and replayed after that (direct launches if use_graph
// is false).
template <class F>
int run_sequence(ieti_handle* h, int which, bool use_graph, F&& body) {
  if (!use_graph) {
    body();
    return IETI_OK;
  }
  if (!h->seq_exec[which]) {
    HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    body();
    HIP_TRY(hipStreamEndCapture(h->stream, &h->seq_graph[which]));
    HIP_TRY(hipGraphInstantiate(&h->seq_exec[which], h->seq_graph[which], nullptr, nullptr, 0));
  }
  HIP_TRY(hipGraphLaunch(h->seq_exec[which], h->stream));
  return IETI_OK;
}

int upload(ieti_handle* h) {
  if (h->uploaded) return IETI_OK;
  const ieti::Plan& P = h->plan;
  const ieti::Model& M = h->model;
  HIP_TRY(hipGetDevice(&h->device));
  if (!h->own_stream) HIP_TRY(hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking));
  if (!h->ev0) {
    HIP_TRY(hipEventCreate(&h->ev0));
    HIP_TRY(hipEventCreate(&h->ev1));
    HIP_TRY(hipEventCreate(&h->ev2));
    HIP_TRY(hipEventCreateWithFlags(&h->ev_chk[0], hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&h->ev_chk[1], hipEventDisableTiming));
  }
  if (!h->flags_h) HIP_TRY(hipHostMalloc(&h->flags_h, 8 * sizeof(int)));
  int rc = 0;
#define UP(buf, vec) \
  if ((rc = dupload(h->buf, vec))) return rc;
  UP(scatter_dst, P.scatter_dst);
  UP(tile_ptr, P.tile_ptr);
  UP(scatter_val, P.scatter_val);
  UP(piv_tol, P.piv_tol);
  UP(potrf, P.potrf_task);
  UP(trsm, P.trsm_task);
  UP(upd, P.upd_task);
  UP(upd_pair, P.upd_pair);
  UP(ffull_pair, P.ffull_pair);
  UP(rec_pair, P.rec_pair);
  UP(bupd_pair, P.bupd_pair);
  UP(copyS, P.copy_task);
  UP(xsinv, P.xsinv_task);
  UP(xphi, P.xphi_task);
  UP(xspi, P.xspi_task);
  UP(fdiag, P.fdiag_task);
  UP(ffull, P.ffull_task);
  UP(rec_task, P.rec_task);
  UP(bdiag, P.bdiag_task);
  UP(bupd, P.bupd_task);
  UP(spi_ptr, P.spi_ptr);
  UP(spi_src, P.spi_src);
  for (int64_t v : P.row_src)
    if (v < 0) return fail(IETI_ERR_TREE, "a multiplier row does not join two interface slots");
  UP(row_src, P.row_src);
  UP(I_aug, P.I_aug);
  UP(A_aug, P.A_aug);
  UP(I_row, P.I_row);
  UP(I_sign, P.I_sign);
  UP(I_sub, P.I_sub);
  UP(glob2loc, P.glob2loc);
  UP(g2l_off, P.g2l_off);
  UP(recP_pos, P.recP_pos);
  UP(recP_glob, P.recP_glob);
  if ((rc = dalloc(h->yj, P.r_total))) return rc;
  UP(out_src, P.out_src);
  UP(out_edge, P.out_edge);
  UP(primal_edges, M.primal_edges);
  UP(d_edges, M.d_edges);
  UP(d_vals, M.d_vals);
  UP(b_aug0, P.b_aug0);
  // per interface slot: start of its row in Phi
  std::vector<int64_t> phirow(P.I_total, 0);
  h->max_ld = 0;
  for (auto& v : h->gemv_task_h) v.clear();
  const int n_prob = int(M.probs.size());
  h->pb_entries.assign(n_prob, 0.0);
  h->pb_sumI.assign(n_prob, 0.0);
  h->pb_sumInp.assign(n_prob, 0.0);
  for (size_t k = 0; k < P.sub.size(); ++k) {
    const auto& sp = P.sub[k];
    const int pk = M.sub_prob[k];
    h->pb_entries[pk] += 0.5 * double(sp.nI) * double(sp.nI + 1);
    h->pb_sumI[pk] += double(sp.nI);
    h->pb_sumInp[pk] += double(sp.nI) * double(sp.nP);
  }
  std::vector<int32_t> tprob[3];
  std::vector<int64_t> tstart(3 * (n_prob + 1), 0);  // per task list: first task of each problem
  for (size_t k = 0; k < P.sub.size(); ++k) {
    const auto& sp = P.sub[k];
    const int pk = M.sub_prob[k];
    for (int64_t t = 0; t < sp.nIp; ++t) phirow[sp.I_off + t] = sp.Phi_off + t * sp.nPp;
    h->max_ld = std::max(h->max_ld, sp.nIp);
    for (int ri = 0; ri < 3; ++ri) {
      const int64_t rows = 8 << ri;
      for (int64_t r0 = 0; r0 < sp.nIp; r0 += rows) {
        h->gemv_task_h[ri].insert(h->gemv_task_h[ri].end(), {sp.S_off + r0 * sp.nIp, sp.I_off + r0,
                                                             std::min<int64_t>(rows, sp.nIp - r0), sp.nIp, sp.I_off});
        tprob[ri].push_back(pk);
      }
      tstart[3 * (pk + 1) + ri] = int64_t(h->gemv_task_h[ri].size() / 5);
    }
  }
  for (int p = 1; p <= n_prob; ++p)  // problems without interface tasks inherit the previous end
    for (int ri = 0; ri < 3; ++ri) tstart[3 * p + ri] = std::max(tstart[3 * p + ri], tstart[3 * (p - 1) + ri]);
  // symmetric GEMV: per subdomain with nt = n_Ip / 64 tile rows, tasks (I, t0) over the lower tiles
  // t0 .. min(t0 + SYM_TILES, I + 1) - 1 of tile row I.  Output block J (64 slots) keeps its partials
  // contiguous: the row partials of its tasks (t0 ascending), then the column partials of tiles (I, J),
  // I > J (I ascending); its value is their sum in that order.  The launch order (below) only decides
  // which workgroup runs a task, never where its partials go.
  std::vector<int64_t> sym_task_h, sym_blk_h, bstart(n_prob + 1, 0);
  std::vector<int32_t> sym_tprob_h, sym_bprob_h;
  {
    const int64_t ST = ieti::dev::SYM_TILES;
    int64_t poff = 0;
    h->sym_elems = 0.0;
    std::vector<std::vector<int64_t>> by_size(ST + 1);  // task records by tile count
    std::vector<std::vector<int32_t>> prob_by_size(ST + 1);
    for (size_t k = 0; k < P.sub.size(); ++k) {
      const auto& sp = P.sub[k];
      const int pk = M.sub_prob[k];
      const int64_t nt = sp.nIp / 64;
      std::vector<int64_t> pbase(nt, 0);
      for (int64_t J = 0; J < nt; ++J) {
        const int64_t cnt = (J + ST) / ST + (nt - 1 - J);  // row partials + column partials
        pbase[J] = poff;
        poff += 64 * cnt;
        sym_blk_h.insert(sym_blk_h.end(), {sp.I_off + 64 * J, pbase[J], cnt});
        sym_bprob_h.push_back(pk);
      }
      bstart[pk + 1] = int64_t(sym_blk_h.size() / 3);
      for (int64_t I = 0; I < nt; ++I)
        for (int64_t t0 = 0; t0 <= I; t0 += ST) {
          const int64_t ntile = std::min(ST, I + 1 - t0);
          auto& rec = by_size[ntile];
          rec.insert(rec.end(), {sp.S_off + 64 * I * sp.nIp + 64 * t0, sp.nIp, 64 * ntile, sp.I_off + 64 * I,
                                 sp.I_off + 64 * t0, pbase[I] + 64 * (t0 / ST),
                                 std::min<int64_t>(64, sp.nI - 64 * I), std::min<int64_t>(64 * ntile, sp.nI - 64 * t0)});
          for (int64_t c = 0; c < ST; ++c) {
            const int64_t t = t0 + c;
            // column partial of tile (I, t), t < I: entry (t / ST + 1) + (I - t - 1) of block t
            rec.push_back(c < ntile && t < I ? pbase[t] + 64 * ((t + ST) / ST + (I - t - 1)) : -1);
          }
          prob_by_size[ntile].push_back(pk);
          h->sym_elems += double(std::min<int64_t>(64, sp.nI - 64 * I)) *
                          double(std::min<int64_t>(64 * ntile, sp.nI - 64 * t0));
        }
    }
    // Launch order.  The tile kernel holds two workgroups per CU; the first
    // n_cu workgroups take one CU each and the next n_cu the second slots in
    // the same order.  When the tasks fit in those two rounds, round one takes
    // the n_cu largest tasks and slot k of round two the task that evens out
    // CU k's tiles (the largest remaining task goes with the smallest
    // first-round task), with empty records (0 columns: the workgroup exits)
    // where a CU gets no second task.  Otherwise the tasks go largest first.
    {
      const size_t rec = size_t(ieti::dev::SYM_TASK);
      std::vector<std::pair<int64_t, int64_t>> order;  // (tile count, index within its size class)
      for (int64_t n = ST; n >= 1; --n)
        for (size_t i = 0; i < prob_by_size[n].size(); ++i) order.emplace_back(n, int64_t(i));
      int ncu = 0;
      if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) ncu = 0;
      const size_t nc = size_t(ncu > 0 ? ncu : 0), nt_all = order.size();
      auto put = [&](const std::pair<int64_t, int64_t>& o) {
        const auto& v = by_size[size_t(o.first)];
        sym_task_h.insert(sym_task_h.end(), v.begin() + o.second * int64_t(rec), v.begin() + (o.second + 1) * int64_t(rec));
        sym_tprob_h.push_back(prob_by_size[size_t(o.first)][size_t(o.second)]);
      };
      if (nc > 0 && nt_all > nc && nt_all <= 2 * nc) {
        for (size_t k = 0; k < nc; ++k) put(order[k]);
        std::vector<size_t> cu(nc);
        for (size_t k = 0; k < nc; ++k) cu[k] = k;
        std::stable_sort(cu.begin(), cu.end(), [&](size_t a, size_t b) { return order[a].first < order[b].first; });
        std::vector<int64_t> second(nc, -1);
        for (size_t j = nc; j < nt_all; ++j) second[cu[j - nc]] = int64_t(j);
        for (size_t k = 0; k < nc; ++k) {
          if (second[k] >= 0) {
            put(order[size_t(second[k])]);
          } else {
            sym_task_h.insert(sym_task_h.end(), rec, int64_t(0));
            for (size_t c = 0; c < size_t(ST); ++c) sym_task_h[sym_task_h.size() - size_t(ST) + c] = -1;
            sym_tprob_h.push_back(0);
          }
        }
      } else {
        for (const auto& o : order) put(o);
      }
    }
    for (int p = 1; p <= n_prob; ++p) bstart[p] = std::max(bstart[p], bstart[p - 1]);
    UP(sym_task, sym_task_h);
    UP(sym_tprob, sym_tprob_h);
    UP(sym_blk, sym_blk_h);
    UP(sym_bprob, sym_bprob_h);
    if ((rc = dalloc(h->sym_part, std::max<int64_t>(poff, 1)))) return rc;
    h->symg.task = h->sym_task.ptr;
    h->symg.task_prob = h->sym_tprob.ptr;
    h->symg.ntask = int64_t(sym_tprob_h.size());
    h->symg.blk = h->sym_blk.ptr;
    h->symg.blk_prob = h->sym_bprob.ptr;
    h->symg.nblk = int64_t(sym_blk_h.size() / 3);
    h->symg.part = h->sym_part.ptr;
  }
  UP(slot_phi_row, phirow);
  for (int ri = 0; ri < 3; ++ri) {
    UP(gemv_tasks[ri], h->gemv_task_h[ri]);
    UP(task_prob[ri], tprob[ri]);
    h->ngemv_r[ri] = int(h->gemv_task_h[ri].size() / 5);
  }
  // row blocks (<= 256 rows of one problem) and per-problem descriptors
  namespace D = ieti::dev;
  h->blk_h.clear();
  h->pd_h.assign(size_t(D::PD_N) * n_prob, 0);
  std::vector<int32_t> cprob_h;
  int64_t hoff = 0, ptoff = 0, max_gp = 0;
  for (int p = 0; p < n_prob; ++p) {
    const auto& pr = M.probs[p];
    int64_t* d = &h->pd_h[size_t(D::PD_N) * p];
    d[D::PD_MR0] = pr.mr_base;
    d[D::PD_MR1] = pr.mr_base + pr.m_r;
    d[D::PD_GP0] = pr.gp_base;
    d[D::PD_NGP] = pr.n_gp;
    d[D::PD_H] = hoff;
    d[D::PD_HT] = hoff;
    d[D::PD_SPI] = P.spi_off[p];
    d[D::PD_B0] = int64_t(h->blk_h.size() / 2);
    for (int64_t r0 = 0; r0 < pr.m_r; r0 += 256) h->blk_h.insert(h->blk_h.end(), {pr.mr_base + r0, int64_t(p)});
    d[D::PD_B1] = int64_t(h->blk_h.size() / 2);
    d[D::PD_PT] = ptoff;
    for (int ri = 0; ri < 3; ++ri) {
      d[D::PD_T0 + 2 * ri] = tstart[3 * p + ri];
      d[D::PD_T0 + 2 * ri + 1] = tstart[3 * (p + 1) + ri];
    }
    d[D::PD_T0 + 6] = bstart[p];
    d[D::PD_T0 + 7] = bstart[p + 1];
    hoff += pr.m_r * pr.n_gp;
    ptoff += (d[D::PD_B1] - d[D::PD_B0]) * pr.n_gp;
    max_gp = std::max(max_gp, pr.n_gp);
    for (int64_t c = 0; c < pr.n_gp; ++c) cprob_h.push_back(p);
  }
  UP(pd, h->pd_h);
  UP(blk, h->blk_h);
  UP(cprob, cprob_h);
  {
    std::vector<ieti::CoarseDims> cd(static_cast<size_t>(n_prob));
    for (int p = 0; p < n_prob; ++p) {
      const int64_t* d = &h->pd_h[size_t(D::PD_N) * p];
      cd[size_t(p)].m = d[D::PD_MR1] - d[D::PD_MR0];
      cd[size_t(p)].n = d[D::PD_NGP];
      cd[size_t(p)].spi_off = d[D::PD_SPI];
      cd[size_t(p)].g_off = d[D::PD_H];
    }
    ieti::build_coarse_plan(cd, D::TILE, h->cplan);
    const auto& C = h->cplan;
    UP(cfill, C.fill_task);
    UP(cpotrf, C.potrf_task);
    UP(ctrsm, C.trsm_task);
    UP(cupd, C.upd_task);
    UP(cupd_pair, C.upd_pair);
    UP(cout_h, C.out_h_task);
    UP(cout_l, C.out_l_task);
    // only non-positive pivots are flagged in the coarse matrix
    UP(ctol, std::vector<double>(size_t(n_prob), 0.0));
    std::vector<int64_t> ct;
    for (int p = 0; p < n_prob; ++p)
      for (int64_t c0 = 0; c0 < cd[size_t(p)].n; c0 += 64) ct.insert(ct.end(), {int64_t(p), c0});
    UP(ctask_red, ct);
  }
  h->B.pd = h->pd.ptr;
  h->B.blk = h->blk.ptr;
  h->B.n_prob = n_prob;
  h->B.n_blk = int(h->blk_h.size() / 2);
  h->B.n_gp_total = M.n_gp;
  h->B.max_gp = max_gp;
  // d~ assembly sources: for each global primal, the augmented indices of its local copies
  {
    std::vector<std::vector<int64_t>> src(M.n_gp);
    for (size_t s = 0; s < P.P_glob.size(); ++s) src[P.P_glob[s]].push_back(P.P_aug[s]);
    std::vector<int64_t> ptr(1, 0), idx;
    for (auto& v : src) {
      idx.insert(idx.end(), v.begin(), v.end());
      ptr.push_back(int64_t(idx.size()));
    }
    UP(dsrc_ptr, ptr);
    UP(dsrc_idx, idx);
  }
#undef UP
  const int64_t m_r = M.m_r, n_gp = M.n_gp;
  h->nblk = std::max(1, h->B.n_blk);
  if ((rc = dalloc(h->pool, P.pool_elems))) return rc;
  if ((rc = dalloc(h->inv, std::max<int64_t>(P.inv_elems, 1)))) return rc;
  if ((rc = dalloc(h->S, P.S_elems))) return rc;
  if ((rc = dalloc(h->Sinv, P.S_elems))) return rc;
  if ((rc = dalloc(h->Phi, std::max<int64_t>(P.Phi_elems, 1)))) return rc;
  if ((rc = dalloc(h->SPi, std::max<int64_t>(P.SPi_elems, 1)))) return rc;
  if ((rc = dalloc(h->Spi_glob, std::max<int64_t>(P.spi_off.back(), 1)))) return rc;
  if ((rc = dalloc(h->Lti, std::max<int64_t>(P.spi_off.back(), 1)))) return rc;
  if ((rc = dalloc(h->cpool, std::max<int64_t>(h->cplan.pool_elems, 1)))) return rc;
  if ((rc = dalloc(h->cinv, std::max<int64_t>(h->cplan.inv_elems, 1)))) return rc;
  if ((rc = dalloc(h->G, std::max<int64_t>(hoff, 1)))) return rc;
  if ((rc = dalloc(h->H, std::max<int64_t>(hoff, 1)))) return rc;
  if ((rc = dalloc(h->Ht, std::max<int64_t>(hoff, 1)))) return rc;
  if ((rc = dalloc(h->y, P.r_total))) return rc;
  const int64_t mm = std::max<int64_t>(m_r, 1), gg = std::max<int64_t>(n_gp, 1);
  DBuf<double>* vecs_m[] = {&h->lam, &h->r, &h->z, &h->p, &h->q, &h->b, &h->e, &h->tmp};
  for (auto* d : vecs_m)
    if ((rc = dalloc(*d, mm))) return rc;
  if ((rc = dalloc(h->v, std::max<int64_t>(P.I_total, 1)))) return rc;
  DBuf<double>* vecs_g[] = {&h->dtil, &h->w, &h->t, &h->pglob};
  for (auto* d : vecs_g)
    if ((rc = dalloc(*d, gg))) return rc;
  if ((rc = dalloc(h->part, 3 * int64_t(h->nblk)))) return rc;
  if ((rc = dalloc(h->xgp, std::max<int64_t>(P.I_total, 1)))) return rc;
  if ((rc = dalloc(h->xgr, std::max<int64_t>(P.I_total, 1)))) return rc;
  if ((rc = dalloc(h->part_g, std::max<int64_t>({int64_t(h->ngemv_r[0]), h->symg.nblk, int64_t(1)})))) return rc;
  if ((rc = dalloc(h->part_t, std::max<int64_t>(ptoff, 1)))) return rc;
  if ((rc = dalloc(h->tvec, std::max<int64_t>(M.n_gp, 1)))) return rc;
  h->cred.part_t = h->part_t.ptr;
  h->cred.task = h->ctask_red.ptr;
  h->cred.ntask = h->ctask_red.n / 2;
  h->cred.t = h->tvec.ptr;
  if ((rc = dalloc(h->pdone, n_prob))) return rc;
  if ((rc = dalloc(h->piters, n_prob))) return rc;
  if (h->pflags_h) (void)hipHostFree(h->pflags_h);
  h->pflags_h = nullptr;
  HIP_TRY(hipHostMalloc(&h->pflags_h, 2 * size_t(n_prob) * sizeof(int)));
  if (h->pchk_h) (void)hipHostFree(h->pchk_h);
  h->pchk_h = nullptr;
  HIP_TRY(hipHostMalloc(&h->pchk_h, 2 * size_t(n_prob) * sizeof(int)));
  if ((rc = dalloc(h->lam_acc, mm))) return rc;
  if ((rc = dalloc(h->rtrue, mm))) return rc;
  drop_graphs(h);
  if ((rc = dalloc(h->scal, 8 * int64_t(n_prob)))) return rc;
  if ((rc = dalloc(h->flags, 8))) return rc;
  if ((rc = dalloc(h->aout, M.n_edges_total))) return rc;
  h->uploaded = true;
  return IETI_OK;
}

hipStream_t pick_stream(ieti_handle* h, void* user) {
  return user ? reinterpret_cast<hipStream_t>(user) : h->own_stream;
}

hipEvent_t next_event(ieti_handle* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

// Record the start event of a timed launch; returns the slot or SIZE_MAX.
size_t prof_begin(ieti_handle* h) {
  if (!h->profiling) return SIZE_MAX;
  const size_t i = h->ev_used;
  hipEvent_t a = next_event(h), b = next_event(h);
  if (!a || !b) return SIZE_MAX;
  (void)hipEventRecord(a, h->stream);
  return i;
}

void prof_end(ieti_handle* h, size_t slot, int kind) {
  if (slot == SIZE_MAX) return;
  (void)hipEventRecord(h->ev_pool[slot + 1], h->stream);
  h->ev_marks.emplace_back(kind, slot);
}

// After the stream is synchronised: accumulate the recorded durations.
void prof_collect(ieti_handle* h) {
  for (const auto& m : h->ev_marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev_pool[m.second], h->ev_pool[m.second + 1]) == hipSuccess) {
      h->k_count[m.first] += 1.0;
      h->k_ms[m.first] += ms;
    }
  }
  h->ev_marks.clear();
  h->ev_used = 0;
}

// The local factorisations of every subdomain (Section 2.1, the blocks of
// K_rr): tile pool from the assembled values, then per level of the schedule
// the S_rIrI copies, diagonal-tile Cholesky, panel solves and deferred updates.
void enqueue_local_factor(ieti_handle* h, hipStream_t s, float* S32 = nullptr) {
  namespace D = ieti::dev;
  const auto& P = h->plan;
  D::assemble_tiles(h->pool.ptr, h->scatter_dst.ptr, h->scatter_val.ptr, h->tile_ptr.ptr,
                    int64_t(P.tile_ptr.size()) - 1, s);
  for (int64_t j = 0; j < P.n_steps; ++j) {
    D::copy_tiles(h->pool.ptr, h->copyS.ptr + 5 * P.copy_ptr[j], P.copy_ptr[j + 1] - P.copy_ptr[j], 1.0, h->S.ptr, s,
                  S32);
    D::potrf_tiles(h->pool.ptr, h->inv.ptr, h->potrf.ptr + 3 * P.potrf_ptr[j], P.potrf_ptr[j + 1] - P.potrf_ptr[j],
                   h->piv_tol.ptr, h->flags.ptr, s);
    D::trsm_tiles(h->pool.ptr, h->inv.ptr, h->trsm.ptr + 2 * P.trsm_ptr[j], P.trsm_ptr[j + 1] - P.trsm_ptr[j], s);
    const int64_t nupd = P.upd_ptr[j + 1] - P.upd_ptr[j];
    const size_t ev = nupd > 0 ? prof_begin(h) : SIZE_MAX;
    D::update_tiles(h->pool.ptr, h->upd.ptr + 3 * P.upd_ptr[j], h->upd_pair.ptr, nupd, s, h->upd_wgs);
    prof_end(h, ev, 1);
    if (ev != SIZE_MAX) {
      const int64_t* t = P.upd_task.data() + 3 * P.upd_ptr[j];
      for (int64_t q = 0; q < nupd; ++q) h->upd_tasks += double(t[3 * q + 2]);
    }
  }
}

// Autotuner of the factorisation's own parameters, run on the first
// factorisation of a handle that asks for it: the persistent update launch's
// workgroup count, then the deferral threshold before and inside the dense
// r_I tail (each a new plan), one parameter at a time, each candidate timed
// as the faster of two factorisations (after a warm-up run) on the handle's
// own matrices.  The
// winner is kept for the life of the handle (later factorisations are
// bitwise repeatable).
int tune_factor(ieti_handle* h, int T, int ordering, void* user_stream) {
  h->ftune_log.clear();
  auto time_it = [&](double* ms_out) -> int {
    int rc = build_plan_if_needed(h, T, ordering);
    if (rc) return rc;
    rc = upload(h);
    if (rc) return rc;
    hipStream_t s = pick_stream(h, user_stream);
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      HIP_TRY(hipEventRecord(h->ev0, s));
      enqueue_local_factor(h, s);
      HIP_TRY(hipEventRecord(h->ev1, s));
      HIP_TRY(hipEventSynchronize(h->ev1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
      if (rep > 0) best = std::min(best, ms);  // the first run warms the caches and the code
    }
    *ms_out = double(best);
    h->ftune_log.insert(h->ftune_log.end(),
                        {double(h->pparams.defer), double(h->pparams.defer_tail), double(h->upd_wgs), *ms_out});
    return IETI_OK;
  };
  // a candidate replaces the current parameters only when it is faster by
  // more than the timing noise, so that repeated tunings settle on the same
  // choice (and so on the same task lists)
  constexpr double margin = 0.99;
  double best_ms = 0.0, ms = 0.0;
  int rc = time_it(&best_ms);
  if (rc) return rc;
  int64_t best_w = h->upd_wgs;
  for (int64_t w : {int64_t(512), int64_t(1024), int64_t(2048)}) {
    if (w == best_w) continue;
    h->upd_wgs = w;
    if ((rc = time_it(&ms))) return rc;
    if (ms < margin * best_ms) {
      best_ms = ms;
      best_w = w;
    }
  }
  h->upd_wgs = best_w;
  for (int pass = 0; pass < 2; ++pass) {
    const int cand[3] = {pass == 0 ? 4 : 2, pass == 0 ? 12 : 6, pass == 0 ? 16 : 8};
    ieti::PlanParams best_p = h->pparams;
    for (int c : cand) {
      ieti::PlanParams tryp = best_p;
      (pass == 0 ? tryp.defer : tryp.defer_tail) = c;
      h->pparams = tryp;
      if ((rc = time_it(&ms))) return rc;
      if (ms < margin * best_ms) {
        best_ms = ms;
        best_p = tryp;
      }
    }
    h->pparams = best_p;
  }
  h->ftuned = true;
  return IETI_OK;
}

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(IETI_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return IETI_OK;
}

// per-slot scaling of the preconditioner's jump operator, or null for D_s = I
const double* dsc(const ieti_handle* h) { return h->scaling == IETI_SCALE_IDENTITY ? nullptr : h->dscale.ptr; }

// Algorithmic bytes of one application of the interface operator (is_F) or
// of the preconditioner for problem p, with s-byte interface-block entries:
// the lower triangle of every symmetric interface block once
// (s sum n_I (n_I + 1) / 2), the interface vectors in and out (16 sum n_I),
// three multiplier vectors (24 m_r), and for the operator the local primal
// coupling in and out (16 sum n_I n_p) and the coarse factor (8 n_gp^2).
double alg_bytes(const ieti_handle* h, int p, double s, bool is_F) {
  const auto& pr = h->model.probs[p];
  double b = s * h->pb_entries[p] + 16.0 * h->pb_sumI[p] + 24.0 * double(pr.m_r);
  if (is_F) b += 16.0 * h->pb_sumInp[p] + 8.0 * double(pr.n_gp) * double(pr.n_gp);
  return b;
}

double problem_pcg_bytes(const ieti_handle* h, int p) {
  double b = 0.0;
  for (int f = 0; f < 2; ++f) {
    const double s = f ? 4.0 : 8.0;
    if (p < int(h->cntF[f].size())) b += h->cntF[f][p] * alg_bytes(h, p, s, true);
    if (p < int(h->cntM[f].size())) b += h->cntM[f][p] * alg_bytes(h, p, s, false);
  }
  return b;
}

// one more application on every problem of the batch
void count_all(std::vector<int>& c) {
  for (int& v : c) ++v;
}

// GEMV launch shape in use for FP64 (fp32 = 0) or FP32 (1) blocks, its task list and task count
int gvariant(const ieti_handle* h, int fp32) { return h->gvar[fp32] >= 0 ? h->gvar[fp32] : ieti::dev::GEMV_DEFAULT; }

// One interface GEMV application with launch shape `variant` (row-streaming
// shapes, or the symmetric lower-tile kernel); partials in part_g by the
// variant's task list (index variant / 4 in the problem descriptors).
// With coarse = true the same step also reduces the coarse partials of the
// PCG (t = H^T p, for the operator's second half): in extra workgroups of the
// symmetric kernel's block reduction, else in a launch of its own.
template <typename MT>
void launch_gemv(ieti_handle* h, const MT* M, int variant, const double* xg, double* v, const int* done,
                 hipEvent_t a = nullptr, hipEvent_t b = nullptr, bool coarse = false) {
  namespace D = ieti::dev;
  const bool cr = coarse && h->cred.ntask > 0;
  if (variant == D::GEMV_SYM) {
    D::gemv_sym(M, h->symg, xg, v, h->part_g.ptr, done, h->stream, a, b, cr ? &h->cred : nullptr, &h->B);
    return;
  }
  const int ri = variant / 4;
  D::gemv(M, h->gemv_tasks[ri].ptr, h->ngemv_r[ri], h->max_ld, xg, v, h->part_g.ptr, done, h->task_prob[ri].ptr,
          h->stream, variant, a, b);
  if (cr) D::coarse_reduce(h->cred, done, h->B, h->stream);
}

// Interface GEMV over all subdomains, timed with launch events when profiling.
template <typename MT>
void gemv_timed(ieti_handle* h, const MT* M, const double* xg, double* v, const int* done = nullptr,
                bool coarse = false) {
  const int fp32 = std::is_same<MT, float>::value ? 1 : 0;
  hipEvent_t a = nullptr, b = nullptr;
  size_t slot = SIZE_MAX;
  if (h->profiling) {
    slot = h->ev_used;
    a = next_event(h);
    b = next_event(h);
    if (!a || !b) a = b = nullptr;
  }
  launch_gemv(h, M, gvariant(h, fp32), xg, v, done, a, b, coarse);
  if (a) h->ev_marks.emplace_back(fp32 ? 2 : 0, slot);
}

// q = F x = sum_k B_k (K_rr^(k))^{-1}_II B_k^T x + H (H^T x)
void apply_F(ieti_handle* h, const double* x, double* out) {
  namespace D = ieti::dev;
  const auto& M = h->model;
  hipStream_t s = h->stream;
  D::gather_rows(x, h->row_src.ptr, M.m_r, h->xgp.ptr, s);
  gemv_timed(h, h->Sinv.ptr, h->xgp.ptr, h->v.ptr);
  if (M.n_gp > 0) D::coarse_project(h->Ht.ptr, x, h->t.ptr, h->cprob.ptr, h->B, s);
  D::combine(h->v.ptr, h->row_src.ptr, M.n_gp > 0 ? h->Ht.ptr : nullptr, h->t.ptr, out, h->B, s);
}

// z = M_D^{-1} x = sum_k B_k S_rIrI^(k) B_k^T x  (D_s = I)
void apply_M(ieti_handle* h, const double* x, double* out) {
  namespace D = ieti::dev;
  const auto& M = h->model;
  hipStream_t s = h->stream;
  D::gather_rows(x, h->row_src.ptr, M.m_r, h->xgr.ptr, s, dsc(h));
  gemv_timed(h, h->S.ptr, h->xgr.ptr, h->v.ptr);
  D::combine(h->v.ptr, h->row_src.ptr, nullptr, nullptr, out, h->B, s, dsc(h));
}

// Coarse rows H (or H^T) stored in the precision MT of the interface blocks.
template <typename MT>
const MT* coarse_rows(const ieti_handle* h, bool transposed);
template <>
const double* coarse_rows<double>(const ieti_handle* h, bool transposed) {
  return transposed ? h->Ht.ptr : h->H.ptr;
}
template <>
const float* coarse_rows<float>(const ieti_handle* h, bool transposed) {
  return transposed ? h->Ht32.ptr : h->H32.ptr;
}

// One PCG iteration of parity `par` as four launches, with the interface
// blocks stored as MT (FP64, or FP32 in the inner solves of the mixed path).
template <typename MT>
void pcg_iteration(ieti_handle* h, int par, const MT* Sinv, const MT* S) {
  namespace D = ieti::dev;
  hipStream_t s = h->stream;
  int* done = h->pdone.ptr;
  int* iters = h->piters.ptr;
  int* perr = h->flags.ptr + 3;
  double* part_rr = h->part.ptr + h->nblk;
  const int fp32 = std::is_same<MT, float>::value ? 1 : 0;
  const int gt = gvariant(h, fp32) / 4;
  // the coarse rows in the blocks' precision (the inner solves of the mixed path read FP32 copies)
  const MT* H = coarse_rows<MT>(h, false);
  const MT* Ht = coarse_rows<MT>(h, true);
  gemv_timed(h, Sinv, h->xgp.ptr, h->v.ptr, done, true);
  D::pcg_F(h->v.ptr, h->row_src.ptr, Ht, h->tvec.ptr, h->part_g.ptr, h->p.ptr, h->lam.ptr, h->r.ptr,
           h->xgr.ptr, part_rr, h->scal.ptr, par, done, perr, h->B, gt, s, dsc(h));
  gemv_timed(h, S, h->xgr.ptr, h->v.ptr, done);
  D::pcg_M(h->v.ptr, h->row_src.ptr, H, h->part_g.ptr, part_rr, h->p.ptr, h->z.ptr, h->xgp.ptr,
           h->part_t.ptr, h->scal.ptr, par, done, iters, 0, h->B, gt, s, dsc(h));
}

void pcg_iteration_prec(ieti_handle* h, int par, bool fp32) {
  if (fp32) pcg_iteration<float>(h, par, h->Sinv32.ptr, h->S32.ptr);
  else pcg_iteration<double>(h, par, h->Sinv.ptr, h->S.ptr);
}


// Autotuner of the interface GEMV: every launch shape is timed on the
// handle's own blocks, alternating the operator and preconditioner blocks as
// the PCG does (so the caches see the same working set): 2 warm-up and 5
// timed pairs per shape, HIP events on the solve stream, in three rounds
// over all shapes; a shape's time is its fastest round (the shapes differ by
// a few per cent, less than the spread of a single round) and the fastest
// shape is kept.  Runs once per handle and precision, after the first
// factorisation, so later solves are repeatable.
template <typename MT>
int tune_gemv(ieti_handle* h, const MT* Ma, const MT* Mb, int fp32) {
  namespace D = ieti::dev;
  hipStream_t s = h->stream;
  float tmin[D::GEMV_SHAPES];
  for (int v = 0; v < D::GEMV_SHAPES; ++v) tmin[v] = 1e30f;
  for (int round = 0; round < 3; ++round)
    for (int v = 0; v < D::GEMV_SHAPES; ++v) {
      auto launch = [&]() {
        launch_gemv(h, Ma, v, h->xgp.ptr, h->v.ptr, nullptr);
        launch_gemv(h, Mb, v, h->xgr.ptr, h->v.ptr, nullptr);
      };
      launch();
      launch();
      HIP_TRY(hipEventRecord(h->ev0, s));
      for (int k = 0; k < 5; ++k) launch();
      HIP_TRY(hipEventRecord(h->ev1, s));
      HIP_TRY(hipEventSynchronize(h->ev1));
      int rc = check_launch();
      if (rc) return rc;
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
      tmin[v] = std::min(tmin[v], ms / 10.f);
    }
  int bv = D::GEMV_DEFAULT;
  for (int v = 0; v < D::GEMV_SHAPES; ++v) {
    h->gtime[fp32][v] = tmin[v];
    if (tmin[v] < tmin[bv]) bv = v;
  }
  if (h->gvar[fp32] != bv) drop_graphs(h);
  h->gvar[fp32] = bv;
  return IETI_OK;
}

int choose_gemv(ieti_handle* h, int forced, int fp32) {
  if (forced > 0) {
    if (h->gvar[fp32] != forced - 1) drop_graphs(h);
    h->gvar[fp32] = forced - 1;
    return IETI_OK;
  }
  if (h->gvar[fp32] >= 0 || h->plan.S_elems == 0) return IETI_OK;
  return fp32 ? tune_gemv(h, h->Sinv32.ptr, h->S32.ptr, 1) : tune_gemv(h, h->Sinv.ptr, h->S.ptr, 0);
}

// Scaling of the preconditioner's jump operator (beyond the paper's
// D_s = I): every multiplier row joins two interface slots s0 (+1) and s1
// (-1); rho-scaling gives them delta_s0 = rho_s1 / (rho_s0 + rho_s1) and
// delta_s1 = rho_s0 / (rho_s0 + rho_s1), with rho the diagonal entry of the
// slot's subdomain stiffness at that DOF (it carries the local
// reluctivity); multiplicity scaling gives 1/2.
int set_scaling(ieti_handle* h, int kind) {
  const double* before = dsc(h);
  if (kind != IETI_SCALE_IDENTITY) {
    const auto& P = h->plan;
    const auto& M = h->model;
    std::vector<double> rho(std::max<int64_t>(P.I_total, 1), 0.0), d(std::max<int64_t>(P.I_total, 1), 0.0);
    for (size_t k = 0; k < P.sub.size(); ++k) {
      const auto& s = M.sd[k];
      for (int64_t t = 0; t < P.sub[k].nI; ++t) {
        const int32_t r = s.I_local[t];
        double dg = 0.0;
        for (int64_t q = s.indptr[r]; q < s.indptr[r + 1]; ++q)
          if (s.indices[q] == r) dg = s.values[q];
        rho[P.sub[k].I_off + t] = dg;
      }
    }
    for (int64_t row = 0; row < M.m_r; ++row) {
      const int64_t s0 = P.row_src[2 * row], s1 = P.row_src[2 * row + 1];
      if (kind == IETI_SCALE_MULTIPLICITY) {
        d[s0] = d[s1] = 0.5;
      } else {
        const double a = rho[s0], b = rho[s1];
        if (!(a > 0.0) || !(b > 0.0)) return fail(IETI_ERR_NOT_SPD, "non-positive stiffness diagonal on an interface");
        d[s0] = b / (a + b);
        d[s1] = a / (a + b);
      }
    }
    if (h->dscale.ptr && h->dscale.n == int64_t(d.size())) {
      HIP_TRY(hipMemcpy(h->dscale.ptr, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
      int rc = dupload(h->dscale, d);
      if (rc) return rc;
    }
  }
  h->scaling = kind;
  if (dsc(h) != before) drop_graphs(h);  // captured graphs hold the scaling pointer (or its absence)
  return IETI_OK;
}

// Capture two PCG iterations (parities 0 and 1) as one graph per precision.
int capture_graph(ieti_handle* h, bool fp32) {
  hipGraph_t& g = fp32 ? h->graph32 : h->graph;
  hipGraphExec_t& ge = fp32 ? h->graph_exec32 : h->graph_exec;
  if (ge) return IETI_OK;
  HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  pcg_iteration_prec(h, 0, fp32);
  pcg_iteration_prec(h, 1, fp32);
  HIP_TRY(hipStreamEndCapture(h->stream, &g));
  HIP_TRY(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
  return IETI_OK;
}

// Forward solve with the factor over all augmented rows (full) or r rows only.
void forward_solve(ieti_handle* h) {
  namespace D = ieti::dev;
  const auto& P = h->plan;
  for (int64_t j = 0; j < P.n_steps; ++j) {
    D::trsv_diag(h->inv.ptr, h->fdiag.ptr + 2 * P.fdiag_ptr[j], P.fdiag_ptr[j + 1] - P.fdiag_ptr[j], h->y.ptr, false,
                 h->stream);
    D::trsv_update(h->pool.ptr, h->ffull.ptr + 3 * P.ffull_ptr[j], h->ffull_pair.ptr,
                   P.ffull_ptr[j + 1] - P.ffull_ptr[j], h->y.ptr, false, h->stream);
  }
}

void backward_solve(ieti_handle* h) {
  namespace D = ieti::dev;
  const auto& P = h->plan;
  for (int64_t s = 0; s < P.n_steps; ++s) {
    D::trsv_diag(h->inv.ptr, h->bdiag.ptr + 2 * P.bdiag_ptr[s], P.bdiag_ptr[s + 1] - P.bdiag_ptr[s], h->y.ptr, true,
                 h->stream);
    D::trsv_update(h->pool.ptr, h->bupd.ptr + 3 * P.bupd_ptr[s], h->bupd_pair.ptr, P.bupd_ptr[s + 1] - P.bupd_ptr[s],
                   h->y.ptr, true, h->stream);
  }
}

// Right-hand side b = e - G S_c^{-1} d~ (positive definite form of Eq. intProb).
int compute_rhs(ieti_handle* h, bool use_graph) {
  namespace D = ieti::dev;
  const auto& P = h->plan;
  const auto& M = h->model;
  hipStream_t s = h->stream;
  int rc = run_sequence(h, 0, use_graph, [&]() {
    D::vec_copy(h->b_aug0.ptr, h->y.ptr, P.r_total, s);
    forward_solve(h);
    D::vec_copy(h->y.ptr, h->yj.ptr, P.r_total, s);  // kept for the recovery
    D::rhs_assemble(h->y.ptr, h->A_aug.ptr, h->row_src.ptr, M.m_r, h->e.ptr, s);
    if (M.n_gp > 0) {
      D::sum_sources(h->y.ptr, h->dsrc_ptr.ptr, h->dsrc_idx.ptr, M.n_gp, h->dtil.ptr, s);
      D::tri_small_inv(h->Lti.ptr, h->dtil.ptr, h->w.ptr, false, h->B, s);
      D::axpy_rows(h->Ht.ptr, h->w.ptr, h->e.ptr, h->b.ptr, h->B, s);
    } else {
      D::vec_copy(h->e.ptr, h->b.ptr, M.m_r, s);
    }
  });
  if (rc) return rc;
  h->rhs_ready = true;
  return check_launch();
}

// Per-problem dot products x.y (block partials on the device, summed in
// block order on the host).
std::vector<double> host_dots(ieti_handle* h, const double* x, const double* y) {
  const int n_prob = h->B.n_prob;
  std::vector<double> out(n_prob, 0.0);
  if (h->B.n_blk <= 0) return out;
  ieti::dev::dot_blocks(x, y, h->part.ptr, h->B, h->stream);
  std::vector<double> part(h->B.n_blk);
  (void)hipMemcpyAsync(part.data(), h->part.ptr, part.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
  (void)hipStreamSynchronize(h->stream);
  for (int b = 0; b < h->B.n_blk; ++b) out[h->blk_h[2 * b + 1]] += part[b];
  return out;
}

// lambda_0 from the attached network: features from the per-patch
// coefficients, forward pass, weighted sum of the output groups, scatter
// into the multiplier rows.
void warm_predict(ieti_handle* h, double* lam) {
  namespace N = ieti::nn;
  auto& W = h->warm;
  hipStream_t s = h->stream;
  N::features(h->nu_d.ptr, h->lscale_d.ptr, W.feat_patch.ptr, W.shift.ptr, W.scale.ptr, W.n_facets, W.n_feat,
              W.comb_patch.ptr, W.n_comb, W.work.H[0].ptr, W.Cf.ptr, s);
  N::forward(W.mlp, W.theta.ptr, W.n_facets, W.work, s);
  N::combine_loss(W.work.Y.ptr, W.Cf.ptr, nullptr, W.n_facets, W.n_comb, W.n_out, W.work.pred.ptr, nullptr, nullptr,
                  s);
  ieti::dev::fill(lam, h->model.m_r, 0.0, s);
  N::scatter_prediction(W.work.pred.ptr, W.out_row.ptr, W.out_sign.ptr, int64_t(W.n_facets) * W.n_out, W.out_scale,
                        lam, s);
}

// Initial multipliers lam0 and residual r0 = b - F lam0 (rr0[p] = ||r0_p||^2
// per problem): the caller's lambda0, else the network's prediction (dropped
// for 0, per problem, when its residual is not below ||b_p|| or not finite),
// else 0.  warm[p]: 1 prediction used, -1 rejected, 0 not asked.
int init_lambda(ieti_handle* h, const ieti_solve_opts* opts, const std::vector<double>& bb, double* lam0, double* r0,
                std::vector<double>& rr0, int* applies, std::vector<int>& warm) {
  namespace D = ieti::dev;
  const int64_t m_r = h->model.m_r;
  const int n_prob = h->B.n_prob;
  hipStream_t s = h->stream;
  warm.assign(n_prob, 0);
  bool have = false;
  if (opts && opts->lambda0) {
    HIP_TRY(hipMemcpyAsync(lam0, opts->lambda0, m_r * sizeof(double), hipMemcpyHostToDevice, s));
    have = true;
  } else if (opts && opts->warm_start) {
    if (!h->warm.on) return fail(IETI_ERR_STATE, "warm_start requested but no network is attached");
    warm_predict(h, lam0);
    have = true;
    warm.assign(n_prob, 1);
  }
  if (have) {
    apply_F(h, lam0, h->q.ptr);
    ++*applies;
    count_all(h->cntF[0]);
    D::axpby(h->b.ptr, h->q.ptr, r0, 1.0, -1.0, m_r, s);
    rr0 = host_dots(h, r0, r0);
    for (int p = 0; p < n_prob; ++p)
      if (warm[p] == 1 && !(std::isfinite(rr0[p]) && rr0[p] < bb[p])) {
        const int64_t* d = &h->pd_h[size_t(D::PD_N) * p];
        const int64_t r0w = d[D::PD_MR0], nr = d[D::PD_MR1] - d[D::PD_MR0];
        D::fill(lam0 + r0w, nr, 0.0, s);
        D::vec_copy(h->b.ptr + r0w, r0 + r0w, nr, s);
        rr0[p] = bb[p];
        warm[p] = -1;
      }
  } else {
    D::fill(lam0, m_r, 0.0, s);
    D::vec_copy(h->b.ptr, r0, m_r, s);
    rr0 = bb;
  }
  return check_launch();
}

// PCG on F x = r_0 for every problem of the batch at once from the state
// prepared by the caller (x in h->lam, r_0 in h->r with ||r_0,p||^2 =
// rr0[p]); problem p stops when ||r_p||^2 <= tol2[p] (it is frozen while the
// others go on), all stop at maxit iterations.
int run_pcg(ieti_handle* h, const std::vector<double>& tol2, const std::vector<double>& rr0, int maxit, int every,
            bool fp32, bool use_graph, std::vector<int>& iters_out, std::vector<double>& rr_out,
            std::vector<int>& status) {
  namespace D = ieti::dev;
  const auto& M = h->model;
  hipStream_t s = h->stream;
  const int64_t m_r = M.m_r;
  const int n_prob = h->B.n_prob;
  double* part_rr = h->part.ptr + h->nblk;
  iters_out.assign(n_prob, 0);
  rr_out = rr0;
  status.assign(n_prob, IETI_OK);
  std::vector<int> done0(n_prob, 0);
  bool all = true;
  for (int p = 0; p < n_prob; ++p) {
    done0[p] = rr0[p] <= tol2[p] ? 1 : 0;
    all = all && done0[p];
  }
  if (all) return IETI_OK;
  count_all(h->cntM[fp32 ? 1 : 0]);  // z_0 = M r_0 below, every problem
  std::vector<double> sc(8 * size_t(n_prob), 0.0);
  for (int p = 0; p < n_prob; ++p) {
    sc[8 * p + 4] = tol2[p];
    sc[8 * p + 5] = rr0[p];
  }
  HIP_TRY(hipMemcpyAsync(h->scal.ptr, sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->pdone.ptr, done0.data(), n_prob * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(h->piters.ptr, 0, n_prob * sizeof(int), s));
  HIP_TRY(hipMemsetAsync(h->flags.ptr + 3, 0, sizeof(int), s));
  if (h->B.hist) D::fill(h->B.hist, 2 * int64_t(h->B.hcap) * n_prob, 0.0, s);
  // z_0 = M r_0, p_0 = z_0, rz_0, partials of H^T p_0
  const int pf = fp32 ? 1 : 0;
  const int gt = gvariant(h, pf) / 4;
  D::gather_rows(h->r.ptr, h->row_src.ptr, m_r, h->xgr.ptr, s, dsc(h));
  if (fp32) launch_gemv(h, h->S32.ptr, gvariant(h, pf), h->xgr.ptr, h->v.ptr, nullptr);
  else launch_gemv(h, h->S.ptr, gvariant(h, pf), h->xgr.ptr, h->v.ptr, nullptr);
  if (fp32)
    D::pcg_M(h->v.ptr, h->row_src.ptr, h->H32.ptr, h->part_g.ptr, part_rr, h->p.ptr, h->z.ptr, h->xgp.ptr,
             h->part_t.ptr, h->scal.ptr, 0, h->pdone.ptr, h->piters.ptr, 1, h->B, gt, s, dsc(h));
  else
    D::pcg_M(h->v.ptr, h->row_src.ptr, h->H.ptr, h->part_g.ptr, part_rr, h->p.ptr, h->z.ptr, h->xgp.ptr,
             h->part_t.ptr, h->scal.ptr, 0, h->pdone.ptr, h->piters.ptr, 1, h->B, gt, s, dsc(h));
  if (use_graph) {
    int rc = capture_graph(h, fp32);
    if (rc) return rc;
  }
  // Convergence checks every `every2` iterations: the done flags are copied
  // to one of two pinned slots behind an event, and a check is read only
  // after the next interval's iterations are queued, so the GPU never waits
  // for the host.  Iterations queued after a problem finishes exit at once
  // (done flag), and the iteration count is kept on the device.  A profiled
  // run reads each check at once instead, so that every timed launch is one
  // that did its work.
  const int every2 = std::max(2, every + (every & 1));
  const bool overlap = !h->profiling;
  int slot = 0, pending = -1;
  for (int it = 0; it < maxit; it += 2) {
    if (it + 1 == maxit) {
      pcg_iteration_prec(h, 0, fp32);  // an odd cap: the last iteration alone
    } else if (use_graph) {
      HIP_TRY(hipGraphLaunch(fp32 ? h->graph_exec32 : h->graph_exec, s));
    } else {
      pcg_iteration_prec(h, 0, fp32);
      pcg_iteration_prec(h, 1, fp32);
    }
    if ((it + 2) % every2 == 0 || it + 2 >= maxit) {
      if (pending >= 0) {
        HIP_TRY(hipEventSynchronize(h->ev_chk[pending]));
        bool fin = true;
        for (int p = 0; p < n_prob && fin; ++p) fin = h->pchk_h[pending * n_prob + p] != 0;
        if (fin) break;
      }
      HIP_TRY(hipMemcpyAsync(h->pchk_h + slot * n_prob, h->pdone.ptr, n_prob * sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipEventRecord(h->ev_chk[slot], s));
      pending = slot;
      slot ^= 1;
      if (!overlap) {
        HIP_TRY(hipEventSynchronize(h->ev_chk[pending]));
        bool fin = true;
        for (int p = 0; p < n_prob && fin; ++p) fin = h->pchk_h[pending * n_prob + p] != 0;
        if (fin) break;
        pending = -1;
      }
    }
  }
  int rc = check_launch();
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(h->pflags_h, h->pdone.ptr, n_prob * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(h->pflags_h + n_prob, h->piters.ptr, n_prob * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(sc.data(), h->scal.ptr, sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  h->hist_n.assign(n_prob, 0);
  for (int p = 0; p < n_prob; ++p) {
    iters_out[p] = h->pflags_h[n_prob + p];
    // an iteration applies F and M to the problem until its done flag is set
    h->cntF[fp32 ? 1 : 0][p] += iters_out[p];
    h->cntM[fp32 ? 1 : 0][p] += iters_out[p];
    h->hist_n[p] = std::min(iters_out[p], h->B.hcap);
    rr_out[p] = sc[8 * p + 5];
    if (h->pflags_h[p] == 3)
      return fail(IETI_ERR_BREAKDOWN, "PCG breakdown (p^T F p <= 0) in problem " + std::to_string(p));
    if (h->pflags_h[p] != 1) status[p] = IETI_ERR_NOT_CONVERGED;
  }
  return IETI_OK;
}

int solve_impl(ieti_handle* h, const ieti_solve_opts* opts, double* a_host, double* a_dev, ieti_stats* st) {
  namespace D = ieti::dev;
  if (!h) return fail(IETI_ERR_INVALID_ARG, "handle is NULL");
  if (!h->factored) return fail(IETI_ERR_STATE, "ieti_solve called before ieti_factor");
  const auto& M = h->model;
  const auto& P = h->plan;
  const double rtol = (opts && opts->rtol > 0) ? opts->rtol : 1e-8;
  const int maxit = (opts && opts->maxit > 0) ? opts->maxit : 1000;
  const int every = (opts && opts->check_every > 0) ? opts->check_every : 8;
  hipStream_t s = h->stream;
  const int64_t m_r = M.m_r;
  const int n_prob = h->B.n_prob;
  // profiled runs use direct launches so every GEMV carries launch events
  const bool use_graph = (!opts || opts->use_graph != 0) && !h->profiling;
  for (int f = 0; f < 2; ++f) {
    h->cntF[f].assign(n_prob, 0);
    h->cntM[f].assign(n_prob, 0);
  }
  Phase ph_solve("ieti_solve");
  HIP_TRY(hipEventRecord(h->ev0, s));
  int rc = 0;
  {
    Phase ph("ieti_solve: right-hand side");
    rc = compute_rhs(h, use_graph);
  }
  if (rc) return rc;
  int it = 0, outer = 0;
  const std::vector<double> bb = host_dots(h, h->b.ptr, h->b.ptr);
  double bb_all = 0.0;
  for (double v : bb) bb_all += v;
  h->bnorm = std::sqrt(bb_all);
  HIP_TRY(hipEventRecord(h->ev1, s));
  int applies = 0;
  std::vector<double> rr(n_prob, 0.0), rr0(n_prob, 0.0);
  std::vector<int> status(n_prob, IETI_OK), iters(n_prob, 0), outers(n_prob, 0), warm(n_prob, 0);
  if (m_r > 0) {
    Phase ph("ieti_solve: PCG on the multipliers");
    if (!h->mixed) {
      // plain FP64: PCG on F lambda = b from lambda_0
      rc = init_lambda(h, opts, bb, h->lam.ptr, h->r.ptr, rr, &applies, warm);
      if (rc) return rc;
      rr0 = rr;
      std::vector<double> tol2(n_prob);
      for (int p = 0; p < n_prob; ++p) tol2[p] = rtol * rtol * bb[p];
      rc = run_pcg(h, tol2, rr, maxit, every, false, use_graph, iters, rr, status);
      if (rc) return rc;
      for (int n : iters) it = std::max(it, n);
      applies += it;
    } else {
      // mixed: outer refinement on the FP64 residual r = b - F lambda, inner PCG
      // with FP32-stored interface blocks on F d = r, lambda += d (per problem)
      rc = init_lambda(h, opts, bb, h->lam_acc.ptr, h->rtrue.ptr, rr, &applies, warm);
      if (rc) return rc;
      rr0 = rr;
      const int max_outer = 20;
      std::vector<int> in_iters, in_status;
      std::vector<double> in_rr;
      for (outer = 0;; ++outer) {
        if (outer > 0) {
          apply_F(h, h->lam_acc.ptr, h->q.ptr);
          ++applies;
          count_all(h->cntF[0]);
          D::axpby(h->b.ptr, h->q.ptr, h->rtrue.ptr, 1.0, -1.0, m_r, s);
          rr = host_dots(h, h->rtrue.ptr, h->rtrue.ptr);
        }
        bool all = true;
        std::vector<double> tol2(n_prob);
        for (int p = 0; p < n_prob; ++p) {
          const bool conv = rr[p] <= rtol * rtol * bb[p] || bb[p] == 0.0;
          status[p] = conv ? IETI_OK : IETI_ERR_NOT_CONVERGED;
          all = all && conv;
          // inner tolerance: a fixed factor below the current true residual,
          // never tighter than what the final step needs; converged problems
          // start (and stay) finished
          const double inner_rel = conv ? 1.0 : std::max(1e-4, 0.5 * rtol * std::sqrt(bb[p] / rr[p]));
          tol2[p] = inner_rel * inner_rel * rr[p];
          if (!conv) outers[p] = outer;
        }
        if (all || outer >= max_outer || it >= maxit) break;
        D::fill(h->lam.ptr, m_r, 0.0, s);
        D::vec_copy(h->rtrue.ptr, h->r.ptr, m_r, s);
        rc = run_pcg(h, tol2, rr, maxit - it, every, true, use_graph, in_iters, in_rr, in_status);
        if (rc) return rc;
        int n = 0;
        for (int p = 0; p < n_prob; ++p) {
          iters[p] += in_iters[p];
          n = std::max(n, in_iters[p]);
        }
        it += n;
        applies += n;
        D::axpby(h->lam_acc.ptr, h->lam.ptr, h->lam_acc.ptr, 1.0, 1.0, m_r, s);
      }
      for (int p = 0; p < n_prob; ++p) outers[p] += status[p] == IETI_OK && outer > 0 ? 1 : 0;
      D::vec_copy(h->lam_acc.ptr, h->lam.ptr, m_r, s);
    }
  }
  HIP_TRY(hipEventRecord(h->ev2, s));
  // ---- recovery: p = S_c^{-1}(d~ + G^T lambda), a_r = K_rr^{-1}(j_r - K_rp C p - B^T lambda)
  Phase ph_rec("ieti_solve: recovery");
  rc = run_sequence(h, 1, use_graph, [&]() {
    if (M.n_gp > 0) {
      // u = L_c^{-1} d~ + H^T lambda, p = L_c^{-T} u  (H = G L_c^{-T}, S_c = L_c L_c^T), per problem
      D::coarse_project(h->Ht.ptr, h->lam.ptr, h->t.ptr, h->cprob.ptr, h->B, s);
      D::axpby(h->w.ptr, h->t.ptr, h->dtil.ptr, 1.0, 1.0, M.n_gp, s);
      D::tri_small_inv(h->Lti.ptr, h->dtil.ptr, h->pglob.ptr, true, h->B, s);
    }
    // y = L_rr^{-1} (j_r - K_rp a_p - B_r^T lambda) = y_j - L_pr^T a_p - L_Er^T u (no forward sweep),
    // then the backward sweep
    D::vec_copy(h->yj.ptr, h->y.ptr, P.r_total, s);
    D::recovery_sources(h->y.ptr, h->recP_pos.ptr, h->recP_glob.ptr, int64_t(P.recP_pos.size()),
                        M.n_gp > 0 ? h->pglob.ptr : nullptr, h->A_aug.ptr, h->I_row.ptr, h->I_sign.ptr, P.I_total,
                        h->lam.ptr, s);
    D::trsv_update(h->pool.ptr, h->rec_task.ptr, h->rec_pair.ptr, int64_t(P.rec_task.size() / 3), h->y.ptr, true,
                   s);
    backward_solve(h);
  });
  if (rc) return rc;
  double* aout = a_dev ? a_dev : h->aout.ptr;
  D::fill(aout, M.n_edges_total, 0.0, s);
  D::write_output(h->y.ptr, h->out_src.ptr, h->out_edge.ptr, int64_t(P.out_src.size()), h->pglob.ptr,
                  h->primal_edges.ptr, M.n_gp, aout, s);
  if (!M.d_edges.empty()) D::scatter(aout, h->d_edges.ptr, h->d_vals.ptr, int64_t(M.d_edges.size()), s);
  hipEvent_t evend;
  HIP_TRY(hipEventCreate(&evend));
  HIP_TRY(hipEventRecord(evend, s));
  rc = check_launch();
  if (rc) return rc;
  if (a_host) HIP_TRY(hipMemcpyAsync(a_host, aout, M.n_edges_total * sizeof(double), hipMemcpyDeviceToHost, s));
  h->lambda_h.assign(m_r, 0.0);
  if (m_r > 0) HIP_TRY(hipMemcpyAsync(h->lambda_h.data(), h->lam.ptr, m_r * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  prof_collect(h);
  float ms_total = 0.f, ms_pcg = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms_total, h->ev0, evend));
  HIP_TRY(hipEventElapsedTime(&ms_pcg, h->ev1, h->ev2));
  HIP_TRY(hipEventDestroy(evend));
  // per-problem results; the stats report the worst problem
  h->p_iters = iters;
  h->p_outer = outers;
  h->p_status = status;
  h->p_warm = warm;
  h->p_relres.assign(n_prob, 0.0);
  h->p_relres0.assign(n_prob, 0.0);
  double rel = 0.0, rel0 = 0.0;
  int st_all = IETI_OK, warm_all = 0, outer_max = 0;
  for (int p = 0; p < n_prob; ++p) {
    h->p_relres[p] = bb[p] > 0 ? std::sqrt(rr[p] / bb[p]) : 0.0;
    h->p_relres0[p] = bb[p] > 0 ? std::sqrt(rr0[p] / bb[p]) : 0.0;
    rel = std::max(rel, h->p_relres[p]);
    rel0 = std::max(rel0, h->p_relres0[p]);
    if (status[p] != IETI_OK) st_all = status[p];
    if (warm[p] == -1) warm_all = -1;
    else if (warm[p] == 1 && warm_all == 0) warm_all = 1;
    outer_max = std::max(outer_max, outers[p]);
  }
  if (st) {
    st->n_global = M.n_g;
    st->n_multipliers = M.m_r;
    st->n_primal = M.n_gp;
    st->n_sub = M.n_sub;
    st->iters = it;
    st->outer_iters = h->mixed ? outer : 0;
    st->status = st_all;
    st->f_applies = applies;
    st->rel_residual = rel;
    st->t_factor_s = h->factor_ms * 1e-3;
    st->t_solve_s = ms_total * 1e-3;
    st->t_pcg_s = ms_pcg * 1e-3;
    st->factor_flops = h->plan.flops;
    st->rel_residual0 = rel0;
    st->warm_start = warm_all;
    st->reserved = 0;
    st->pcg_bytes = 0.0;
    for (int p = 0; p < n_prob; ++p) st->pcg_bytes += problem_pcg_bytes(h, p);
  }
  (void)outer_max;
  if (st_all != IETI_OK) return fail(st_all, "PCG did not reach the tolerance within maxit");
  return IETI_OK;
}

// Validation, topology, gauge and assembly of one problem into m (host).
int assemble_model(const ieti_problem* prob, ieti::Model& m, bool primal = true) {
  int rc = validate(prob);
  if (rc) return rc;
  m.prob = *prob;
  m.primal_enabled = primal;
  const int64_t np = int64_t(prob->patches[0]) * prob->patches[1] * prob->patches[2];
  m.part.assign(prob->patch_to_subdomain, prob->patch_to_subdomain + np);
  m.nu.assign(prob->nu_per_patch, prob->nu_per_patch + np);
  int maxs = -1;
  for (int64_t q = 0; q < np; ++q) {
    if (m.part[q] < 0) return fail(IETI_ERR_INVALID_ARG, "negative subdomain id");
    if (!(m.nu[q] > 0.0)) return fail(IETI_ERR_INVALID_ARG, "reluctivity must be positive");
    maxs = std::max(maxs, m.part[q]);
  }
  m.n_sub = maxs + 1;
  ieti::Error err{0, ""};
  if (ieti::check_partition(*prob, m.part, m.n_sub, err)) return fail(err.code, err.msg);
  m.mesh.init(*prob);
  rc = ieti::build_topology(m, err);
  if (!rc) rc = ieti::assemble_local_systems(m, err);
  if (rc) return fail(rc, err.msg);
  m.prob.J = nullptr;  // the callbacks are not kept beyond the assembly call
  m.prob.J_user = nullptr;
  m.prob.A_D = nullptr;
  m.prob.A_D_user = nullptr;
  ieti::finalize_single(m);
  return IETI_OK;
}

}  // namespace

// ---- allocation-free operator application
//
// The work vectors of ieti_apply_F_noalloc live in this array, one copy per
// GPU (part of the library's code object, so it exists from the moment the
// library is loaded on a device until the process ends).  Host code never
// uses the symbol itself as an address: each device's copy is resolved once
// with hipGetSymbolAddress while that device is current, and that address
// is what the kernels receive.
static constexpr int64_t NOALLOC_DOUBLES = IETI_NOALLOC_SCRATCH_BYTES / int64_t(sizeof(double));
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

int scratch_for_device(int dev, double** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(IETI_ERR_INVALID_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(IETI_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return IETI_OK;
}

// 256-byte aligned carve-outs of the scratch array, in doubles
int64_t carve(int64_t n) { return (std::max<int64_t>(n, 1) + 31) / 32 * 32; }

}  // namespace

extern "C" {

const char* ieti_last_error(void) { return ieti::rt::last_error().c_str(); }

int ieti_assemble(const ieti_problem* prob, ieti_handle** out) { return ieti_assemble_batch(prob, 1, out); }

int ieti_assemble_batch(const ieti_problem* probs, int32_t n, ieti_handle** out) {
  Phase ph("ieti_assemble");
  if (!out) return fail(IETI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!probs || n < 1) return fail(IETI_ERR_INVALID_ARG, "a batch needs at least one problem");
  std::vector<ieti::Model> parts(n);
  for (int32_t i = 0; i < n; ++i) {
    int rc = assemble_model(&probs[i], parts[i]);
    if (rc) {
      if (n > 1) ieti::rt::last_error() = "problem " + std::to_string(i) + ": " + ieti::rt::last_error();
      return rc;
    }
  }
  auto* h = new ieti_handle();
  if (n == 1) {
    h->model = std::move(parts[0]);
  } else {
    ieti::Error err{0, ""};
    if (int rc = ieti::merge_models(parts, h->model, err)) {
      delete h;
      return fail(rc, err.msg);
    }
  }
  int rc = build_plan_if_needed(h, ieti::dev::TILE, 0);
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return IETI_OK;
}

int ieti_assemble_ex(const ieti_problem* prob, const ieti_assemble_opts* opts, ieti_handle** out) {
  Phase ph("ieti_assemble");
  if (!out) return fail(IETI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!prob) return fail(IETI_ERR_INVALID_ARG, "problem is NULL");
  bool primal = true;
  if (opts) {
    if (opts->version != IETI_ABI_VERSION) return fail(IETI_ERR_INVALID_ARG, "ieti_assemble_opts version mismatch");
    if (opts->primal != 0 && opts->primal != 1) return fail(IETI_ERR_INVALID_ARG, "primal must be 0 or 1");
    primal = opts->primal == 1;
  }
  auto* h = new ieti_handle();
  int rc = assemble_model(prob, h->model, primal);
  if (!rc) rc = build_plan_if_needed(h, ieti::dev::TILE, 0);
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return IETI_OK;
}

int ieti_batch_of(const ieti_handle* const* hs, int32_t n, ieti_handle** out) {
  if (!out) return fail(IETI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!hs || n < 1) return fail(IETI_ERR_INVALID_ARG, "a batch needs at least one handle");
  std::vector<ieti::Model> parts;
  parts.reserve(n);
  for (int32_t i = 0; i < n; ++i) {
    if (!hs[i]) return fail(IETI_ERR_INVALID_ARG, "handle " + std::to_string(i) + " is NULL");
    if (hs[i]->model.batch()) return fail(IETI_ERR_INVALID_ARG, "handle " + std::to_string(i) + " is a batch");
    parts.push_back(hs[i]->model);
  }
  auto* h = new ieti_handle();
  ieti::Error err{0, ""};
  int rc = ieti::merge_models(parts, h->model, err);
  if (rc) {
    delete h;
    return fail(rc, err.msg);
  }
  if (n == 1) ieti::finalize_single(h->model);
  rc = build_plan_if_needed(h, ieti::dev::TILE, 0);
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return IETI_OK;
}

int ieti_get_batch_info(const ieti_handle* h, int64_t* ranges, int32_t* iters, double* rel_residual) {
  if (!h) return fail(IETI_ERR_INVALID_ARG, "handle is NULL");
  const auto& M = h->model;
  for (size_t p = 0; p < M.probs.size(); ++p) {
    const auto& r = M.probs[p];
    if (ranges) {
      const int64_t v[8] = {r.edge_base, r.n_edges, r.mr_base, r.m_r, r.gp_base, r.n_gp, r.sub_base, r.n_sub};
      std::memcpy(ranges + 8 * p, v, sizeof(v));
    }
    if (iters) iters[p] = p < h->p_iters.size() ? h->p_iters[p] : 0;
    if (rel_residual) rel_residual[p] = p < h->p_relres.size() ? h->p_relres[p] : 0.0;
  }
  return IETI_OK;
}

int ieti_get_problem_stats(const ieti_handle* h, int32_t prob, ieti_problem_stats* out) {
  if (!h || !out) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  if (prob < 0 || prob >= int32_t(h->model.probs.size())) return fail(IETI_ERR_INVALID_ARG, "problem out of range");
  if (!h->uploaded) return fail(IETI_ERR_STATE, "not factored");
  std::memset(out, 0, sizeof(*out));
  const size_t p = size_t(prob);
  auto at = [p](const std::vector<int>& v) { return p < v.size() ? v[p] : 0; };
  auto atd = [p](const std::vector<double>& v) { return p < v.size() ? v[p] : 0.0; };
  out->iters = at(h->p_iters);
  out->outer_iters = at(h->p_outer);
  out->status = at(h->p_status);
  out->warm_start = at(h->p_warm);
  for (int f = 0; f < 2; ++f) {
    out->f_applies[f] = at(h->cntF[f]);
    out->m_applies[f] = at(h->cntM[f]);
    const double sz = f ? 4.0 : 8.0;
    out->bytes_F[f] = alg_bytes(h, prob, sz, true);
    out->bytes_M[f] = alg_bytes(h, prob, sz, false);
  }
  out->rel_residual = atd(h->p_relres);
  out->rel_residual0 = atd(h->p_relres0);
  out->block_entries = h->pb_entries[p];
  out->pcg_bytes = problem_pcg_bytes(h, prob);
  return IETI_OK;
}

int ieti_factor(ieti_handle* h, const ieti_factor_opts* opts) {
  namespace D = ieti::dev;
  if (!h) return fail(IETI_ERR_INVALID_ARG, "handle is NULL");
  Phase ph("ieti_factor");
  const int T = (opts && opts->tile) ? opts->tile : D::TILE;
  if (T != D::TILE) return fail(IETI_ERR_INVALID_ARG, "only tile size 64 is built");
  if (opts && opts->precision != IETI_PREC_FP64 && opts->precision != IETI_PREC_MIXED)
    return fail(IETI_ERR_INVALID_ARG, "unknown precision");
  const int scaling = opts ? opts->scaling : IETI_SCALE_IDENTITY;
  if (scaling != IETI_SCALE_IDENTITY && scaling != IETI_SCALE_STIFFNESS && scaling != IETI_SCALE_MULTIPLICITY)
    return fail(IETI_ERR_INVALID_ARG, "unknown scaling");
  int rc = 0;
  if (opts && opts->factor_tune == 1 && !h->ftuned) {
    rc = tune_factor(h, T, opts->ordering, opts->hip_stream);
    if (rc) return rc;
  }
  rc = build_plan_if_needed(h, T, opts ? opts->ordering : 0);
  if (rc) return rc;
  rc = upload(h);
  if (rc) return rc;
  h->stream = pick_stream(h, opts ? opts->hip_stream : nullptr);
  hipStream_t s = h->stream;
  const auto& P = h->plan;
  const auto& M = h->model;
  h->factored = false;
  h->rhs_ready = false;
  HIP_TRY(hipMemsetAsync(h->flags.ptr, 0, 8 * sizeof(int), s));
  // the padded interface slots of the gathered vectors must read 0 (gathers
  // write the real slots only); cleared on the solve stream itself
  D::fill(h->xgp.ptr, h->xgp.n, 0.0, s);
  D::fill(h->xgr.ptr, h->xgr.n, 0.0, s);
  // mixed precision: FP32 copies of the interface blocks for the inner PCG,
  // written by the same tile copies as the FP64 blocks
  const bool mixed = opts && opts->precision == IETI_PREC_MIXED;
  if (mixed && !h->S32.ptr) {
    if ((rc = dalloc(h->S32, P.S_elems))) return rc;
    if ((rc = dalloc(h->Sinv32, P.S_elems))) return rc;
    if (P.S_elems > 0) {
      HIP_TRY(hipMemset(h->S32.ptr, 0, size_t(P.S_elems) * sizeof(float)));
      HIP_TRY(hipMemset(h->Sinv32.ptr, 0, size_t(P.S_elems) * sizeof(float)));
    }
  }
  HIP_TRY(hipEventRecord(h->ev0, s));
  enqueue_local_factor(h, s, mixed ? h->S32.ptr : nullptr);
  D::copy_tiles(h->pool.ptr, h->xsinv.ptr, int64_t(P.xsinv_task.size() / 5), -1.0, h->Sinv.ptr, s,
                mixed ? h->Sinv32.ptr : nullptr);
  D::copy_tiles(h->pool.ptr, h->xphi.ptr, int64_t(P.xphi_task.size() / 5), -1.0, h->Phi.ptr, s);
  D::copy_tiles(h->pool.ptr, h->xspi.ptr, int64_t(P.xspi_task.size() / 5), 1.0, h->SPi.ptr, s);
  if (M.n_gp > 0) {
    D::sum_sources(h->SPi.ptr, h->spi_ptr.ptr, h->spi_src.ptr, P.spi_off.back(), h->Spi_glob.ptr, s);
    D::build_G(h->Phi.ptr, h->row_src.ptr, h->slot_phi_row.ptr, h->I_sub.ptr, h->glob2loc.ptr, h->g2l_off.ptr,
               h->G.ptr, h->B, s);
    // Cholesky of S_c with H = G L_c^{-T} and U = L_c^{-T} as one tile
    // factorisation of the column block [S_c; G; I]
    const auto& C = h->cplan;
    D::fill(h->cpool.ptr, C.pool_elems, 0.0, s);
    D::dense_to_tiles(h->cpool.ptr, h->cfill.ptr, int64_t(C.fill_task.size() / 7), h->Spi_glob.ptr, h->G.ptr, s);
    for (int64_t c = 0; c < C.n_levels; ++c) {
      D::potrf_tiles(h->cpool.ptr, h->cinv.ptr, h->cpotrf.ptr + 3 * C.potrf_ptr[c], C.potrf_ptr[c + 1] - C.potrf_ptr[c],
                     h->ctol.ptr, h->flags.ptr + 4, s);
      D::trsm_tiles(h->cpool.ptr, h->cinv.ptr, h->ctrsm.ptr + 2 * C.trsm_ptr[c], C.trsm_ptr[c + 1] - C.trsm_ptr[c], s);
      D::update_tiles(h->cpool.ptr, h->cupd.ptr + 3 * C.upd_ptr[c], h->cupd_pair.ptr, C.upd_ptr[c + 1] - C.upd_ptr[c],
                      s);
    }
    D::tiles_to_dense(h->cpool.ptr, h->cout_h.ptr, int64_t(C.out_h_task.size() / 7), h->H.ptr, h->Ht.ptr, s);
    D::tiles_to_dense(h->cpool.ptr, h->cout_l.ptr, int64_t(C.out_l_task.size() / 7), h->Lti.ptr, nullptr, s);
  }
  // mixed precision: FP32 copies of the coarse rows
  h->mixed = mixed;
  if (h->mixed) {
    if (M.n_gp > 0) {
      if (h->H32.n != h->H.n) {
        if ((rc = dalloc(h->H32, h->H.n))) return rc;
        if ((rc = dalloc(h->Ht32, h->Ht.n))) return rc;
      }
      D::to_float(h->H.ptr, h->H32.ptr, h->H.n, s);
      D::to_float(h->Ht.ptr, h->Ht32.ptr, h->Ht.n, s);
    }
  }
  HIP_TRY(hipEventRecord(h->ev1, s));
  rc = check_launch();
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(h->flags_h, h->flags.ptr, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  h->factor_ms = ms;
  prof_collect(h);
  if (h->flags_h[0] > 0) {
    const int k = h->flags_h[0] - 1;
    std::string where = "subdomain " + std::to_string(k);
    if (M.batch())
      where = "subdomain " + std::to_string(k - M.probs[M.sub_prob[k]].sub_base) + " of problem " +
              std::to_string(M.sub_prob[k]);
    return fail(IETI_ERR_NOT_SPD, "pivot at or below " + std::to_string(ieti::Plan::PIVOT_REL) +
                                      " of the largest diagonal entry (K_rr numerically singular) in the local "
                                      "factorisation of " + where);
  }
  if (h->flags_h[4] > 0)
    return fail(IETI_ERR_NOT_SPD, "coarse matrix of problem " + std::to_string(h->flags_h[4] - 1) +
                                      " is not positive definite");
  const int forced = opts ? opts->gemv_variant : 0;
  if (forced < 0 || forced > D::GEMV_SHAPES) return fail(IETI_ERR_INVALID_ARG, "gemv_variant out of range");
  if ((rc = choose_gemv(h, forced, 0))) return rc;
  if (h->mixed && (rc = choose_gemv(h, forced, 1))) return rc;
  // recomputed on every factorisation: it follows the assembled stiffness (set_coefficients)
  if ((rc = set_scaling(h, scaling))) return rc;
  h->factored = true;
  return IETI_OK;
}

int ieti_solve(ieti_handle* h, const ieti_solve_opts* opts, double* a_out, ieti_stats* stats) {
  return solve_impl(h, opts, a_out, nullptr, stats);
}

int ieti_solve_device(ieti_handle* h, const ieti_solve_opts* opts, double* d_a_out, ieti_stats* stats) {
  if (!d_a_out) return fail(IETI_ERR_INVALID_ARG, "d_a_out is NULL");
  return solve_impl(h, opts, nullptr, d_a_out, stats);
}

int ieti_get_sizes(const ieti_handle* h, int64_t* sizes) {
  if (!h || !sizes) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  const auto& m = h->model;
  int64_t sum_r = 0, max_nI = 0;
  for (const auto& s : m.sd) {
    sum_r += int64_t(s.r_edges.size());
    max_nI = std::max<int64_t>(max_nI, int64_t(s.I_local.size()));
  }
  int64_t n_nodes = 0;
  for (const auto& me : m.meshes) n_nodes += me.n_nodes;
  const int64_t v[8] = {m.n_edges_total, m.n_g, sum_r, m.m_r, m.n_gp, m.n_sub, n_nodes, max_nI};
  std::memcpy(sizes, v, sizeof(v));
  return IETI_OK;
}

int ieti_get_maps(const ieti_handle* h, uint8_t* weight, uint8_t* tree_mask, uint8_t* dirichlet,
                  int64_t* primal_edges, int64_t* mult_rows, int64_t* sub_offsets, int64_t* sub_r_edges) {
  if (!h) return fail(IETI_ERR_INVALID_ARG, "handle is NULL");
  const auto& m = h->model;
  if (m.batch()) return fail(IETI_ERR_STATE, "the integer maps are per problem; not available on a batch handle");
  if (weight) std::copy(m.weight.begin(), m.weight.end(), weight);
  if (tree_mask) std::copy(m.tree.begin(), m.tree.end(), tree_mask);
  if (dirichlet) std::copy(m.dirichlet.begin(), m.dirichlet.end(), dirichlet);
  if (primal_edges) std::copy(m.primal_edges.begin(), m.primal_edges.end(), primal_edges);
  if (mult_rows) std::copy(m.mult.begin(), m.mult.end(), mult_rows);
  int64_t acc = 0;
  for (int k = 0; k < m.n_sub; ++k) {
    if (sub_offsets) sub_offsets[k] = acc;
    if (sub_r_edges) std::copy(m.sd[k].r_edges.begin(), m.sd[k].r_edges.end(), sub_r_edges + acc);
    acc += int64_t(m.sd[k].r_edges.size());
  }
  if (sub_offsets) sub_offsets[m.n_sub] = acc;
  return IETI_OK;
}

int ieti_get_local_system(const ieti_handle* h, int32_t k, int64_t* n, int64_t* nnz, int64_t* indptr,
                          int32_t* indices, double* values, double* load) {
  if (!h || !n || !nnz) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  if (k < 0 || k >= h->model.n_sub) return fail(IETI_ERR_INVALID_ARG, "subdomain out of range");
  const auto& s = h->model.sd[k];
  *n = s.n_loc;
  *nnz = int64_t(s.indices.size());
  if (indptr) std::copy(s.indptr.begin(), s.indptr.end(), indptr);
  if (indices) std::copy(s.indices.begin(), s.indices.end(), indices);
  if (values) std::copy(s.values.begin(), s.values.end(), values);
  if (load) std::copy(s.load.begin(), s.load.end(), load);
  return IETI_OK;
}

int ieti_get_schur(const ieti_handle* h, int32_t k, int64_t* n_I_out, double* S, double* Sinv) {
  if (!h || !n_I_out) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  if (k < 0 || k >= h->model.n_sub) return fail(IETI_ERR_INVALID_ARG, "subdomain out of range");
  if (!h->factored) return fail(IETI_ERR_STATE, "not factored");
  const auto& sp = h->plan.sub[k];
  *n_I_out = sp.nI;
  std::vector<double> buf(sp.nIp * sp.nIp);
  const DBuf<double>* srcs[2] = {&h->S, &h->Sinv};
  double* dsts[2] = {S, Sinv};
  for (int w = 0; w < 2; ++w) {
    if (!dsts[w] || sp.nI == 0) continue;
    HIP_TRY(hipMemcpy(buf.data(), srcs[w]->ptr + sp.S_off, buf.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < sp.nI; ++i)
      for (int64_t j = 0; j < sp.nI; ++j) dsts[w][i * sp.nI + j] = buf[i * sp.nIp + j];
  }
  return IETI_OK;
}

int ieti_apply_F(ieti_handle* h, const double* lambda, double* q) {
  if (!h || !lambda || !q) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  if (!h->factored) return fail(IETI_ERR_STATE, "not factored");
  const int64_t m_r = h->model.m_r;
  if (m_r == 0) return IETI_OK;
  HIP_TRY(hipMemcpyAsync(h->tmp.ptr, lambda, m_r * sizeof(double), hipMemcpyHostToDevice, h->stream));
  apply_F(h, h->tmp.ptr, h->q.ptr);
  int rc = check_launch();
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(q, h->q.ptr, m_r * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return IETI_OK;
}

int ieti_apply_M(ieti_handle* h, const double* r, double* z) {
  if (!h || !r || !z) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  if (!h->factored) return fail(IETI_ERR_STATE, "not factored");
  const int64_t m_r = h->model.m_r;
  if (m_r == 0) return IETI_OK;
  HIP_TRY(hipMemcpyAsync(h->tmp.ptr, r, m_r * sizeof(double), hipMemcpyHostToDevice, h->stream));
  apply_M(h, h->tmp.ptr, h->z.ptr);
  int rc = check_launch();
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(z, h->z.ptr, m_r * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return IETI_OK;
}

int ieti_apply_F_noalloc(ieti_handle* h, const double* d_lambda, double* d_q, void* hip_stream) {
  namespace D = ieti::dev;
  if (!h || !d_lambda || !d_q) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  if (d_lambda == d_q) return fail(IETI_ERR_INVALID_ARG, "d_lambda and d_q must be distinct");
  if (!h->factored) return fail(IETI_ERR_STATE, "not factored");
  const auto& M = h->model;
  if (M.m_r == 0) return IETI_OK;
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != h->device)
    return fail(IETI_ERR_STATE, "the handle's device " + std::to_string(h->device) + " is not current");
  // work vectors: gathered values and local products per interface slot,
  // GEMV partials (the symmetric kernel's partial lists, the per-block sums)
  // and the coarse projection
  const int variant = gvariant(h, 0);
  const bool sym = variant == D::GEMV_SYM;
  const int64_t n_xg = carve(h->xgp.n), n_v = carve(h->v.n), n_pg = carve(h->part_g.n);
  const int64_t n_sp = sym ? carve(h->sym_part.n) : 0, n_t = M.n_gp > 0 ? carve(M.n_gp) : 0;
  const int64_t need = n_xg + n_v + n_pg + n_sp + n_t;
  if (need > NOALLOC_DOUBLES)
    return fail(IETI_ERR_INVALID_ARG, "the work vectors of this handle need " + std::to_string(need * 8) +
                                          " bytes; the allocation-free path holds " +
                                          std::to_string(int64_t(IETI_NOALLOC_SCRATCH_BYTES)));
  double* base = nullptr;
  int rc = scratch_for_device(cur, &base);
  if (rc) return rc;
  double* xg = base;
  double* v = xg + n_xg;
  double* part_g = v + n_v;
  double* sym_part = part_g + n_pg;
  double* t = sym_part + n_sp;
  hipStream_t s = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : h->stream;
  // padding slots are read by the GEMV and written by no gather: clear the
  // whole gathered vector (a fill kernel, which graph capture accepts)
  D::fill(xg, h->xgp.n, 0.0, s);
  D::gather_rows(d_lambda, h->row_src.ptr, M.m_r, xg, s);
  if (sym) {
    D::SymGemv g = h->symg;
    g.part = sym_part;
    D::gemv_sym(h->Sinv.ptr, g, xg, v, part_g, nullptr, s);
  } else {
    const int ri = variant / 4;
    D::gemv(h->Sinv.ptr, h->gemv_tasks[ri].ptr, h->ngemv_r[ri], h->max_ld, xg, v, part_g, nullptr,
            h->task_prob[ri].ptr, s, variant);
  }
  if (M.n_gp > 0) D::coarse_project(h->Ht.ptr, d_lambda, t, h->cprob.ptr, h->B, s);
  D::combine(v, h->row_src.ptr, M.n_gp > 0 ? h->Ht.ptr : nullptr, t, d_q, h->B, s);
  return check_launch();
}

int ieti_get_rhs(ieti_handle* h, double* b) {
  if (!h || !b) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  if (!h->factored) return fail(IETI_ERR_STATE, "not factored");
  int rc = compute_rhs(h, false);
  if (rc) return rc;
  const int64_t m_r = h->model.m_r;
  if (m_r > 0) HIP_TRY(hipMemcpyAsync(b, h->b.ptr, m_r * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return IETI_OK;
}

int ieti_get_plan_info(const ieti_handle* h, double* info) {
  if (!h || !info) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  const auto& P = h->plan;
  double sum_nI2 = 0.0, max_ld = 0.0;
  for (const auto& sp : P.sub) {
    sum_nI2 += double(sp.nI) * double(sp.nI);
    max_ld = std::max(max_ld, double(sp.nIp));
  }
  const double v[12] = {double(P.pool_elems), double(P.S_elems), P.flops, P.dense_flops, double(P.n_steps),
                        double(P.n_update_tasks), sum_nI2, double(P.I_total), max_ld, double(P.T),
                        P.flops_scalar_rr, P.flops_scalar_aug};
  std::memcpy(info, v, sizeof(v));
  return IETI_OK;
}

int ieti_set_factor_params(ieti_handle* h, int32_t defer, int32_t defer_tail, int32_t update_wgs) {
  if (!h) return fail(IETI_ERR_INVALID_ARG, "handle is NULL");
  if (defer < 1 || defer > 64 || defer_tail < 1 || defer_tail > 64 || update_wgs < 1 || update_wgs > 65536)
    return fail(IETI_ERR_INVALID_ARG, "factorisation parameters out of range");
  h->pparams.defer = defer;
  h->pparams.defer_tail = defer_tail;
  h->upd_wgs = update_wgs;
  h->ftuned = true;  // explicit parameters: no autotuning on this handle
  return IETI_OK;
}

int ieti_get_factor_tuning(const ieti_handle* h, int32_t* params, double* log, int32_t* n_log) {
  if (!h) return fail(IETI_ERR_INVALID_ARG, "handle is NULL");
  if (params) {
    params[0] = h->pparams.defer;
    params[1] = h->pparams.defer_tail;
    params[2] = int32_t(h->upd_wgs);
  }
  if (n_log) *n_log = int32_t(h->ftune_log.size() / 4);
  if (log) std::copy(h->ftune_log.begin(), h->ftune_log.end(), log);
  return IETI_OK;
}

int ieti_get_gemv_tuning(const ieti_handle* h, int32_t* variant, float* ms) {
  if (!h) return fail(IETI_ERR_INVALID_ARG, "handle is NULL");
  if (variant) {
    variant[0] = h->gvar[0];
    variant[1] = h->gvar[1];
  }
  if (ms)
    for (int f = 0; f < 2; ++f)
      for (int v = 0; v < ieti::dev::GEMV_SHAPES; ++v) ms[f * ieti::dev::GEMV_SHAPES + v] = h->gtime[f][v];
  return IETI_OK;
}

int ieti_set_profiling(ieti_handle* h, int32_t enable) {
  if (!h) return fail(IETI_ERR_INVALID_ARG, "handle is NULL");
  h->profiling = enable != 0;
  for (int k = 0; k < 3; ++k) h->k_count[k] = h->k_ms[k] = 0.0;
  h->upd_tasks = 0.0;
  h->ev_marks.clear();
  h->ev_used = 0;
  return IETI_OK;
}

int ieti_record_pcg(ieti_handle* h, int32_t cap) {
  if (!h) return fail(IETI_ERR_INVALID_ARG, "handle is NULL");
  if (cap < 0 || cap > (1 << 20)) return fail(IETI_ERR_INVALID_ARG, "cap must lie in [0, 2^20]");
  drop_graphs(h);  // captured launches carry the record pointer
  h->hist.release();
  h->B.hist = nullptr;
  h->B.hcap = 0;
  h->hist_n.clear();
  if (cap == 0) return IETI_OK;
  const int n_prob = std::max<int>(1, int(h->model.probs.size()));
  int rc = dalloc(h->hist, 2 * int64_t(cap) * n_prob);
  if (rc) return rc;
  h->B.hist = h->hist.ptr;
  h->B.hcap = cap;
  return IETI_OK;
}

int ieti_get_pcg_coefficients(const ieti_handle* h, int32_t prob, double* alpha, double* beta, int32_t* n_out) {
  if (!h || !n_out) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  if (!h->B.hist) return fail(IETI_ERR_STATE, "PCG recording is off (ieti_record_pcg)");
  if (prob < 0 || prob >= int(h->hist_n.size())) return fail(IETI_ERR_STATE, "no recorded solve for this problem");
  const int n = h->hist_n[prob];
  *n_out = n;
  if (n == 0 || (!alpha && !beta)) return IETI_OK;
  std::vector<double> v(2 * size_t(n));
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(v.data(), h->B.hist + 2 * int64_t(prob) * h->B.hcap, v.size() * sizeof(double),
                    hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) {
    if (alpha) alpha[i] = v[2 * i];
    if (beta) beta[i] = v[2 * i + 1];
  }
  return IETI_OK;
}

int ieti_get_condition(const ieti_handle* h, int32_t prob, double* lambda_min, double* lambda_max) {
  if (!lambda_min || !lambda_max) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  int32_t k = 0;
  int rc = ieti_get_pcg_coefficients(h, prob, nullptr, nullptr, &k);
  if (rc) return rc;
  if (k == 0) {
    *lambda_min = *lambda_max = 1.0;
    return IETI_OK;
  }
  std::vector<double> al(k), be(k);
  if ((rc = ieti_get_pcg_coefficients(h, prob, al.data(), be.data(), &k))) return rc;
  // Lanczos tridiagonal of the preconditioned operator from the PCG
  // coefficients: d_i = 1/alpha_i + beta_{i-1}/alpha_{i-1}, e_i = sqrt(beta_i)/alpha_i
  std::vector<double> d(k), e2(k > 1 ? k - 1 : 1, 0.0);
  for (int i = 0; i < k; ++i) {
    if (!(al[i] > 0.0)) return fail(IETI_ERR_STATE, "recorded step lengths are not positive");
    d[i] = 1.0 / al[i] + (i > 0 ? be[i - 1] / al[i - 1] : 0.0);
  }
  for (int i = 0; i + 1 < k; ++i) e2[i] = be[i] / (al[i] * al[i]);
  // eigenvalues below x: sign changes of the LDL^T pivots of T - x I (Sturm count)
  auto below = [&](double x) {
    int c = 0;
    double q = d[0] - x;
    const double tiny = 1e-300;
    for (int i = 0;; ++i) {
      if (q == 0.0) q = -tiny;
      if (q < 0.0) ++c;
      if (i + 1 == k) break;
      q = d[i + 1] - x - e2[i] / q;
    }
    return c;
  };
  double lo = d[0], hi = d[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::sqrt(e2[i - 1]) : 0.0) + (i + 1 < k ? std::sqrt(e2[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  // the j-th smallest eigenvalue by bisection on the Sturm count
  auto eig = [&](int j) {
    double a = lo, b = hi;
    for (int it = 0; it < 200 && b - a > 1e-15 * std::max(std::abs(a), std::abs(b)); ++it) {
      const double m = 0.5 * (a + b);
      if (below(m) > j) b = m;
      else a = m;
    }
    return 0.5 * (a + b);
  };
  *lambda_min = eig(0);
  *lambda_max = eig(k - 1);
  return IETI_OK;
}

int ieti_get_kernel_times(const ieti_handle* h, double* times) {
  if (!h || !times) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  double full = 0.0;
  for (const auto& sp : h->plan.sub) full += double(sp.nIp) * double(sp.nIp) * sizeof(double);
  const double lower = h->sym_elems * sizeof(double);
  const double bytes = h->gvar[0] == ieti::dev::GEMV_SYM ? lower : full;
  double entries = 0.0;
  for (double e : h->pb_entries) entries += e;
  const double v[12] = {h->k_count[0], h->k_ms[0], h->k_count[1], h->k_ms[1], h->upd_tasks, bytes, full, lower,
                        entries * sizeof(double), h->k_count[2], h->k_ms[2], 0.0};
  std::memcpy(times, v, sizeof(v));
  return IETI_OK;
}

int ieti_get_lambda(const ieti_handle* h, double* lambda_out) {
  if (!h || !lambda_out) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  std::copy(h->lambda_h.begin(), h->lambda_h.end(), lambda_out);
  return IETI_OK;
}

void ieti_destroy(ieti_handle* h) { delete h; }

int ieti_set_coefficients(ieti_handle* h, const double* nu_per_patch, const double* load_scale) {
  if (!h) return fail(IETI_ERR_INVALID_ARG, "handle is NULL");
  auto& M = h->model;
  if (h->stream) HIP_TRY(hipStreamSynchronize(h->stream));
  const std::vector<double> nu(nu_per_patch ? std::vector<double>(nu_per_patch, nu_per_patch + M.part.size()) : M.nu);
  const std::vector<double> sc(load_scale ? std::vector<double>(load_scale, load_scale + M.part.size())
                                          : M.load_scale);
  ieti::Error err{0, ""};
  if (ieti::set_coefficients(M, nu.data(), sc.data(), err)) return fail(err.code, err.msg);
  h->factored = false;
  h->rhs_ready = false;
  if (h->plan_T > 0) {
    ieti::refill_values(M, h->plan);
    if (h->uploaded) {
      const auto& P = h->plan;
      HIP_TRY(hipMemcpy(h->scatter_val.ptr, P.scatter_val.data(), P.scatter_val.size() * sizeof(double),
                        hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(h->b_aug0.ptr, P.b_aug0.data(), P.b_aug0.size() * sizeof(double), hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(h->piv_tol.ptr, P.piv_tol.data(), P.piv_tol.size() * sizeof(double), hipMemcpyHostToDevice));
    }
  }
  if (h->nu_d.ptr) {
    HIP_TRY(hipMemcpy(h->nu_d.ptr, M.nu.data(), M.nu.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->lscale_d.ptr, M.load_scale.data(), M.load_scale.size() * sizeof(double),
                      hipMemcpyHostToDevice));
  }
  return IETI_OK;
}

namespace {

// Checks a warm-start layout against the handle (and the network's sizes when given).
int check_layout(const ieti_handle* h, const ieti_warm_layout* L, const ieti::nn::Mlp* mlp) {
  const auto& M = h->model;
  const int64_t np = int64_t(M.part.size());
  if (!L) return fail(IETI_ERR_INVALID_ARG, "layout is NULL");
  if (L->n_facets < 1 || L->n_feat < 1 || L->n_comb < 1 || L->n_out < 1)
    return fail(IETI_ERR_INVALID_ARG, "layout sizes must be >= 1");
  if (mlp && (L->n_feat != mlp->arch.n_in || L->n_comb != mlp->arch.n_comb || L->n_out != mlp->arch.n_out))
    return fail(IETI_ERR_INVALID_ARG, "layout sizes do not match the network");
  if (!L->feat_patch || !L->comb_patch || !L->out_row || !L->out_sign)
    return fail(IETI_ERR_INVALID_ARG, "layout arrays are required");
  const int64_t nf = L->n_facets;
  for (int64_t i = 0; i < nf * L->n_feat; ++i)
    if (L->feat_patch[i] < 0 || L->feat_patch[i] >= np) return fail(IETI_ERR_INVALID_ARG, "feature patch out of range");
  for (int64_t i = 0; i < nf * L->n_comb; ++i)
    if (L->comb_patch[i] < 0 || L->comb_patch[i] >= np)
      return fail(IETI_ERR_INVALID_ARG, "coefficient patch out of range");
  std::vector<uint8_t> seen(M.m_r, 0);
  for (int64_t i = 0; i < nf * L->n_out; ++i) {
    const int32_t r = L->out_row[i];
    if (r < -1 || r >= M.m_r) return fail(IETI_ERR_INVALID_ARG, "output row out of range");
    if (r >= 0 && seen[r]++) return fail(IETI_ERR_INVALID_ARG, "output rows must be distinct");
    if (L->out_sign[i] != 1 && L->out_sign[i] != -1) return fail(IETI_ERR_INVALID_ARG, "output signs must be +-1");
  }
  return IETI_OK;
}

}  // namespace

int ieti_set_warm_start(ieti_handle* h, const ieti_nn* nn, const ieti_warm_layout* L) {
  if (!h || !nn || !L) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  const auto& mlp = ieti::nn::mlp_of(nn);
  const auto& M = h->model;
  int rc = check_layout(h, L, &mlp);
  if (rc) return rc;
  const int64_t nf = L->n_facets;
  auto& W = h->warm;
  W.release();
  W.mlp = mlp;
  W.n_facets = L->n_facets;
  W.n_feat = L->n_feat;
  W.n_comb = L->n_comb;
  W.n_out = L->n_out;
  W.out_scale = ieti::nn::out_scale_of(nn);
  HIP_TRY(hipStreamSynchronize(ieti::nn::stream_of(nn)));
  if ((rc = dalloc(W.theta, mlp.n_params))) return rc;
  HIP_TRY(hipMemcpy(W.theta.ptr, ieti::nn::params_of(nn), mlp.n_params * sizeof(float), hipMemcpyDeviceToDevice));
  if ((rc = dupload(W.feat_patch, L->feat_patch, nf * L->n_feat))) return rc;
  if ((rc = dupload(W.shift, ieti::nn::shift_of(nn)))) return rc;
  if ((rc = dupload(W.scale, ieti::nn::scale_of(nn)))) return rc;
  if ((rc = dupload(W.comb_patch, L->comb_patch, nf * L->n_comb))) return rc;
  if ((rc = dupload(W.out_row, L->out_row, nf * L->n_out))) return rc;
  if ((rc = dupload(W.out_sign, L->out_sign, nf * L->n_out))) return rc;
  if ((rc = dalloc(W.Cf, nf * L->n_comb))) return rc;
  if ((rc = W.work.reserve(W.mlp, nf, nullptr))) return rc;
  if ((rc = dupload(h->nu_d, M.nu))) return rc;
  if ((rc = dupload(h->lscale_d, M.load_scale))) return rc;
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(nullptr));
  W.on = true;
  return IETI_OK;
}

int ieti_warm_rows(const ieti_handle* h, const ieti_warm_layout* L, float* X, float* C, float* Y) {
  if (!h) return fail(IETI_ERR_INVALID_ARG, "handle is NULL");
  int rc = check_layout(h, L, nullptr);
  if (rc) return rc;
  const auto& M = h->model;
  const int64_t nf = L->n_facets;
  if (X)
    for (int64_t i = 0; i < nf * L->n_feat; ++i) X[i] = float(std::log(M.nu[L->feat_patch[i]]));
  if (C)
    for (int64_t i = 0; i < nf * L->n_comb; ++i) C[i] = float(M.load_scale[L->comb_patch[i]]);
  if (Y) {
    if (int64_t(h->lambda_h.size()) != M.m_r) return fail(IETI_ERR_STATE, "no solve has produced multipliers");
    for (int64_t i = 0; i < nf * L->n_out; ++i)
      Y[i] = L->out_row[i] >= 0 ? float(double(L->out_sign[i]) * h->lambda_h[L->out_row[i]]) : 0.f;
  }
  return IETI_OK;
}

int ieti_warm_append(const ieti_handle* h, const ieti_warm_layout* L, const char* dataset_path) {
  if (!h || !dataset_path) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  int rc = check_layout(h, L, nullptr);
  if (rc) return rc;
  const int64_t nf = L->n_facets;
  std::vector<float> X(nf * L->n_feat), C(nf * L->n_comb), Y(nf * L->n_out);
  if ((rc = ieti_warm_rows(h, L, X.data(), C.data(), Y.data()))) return rc;
  return ieti_nn_dataset_append(dataset_path, X.data(), C.data(), Y.data(), nf, L->n_feat, L->n_comb, L->n_out);
}

int ieti_warm_load(ieti_handle* h, const char* model_path, const ieti_warm_layout* L) {
  if (!h || !model_path || !L) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  ieti_nn* nn = nullptr;
  int rc = ieti_nn_load(model_path, &nn);
  if (rc) return rc;
  rc = ieti_set_warm_start(h, nn, L);
  ieti_nn_destroy(nn);
  return rc;
}

int ieti_warm_predict(ieti_handle* h, double* lambda0) {
  if (!h || !lambda0) return fail(IETI_ERR_INVALID_ARG, "NULL argument");
  if (!h->warm.on) return fail(IETI_ERR_STATE, "no network is attached");
  if (!h->factored) return fail(IETI_ERR_STATE, "not factored");
  const int64_t m_r = h->model.m_r;
  if (m_r == 0) return IETI_OK;
  warm_predict(h, h->tmp.ptr);
  int rc = check_launch();
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(lambda0, h->tmp.ptr, m_r * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return IETI_OK;
}

}  // extern "C"
