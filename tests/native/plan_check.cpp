// Host-side check of the factorisation schedule (test program, CPU only).
//
// Builds the library's plan for a box problem and runs its task lists in
// plain loops, as the GPU kernels define them (the tile pool from the
// destination-ordered entries, each tile's entries one range of the list):
// per level the S_rIrI copies,
// the diagonal-tile Cholesky with the inverse of its factor, the panel
// solves A L^{-T}, and the deferred updates C -= sum A B^T.  Then every tile
// of every subdomain is compared with the definition of the partial
// factorisation of the augmented matrix:
//   column tile l of r:        A_il = sum_{j <= l} L_ij L_lj^T
//   trailing (p, E_I) columns: tile = A_il - sum_{j in r} L_ij L_lj^T
//   S_rIrI copy:               A_il - sum_{j in r_V} L_ij L_lj^T   (i, l in r_I)
// and the lists are checked for offsets inside the pool, no target twice in
// one update launch, and no tile both written and read by one update launch.
//
// usage: plan_check P0 P1 P2 p n_el n_sub [defer defer_tail]   (patches per
// direction, degree, elements per patch, subdomains as contiguous ranges of
// patches, deferral thresholds of the updates)
// prints one line and exits 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

#include "host/model.hpp"
#include "host/plan.hpp"

using namespace ieti;

static void source(const double* x, int64_t n, double* o, void*) {
  for (int64_t i = 0; i < n; ++i) {
    o[3 * i] = std::sin(3 * x[3 * i + 1]);
    o[3 * i + 1] = std::cos(2 * x[3 * i + 2]);
    o[3 * i + 2] = x[3 * i];
  }
}

int main(int argc, char** argv) {
  if (argc != 7 && argc != 9) {
    std::fprintf(stderr, "usage: plan_check P0 P1 P2 p n_el n_sub [defer defer_tail]\n");
    return 2;
  }
  const int P0 = std::atoi(argv[1]), P1 = std::atoi(argv[2]), P2 = std::atoi(argv[3]);
  const int p = std::atoi(argv[4]), nel = std::atoi(argv[5]), nsub = std::atoi(argv[6]);
  const int np = P0 * P1 * P2;
  ieti_problem pr{};
  pr.version = IETI_ABI_VERSION;
  pr.geom_kind = 0;
  pr.patches[0] = P0;
  pr.patches[1] = P1;
  pr.patches[2] = P2;
  const double box[6] = {0, 1, 0, 1, 0, 1};
  for (int i = 0; i < 6; ++i) pr.geom_params[i] = box[i];
  pr.degree_p = p;
  pr.n_el = nel;
  std::vector<int32_t> part(np);
  for (int i = 0; i < np; ++i) part[i] = int32_t(int64_t(i) * nsub / np);
  std::vector<double> nu(np);
  for (int i = 0; i < np; ++i) nu[i] = 1.0 + 0.37 * i;
  pr.patch_to_subdomain = part.data();
  pr.nu_per_patch = nu.data();
  pr.J = source;
  Model m;
  m.prob = pr;
  m.part = part;
  m.nu = nu;
  m.n_sub = nsub;
  m.mesh.init(pr);
  Error err{0, ""};
  if (build_topology(m, err) || assemble_local_systems(m, err)) {
    std::printf("assembly failed: %s\n", err.msg.c_str());
    return 1;
  }
  finalize_single(m);
  Plan plan;
  PlanParams pp;
  if (argc == 9) {
    pp.defer = std::atoi(argv[7]);
    pp.defer_tail = std::atoi(argv[8]);
  }
  if (build_plan(m, 64, 0, plan, err, pp)) {
    std::printf("plan failed: %s\n", err.msg.c_str());
    return 1;
  }
  const int T = 64;
  const int64_t TT = int64_t(T) * T;
  auto in_pool = [&](int64_t o) { return o >= 0 && o + TT <= plan.pool_elems; };
  std::vector<double> pool(size_t(plan.pool_elems), 0.0), inv(size_t(plan.inv_elems), 0.0);
  std::set<int64_t> seen;
  for (size_t i = 0; i < plan.scatter_dst.size(); ++i) {
    if (!seen.insert(plan.scatter_dst[i]).second) {
      std::printf("scatter: destination %ld repeated\n", long(plan.scatter_dst[i]));
      return 1;
    }
    pool[size_t(plan.scatter_dst[i])] = plan.scatter_val[i];
  }
  // the per-tile ranges of the destination-ordered list (the tile assembly's input)
  if (plan.tile_ptr.size() != size_t(plan.pool_elems / TT) + 1 || plan.tile_ptr.front() != 0 ||
      plan.tile_ptr.back() != int64_t(plan.scatter_dst.size())) {
    std::printf("scatter: tile ranges do not cover the list\n");
    return 1;
  }
  for (size_t t = 0; t + 1 < plan.tile_ptr.size(); ++t)
    for (int64_t i = plan.tile_ptr[t]; i < plan.tile_ptr[t + 1]; ++i)
      if (plan.scatter_dst[size_t(i)] / TT != int64_t(t)) {
        std::printf("scatter: entry %ld outside its tile range\n", long(i));
        return 1;
      }
  const std::vector<double> A0 = pool;
  std::vector<double> S(size_t(plan.S_elems), 0.0);
  int64_t products = 0;
  for (int64_t lv = 0; lv < plan.n_steps; ++lv) {
    for (int64_t t = plan.copy_ptr[lv]; t < plan.copy_ptr[lv + 1]; ++t) {
      const int64_t* c = &plan.copy_task[5 * t];
      for (int b = 0; b < T; ++b)
        for (int a = 0; a < T; ++a) {
          if (c[4] && a < b) continue;
          const double v = pool[size_t(c[0] + b * T + a)];
          S[size_t(c[1] + a * c[3] + b)] = v;
          if (c[2] >= 0 && !(c[4] && a == b)) S[size_t(c[2] + b * c[3] + a)] = v;
        }
    }
    for (int64_t t = plan.potrf_ptr[lv]; t < plan.potrf_ptr[lv + 1]; ++t) {
      double* A = &pool[size_t(plan.potrf_task[3 * t])];
      double* X = &inv[size_t(plan.potrf_task[3 * t + 2])];
      for (int k = 0; k < T; ++k) {
        if (!(A[k * T + k] > 0.0)) {
          std::printf("potrf: non-positive pivot at level %ld\n", long(lv));
          return 1;
        }
        const double piv = std::sqrt(A[k * T + k]);
        A[k * T + k] = piv;
        for (int i = k + 1; i < T; ++i) A[k * T + i] /= piv;
        for (int jj = k + 1; jj < T; ++jj)
          for (int i = jj; i < T; ++i) A[jj * T + i] -= A[k * T + i] * A[k * T + jj];
      }
      for (int b = 0; b < T; ++b)
        for (int a = 0; a < b; ++a) A[b * T + a] = 0.0;
      for (int c = 0; c < T; ++c)
        for (int r = 0; r < T; ++r) {
          if (r < c) {
            X[c * T + r] = 0.0;
            continue;
          }
          if (r == c) {
            X[c * T + r] = 1.0 / A[c * T + c];
            continue;
          }
          double v = 0.0;
          for (int q = c; q < r; ++q) v += A[q * T + r] * X[c * T + q];
          X[c * T + r] = -v / A[r * T + r];
        }
    }
    for (int64_t t = plan.trsm_ptr[lv]; t < plan.trsm_ptr[lv + 1]; ++t) {
      double* A = &pool[size_t(plan.trsm_task[2 * t])];
      const double* Li = &inv[size_t(plan.trsm_task[2 * t + 1])];
      std::vector<double> O(size_t(TT), 0.0);
      for (int col = 0; col < T; ++col)
        for (int row = 0; row < T; ++row) {
          double s = 0.0;
          for (int k = 0; k < T; ++k) s += A[k * T + row] * Li[k * T + col];
          O[size_t(col * T + row)] = s;
        }
      for (int q = 0; q < T * T; ++q) A[q] = O[size_t(q)];
    }
    std::set<int64_t> written, read;
    for (int64_t t = plan.upd_ptr[lv]; t < plan.upd_ptr[lv + 1]; ++t) {
      const int64_t* tk = &plan.upd_task[3 * t];
      if (tk[2] <= 0 || !in_pool(tk[0]) || !written.insert(tk[0]).second) {
        std::printf("update: bad or repeated target at level %ld\n", long(lv));
        return 1;
      }
      std::vector<double> acc(size_t(TT), 0.0);
      for (int64_t q = 0; q < tk[2]; ++q) {
        const int64_t* o = &plan.upd_pair[2 * (tk[1] + q)];
        if (!in_pool(o[0]) || !in_pool(o[1])) {
          std::printf("update: operand outside the pool at level %ld\n", long(lv));
          return 1;
        }
        read.insert(o[0]);
        read.insert(o[1]);
        const double* A = &pool[size_t(o[0])];
        const double* B = &pool[size_t(o[1])];
        for (int col = 0; col < T; ++col)
          for (int k = 0; k < T; ++k) {
            const double bv = B[k * T + col];
            for (int row = 0; row < T; ++row) acc[size_t(col * T + row)] += A[k * T + row] * bv;
          }
        ++products;
      }
      double* C = &pool[size_t(tk[0])];
      for (int q = 0; q < T * T; ++q) C[q] -= acc[size_t(q)];
    }
    for (int64_t x : written)
      if (read.count(x)) {
        std::printf("update: tile written and read in one launch at level %ld\n", long(lv));
        return 1;
      }
  }
  if (products != plan.n_update_tasks) {
    std::printf("update: %ld products run, plan counts %ld\n", long(products), long(plan.n_update_tasks));
    return 1;
  }
  double worst = 0.0, worstS = 0.0;
  for (const SubPlan& sp : plan.sub) {
    const int64_t nt = sp.nt;
    auto off = [&](int64_t i, int64_t l) { return sp.tile_off[size_t(i * nt + l)]; };
    double scale = 0.0;
    for (int64_t a = 0; a < nt; ++a)
      if (off(a, a) >= 0)
        for (int q = 0; q < T * T; ++q) scale = std::max(scale, std::fabs(A0[size_t(off(a, a) + q)]));
    for (int64_t i = 0; i < nt; ++i)
      for (int64_t l = 0; l <= i; ++l) {
        const int64_t o = off(i, l);
        const bool inS = i >= sp.ntV && i < sp.ntr && l >= sp.ntV && l < sp.ntr;
        std::vector<double> M(size_t(TT), 0.0), MS;
        if (o >= 0)
          for (int q = 0; q < T * T; ++q) M[size_t(q)] = A0[size_t(o + q)];
        if (inS) MS = M;
        const int64_t jm = std::min<int64_t>(l + 1, sp.ntr);
        for (int64_t j = 0; j < jm; ++j) {
          if (off(i, j) < 0 || off(l, j) < 0) continue;
          const double* A = &pool[size_t(off(i, j))];
          const double* B = &pool[size_t(off(l, j))];
          for (int col = 0; col < T; ++col)
            for (int k = 0; k < T; ++k) {
              const double bv = B[k * T + col];
              for (int row = 0; row < T; ++row) {
                M[size_t(col * T + row)] -= A[k * T + row] * bv;
                if (inS && j < sp.ntV) MS[size_t(col * T + row)] -= A[k * T + row] * bv;
              }
            }
        }
        for (int col = 0; col < T; ++col)
          for (int row = 0; row < T; ++row) {
            if (i == l && row < col) continue;
            const double want = l < sp.ntr ? 0.0 : (o >= 0 ? pool[size_t(o + col * T + row)] : 0.0);
            worst = std::max(worst, std::fabs(M[size_t(col * T + row)] - want) / scale);
            if (inS) {
              const int64_t r0 = (i - sp.ntV) * T + row, c0 = (l - sp.ntV) * T + col;
              const double v = MS[size_t(col * T + row)];
              worstS = std::max(worstS, std::fabs(S[size_t(sp.S_off + r0 * sp.nIp + c0)] - v) / scale);
              worstS = std::max(worstS, std::fabs(S[size_t(sp.S_off + c0 * sp.nIp + r0)] - v) / scale);
            }
          }
      }
  }
  std::printf("levels %ld update tasks %ld products %ld factor residual %.3e S residual %.3e\n", long(plan.n_steps),
              long(plan.upd_task.size() / 3), long(products), worst, worstS);
  return (worst < 1e-12 && worstS < 1e-12) ? 0 : 1;
}
