// Ordering, padding, tile-level symbolic factorisation and task lists.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>

namespace ieti {

namespace {

// Nested dissection of the r_V DOFs by recursive coordinate bisection with
// one-sided vertex separators taken from the sparsity graph of K_VV.
// Blocks (leaves and separators) are appended to `out` in elimination order.
void nested_dissection(const std::vector<std::vector<int32_t>>& adj, const std::vector<double>& xyz,
                       std::vector<int32_t>& ids, std::vector<std::vector<int32_t>>& out, std::vector<int8_t>& side,
                       int leaf) {
  if (int(ids.size()) <= leaf) {
    if (!ids.empty()) out.push_back(ids);
    return;
  }
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int32_t v : ids)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], xyz[3 * v + a]);
      hi[a] = std::max(hi[a], xyz[3 * v + a]);
    }
  int ax = 0;
  for (int a = 1; a < 3; ++a)
    if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
  std::vector<double> c(ids.size());
  for (size_t i = 0; i < ids.size(); ++i) c[i] = xyz[3 * ids[i] + ax];
  std::vector<double> cs = c;
  std::nth_element(cs.begin(), cs.begin() + cs.size() / 2, cs.end());
  const double mid = cs[cs.size() / 2];
  std::vector<int32_t> left, right, sep;
  for (size_t i = 0; i < ids.size(); ++i) {
    if (c[i] < mid) {
      left.push_back(ids[i]);
      side[ids[i]] = 1;
    } else {
      right.push_back(ids[i]);
      side[ids[i]] = 2;
    }
  }
  if (left.empty() || right.empty()) {
    for (int32_t v : ids) side[v] = 0;
    out.push_back(ids);
    return;
  }
  std::vector<int32_t> right2;
  for (int32_t v : right) {
    bool touches = false;
    for (int32_t u : adj[v])
      if (side[u] == 1) {
        touches = true;
        break;
      }
    (touches ? sep : right2).push_back(v);
  }
  for (int32_t v : ids) side[v] = 0;
  nested_dissection(adj, xyz, left, out, side, leaf);
  nested_dissection(adj, xyz, right2, out, side, leaf);
  if (!sep.empty()) out.push_back(sep);
}

int64_t round_up(int64_t x, int64_t t) { return (x + t - 1) / t * t; }


// Scalar-level work of the Cholesky factorisation in the plan's elimination
// order (r_V by nested dissection, then r_I), from the elimination tree and
// the row subtrees (no tiles, no padding):
//   rr  = sum_j c_j^2 over the r columns, c_j the off-diagonal count of
//         column j of L with L L^T = K_rr (the local factorisation itself);
//   aug = the same sum when the columns also carry the trailing rows of the
//         augmented matrix (K_pr and E_I^T), i.e. the scalar work of the
//         partial factorisation that yields the explicit interface blocks.
void scalar_factor_work(const Subdomain& s, const SubPlan& sp, double& rr, double& aug) {
  const int64_t nr = int64_t(s.r_edges.size());
  rr = aug = 0.0;
  if (nr == 0) return;
  // elimination order of the r DOFs: increasing augmented position
  std::vector<int32_t> order(nr);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return sp.pos_of_local[a] < sp.pos_of_local[b]; });
  std::vector<int32_t> newi(nr);
  for (int64_t q = 0; q < nr; ++q) newi[order[q]] = int32_t(q);
  // lower entries of each row (columns before it) in the new order
  std::vector<std::vector<int32_t>> lower(nr);
  for (int64_t r = 0; r < nr; ++r)
    for (int64_t q = s.indptr[r]; q < s.indptr[r + 1]; ++q) {
      const int32_t c = s.indices[q];
      if (c < nr && newi[c] < newi[r]) lower[newi[r]].push_back(newi[c]);
    }
  // elimination tree (Liu, with path compression through `anc`)
  std::vector<int32_t> parent(nr, -1), anc(nr, -1);
  for (int32_t i = 0; i < int32_t(nr); ++i)
    for (int32_t j : lower[i])
      while (j != -1 && j < i) {
        const int32_t nx = anc[j];
        anc[j] = i;
        if (nx == -1) {
          parent[j] = i;
          break;
        }
        j = nx;
      }
  // column counts: row i of L is the union of the tree paths from its
  // entries up to i; trailing rows take the paths up to the root
  std::vector<int64_t> cnt(nr, 0), tcnt(nr, 0);
  std::vector<int32_t> mark(nr, -1);
  for (int32_t i = 0; i < int32_t(nr); ++i) {
    mark[i] = i;
    for (int32_t j : lower[i])
      for (int32_t k = j; k != -1 && mark[k] != i; k = parent[k]) {
        mark[k] = i;
        ++cnt[k];
      }
  }
  int32_t tag = int32_t(nr);
  auto trailing_row = [&](const std::vector<int32_t>& cols) {
    std::vector<int32_t>& mk = mark;
    for (int32_t j : cols)
      for (int32_t k = j; k != -1 && mk[k] != tag; k = parent[k]) {
        mk[k] = tag;
        ++tcnt[k];
      }
    ++tag;
  };
  std::fill(mark.begin(), mark.end(), -1);
  const int64_t np = s.n_loc - nr;
  std::vector<std::vector<int32_t>> prow(np);
  for (int64_t r = 0; r < nr; ++r)
    for (int64_t q = s.indptr[r]; q < s.indptr[r + 1]; ++q)
      if (s.indices[q] >= nr) prow[s.indices[q] - nr].push_back(newi[r]);
  for (auto& row : prow) trailing_row(row);
  for (int32_t t : s.I_local) trailing_row(std::vector<int32_t>{newi[t]});
  for (int64_t j = 0; j < nr; ++j) {
    rr += double(cnt[j]) * double(cnt[j]);
    aug += double(cnt[j] + tcnt[j]) * double(cnt[j] + tcnt[j]);
  }
}

}  // namespace

// Deferred updates: the contribution L_ij L_lj^T of column j to the target
// tile (i, l) may be applied at any level from level(j) up to the last level
// before the target is read (level(l) - 1 for a column of r, the level
// before the S copy for r_V contributions to the r_I block, the subdomain's
// last level for the trailing p / E_I columns).  Contributions are held back
// until pp.defer of them are pending (pp.defer_tail inside the subdomain's
// dense r_I tail, where one column per level leaves few targets and a task's
// pairs run in series) or the deadline is reached, so that a target tile is
// read and written once per batch of contributions instead of once per
// contributing level.  The decision depends on the subdomain and the
// parameters alone, so a subdomain gets the same tasks in a batch as on its
// own.  Only these lists depend on the parameters.
int build_update_tasks(Plan& plan, const PlanParams& pp, Error& err) {
  const int S = int(plan.sub.size());
  const int64_t n_levels = plan.n_steps;
  plan.upd_task.clear();
  plan.upd_pair.clear();
  plan.upd_ptr.assign(1, 0);
  struct Pending {
    std::vector<int64_t> cols;  // contributing columns in order of arrival
    int64_t deadline = 0;
  };
  struct LevelUpdates {
    std::vector<int64_t> upd, pair;
  };
  std::vector<std::vector<LevelUpdates>> lt(S);
  std::vector<int> left_over(S, 0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < S; ++k) {
    const SubPlan& sp = plan.sub[k];
    const int64_t nt = sp.nt;
    const auto& lev = plan.col_level[k];
    auto off = [&](int64_t i, int64_t l) { return sp.tile_off[i * nt + l]; };
    std::vector<std::vector<int64_t>> cols(size_t(sp.nlev));
    for (int64_t j = 0; j < sp.ntr; ++j) cols[size_t(lev[j])].push_back(j);
    std::map<int64_t, Pending> P;  // keyed by target i * nt + l
    lt[k].resize(size_t(sp.nlev));
    for (int64_t lv = 0; lv < sp.nlev; ++lv) {
      LevelUpdates& out = lt[k][size_t(lv)];
      for (int64_t j : cols[size_t(lv)]) {
        std::vector<int64_t> rows;
        for (int64_t i = j + 1; i < nt; ++i)
          if (off(i, j) >= 0) rows.push_back(i);
        for (size_t x = 0; x < rows.size(); ++x)
          for (size_t y = 0; y <= x; ++y) {
            const int64_t i = rows[x], l = rows[y];
            int64_t dl = l < sp.ntr ? lev[l] - 1 : sp.nlev - 1;
            if (j < sp.ntV && l >= sp.ntV && l < sp.ntr) dl = std::min<int64_t>(dl, sp.levS - 1);
            auto it = P.find(i * nt + l);
            if (it == P.end()) {
              it = P.emplace(i * nt + l, Pending{}).first;
              it->second.deadline = dl;
            }
            it->second.cols.push_back(j);
            it->second.deadline = std::min(it->second.deadline, dl);
          }
      }
      for (auto it = P.begin(); it != P.end();) {
        const Pending& q = it->second;
        if (int64_t(q.cols.size()) < (lv >= sp.levS ? pp.defer_tail : pp.defer) && q.deadline > lv) {
          ++it;
          continue;
        }
        const int64_t i = it->first / nt, l = it->first % nt;
        const int64_t p0 = int64_t(out.pair.size() / 2);  // local; made global when concatenated
        for (int64_t j : q.cols) out.pair.insert(out.pair.end(), {off(i, j), off(l, j)});
        out.upd.insert(out.upd.end(), {off(i, l), p0, int64_t(q.cols.size())});
        it = P.erase(it);
      }
    }
    left_over[k] = P.empty() ? 0 : 1;
  }
  for (int k = 0; k < S; ++k)
    if (left_over[k]) {
      err = Error{IETI_ERR_STATE, "plan: deferred tile updates left at the end of the schedule"};
      return err.code;
    }
  for (int64_t lv = 0; lv < n_levels; ++lv) {
    for (int k = 0; k < S; ++k) {
      if (lv >= int64_t(lt[k].size())) continue;
      const LevelUpdates& t = lt[k][size_t(lv)];
      const int64_t base = int64_t(plan.upd_pair.size() / 2);
      plan.upd_pair.insert(plan.upd_pair.end(), t.pair.begin(), t.pair.end());
      for (size_t q = 0; q < t.upd.size(); q += 3)
        plan.upd_task.insert(plan.upd_task.end(), {t.upd[q], t.upd[q + 1] + base, t.upd[q + 2]});
    }
    plan.upd_ptr.push_back(int64_t(plan.upd_task.size() / 3));
  }
  plan.n_update_tasks = int64_t(plan.upd_pair.size() / 2);
  plan.params = pp;
  return IETI_OK;
}

int build_plan(const Model& m, int T, int ordering, Plan& plan, Error& err, const PlanParams& pp) {
  plan = Plan();
  plan.T = T;
  const int S = m.n_sub;
  plan.sub.resize(S);
  // ---------------------------------------------------------------- per subdomain
  std::vector<std::vector<std::vector<uint64_t>>> present(S);  // column bitsets
  int64_t pool = 0, S_elems = 0, I_total = 0, P_total = 0, r_total = 0;
  // ordering and tile structure are independent per subdomain (host threads);
  // offsets are assigned afterwards in subdomain order
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < S; ++k) {
    const Subdomain& s = m.sd[k];
    SubPlan& sp = plan.sub[k];
    const Mesh& M = m.mesh_of(k);
    sp.nV = int64_t(s.V_local.size());
    sp.nI = int64_t(s.I_local.size());
    sp.nP = int64_t(s.p_edges.size());
    sp.nIp = round_up(sp.nI, T);
    sp.nPp = round_up(sp.nP, T);
    const int64_t nr = int64_t(s.r_edges.size());
    // ---- ordering of r_V: nested-dissection blocks, each padded to whole
    // tiles with identity dummies so that independent subtrees never share
    // a tile (their columns then sit on independent levels of the schedule)
    std::vector<int32_t> vslot;  // augmented position -> V index, -1 = dummy
    if (ordering == 0 && sp.nV > 0) {
      std::vector<int32_t> vidx(nr, -1);
      for (int32_t t = 0; t < int32_t(sp.nV); ++t) vidx[s.V_local[t]] = t;
      std::vector<std::vector<int32_t>> adj(sp.nV);
      for (int32_t t = 0; t < int32_t(sp.nV); ++t) {
        const int32_t r = s.V_local[t];
        for (int64_t q = s.indptr[r]; q < s.indptr[r + 1]; ++q) {
          const int32_t c = s.indices[q];
          if (c < nr && vidx[c] >= 0 && vidx[c] != t) adj[t].push_back(vidx[c]);
        }
      }
      std::vector<double> xyz(3 * sp.nV);
      for (int32_t t = 0; t < int32_t(sp.nV); ++t) {
        int d;
        int64_t X[3];
        M.decode_edge(s.r_edges[s.V_local[t]], d, X);
        for (int a = 0; a < 3; ++a) xyz[3 * t + a] = double(X[a]) + (a == d ? 0.5 : 0.0);
        // periodic axes: unwrap around the subdomain's first DOF
        for (int a = 0; a < 3; ++a)
          if (M.per[a] && t > 0) {
            const double ref = xyz[a];
            const double L = double(M.N[a]);
            while (xyz[3 * t + a] - ref > 0.5 * L) xyz[3 * t + a] -= L;
            while (xyz[3 * t + a] - ref < -0.5 * L) xyz[3 * t + a] += L;
          }
      }
      std::vector<int32_t> ids(sp.nV);
      std::iota(ids.begin(), ids.end(), 0);
      std::vector<int8_t> side(sp.nV, 0);
      std::vector<std::vector<int32_t>> blocks;
      nested_dissection(adj, xyz, ids, blocks, side, 4 * T);
      for (const auto& b : blocks) {
        vslot.insert(vslot.end(), b.begin(), b.end());
        while (vslot.size() % T) vslot.push_back(-1);
      }
    } else {
      for (int32_t t = 0; t < int32_t(sp.nV); ++t) vslot.push_back(t);
      while (vslot.size() % T) vslot.push_back(-1);
    }
    sp.nVp = int64_t(vslot.size());
    sp.ntV = sp.nVp / T;
    sp.ntr = sp.ntV + sp.nIp / T;
    sp.nt = sp.ntr + sp.nPp / T + sp.nIp / T;
    sp.vdummy.clear();
    for (int64_t q = 0; q < sp.nVp; ++q)
      if (vslot[q] < 0) sp.vdummy.push_back(q);
    // ---- augmented positions of local [r, p] DOFs
    sp.pos_of_local.assign(s.n_loc, -1);
    for (int64_t q = 0; q < sp.nVp; ++q)
      if (vslot[q] >= 0) sp.pos_of_local[s.V_local[vslot[q]]] = int32_t(q);
    for (int64_t t = 0; t < sp.nI; ++t) sp.pos_of_local[s.I_local[t]] = int32_t(sp.nVp + t);
    for (int64_t t = 0; t < sp.nP; ++t) sp.pos_of_local[nr + t] = int32_t(sp.nVp + sp.nIp + t);
    const int64_t a0 = sp.nVp + sp.nIp + sp.nPp;  // first augmented (E_I) position
    // ---- tile structure: initial nonzero tiles
    const int64_t nt = sp.nt;
    const int64_t words = (nt + 63) / 64;
    auto& col = present[k];
    col.assign(nt, std::vector<uint64_t>(words, 0));
    auto mark = [&](int64_t i, int64_t j) { col[j][i >> 6] |= (uint64_t(1) << (i & 63)); };
    auto has = [&](int64_t i, int64_t j) { return (col[j][i >> 6] >> (i & 63)) & 1; };
    for (int64_t t = 0; t < nt; ++t) mark(t, t);
    for (int64_t r = 0; r < s.n_loc; ++r) {
      const int64_t pr = sp.pos_of_local[r];
      for (int64_t q = s.indptr[r]; q < s.indptr[r + 1]; ++q) {
        const int64_t pc = sp.pos_of_local[s.indices[q]];
        if (pr >= pc) mark(pr / T, pc / T);
      }
    }
    for (int64_t t = 0; t < sp.nI; ++t) mark((a0 + t) / T, (sp.nVp + t) / T);
    // ---- symbolic right-looking fill over the r tiles
    for (int64_t j = 0; j < sp.ntr; ++j) {
      std::vector<int64_t> rows;
      for (int64_t i = j + 1; i < nt; ++i)
        if (has(i, j)) rows.push_back(i);
      for (size_t x = 0; x < rows.size(); ++x)
        for (size_t y = 0; y <= x; ++y) mark(rows[x], rows[y]);
    }
  }
  for (int k = 0; k < S; ++k) {
    SubPlan& sp = plan.sub[k];
    const int64_t nt = sp.nt;
    const auto& col = present[k];
    auto has = [&](int64_t i, int64_t j) { return (col[j][i >> 6] >> (i & 63)) & 1; };
    // ---- pool offsets
    sp.tile_off.assign(nt * nt, -1);
    for (int64_t j = 0; j < nt; ++j)
      for (int64_t i = j; i < nt; ++i)
        if (has(i, j)) {
          sp.tile_off[i * nt + j] = pool;
          pool += int64_t(T) * T;
        }
    sp.S_off = S_elems;
    S_elems += sp.nIp * sp.nIp;
    sp.I_off = I_total;
    I_total += sp.nIp;
    sp.P_off = P_total;
    P_total += sp.nP;
    sp.r_off = r_total;
    r_total += nt * T;
    sp.Phi_off = plan.Phi_elems;
    plan.Phi_elems += sp.nIp * sp.nPp;
    sp.SPi_off = plan.SPi_elems;
    plan.SPi_elems += sp.nPp * sp.nPp;
  }
  plan.pool_elems = pool;
  plan.S_elems = S_elems;
  {
    std::vector<double> rr(S, 0.0), aug(S, 0.0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < S; ++k) scalar_factor_work(m.sd[k], plan.sub[k], rr[k], aug[k]);
    for (int k = 0; k < S; ++k) {
      plan.flops_scalar_rr += rr[k];
      plan.flops_scalar_aug += aug[k];
    }
  }
  plan.I_total = I_total;
  plan.P_total = P_total;
  plan.r_total = r_total;
  // ---------------------------------------------------------------- scatter list
  {
  std::vector<int64_t> voffs(S + 1, 0);
  for (int k = 0; k < S; ++k) voffs[k + 1] = voffs[k] + m.sd[k].indptr[m.sd[k].n_loc];
  std::vector<std::vector<int64_t>> sdst(S), ssrc(S);
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < S; ++k) {
    const Subdomain& s = m.sd[k];
    const SubPlan& sp = plan.sub[k];
    const int64_t nt = sp.nt;
    const int64_t voff = voffs[k];
    auto put = [&](int64_t pr, int64_t pc, int64_t src) {
      const int64_t ti = pr / T, tj = pc / T;
      const int64_t off = sp.tile_off[ti * nt + tj];
      sdst[k].push_back(off + (pc % T) * T + (pr % T));
      ssrc[k].push_back(src);
    };
    for (int64_t r = 0; r < s.n_loc; ++r) {
      const int64_t pr = sp.pos_of_local[r];
      for (int64_t q = s.indptr[r]; q < s.indptr[r + 1]; ++q) {
        const int64_t pc = sp.pos_of_local[s.indices[q]];
        if (pr / T > pc / T || (pr / T == pc / T)) put(pr, pc, voff + q);
      }
    }
    for (int64_t q : sp.vdummy) put(q, q, -2 - k);
    for (int64_t t = sp.nVp + sp.nI; t < sp.nVp + sp.nIp; ++t) put(t, t, -2 - k);
    const int64_t a0 = sp.nVp + sp.nIp + sp.nPp;
    for (int64_t t = 0; t < sp.nI; ++t) put(a0 + t, sp.nVp + t, -1);
    // Destination order, so that consecutive threads of the scatter write
    // consecutive pool entries (CSR order writes one entry per 512-byte tile
    // column): two stable counting passes, by offset inside the tile, then by
    // tile.  A subdomain's tiles occupy a range of the pool of their own, so
    // sorting each subdomain's entries sorts the whole list; destinations are
    // distinct, so the order changes no value.
    auto& dk = sdst[k];
    auto& sk = ssrc[k];
    const size_t n = dk.size();
    if (n > 0) {
      const int64_t TT = int64_t(T) * T;
      int64_t t0 = dk[0] / TT, t1 = t0;
      for (int64_t d : dk) {
        t0 = std::min(t0, d / TT);
        t1 = std::max(t1, d / TT);
      }
      std::vector<int64_t> d2(n), s2(n);
      auto pass = [n](const std::vector<int64_t>& da, const std::vector<int64_t>& sa, std::vector<int64_t>& dd,
                      std::vector<int64_t>& sd, int64_t nb, auto key) {
        std::vector<int64_t> cnt(size_t(nb) + 1, 0);
        for (size_t i = 0; i < n; ++i) ++cnt[size_t(key(da[i])) + 1];
        for (int64_t b = 0; b < nb; ++b) cnt[size_t(b) + 1] += cnt[size_t(b)];
        for (size_t i = 0; i < n; ++i) {
          const int64_t q = cnt[size_t(key(da[i]))]++;
          dd[size_t(q)] = da[i];
          sd[size_t(q)] = sa[i];
        }
      };
      pass(dk, sk, d2, s2, TT, [TT](int64_t d) { return d % TT; });
      pass(d2, s2, dk, sk, t1 - t0 + 1, [TT, t0](int64_t d) { return d / TT - t0; });
    }
  }
  {
    size_t total = 0;
    for (int k = 0; k < S; ++k) total += sdst[k].size();
    plan.scatter_dst.reserve(total);
    plan.scatter_src.reserve(total);
  }
  for (int k = 0; k < S; ++k) {
    plan.scatter_dst.insert(plan.scatter_dst.end(), sdst[k].begin(), sdst[k].end());
    plan.scatter_src.insert(plan.scatter_src.end(), ssrc[k].begin(), ssrc[k].end());
    std::vector<int64_t>().swap(sdst[k]);
    std::vector<int64_t>().swap(ssrc[k]);
  }
  // the pool is whole tiles and the list is in destination order: each
  // tile's entries form one range
  {
    const int64_t TT = int64_t(T) * T;
    plan.tile_ptr.assign(size_t(plan.pool_elems / TT) + 1, 0);
    for (int64_t d : plan.scatter_dst) ++plan.tile_ptr[size_t(d / TT) + 1];
    for (size_t t = 1; t < plan.tile_ptr.size(); ++t) plan.tile_ptr[t] += plan.tile_ptr[t - 1];
  }
  }
  // ---------------------------------------------------------------- level schedule
  // Column j of the tile factor depends on every column k < j with a tile
  // (j, k); level(j) = 1 + max level(k).  Columns of one level are
  // independent, so each level is one batched potrf, trsm and update launch.
  // The r_I columns (a dense block) follow all r_V columns, so that S_rIrI
  // is complete at the start of the first r_I level.
  std::vector<std::vector<int32_t>> lev(S);
  std::vector<std::vector<int64_t>> inv_off(S);
  int64_t n_levels = 0, inv_elems = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < S; ++k) {
    SubPlan& sp = plan.sub[k];
    const int64_t nt = sp.nt;
    auto& L = lev[k];
    L.assign(sp.ntr, 0);
    int32_t maxV = -1;
    for (int64_t j = 0; j < sp.ntV; ++j) {
      maxV = std::max(maxV, L[j]);
      for (int64_t i = j + 1; i < sp.ntV; ++i)
        if (sp.tile_off[i * nt + j] >= 0) L[i] = std::max(L[i], L[j] + 1);
    }
    for (int64_t j = sp.ntV; j < sp.ntr; ++j) L[j] = maxV + 1 + int32_t(j - sp.ntV);
    sp.levS = maxV + 1;
    sp.nlev = sp.ntr > 0 ? (sp.ntr > sp.ntV ? L[sp.ntr - 1] + 1 : maxV + 1) : 0;
  }
  for (int k = 0; k < S; ++k) {
    const SubPlan& sp = plan.sub[k];
    n_levels = std::max<int64_t>(n_levels, sp.nlev);
    inv_off[k].assign(sp.ntr, 0);
    for (int64_t j = 0; j < sp.ntr; ++j) {
      inv_off[k][j] = inv_elems;
      inv_elems += int64_t(T) * T;
    }
  }
  plan.n_steps = n_levels;
  plan.inv_elems = inv_elems;
  // columns of each level, per subdomain
  std::vector<std::vector<std::vector<int64_t>>> cols(S);
  for (int k = 0; k < S; ++k) {
    cols[k].assign(n_levels, {});
    for (int64_t j = 0; j < plan.sub[k].ntr; ++j) cols[k][lev[k][j]].push_back(j);
  }
  plan.potrf_ptr.assign(1, 0);
  plan.trsm_ptr.assign(1, 0);
  plan.copy_ptr.assign(1, 0);
  const double T3 = double(T) * T * T;
  // Each subdomain's task lists are built on its own (host threads), level
  // by level, then concatenated level by level in subdomain order.
  struct LevelTasks {
    std::vector<int64_t> copy, potrf, trsm;
  };
  std::vector<std::vector<LevelTasks>> lt(S);
  std::vector<double> sub_flops(S, 0.0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < S; ++k) {
    const SubPlan& sp = plan.sub[k];
    const int64_t nt = sp.nt;
    auto off = [&](int64_t i, int64_t l) { return sp.tile_off[i * nt + l]; };
    lt[k].resize(size_t(sp.nlev));
    double fl = 0.0;
    for (int64_t lv = 0; lv < sp.nlev; ++lv) {
      LevelTasks& out = lt[k][size_t(lv)];
      if (lv == sp.levS && sp.nIp > 0) {
        for (int64_t i = sp.ntV; i < sp.ntr; ++i)
          for (int64_t l = sp.ntV; l <= i; ++l) {
            const int64_t o = off(i, l);
            if (o < 0) continue;
            const int64_t r0 = (i - sp.ntV) * T, c0 = (l - sp.ntV) * T;
            out.copy.insert(out.copy.end(),
                            {o, sp.S_off + r0 * sp.nIp + c0, sp.S_off + c0 * sp.nIp + r0, sp.nIp, i == l ? 1 : 0});
          }
      }
      for (int64_t j : cols[k][lv]) {
        out.potrf.insert(out.potrf.end(), {off(j, j), int64_t(k), inv_off[k][j]});
        fl += T3 / 3.0;
        int64_t nrow = 0;
        for (int64_t i = j + 1; i < nt; ++i)
          if (off(i, j) >= 0) {
            out.trsm.insert(out.trsm.end(), {off(i, j), inv_off[k][j]});
            fl += T3;
            ++nrow;
          }
        fl += 2.0 * T3 * double(nrow) * double(nrow + 1) / 2.0;  // one product per target (i, l), l <= i
      }
    }
    sub_flops[k] = fl;
  }
  for (int k = 0; k < S; ++k) plan.flops += sub_flops[k];
  for (int64_t lv = 0; lv < n_levels; ++lv) {
    for (int k = 0; k < S; ++k) {
      if (lv >= int64_t(lt[k].size())) continue;
      const LevelTasks& t = lt[k][size_t(lv)];
      plan.copy_task.insert(plan.copy_task.end(), t.copy.begin(), t.copy.end());
      plan.potrf_task.insert(plan.potrf_task.end(), t.potrf.begin(), t.potrf.end());
      plan.trsm_task.insert(plan.trsm_task.end(), t.trsm.begin(), t.trsm.end());
    }
    plan.potrf_ptr.push_back(int64_t(plan.potrf_task.size() / 3));
    plan.trsm_ptr.push_back(int64_t(plan.trsm_task.size() / 2));
    plan.copy_ptr.push_back(int64_t(plan.copy_task.size() / 5));
  }
  std::vector<std::vector<LevelTasks>>().swap(lt);
  plan.col_level = lev;
  if (int rc = build_update_tasks(plan, pp, err)) return rc;
  // ---------------------------------------------------------------- extraction lists
  for (int k = 0; k < S; ++k) {
    const SubPlan& sp = plan.sub[k];
    const int64_t nt = sp.nt;
    const int64_t tP = sp.ntr, tA = sp.ntr + sp.nPp / T;
    auto off = [&](int64_t i, int64_t l) { return sp.tile_off[i * nt + l]; };
    for (int64_t i = tA; i < nt; ++i)
      for (int64_t l = tA; l <= i; ++l) {
        const int64_t o = off(i, l);
        if (o < 0) continue;
        const int64_t r0 = (i - tA) * T, c0 = (l - tA) * T;
        plan.xsinv_task.insert(plan.xsinv_task.end(),
                               {o, sp.S_off + r0 * sp.nIp + c0, sp.S_off + c0 * sp.nIp + r0, sp.nIp, i == l ? 1 : 0});
      }
    for (int64_t i = tA; i < nt; ++i)
      for (int64_t l = tP; l < tA; ++l) {
        const int64_t o = off(i, l);
        if (o < 0) continue;
        const int64_t r0 = (i - tA) * T, c0 = (l - tP) * T;
        plan.xphi_task.insert(plan.xphi_task.end(), {o, sp.Phi_off + r0 * sp.nPp + c0, -1, sp.nPp, 0});
      }
    for (int64_t i = tP; i < tA; ++i)
      for (int64_t l = tP; l <= i; ++l) {
        const int64_t o = off(i, l);
        if (o < 0) continue;
        const int64_t r0 = (i - tP) * T, c0 = (l - tP) * T;
        plan.xspi_task.insert(plan.xspi_task.end(),
                              {o, sp.SPi_off + r0 * sp.nPp + c0, sp.SPi_off + c0 * sp.nPp + r0, sp.nPp, i == l ? 1 : 0});
      }
  }
  // ---------------------------------------------------------------- triangular-solve lists
  // Forward: per level, x_j = L_jj^{-1} y_j for the level's columns, then every
  // target row tile i gets y_i -= sum_j L_ij x_j over the level's columns.
  // Backward: levels in reverse, x_j = L_jj^{-T} y_j, then y_k -= sum_j L_jk^T x_j.
  plan.fdiag_ptr.assign(1, 0);
  plan.ffull_ptr.assign(1, 0);
  auto emit_targets = [&](std::vector<std::pair<int64_t, std::pair<int64_t, int64_t>>>& c, std::vector<int64_t>& task,
                          std::vector<int64_t>& pair) {
    std::stable_sort(c.begin(), c.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    size_t q = 0;
    while (q < c.size()) {
      size_t e = q;
      const int64_t p0 = int64_t(pair.size() / 2);
      while (e < c.size() && c[e].first == c[q].first) {
        pair.insert(pair.end(), {c[e].second.first, c[e].second.second});
        ++e;
      }
      task.insert(task.end(), {c[q].first, p0, int64_t(e - q)});
      q = e;
    }
  };
  // per subdomain and level (host threads), concatenated level by level in subdomain order
  struct SweepTasks {
    std::vector<int64_t> diag, task, pair;
  };
  std::vector<std::vector<SweepTasks>> fw(S), bw(S);
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < S; ++k) {
    const SubPlan& sp = plan.sub[k];
    const int64_t nt = sp.nt;
    fw[k].resize(size_t(sp.nlev));
    bw[k].resize(size_t(sp.nlev));
    for (int64_t lv = 0; lv < sp.nlev; ++lv) {
      std::vector<std::pair<int64_t, std::pair<int64_t, int64_t>>> full;  // (vec_i, (tile, vec_j))
      std::vector<std::pair<int64_t, std::pair<int64_t, int64_t>>> c;     // (vec_k, (tile (j,k), vec_j))
      for (int64_t j : cols[k][lv]) {
        fw[k][size_t(lv)].diag.insert(fw[k][size_t(lv)].diag.end(), {inv_off[k][j], sp.r_off + j * T});
        bw[k][size_t(lv)].diag.insert(bw[k][size_t(lv)].diag.end(), {inv_off[k][j], sp.r_off + j * T});
        for (int64_t i = j + 1; i < nt; ++i) {
          const int64_t o = sp.tile_off[i * nt + j];
          if (o < 0) continue;
          full.push_back({sp.r_off + i * T, {o, sp.r_off + j * T}});
        }
        for (int64_t i = 0; i < j; ++i) {
          const int64_t o = sp.tile_off[j * nt + i];
          if (o < 0) continue;
          c.push_back({sp.r_off + i * T, {o, sp.r_off + j * T}});
        }
      }
      emit_targets(full, fw[k][size_t(lv)].task, fw[k][size_t(lv)].pair);
      emit_targets(c, bw[k][size_t(lv)].task, bw[k][size_t(lv)].pair);
    }
  }
  auto append = [](const SweepTasks& t, std::vector<int64_t>& diag, std::vector<int64_t>& task,
                   std::vector<int64_t>& pair) {
    diag.insert(diag.end(), t.diag.begin(), t.diag.end());
    const int64_t base = int64_t(pair.size() / 2);
    pair.insert(pair.end(), t.pair.begin(), t.pair.end());
    for (size_t q = 0; q < t.task.size(); q += 3) task.insert(task.end(), {t.task[q], t.task[q + 1] + base, t.task[q + 2]});
  };
  for (int64_t lv = 0; lv < n_levels; ++lv) {
    for (int k = 0; k < S; ++k)
      if (lv < int64_t(fw[k].size())) append(fw[k][size_t(lv)], plan.fdiag_task, plan.ffull_task, plan.ffull_pair);
    plan.fdiag_ptr.push_back(int64_t(plan.fdiag_task.size() / 2));
    plan.ffull_ptr.push_back(int64_t(plan.ffull_task.size() / 3));
  }
  plan.bdiag_ptr.assign(1, 0);
  plan.bupd_ptr.assign(1, 0);
  for (int64_t lv = n_levels - 1; lv >= 0; --lv) {
    for (int k = 0; k < S; ++k)
      if (lv < int64_t(bw[k].size())) append(bw[k][size_t(lv)], plan.bdiag_task, plan.bupd_task, plan.bupd_pair);
    plan.bdiag_ptr.push_back(int64_t(plan.bdiag_task.size() / 2));
    plan.bupd_ptr.push_back(int64_t(plan.bupd_task.size() / 3));
  }
  // Recovery (Eq. localProb) without a forward sweep: the factor's primal rows
  // are L_pr = K_pr L_rr^{-T} and its E_I rows L_Er = E_I^T L_rr^{-T}, so
  // L_rr^{-1} (j_r - K_rp a_p - E_I u) = y_j - L_pr^T a_p - L_Er^T u with
  // y_j = L_rr^{-1} j_r from the right-hand side's forward solve: one
  // transposed update per r column tile over the primal and E_I row tiles.
  for (int k = 0; k < S; ++k) {
    const SubPlan& sp = plan.sub[k];
    const int64_t nt = sp.nt;
    for (int64_t c = 0; c < sp.ntr; ++c) {
      const int64_t p0 = int64_t(plan.rec_pair.size() / 2);
      for (int64_t i = sp.ntr; i < nt; ++i) {
        const int64_t o = sp.tile_off[i * nt + c];
        if (o >= 0) plan.rec_pair.insert(plan.rec_pair.end(), {o, sp.r_off + i * T});
      }
      const int64_t np = int64_t(plan.rec_pair.size() / 2) - p0;
      if (np > 0) plan.rec_task.insert(plan.rec_task.end(), {sp.r_off + c * T, p0, np});
    }
    const Subdomain& s = m.sd[k];
    for (int64_t t = 0; t < sp.nPp; ++t) {
      plan.recP_pos.push_back(sp.r_off + sp.nVp + sp.nIp + t);
      plan.recP_glob.push_back(t < sp.nP ? s.p_global[t] : -1);
    }
  }
  // ---------------------------------------------------------------- interface and primal maps
  plan.I_row.assign(I_total, -1);
  plan.I_sign.assign(I_total, 0.0);
  plan.I_aug.assign(I_total, 0);
  plan.A_aug.assign(I_total, 0);
  plan.I_sub.assign(I_total, 0);
  plan.row_src.assign(2 * m.m_r, -1);
  // ragged subdomain x (primal DOFs of the subdomain's problem) map
  plan.g2l_off.assign(S + 1, 0);
  for (int k = 0; k < S; ++k) plan.g2l_off[k + 1] = plan.g2l_off[k] + m.probs[m.sub_prob[k]].n_gp;
  plan.glob2loc.assign(size_t(plan.g2l_off[S]), -1);
  for (int k = 0; k < S; ++k) {
    const Subdomain& s = m.sd[k];
    const SubPlan& sp = plan.sub[k];
    const int64_t a0 = sp.nVp + sp.nIp + sp.nPp;
    for (int64_t t = 0; t < sp.nIp; ++t) {
      const int64_t slot = sp.I_off + t;
      plan.I_aug[slot] = sp.r_off + sp.nVp + t;
      plan.A_aug[slot] = sp.r_off + a0 + t;
      plan.I_sub[slot] = k;
      if (t < sp.nI) {
        plan.I_row[slot] = s.I_row[t];
        plan.I_sign[slot] = double(s.I_sign[t]);
        plan.row_src[2 * s.I_row[t] + (s.I_sign[t] > 0 ? 0 : 1)] = slot;
      }
    }
    for (int64_t t = 0; t < sp.nP; ++t) {
      plan.P_glob.push_back(s.p_global[t]);
      plan.P_aug.push_back(sp.r_off + sp.nVp + sp.nIp + t);
      plan.P_sub.push_back(k);
      plan.glob2loc[size_t(plan.g2l_off[k] + s.p_global[t] - m.probs[m.sub_prob[k]].gp_base)] = int32_t(t);
    }
  }
  // coarse matrices: per problem the sum over its subdomains of C_k^T SPi_k C_k
  // (dense n_gp,p x n_gp,p blocks, concatenated), sources in fixed order
  {
    plan.spi_off.assign(m.probs.size() + 1, 0);
    for (size_t q = 0; q < m.probs.size(); ++q)
      plan.spi_off[q + 1] = plan.spi_off[q] + m.probs[q].n_gp * m.probs[q].n_gp;
    std::vector<std::vector<int64_t>> src(size_t(plan.spi_off.back()));
    for (int k = 0; k < S; ++k) {
      const Subdomain& s = m.sd[k];
      const SubPlan& sp = plan.sub[k];
      const ProblemRange& pr = m.probs[m.sub_prob[k]];
      const int64_t base = plan.spi_off[m.sub_prob[k]];
      for (int64_t a = 0; a < sp.nP; ++a)
        for (int64_t b = 0; b < sp.nP; ++b)
          src[size_t(base + (s.p_global[a] - pr.gp_base) * pr.n_gp + (s.p_global[b] - pr.gp_base))].push_back(
              sp.SPi_off + a * sp.nPp + b);
    }
    plan.spi_ptr.assign(1, 0);
    for (auto& v : src) {
      plan.spi_src.insert(plan.spi_src.end(), v.begin(), v.end());
      plan.spi_ptr.push_back(int64_t(plan.spi_src.size()));
    }
  }
  // output map: augmented index and edge id of every owned r DOF
  for (int64_t k = 0; k < S; ++k) {
    const Subdomain& s = m.sd[k];
    const SubPlan& sp = plan.sub[k];
    const int64_t nr = int64_t(s.r_edges.size());
    for (int64_t r = 0; r < nr; ++r)
      if (s.owner[r]) {
        plan.out_src.push_back(sp.r_off + sp.pos_of_local[r]);
        plan.out_edge.push_back(s.r_edges[r] + m.probs[m.sub_prob[k]].edge_base);
      }
  }
  refill_values(m, plan);
  for (const auto& sp : plan.sub) {
    const double n = double(sp.nVp + sp.nIp);
    const double a = double(sp.nPp + sp.nIp);
    plan.dense_flops += n * n * n / 3.0 + n * n * a;
  }
  (void)err;
  return IETI_OK;
}

void refill_values(const Model& m, Plan& plan) {
  std::vector<const double*> vals;
  std::vector<int64_t> voff(1, 0);
  for (const auto& s : m.sd) {
    vals.push_back(s.values.data());
    voff.push_back(voff.back() + s.indptr[s.n_loc]);
  }
  auto value = [&](int64_t src) {
    const int64_t k = std::upper_bound(voff.begin(), voff.end(), src) - voff.begin() - 1;
    return vals[k][src - voff[k]];
  };
  // largest diagonal entry of each K_rr (local numbering [r, p], r first)
  std::vector<double> dmax(m.sd.size(), 0.0);
  for (size_t k = 0; k < m.sd.size(); ++k) {
    const Subdomain& s = m.sd[k];
    const int64_t nr = int64_t(s.r_edges.size());
    for (int64_t r = 0; r < nr; ++r)
      for (int64_t q = s.indptr[r]; q < s.indptr[r + 1]; ++q)
        if (s.indices[q] == r) dmax[k] = std::max(dmax[k], std::abs(s.values[q]));
    if (!(dmax[k] > 0.0)) dmax[k] = 1.0;
  }
  plan.piv_tol.resize(m.sd.size());
  for (size_t k = 0; k < m.sd.size(); ++k) plan.piv_tol[k] = Plan::PIVOT_REL * dmax[k];
  // the list is in destination order, so its sources are read out of order:
  // the entries are independent and split over the host threads
  plan.scatter_val.resize(plan.scatter_src.size());
  const int64_t ns = int64_t(plan.scatter_src.size());
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ns; ++i) {
    const int64_t src = plan.scatter_src[size_t(i)];
    plan.scatter_val[size_t(i)] = src >= 0 ? value(src) : src == -1 ? 1.0 : dmax[size_t(-2 - src)];
  }
  plan.b_aug0.assign(plan.r_total, 0.0);
  for (size_t k = 0; k < m.sd.size(); ++k) {
    const Subdomain& s = m.sd[k];
    const SubPlan& sp = plan.sub[k];
    for (int64_t r = 0; r < s.n_loc; ++r) plan.b_aug0[sp.r_off + sp.pos_of_local[r]] = s.load[r];
  }
}

void build_coarse_plan(const std::vector<CoarseDims>& dims, int T, CoarsePlan& cp) {
  cp = CoarsePlan();
  const int64_t TT = int64_t(T) * T;
  struct Prob {
    int64_t nc = 0, mt = 0;
    std::vector<int64_t> D, G, E;  // tile offsets: D[ci * nc + cj] (cj <= ci), G[r * nc + c], E[i * nc + c] (i <= c)
    int64_t inv0 = 0;
  };
  std::vector<Prob> pr(dims.size());
  int64_t off = 0, inv = 0;
  for (size_t p = 0; p < dims.size(); ++p) {
    const auto& d = dims[p];
    auto& q = pr[p];
    if (d.n <= 0) continue;
    q.nc = (d.n + T - 1) / T;
    q.mt = (d.m + T - 1) / T;
    q.D.assign(size_t(q.nc * q.nc), -1);
    q.G.assign(size_t(q.mt * q.nc), -1);
    q.E.assign(size_t(q.nc * q.nc), -1);
    for (int64_t ci = 0; ci < q.nc; ++ci)
      for (int64_t cj = 0; cj <= ci; ++cj) {
        q.D[size_t(ci * q.nc + cj)] = off;
        off += TT;
      }
    for (int64_t r = 0; r < q.mt; ++r)
      for (int64_t c = 0; c < q.nc; ++c) {
        q.G[size_t(r * q.nc + c)] = off;
        off += TT;
      }
    for (int64_t i = 0; i < q.nc; ++i)
      for (int64_t c = i; c < q.nc; ++c) {
        q.E[size_t(i * q.nc + c)] = off;
        off += TT;
      }
    q.inv0 = inv;
    inv += q.nc * TT;
    cp.n_levels = std::max(cp.n_levels, q.nc);
    // tile fill
    for (int64_t ci = 0; ci < q.nc; ++ci)
      for (int64_t cj = 0; cj <= ci; ++cj)
        cp.fill_task.insert(cp.fill_task.end(),
                            {q.D[size_t(ci * q.nc + cj)], 0, d.spi_off + ci * T * d.n + cj * T, d.n,
                             std::min<int64_t>(T, d.n - ci * T), std::min<int64_t>(T, d.n - cj * T), ci == cj ? 1 : 0});
    for (int64_t r = 0; r < q.mt; ++r)
      for (int64_t c = 0; c < q.nc; ++c)
        cp.fill_task.insert(cp.fill_task.end(),
                            {q.G[size_t(r * q.nc + c)], 1, d.g_off + r * T * d.n + c * T, d.n,
                             std::min<int64_t>(T, d.m - r * T), std::min<int64_t>(T, d.n - c * T), 0});
    for (int64_t i = 0; i < q.nc; ++i)
      for (int64_t c = i; c < q.nc; ++c)
        cp.fill_task.insert(cp.fill_task.end(), {q.E[size_t(i * q.nc + c)], -1, 0, 0, 0, 0, c == i ? 1 : 0});
    // extraction
    for (int64_t r = 0; r < q.mt; ++r)
      for (int64_t c = 0; c < q.nc; ++c)
        cp.out_h_task.insert(cp.out_h_task.end(),
                             {q.G[size_t(r * q.nc + c)], d.g_off + r * T * d.n + c * T, d.g_off + c * T * d.m + r * T,
                              d.n, d.m, std::min<int64_t>(T, d.m - r * T), std::min<int64_t>(T, d.n - c * T)});
    for (int64_t i = 0; i < q.nc; ++i)
      for (int64_t c = i; c < q.nc; ++c)
        cp.out_l_task.insert(cp.out_l_task.end(),
                             {q.E[size_t(i * q.nc + c)], d.spi_off + i * T * d.n + c * T, -1, d.n, 0,
                              std::min<int64_t>(T, d.n - i * T), std::min<int64_t>(T, d.n - c * T)});
  }
  cp.pool_elems = off;
  cp.inv_elems = inv;
  // level c: Cholesky of D(c, c); panel solves of every tile of column c below it
  // (D(ci, c), ci > c; G(r, c); E(i, c), i <= c); one update per target tile of a
  // later column c' with the column-c contribution X(., c) D(c', c)^T
  cp.potrf_ptr.push_back(0);
  cp.trsm_ptr.push_back(0);
  cp.upd_ptr.push_back(0);
  for (int64_t c = 0; c < cp.n_levels; ++c) {
    for (size_t p = 0; p < pr.size(); ++p) {
      const auto& q = pr[p];
      if (c >= q.nc) continue;
      cp.potrf_task.insert(cp.potrf_task.end(), {q.D[size_t(c * q.nc + c)], int64_t(p), q.inv0 + c * TT});
      const int64_t iv = q.inv0 + c * TT;
      for (int64_t ci = c + 1; ci < q.nc; ++ci) cp.trsm_task.insert(cp.trsm_task.end(), {q.D[size_t(ci * q.nc + c)], iv});
      for (int64_t r = 0; r < q.mt; ++r) cp.trsm_task.insert(cp.trsm_task.end(), {q.G[size_t(r * q.nc + c)], iv});
      for (int64_t i = 0; i <= c; ++i) cp.trsm_task.insert(cp.trsm_task.end(), {q.E[size_t(i * q.nc + c)], iv});
      for (int64_t c2 = c + 1; c2 < q.nc; ++c2) {
        const int64_t B = q.D[size_t(c2 * q.nc + c)];
        auto add = [&](int64_t target, int64_t A) {
          cp.upd_task.insert(cp.upd_task.end(), {target, int64_t(cp.upd_pair.size() / 2), 1});
          cp.upd_pair.insert(cp.upd_pair.end(), {A, B});
        };
        for (int64_t ci = c2; ci < q.nc; ++ci) add(q.D[size_t(ci * q.nc + c2)], q.D[size_t(ci * q.nc + c)]);
        for (int64_t r = 0; r < q.mt; ++r) add(q.G[size_t(r * q.nc + c2)], q.G[size_t(r * q.nc + c)]);
        for (int64_t i = 0; i <= c; ++i) add(q.E[size_t(i * q.nc + c2)], q.E[size_t(i * q.nc + c)]);
      }
    }
    cp.potrf_ptr.push_back(int64_t(cp.potrf_task.size() / 3));
    cp.trsm_ptr.push_back(int64_t(cp.trsm_task.size() / 2));
    cp.upd_ptr.push_back(int64_t(cp.upd_task.size() / 3));
  }
}

}  // namespace ieti
