// Batches of independent problems: one model whose subdomains, multiplier
// rows, primal DOFs, patches and output coefficients are the concatenation
// of the problems', so that one factorisation plan and one set of launches
// covers all of them.  The coarse problem stays per problem (block
// diagonal); the ranges below tell the device code where each block lives.
#include <string>
#include <utility>
#include <vector>

#include "model.hpp"

namespace ieti {

void finalize_single(Model& m) {
  ProblemRange r;
  r.n_edges = m.mesh.n_edges;
  r.m_r = m.m_r;
  r.n_gp = m.n_gp;
  r.n_sub = m.n_sub;
  r.n_patches = int64_t(m.part.size());
  r.n_g = m.n_g;
  m.probs.assign(1, r);
  m.meshes.assign(1, m.mesh);
  m.sub_prob.assign(m.n_sub, 0);
  m.n_edges_total = m.mesh.n_edges;
}

int merge_models(std::vector<Model>& parts, Model& out, Error& err) {
  if (parts.empty()) {
    err = {IETI_ERR_INVALID_ARG, "empty batch"};
    return err.code;
  }
  out = Model();
  out.prob = parts[0].prob;
  out.mesh = parts[0].mesh;
  ProblemRange acc;
  for (size_t p = 0; p < parts.size(); ++p) {
    Model& m = parts[p];
    ProblemRange r;
    r.edge_base = acc.edge_base;
    r.n_edges = m.mesh.n_edges;
    r.mr_base = acc.mr_base;
    r.m_r = m.m_r;
    r.gp_base = acc.gp_base;
    r.n_gp = m.n_gp;
    r.sub_base = acc.sub_base;
    r.n_sub = m.n_sub;
    r.patch_base = acc.patch_base;
    r.n_patches = int64_t(m.part.size());
    r.n_g = m.n_g;
    out.probs.push_back(r);
    out.meshes.push_back(m.mesh);
    for (int k = 0; k < m.n_sub; ++k) {
      Subdomain s = std::move(m.sd[k]);
      for (auto& row : s.I_row) row += int32_t(r.mr_base);
      for (auto& g : s.p_global) g += int32_t(r.gp_base);
      for (auto& q : s.tr_patch) q += int32_t(r.patch_base);
      out.sd.push_back(std::move(s));
      out.sub_prob.push_back(int32_t(p));
    }
    for (int64_t i = 0; i < m.m_r; ++i) {
      const int64_t* row = &m.mult[5 * i];
      out.mult.insert(out.mult.end(), {row[0], row[1] + r.sub_base, row[2] + r.sub_base, row[3], row[4]});
    }
    for (int64_t e : m.primal_edges) out.primal_edges.push_back(e + r.edge_base);
    for (int32_t k : m.part) out.part.push_back(k + int32_t(r.sub_base));
    out.nu.insert(out.nu.end(), m.nu.begin(), m.nu.end());
    out.load_scale.insert(out.load_scale.end(), m.load_scale.begin(), m.load_scale.end());
    for (auto& pl : m.patch_load) out.patch_load.push_back(std::move(pl));
    if (m.patch_lift.empty()) m.patch_lift.assign(m.part.size(), {});
    for (auto& pl : m.patch_lift) out.patch_lift.push_back(std::move(pl));
    for (size_t i = 0; i < m.d_edges.size(); ++i) {
      out.d_edges.push_back(m.d_edges[i] + r.edge_base);
      out.d_vals.push_back(m.d_vals[i]);
    }
    acc.edge_base += r.n_edges;
    acc.mr_base += r.m_r;
    acc.gp_base += r.n_gp;
    acc.sub_base += r.n_sub;
    acc.patch_base += r.n_patches;
    out.n_g += r.n_g;
    Model().sd.swap(m.sd);
  }
  if (acc.mr_base > (int64_t(1) << 31) - 1 || acc.gp_base > (int64_t(1) << 31) - 1) {
    err = {IETI_ERR_INVALID_ARG, "batch too large for 32-bit row indices"};
    return err.code;
  }
  out.n_sub = int(acc.sub_base);
  out.m_r = acc.mr_base;
  out.n_gp = acc.gp_base;
  out.n_edges_total = acc.edge_base;
  return IETI_OK;
}

}  // namespace ieti
