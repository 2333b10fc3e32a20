// Numbering, decomposition topology, tree-cotree gauge and dual-primal maps.
//
// Section 2 defines facets (interfaces, Dirichlet parts, never two
// patch-facets of one patch sharing a patch-line) and the wire basket (edges
// on facet boundaries).  Section 3 grows a global spanning tree with
// Kruskal's algorithm under the weights of Fig. weights and makes every
// cotree edge of weight 2 primal.  Eq. gloDP keeps one multiplier per
// remaining interface DOF.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "model.hpp"

namespace ieti {

void Mesh::init(const ieti_problem& pr) {
  p = pr.degree_p;
  n_el = pr.n_el;
  n = n_el + p;
  for (int d = 0; d < 3; ++d) {
    P[d] = pr.patches[d];
    per[d] = pr.periodic[d] != 0;
    N[d] = int64_t(P[d]) * (n - 1) + (per[d] ? 0 : 1);
  }
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 3; ++c) ext[d][c] = (c == d && !per[c]) ? N[c] - 1 : N[c];
  int64_t acc = 0;
  for (int d = 0; d < 3; ++d) {
    off[d] = acc;
    acc += ext[d][0] * ext[d][1] * ext[d][2];
  }
  n_edges = acc;
  n_nodes = N[0] * N[1] * N[2];
}

void Mesh::decode_edge(int64_t e, int& d, int64_t X[3]) const {
  d = (e >= off[2]) ? 2 : (e >= off[1] ? 1 : 0);
  int64_t r = e - off[d];
  X[0] = r % ext[d][0];
  r /= ext[d][0];
  X[1] = r % ext[d][1];
  X[2] = r / ext[d][1];
}

namespace {

struct UnionFind {
  std::vector<int64_t> parent;
  std::vector<int32_t> size;
  explicit UnionFind(int64_t n) : parent(n), size(n, 1) { std::iota(parent.begin(), parent.end(), 0); }
  int64_t find(int64_t x) {
    int64_t root = x;
    while (parent[root] != root) root = parent[root];
    while (parent[x] != root) {
      int64_t nx = parent[x];
      parent[x] = root;
      x = nx;
    }
    return root;
  }
  bool unite(int64_t a, int64_t b) {
    a = find(a);
    b = find(b);
    if (a == b) return false;
    if (size[a] < size[b]) std::swap(a, b);
    parent[b] = a;
    size[a] += size[b];
    return true;
  }
};

// Patch-facet type.  kind: 0 = does not exist, 1 = internal (same subdomain
// on both sides: not part of any facet), 2 = Dirichlet facet of subdomain k,
// 3 = interface between subdomains k < l.
struct FaceType {
  int kind = 0, k = -1, l = -1;
  bool typed() const { return kind >= 2; }
  bool operator==(const FaceType& o) const { return kind == o.kind && k == o.k && l == o.l; }
};

struct PatchGrid {
  const Model* m;
  // patch index for patch coordinates, or -1 outside a non-periodic grid
  int64_t patch(int64_t c0, int64_t c1, int64_t c2) const {
    int64_t c[3] = {c0, c1, c2};
    for (int a = 0; a < 3; ++a) {
      const int Pa = m->mesh.P[a];
      if (m->mesh.per[a]) {
        c[a] = ((c[a] % Pa) + Pa) % Pa;
      } else if (c[a] < 0 || c[a] >= Pa) {
        return -1;
      }
    }
    return c[0] + int64_t(m->mesh.P[0]) * (c[1] + int64_t(m->mesh.P[1]) * c[2]);
  }
  FaceType between(int64_t pa, int64_t pb) const {
    FaceType t;
    if (pa < 0 && pb < 0) return t;
    if (pa < 0 || pb < 0) {
      t.kind = 2;
      t.k = m->part[pa < 0 ? pb : pa];
      return t;
    }
    int ka = m->part[pa], kb = m->part[pb];
    if (ka == kb) {
      t.kind = 1;
      return t;
    }
    t.kind = 3;
    t.k = std::min(ka, kb);
    t.l = std::max(ka, kb);
    return t;
  }
  bool row_exists(int axis, int64_t s) const {
    return m->mesh.per[axis] || (s >= 0 && s < m->mesh.P[axis]);
  }
};

// A patch-line along axis d (segment seg) at patch-vertex coordinates (a, b)
// of the transverse axes u < v lies on a facet boundary iff a typed
// patch-facet incident to it has no coplanar continuation of the same type
// across the line.  On aligned grids patch-facets at a line either are
// coplanar or belong to a common patch, so this is the facet rule of
// Section 2 expressed locally.
bool facet_boundary_line(const PatchGrid& g, int d, int64_t seg, int u, int v, int64_t a, int64_t b) {
  auto P = [&](int64_t su, int64_t sv) {
    int64_t c[3];
    c[d] = seg;
    c[u] = su;
    c[v] = sv;
    return g.patch(c[0], c[1], c[2]);
  };
  // faces in the plane normal to u (one on each side of the line along v)
  FaceType fu[2], fv[2];
  bool eu[2], ev[2];
  for (int s = 0; s < 2; ++s) {
    int64_t sv = b - 1 + s;
    eu[s] = g.row_exists(v, sv);
    if (eu[s]) fu[s] = g.between(P(a - 1, sv), P(a, sv));
    int64_t su = a - 1 + s;
    ev[s] = g.row_exists(u, su);
    if (ev[s]) fv[s] = g.between(P(su, b - 1), P(su, b));
  }
  for (int s = 0; s < 2; ++s) {
    if (eu[s] && fu[s].typed() && (!eu[1 - s] || !(fu[1 - s] == fu[s]))) return true;
    if (ev[s] && fv[s].typed() && (!ev[1 - s] || !(fv[1 - s] == fv[s]))) return true;
  }
  return false;
}

}  // namespace

int build_topology(Model& m, Error& err) {
  Mesh& M = m.mesh;
  const int64_t ne = M.n_edges;
  const int n1 = M.n - 1;
  const int64_t n_patches = int64_t(M.P[0]) * M.P[1] * M.P[2];
  // ---- subdomain sets: every patch marks the edges of its closure
  m.subs.assign(ne * 4, -1);
  m.nsubs.assign(ne, 0);
  for (int64_t q = 0; q < n_patches; ++q) {
    const int64_t pc[3] = {q % M.P[0], (q / M.P[0]) % M.P[1], q / (int64_t(M.P[0]) * M.P[1])};
    const int k = m.part[q];
    for (int d = 0; d < 3; ++d) {
      int64_t lo[3], cnt[3];
      for (int c = 0; c < 3; ++c) {
        lo[c] = pc[c] * n1;
        cnt[c] = (c == d) ? n1 : n1 + 1;
      }
      for (int64_t z = 0; z < cnt[2]; ++z)
        for (int64_t y = 0; y < cnt[1]; ++y)
          for (int64_t x = 0; x < cnt[0]; ++x) {
            int64_t e = M.edge_id(d, M.wrap(0, lo[0] + x), M.wrap(1, lo[1] + y), M.wrap(2, lo[2] + z));
            int32_t* s = &m.subs[e * 4];
            int ns = m.nsubs[e];
            bool have = false;
            for (int t = 0; t < ns; ++t) have |= (s[t] == k);
            if (have) continue;
            if (ns >= 4) {
              err = {IETI_ERR_INVALID_ARG, "edge shared by more than four patches"};
              return err.code;
            }
            int pos = ns;
            while (pos > 0 && s[pos - 1] > k) {
              s[pos] = s[pos - 1];
              --pos;
            }
            s[pos] = k;
            m.nsubs[e] = uint8_t(ns + 1);
          }
    }
  }
  // ---- Dirichlet edges: tangential to the boundary
  m.dirichlet.assign(ne, 0);
  for (int64_t e = 0; e < ne; ++e) {
    int d;
    int64_t X[3];
    M.decode_edge(e, d, X);
    for (int c = 0; c < 3; ++c)
      if (c != d && M.on_boundary_node(c, X[c])) m.dirichlet[e] = 1;
  }
  // ---- wire basket: edges on facet-boundary patch-lines
  std::vector<uint8_t> wire(ne, 0);
  PatchGrid grid{&m};
  for (int d = 0; d < 3; ++d) {
    int u = (d == 0) ? 1 : 0;
    int v = (d == 2) ? 1 : 2;
    int64_t na = M.per[u] ? M.P[u] : M.P[u] + 1;
    int64_t nb = M.per[v] ? M.P[v] : M.P[v] + 1;
    for (int64_t seg = 0; seg < M.P[d]; ++seg)
      for (int64_t a = 0; a < na; ++a)
        for (int64_t b = 0; b < nb; ++b) {
          if (!facet_boundary_line(grid, d, seg, u, v, a, b)) continue;
          for (int64_t t = 0; t < n1; ++t) {
            int64_t X[3];
            X[d] = seg * n1 + t;
            X[u] = M.wrap(u, a * n1);
            X[v] = M.wrap(v, b * n1);
            wire[M.edge_id(d, X[0], X[1], X[2])] = 1;
          }
        }
  }
  // ---- weights (Fig. weights; smallest applicable)
  m.weight.assign(ne, 5);
  for (int64_t e = 0; e < ne; ++e) {
    const bool dir = m.dirichlet[e];
    const int ns = m.nsubs[e];
    uint8_t w = 5;
    if (dir || ns >= 2) w = 4;
    if (wire[e]) w = 3;
    if (!dir && ns >= 3) w = 2;
    if (dir && ns >= 2) w = 1;
    m.weight[e] = w;
  }
  // ---- Kruskal: weight buckets, increasing edge id inside each bucket
  m.tree.assign(ne, 0);
  {
    UnionFind uf(M.n_nodes);
    for (int w = 1; w <= 5; ++w)
      for (int64_t e = 0; e < ne; ++e) {
        if (m.weight[e] != w) continue;
        int d;
        int64_t X[3];
        M.decode_edge(e, d, X);
        int64_t Y[3] = {X[0], X[1], X[2]};
        Y[d] = M.wrap(d, Y[d] + 1);
        if (uf.unite(M.node_id(X[0], X[1], X[2]), M.node_id(Y[0], Y[1], Y[2]))) m.tree[e] = 1;
      }
  }
  // ---- Section 3: tree restricted to the Dirichlet boundary must be a tree
  {
    UnionFind uf(M.n_nodes);
    int64_t n_bnodes = 0, n_btree = 0;
    int64_t any_bnode = -1;
    for (int64_t K = 0; K < M.N[2]; ++K)
      for (int64_t J = 0; J < M.N[1]; ++J)
        for (int64_t I = 0; I < M.N[0]; ++I)
          if (M.on_boundary_node(0, I) || M.on_boundary_node(1, J) || M.on_boundary_node(2, K)) {
            ++n_bnodes;
            any_bnode = M.node_id(I, J, K);
          }
    bool ok = true;
    for (int64_t e = 0; e < ne; ++e) {
      if (!(m.tree[e] && m.dirichlet[e])) continue;
      ++n_btree;
      int d;
      int64_t X[3];
      M.decode_edge(e, d, X);
      int64_t Y[3] = {X[0], X[1], X[2]};
      Y[d] = M.wrap(d, Y[d] + 1);
      ok &= uf.unite(M.node_id(X[0], X[1], X[2]), M.node_id(Y[0], Y[1], Y[2]));
    }
    if (n_bnodes > 0) {
      ok &= (n_btree == n_bnodes - 1);
      int64_t root = uf.find(any_bnode);
      for (int64_t K = 0; K < M.N[2] && ok; ++K)
        for (int64_t J = 0; J < M.N[1] && ok; ++J)
          for (int64_t I = 0; I < M.N[0]; ++I)
            if (M.on_boundary_node(0, I) || M.on_boundary_node(1, J) || M.on_boundary_node(2, K))
              if (uf.find(M.node_id(I, J, K)) != root) {
                ok = false;
                break;
              }
    }
    if (!ok) {
      err = {IETI_ERR_TREE, "spanning tree restricted to the Dirichlet boundary is not a tree"};
      return err.code;
    }
  }
  // ---- primal DOFs: cotree edges of weight 2
  m.primal.assign(ne, 0);
  m.primal_edges.clear();
  std::vector<int32_t> gp(ne, -1);
  m.n_g = 0;
  for (int64_t e = 0; e < ne; ++e) {
    const bool free_dof = !m.dirichlet[e] && !m.tree[e];
    if (free_dof) ++m.n_g;
    if (free_dof && m.weight[e] == 2 && m.primal_enabled) {
      m.primal[e] = 1;
      gp[e] = int32_t(m.primal_edges.size());
      m.primal_edges.push_back(e);
    }
  }
  m.n_gp = int64_t(m.primal_edges.size());
  // ---- per-subdomain DOF lists
  m.sd.assign(m.n_sub, Subdomain());
  for (int64_t e = 0; e < ne; ++e) {
    if (m.dirichlet[e] || m.tree[e]) continue;
    for (int t = 0; t < m.nsubs[e]; ++t) {
      Subdomain& s = m.sd[m.subs[e * 4 + t]];
      if (m.primal[e]) {
        s.p_edges.push_back(e);
        s.p_global.push_back(gp[e]);
      } else {
        s.r_edges.push_back(e);
        // without primal DOFs an edge of three or more subdomains gets one
        // multiplier between its first two; the others keep it interior
        s.is_I.push_back(m.nsubs[e] >= 2 && t < 2 ? 1 : 0);
        s.owner.push_back(t == 0 ? 1 : 0);
      }
    }
  }
  for (int k = 0; k < m.n_sub; ++k) {
    if (m.sd[k].r_edges.empty() && m.sd[k].p_edges.empty()) {
      err = {IETI_ERR_PARTITION, "subdomain " + std::to_string(k) + " has no free DOFs"};
      return err.code;
    }
  }
  // ---- multipliers: one row per remaining interface DOF (two subdomains)
  m.mult.clear();
  for (int64_t e = 0; e < ne; ++e) {
    if (m.dirichlet[e] || m.tree[e] || m.primal[e] || m.nsubs[e] < 2) continue;
    if (m.nsubs[e] != 2 && m.primal_enabled) {
      err = {IETI_ERR_TREE, "a dual DOF is shared by more than two subdomains"};
      return err.code;
    }
    const int k = m.subs[e * 4], l = m.subs[e * 4 + 1];
    auto loc = [&](int s) {
      const auto& r = m.sd[s].r_edges;
      return int64_t(std::lower_bound(r.begin(), r.end(), e) - r.begin());
    };
    const int64_t row = int64_t(m.mult.size() / 5);
    const int64_t lk = loc(k), ll = loc(l);
    m.mult.insert(m.mult.end(), {e, int64_t(k), int64_t(l), lk, ll});
    m.sd[k].I_local.push_back(int32_t(lk));
    m.sd[k].I_row.push_back(int32_t(row));
    m.sd[k].I_sign.push_back(1);
    m.sd[l].I_local.push_back(int32_t(ll));
    m.sd[l].I_row.push_back(int32_t(row));
    m.sd[l].I_sign.push_back(-1);
  }
  m.m_r = int64_t(m.mult.size() / 5);
  for (auto& s : m.sd) {
    for (int32_t i = 0; i < int32_t(s.r_edges.size()); ++i)
      if (!s.is_I[i]) s.V_local.push_back(i);
  }
  return IETI_OK;
}

}  // namespace ieti
