// Admissibility of the patch-to-subdomain map (Section 2): every subdomain
// is a non-empty union of patches that is connected through shared patch
// faces (the dual graph of the multipatch structure) and simply connected.
//
// Simple connectivity is decided on the closed union U of the subdomain's
// patch cubes, a cubical complex on the patch grid: its Euler
// characteristic chi = V - E + F - C (vertices, edges, faces and cubes of
// the complex) equals b0 - b1 + b2.  A face-connected union has b0 = 1; b2
// is the number of bounded components of the complement (cavities), found
// by a flood fill of the complement's grid cells, which are connected when
// they share a face (a face between two cells outside U is not in U, and a
// complement cell that meets another only along an edge or at a vertex
// reaches it through a common face neighbour outside U).  Hence
// b1 = 1 + b2 - chi, and the subdomain is simply connected iff b1 = 0.
// Periodic directions wrap both the complex and the complement.
#include <cstdint>
#include <string>
#include <unordered_set>
#include <vector>

#include "model.hpp"

namespace ieti {

namespace {

struct Grid {
  int64_t P[3];
  bool per[3];
  // cell / vertex coordinates with wrap in periodic directions
  int64_t wrapc(int d, int64_t x) const { return per[d] ? ((x % P[d]) + P[d]) % P[d] : x; }
  int64_t wrapv(int d, int64_t x) const { return per[d] ? ((x % P[d]) + P[d]) % P[d] : x; }
};

// Key of a k-cell of the cubical complex: lower corner (wrapped) and the
// set of directions it extends along (bit mask).
uint64_t key(const Grid& g, int64_t x, int64_t y, int64_t z, int mask) {
  const int64_t X = g.wrapv(0, x), Y = g.wrapv(1, y), Z = g.wrapv(2, z);
  return (uint64_t(X) | (uint64_t(Y) << 20) | (uint64_t(Z) << 40)) * 8u + uint64_t(mask);
}

}  // namespace

int check_partition(const ieti_problem& pr, const std::vector<int32_t>& part, int n_sub, Error& err) {
  Grid g{};
  for (int d = 0; d < 3; ++d) {
    g.P[d] = pr.patches[d];
    g.per[d] = pr.periodic[d] != 0;
  }
  if (g.P[0] >= (1 << 19) || g.P[1] >= (1 << 19) || g.P[2] >= (1 << 19)) {
    err = {IETI_ERR_INVALID_ARG, "patch grid too large"};
    return err.code;
  }
  const int64_t np = g.P[0] * g.P[1] * g.P[2];
  auto cell = [&](int64_t i, int64_t j, int64_t k) { return i + g.P[0] * (j + g.P[1] * k); };
  std::vector<std::vector<int64_t>> members(n_sub);
  for (int64_t q = 0; q < np; ++q) members[part[q]].push_back(q);
  for (int s = 0; s < n_sub; ++s) {
    const auto& mem = members[s];
    if (mem.empty()) {
      err = {IETI_ERR_PARTITION, "subdomain " + std::to_string(s) + " has no patch"};
      return err.code;
    }
    // ---- connectivity through shared patch faces
    std::vector<uint8_t> seen(np, 0);
    std::vector<int64_t> stack{mem[0]};
    seen[mem[0]] = 1;
    int64_t reached = 0;
    while (!stack.empty()) {
      const int64_t q = stack.back();
      stack.pop_back();
      ++reached;
      const int64_t c[3] = {q % g.P[0], (q / g.P[0]) % g.P[1], q / (g.P[0] * g.P[1])};
      for (int d = 0; d < 3; ++d)
        for (int step = -1; step <= 1; step += 2) {
          int64_t n[3] = {c[0], c[1], c[2]};
          n[d] += step;
          if (!g.per[d] && (n[d] < 0 || n[d] >= g.P[d])) continue;
          n[d] = g.wrapc(d, n[d]);
          const int64_t r = cell(n[0], n[1], n[2]);
          if (r != q && part[r] == s && !seen[r]) {
            seen[r] = 1;
            stack.push_back(r);
          }
        }
    }
    if (reached != int64_t(mem.size())) {
      err = {IETI_ERR_PARTITION, "subdomain " + std::to_string(s) + " is not connected through patch faces"};
      return err.code;
    }
    // ---- Euler characteristic of the closed union of its cubes
    std::unordered_set<uint64_t> cells[4];
    for (int64_t q : mem) {
      const int64_t c[3] = {q % g.P[0], (q / g.P[0]) % g.P[1], q / (g.P[0] * g.P[1])};
      for (int mask = 0; mask < 8; ++mask) {
        const int dim = (mask & 1) + ((mask >> 1) & 1) + ((mask >> 2) & 1);
        // every face of the cube extending along `mask`: the free corner offsets
        // in the other directions take 0 or 1
        for (int off = 0; off < 8; ++off) {
          if (off & mask) continue;
          cells[dim].insert(key(g, c[0] + (off & 1), c[1] + ((off >> 1) & 1), c[2] + ((off >> 2) & 1), mask));
        }
      }
    }
    const int64_t chi = int64_t(cells[0].size()) - int64_t(cells[1].size()) + int64_t(cells[2].size()) -
                        int64_t(cells[3].size());
    // ---- cavities: components of the complement (padded by one cell in the
    // non-periodic directions) that do not reach the padding
    int64_t Q[3], lo[3];
    for (int d = 0; d < 3; ++d) {
      Q[d] = g.per[d] ? g.P[d] : g.P[d] + 2;
      lo[d] = g.per[d] ? 0 : 1;
    }
    const int64_t nq = Q[0] * Q[1] * Q[2];
    std::vector<int8_t> in(nq, 0);  // 1 = cell of the subdomain
    for (int64_t q : mem) {
      const int64_t c[3] = {q % g.P[0], (q / g.P[0]) % g.P[1], q / (g.P[0] * g.P[1])};
      in[(c[0] + lo[0]) + Q[0] * ((c[1] + lo[1]) + Q[1] * (c[2] + lo[2]))] = 1;
    }
    std::vector<int32_t> comp(nq, -1);
    int64_t cavities = 0;
    int32_t ncomp = 0;
    for (int64_t start = 0; start < nq; ++start) {
      if (in[start] || comp[start] >= 0) continue;
      bool outer = false;
      std::vector<int64_t> st{start};
      comp[start] = ncomp;
      while (!st.empty()) {
        const int64_t v = st.back();
        st.pop_back();
        const int64_t c[3] = {v % Q[0], (v / Q[0]) % Q[1], v / (Q[0] * Q[1])};
        for (int d = 0; d < 3; ++d)
          if (!g.per[d] && (c[d] == 0 || c[d] == Q[d] - 1)) outer = true;
        for (int d = 0; d < 3; ++d)
          for (int step = -1; step <= 1; step += 2) {
            int64_t n[3] = {c[0], c[1], c[2]};
            n[d] += step;
            if (g.per[d]) n[d] = ((n[d] % Q[d]) + Q[d]) % Q[d];
            else if (n[d] < 0 || n[d] >= Q[d]) continue;
            const int64_t w = n[0] + Q[0] * (n[1] + Q[1] * n[2]);
            if (!in[w] && comp[w] < 0) {
              comp[w] = ncomp;
              st.push_back(w);
            }
          }
      }
      ++ncomp;
      if (!outer) ++cavities;
    }
    const int64_t b1 = 1 + cavities - chi;
    if (b1 != 0) {
      err = {IETI_ERR_PARTITION, "subdomain " + std::to_string(s) + " is not simply connected (first Betti number " +
                                     std::to_string(b1) + ")"};
      return err.code;
    }
  }
  return IETI_OK;
}

}  // namespace ieti
