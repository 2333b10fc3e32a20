// Host-side model of one IETI-DP problem: numbering, topology, gauge,
// dual-primal maps, assembled local blocks and the GPU factorisation plan.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "ietidp.h"

namespace ieti {

struct Error {
  int code;
  std::string msg;
};

// Structured control mesh of the multipatch domain (Section 2).
struct Mesh {
  int p = 0, n_el = 0, n = 0;  // n = B-splines per patch and direction
  int P[3] = {0, 0, 0};
  bool per[3] = {false, false, false};
  int64_t N[3] = {0, 0, 0};     // control nodes per axis
  int64_t ext[3][3] = {};       // ext[d][c]: positions of direction-d edges along axis c
  int64_t off[3] = {0, 0, 0};
  int64_t n_edges = 0, n_nodes = 0;

  void init(const ieti_problem& pr);
  int64_t edge_id(int d, int64_t I, int64_t J, int64_t K) const {
    return off[d] + I + ext[d][0] * (J + ext[d][1] * K);
  }
  int64_t node_id(int64_t I, int64_t J, int64_t K) const { return I + N[0] * (J + N[1] * K); }
  void decode_edge(int64_t e, int& d, int64_t X[3]) const;
  int64_t wrap(int c, int64_t X) const { return per[c] ? ((X % N[c]) + N[c]) % N[c] : X; }
  bool on_boundary_node(int c, int64_t X) const { return !per[c] && (X == 0 || X == N[c] - 1); }
};

// Per-subdomain dual-primal data.
struct Subdomain {
  std::vector<int64_t> r_edges;   // remaining DOFs, increasing edge id
  std::vector<int64_t> p_edges;   // primal DOFs, increasing edge id
  std::vector<int32_t> p_global;  // global primal index of each primal DOF
  std::vector<uint8_t> is_I;      // per r DOF: on an interface
  std::vector<int32_t> I_local;   // local r index of each interface DOF (multiplier order)
  std::vector<int32_t> I_row;     // multiplier row of each interface DOF
  std::vector<int8_t> I_sign;     // +1 / -1 entry of B
  std::vector<int32_t> V_local;   // local r index of each non-interface DOF
  // assembled blocks over [r, p] local numbering (CSR, full symmetric)
  int64_t n_loc = 0;
  std::vector<int64_t> indptr;
  std::vector<int32_t> indices;
  std::vector<double> values;
  std::vector<double> load;
  // unscaled per-patch contributions of every CSR entry, in increasing patch
  // order: values[i] = sum over t in [tr_seg[i], tr_seg[i+1]) of
  // nu[tr_patch[t]] * tr_val[t] (the Galerkin matrix is linear in the
  // piecewise-constant reluctivity)
  std::vector<int64_t> tr_seg;
  std::vector<int32_t> tr_patch;
  std::vector<double> tr_val;
  std::vector<uint8_t> owner;     // per r DOF: 1 if this subdomain writes the global value
};

// One problem of a batch: its ranges in the batch's concatenated numbering
// (a single problem is a batch of one with every base 0).
struct ProblemRange {
  int64_t edge_base = 0, n_edges = 0;     // coefficients of the output vector
  int64_t mr_base = 0, m_r = 0;           // multiplier rows
  int64_t gp_base = 0, n_gp = 0;          // global primal DOFs
  int64_t sub_base = 0, n_sub = 0;        // subdomains
  int64_t patch_base = 0, n_patches = 0;  // patches (coefficient arrays)
  int64_t n_g = 0;
};

struct Model {
  ieti_problem prob{};
  std::vector<int32_t> part;
  std::vector<double> nu;
  std::vector<double> load_scale;  // per patch, multiplies the patch's assembled load
  // per patch: unscaled load entries (local DOF in the patch's subdomain, value)
  std::vector<std::vector<std::pair<int32_t, double>>> patch_load;
  // per patch: Dirichlet lifting (K a_D with nu = 1) at local DOFs; load -= nu * lift
  std::vector<std::vector<std::pair<int32_t, double>>> patch_lift;
  // prescribed boundary coefficients (non-homogeneous Dirichlet data), edge ids batch-global
  std::vector<int64_t> d_edges;
  std::vector<double> d_vals;
  Mesh mesh;
  int n_sub = 0;
  // Section 3's primal DOFs (cotree edges of weight 2); false: none, the local
  // problems the paper shows to be singular (only for checking that)
  bool primal_enabled = true;
  // per edge
  std::vector<uint8_t> dirichlet, weight, tree, primal;
  std::vector<int32_t> subs;     // up to 4 subdomain ids per edge (-1 padded), sorted
  std::vector<uint8_t> nsubs;
  std::vector<int64_t> primal_edges;
  std::vector<int64_t> mult;     // m_r x 5: edge, k, l, loc_k, loc_l
  int64_t m_r = 0, n_gp = 0, n_g = 0;
  std::vector<Subdomain> sd;
  // batch structure: problems, their meshes, problem of every subdomain.
  // Subdomain fields I_row and p_global are batch-global; r_edges, p_edges
  // and mult edge ids stay local to the subdomain's problem.
  std::vector<ProblemRange> probs;
  std::vector<Mesh> meshes;
  std::vector<int32_t> sub_prob;
  int64_t n_edges_total = 0;
  bool batch() const { return probs.size() > 1; }
  const Mesh& mesh_of(int k) const { return meshes[sub_prob[k]]; }
};

// partition_check.cpp: every subdomain non-empty, connected through patch
// faces and simply connected (IETI_ERR_PARTITION otherwise)
int check_partition(const ieti_problem& pr, const std::vector<int32_t>& part, int n_sub, Error& err);
// mesh_topology.cpp
int build_topology(Model& m, Error& err);
// assemble.cpp
int assemble_local_systems(Model& m, Error& err);
// batch.cpp: ranges of a single assembled problem; concatenation of several
void finalize_single(Model& m);
int merge_models(std::vector<Model>& parts, Model& out, Error& err);
// new reluctivity and load scale per patch, from the stored contributions
int set_coefficients(Model& m, const double* nu, const double* load_scale, Error& err);

}  // namespace ieti
