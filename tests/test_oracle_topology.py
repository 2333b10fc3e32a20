"""Pins of the oracle's decomposition topology (Sections 2 and 3)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.space import Space
from oracle.topology import build_topology, kruskal
from workloads import configs
from workloads.partition import partition_is_admissible


@pytest.fixture(scope="module")
def cube8_topo():
    prob = configs.cube8()
    S = Space(prob)
    return prob, S, build_topology(S)


def test_cube8_counts_match_hand_derivation(cube8_topo, golden_dir):
    _, S, T = cube8_topo
    g = json.load(open(os.path.join(golden_dir, "cube8_counts.json")))
    assert S.n_edges == g["n_edges"]
    assert int(S.dirichlet.sum()) == g["n_dirichlet"]
    counts = np.bincount(T.weight, minlength=6)
    for w in range(1, 6):
        assert counts[w] == g["weight_counts"][str(w)]
    assert T.n_g == g["n_g"]
    assert T.n_gp == g["n_gp"]
    assert T.m_r == g["m_r"]
    assert all(len(r) == g["n_r"] for r in T.sub_r)
    assert all(int(i.sum()) == g["n_I"] for i in T.sub_I)
    # sum n_r - m_r + n_gp = n_g: every multiplier glues one pair of copies
    assert sum(len(r) for r in T.sub_r) - T.m_r + T.n_gp == T.n_g


def test_tree_is_spanning_tree(cube8_topo):
    _, S, T = cube8_topo
    tree_edges = np.flatnonzero(T.tree)
    assert tree_edges.size == S.n_nodes - 1
    G = sp.coo_matrix((np.ones(tree_edges.size), (S.edge_nodes[tree_edges, 0], S.edge_nodes[tree_edges, 1])),
                      shape=(S.n_nodes, S.n_nodes))
    ncomp, _ = sp.csgraph.connected_components(G, directed=False)
    assert ncomp == 1
    assert T.tree_consistent  # Section 3: tree restricted to the Dirichlet boundary is a tree


def test_primal_is_cotree_weight_two(cube8_topo):
    _, S, T = cube8_topo
    assert np.all(T.weight[T.primal_edges] == 2)
    assert not np.any(T.tree[T.primal_edges])
    w2 = np.flatnonzero(T.weight == 2)
    assert set(w2) == set(np.flatnonzero(T.tree & (T.weight == 2))) | set(T.primal_edges)


def test_kruskal_prefers_lower_weights(cube8_topo):
    """Every cotree edge closes a cycle made of tree edges of weight <= its own."""
    _, S, T = cube8_topo
    rng = np.random.default_rng(0)
    cot = np.flatnonzero(~T.tree)
    for e in rng.choice(cot, 20, replace=False):
        w = T.weight[e]
        allowed = np.flatnonzero(T.tree & (T.weight <= w))
        G = sp.coo_matrix((np.ones(allowed.size), (S.edge_nodes[allowed, 0], S.edge_nodes[allowed, 1])),
                          shape=(S.n_nodes, S.n_nodes))
        _, lab = sp.csgraph.connected_components(G, directed=False)
        assert lab[S.edge_nodes[e, 0]] == lab[S.edge_nodes[e, 1]]


@pytest.mark.parametrize("p,n_el", [(1, 2), (2, 2), (2, 4), (3, 2), (3, 4)])
def test_ngp_independent_of_h_and_p(p, n_el):
    """Section 3: n_gp does not depend on h or p for a fixed decomposition."""
    prob = configs.cube8(degree=p, n_el=n_el)
    T = build_topology(Space(prob))
    assert T.n_gp == 5
    prob2 = configs.small_cube(P=(3, 2, 2), part=[0, 0, 1, 2, 2, 1, 0, 3, 1, 2, 3, 3], degree=p, n_el=n_el)
    ok, why = partition_is_admissible(prob2.patch_to_sub, prob2.patches)
    assert ok, why
    T2 = build_topology(Space(prob2))
    ref = build_topology(Space(prob2.with_refinement(degree=1, n_el=1)))
    assert T2.n_gp == ref.n_gp > 0


def test_multiplier_structure(cube8_topo):
    _, S, T = cube8_topo
    # two subdomains per row, +1 in the lower index, rows sorted by edge id
    assert np.all(np.diff(T.mult[:, 0]) > 0)
    assert np.all(T.mult[:, 1] < T.mult[:, 2])
    # each remaining interface DOF appears in exactly one row
    for k in range(T.n_sub):
        nI = int(T.sub_I[k].sum())
        locs = np.concatenate([T.mult[T.mult[:, 1] == k, 3], T.mult[T.mult[:, 2] == k, 4]])
        assert len(locs) == nI == len(set(locs.tolist()))
        assert np.all(T.sub_I[k][locs])


def test_B_annihilates_restrictions(cube8_topo):
    """B_r R = 0 for the stacked restriction R of any global vector (Eq. fetiNaive constraint)."""
    _, S, T = cube8_topo
    x = np.random.default_rng(3).standard_normal(S.n_edges)
    jump = np.zeros(T.m_r)
    for row, (e, k, l, lk, ll) in enumerate(T.mult):
        xk = x[T.sub_r[k]]
        xl = x[T.sub_r[l]]
        jump[row] = xk[lk] - xl[ll]
    assert np.all(jump == 0.0)


def test_single_subdomain_has_no_multipliers():
    prob = configs.cube8().with_partition(np.zeros(8, dtype=np.int32))
    T = build_topology(Space(prob))
    assert T.m_r == 0 and T.n_gp == 0
    assert len(T.sub_r[0]) == T.n_g


def test_workload_partitions_are_admissible():
    for name in ("cube64", "cube256"):
        prob = configs.make_config(name)
        ok, why = partition_is_admissible(prob.patch_to_sub, prob.patches)
        assert ok, why
        assert prob.patch_to_sub.max() + 1 == {"cube64": 16, "cube256": 64}[name]
        sizes = np.bincount(prob.patch_to_sub)
        assert sizes.min() >= 1 and sizes.max() <= 8


def test_partition_checker_rejects_bad_partitions():
    P = (3, 3, 1)
    # ring around the centre patch: not simply connected
    ring = [0, 0, 0, 0, 1, 0, 0, 0, 0]
    ok, why = partition_is_admissible(ring, P)
    assert not ok and "simply" in why
    # two patches of one subdomain touching only along an edge
    diag = [0, 1, 2, 1, 0, 3, 4, 5, 6]
    ok, why = partition_is_admissible(diag, P)
    assert not ok


def test_dirichlet_tree_consistency_on_workloads():
    prob = configs.make_config("cube64").with_refinement(degree=1, n_el=1)
    T = build_topology(Space(prob))
    assert T.tree_consistent
    assert T.n_gp > 0


def _subdomain_edges(space, T):
    """Maximal runs of consecutive weight-2 control edges on one patch-line
    with one subdomain set: the subdomain edges (cross-edges) of Section 3."""
    groups = {}
    for e in np.flatnonzero(T.weight == 2):
        d = int(space.edge_dir[e])
        X = space.edge_coord[e]
        u, v = [c for c in range(3) if c != d]
        groups.setdefault((d, int(X[u]), int(X[v]), tuple(T.subsets[e])), []).append((int(X[d]), int(e)))
    runs = []
    for lst in groups.values():
        lst.sort()
        cur = [lst[0][1]]
        for a, b in zip(lst[:-1], lst[1:]):
            if b[0] == a[0] + 1:
                cur.append(b[1])
            else:
                runs.append(cur)
                cur = [b[1]]
        runs.append(cur)
    return runs


@pytest.mark.parametrize("name,prob", [
    ("cube8", configs.cube8()),
    ("cube64_p2", configs.cube64(degree=2, n_el=2)),
    ("paper_cube6", configs.paper_cube(degree=2, n_el=2, n_sub=6)),
    ("paper_cube12", configs.paper_cube(degree=1, n_el=3, n_sub=12)),
    ("stream5", configs.stream_problem(5)),
])
def test_edge_average_primal_coincides_with_cotree_primal(name, prob):
    """Whole-edge tangential averages as primal constraints (the alternative
    to Section 3's single cotree DOFs) impose the same continuity under the
    tree gauge: every subdomain edge carries at most one cotree edge, the
    others are tree edges fixed to zero in every subdomain, so its average
    is that DOF divided by the edge count (or identically zero)."""
    space = Space(prob)
    T = build_topology(space)
    runs = _subdomain_edges(space, T)
    counts = [int(np.count_nonzero(T.primal[r])) for r in runs]
    assert max(counts) <= 1
    assert sum(counts) == T.n_gp
    for r in runs:
        assert np.all(T.tree[r] | T.primal[r])
