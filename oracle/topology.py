"""Decomposition topology, tree-cotree gauge and primal selection (oracle).

TEST INFRASTRUCTURE ONLY.

Follows Section 2 (facets, wire basket) and Section 3 (tree-cotree gauging):

* Each control edge lies in exactly one patch-grid entity (a patch
  interior, a patch-facet or a patch-line).  The patches containing it give
  its subdomain set S(e).
* Facets (Section 2): interfaces and Dirichlet parts are unions of
  patch-facets of one type (interface between subdomains k<l, or Dirichlet
  boundary of k); two patch-facets of the same patch that share a patch-line
  are never in the same facet.  On the aligned patch grids used here, two
  patch-facets that share a patch-line either are coplanar (then they merge
  if they have the same type) or share a patch (then they are separate).
  A patch-line is on a facet boundary iff some typed patch-facet at the line
  has its coplanar continuation across the line missing or of another type.
  The wire basket is the set of control edges on facet-boundary patch-lines.
* Edge weights (Fig. weights), smallest applicable wins:
    1 Dirichlet edge shared by two or more subdomains (interface meets the
      Dirichlet boundary),
    2 non-Dirichlet edge shared by more than two subdomains (cross-edge),
    3 other wire-basket edge,
    4 other edge on the Dirichlet boundary or on an interface,
    5 remaining (subdomain interior) edge.
* Kruskal's algorithm on the whole control mesh with edges taken in
  increasing (weight, global edge id) order; the tie-break by edge id is a
  reading (the paper does not fix it).
* Primal DOFs: every cotree edge of weight 2 (Section 3).
* Redundant constraints removed (Eq. gloDP): each remaining interface DOF
  (cotree, not primal, not Dirichlet) is shared by exactly two subdomains
  k < l and gets one multiplier row with +1 in k and -1 in l; rows are sorted
  by global edge id.
* Local numbering (a reading): the remaining DOFs of subdomain k are its
  non-Dirichlet, non-tree, non-primal edges in increasing global edge id.
"""
from __future__ import annotations

import numpy as np

from workloads.problem import patch_index


class Topology:
    pass


def _patch_options(X, n1, P, per):
    """Patch indices along one axis that contain transverse node coordinate X."""
    if X % n1 == 0:
        j = X // n1
        cand = [j - 1, j]
    else:
        cand = [X // n1]
    out = []
    for c in cand:
        if per:
            out.append(c % P)
        elif 0 <= c < P:
            out.append(c)
    return sorted(set(out))


def _line_is_facet_boundary(prob, d, seg, a, b, u, v):
    P, per = prob.patches, prob.periodic

    def patch(su, sv):
        c = [0, 0, 0]
        c[d] = seg
        for ax, s in ((u, su), (v, sv)):
            if per[ax]:
                s = s % P[ax]
            elif not (0 <= s < P[ax]):
                return None
            c[ax] = s
        return patch_index(c[0], c[1], c[2], P)

    def exists_row(ax, s):
        return per[ax] or (0 <= s < P[ax])

    def ftype(X, Y):
        if X is None and Y is None:
            return "none"
        if X is None or Y is None:
            Z = X if Y is None else Y
            return ("D", int(prob.patch_to_sub[Z]))
        kx, ky = int(prob.patch_to_sub[X]), int(prob.patch_to_sub[Y])
        if kx == ky:
            return None
        return ("I", min(kx, ky), max(kx, ky))

    faces = {}
    for sv in (b - 1, b):  # faces in the plane normal to u through the line
        if exists_row(v, sv):
            faces[("u", sv)] = ftype(patch(a - 1, sv), patch(a, sv))
        else:
            faces[("u", sv)] = "missing"
    for su in (a - 1, a):  # faces in the plane normal to v through the line
        if exists_row(u, su):
            faces[("v", su)] = ftype(patch(su, b - 1), patch(su, b))
        else:
            faces[("v", su)] = "missing"
    pairs = [(("u", b - 1), ("u", b)), (("v", a - 1), ("v", a))]
    for f1, f2 in pairs:
        for f, g in ((f1, f2), (f2, f1)):
            tf = faces[f]
            if tf is None or tf == "missing" or tf == "none":
                continue
            tg = faces[g]
            if tg == "missing" or tg != tf:
                return True
    return False


def classify_edges(space):
    """Subdomain sets, Dirichlet flags, wire basket and weights of all edges."""
    prob = space.prob
    P, per = prob.patches, prob.periodic
    n1 = space.n - 1
    ne = space.n_edges
    subsets = -np.ones((ne, 4), dtype=np.int64)
    nsub = np.zeros(ne, dtype=np.int64)
    wire = np.zeros(ne, dtype=bool)
    line_cache = {}
    for e in range(ne):
        d = int(space.edge_dir[e])
        X = space.edge_coord[e]
        opts = []
        for c in range(3):
            if c == d:
                opts.append([int(X[c]) // n1])
            else:
                opts.append(_patch_options(int(X[c]), n1, P[c], per[c]))
        subs = set()
        for i in opts[0]:
            for j in opts[1]:
                for k in opts[2]:
                    subs.add(int(prob.patch_to_sub[patch_index(i, j, k, P)]))
        s = sorted(subs)
        subsets[e, :len(s)] = s
        nsub[e] = len(s)
        u, v = [c for c in range(3) if c != d]
        if X[u] % n1 == 0 and X[v] % n1 == 0:
            key = (d, int(X[d]) // n1, int(X[u]) // n1, int(X[v]) // n1)
            if key not in line_cache:
                line_cache[key] = _line_is_facet_boundary(prob, d, key[1], key[2], key[3], u, v)
            wire[e] = line_cache[key]
    dirichlet = space.dirichlet
    weight = np.full(ne, 5, dtype=np.int64)
    w4 = dirichlet | (nsub >= 2)
    weight[w4] = 4
    weight[wire] = 3
    weight[(~dirichlet) & (nsub >= 3)] = 2
    weight[dirichlet & (nsub >= 2)] = 1
    return subsets, nsub, wire, weight


class _UnionFind:
    def __init__(self, n):
        self.parent = list(range(n))

    def find(self, x):
        par = self.parent
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x

    def union(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra == rb:
            return False
        self.parent[ra] = rb
        return True


def kruskal(space, weight):
    """Spanning tree of the control mesh, edges in (weight, edge id) order."""
    order = np.lexsort((np.arange(space.n_edges), weight))
    uf = _UnionFind(space.n_nodes)
    tree = np.zeros(space.n_edges, dtype=bool)
    nodes = space.edge_nodes
    for e in order:
        if uf.union(int(nodes[e, 0]), int(nodes[e, 1])):
            tree[e] = True
    return tree


def dirichlet_tree_is_spanning(space, tree):
    """Section 3: the tree restricted to the Dirichlet boundary mesh must be a tree."""
    bnodes = np.flatnonzero(space.node_boundary)
    if bnodes.size == 0:
        return True
    be = np.flatnonzero(tree & space.dirichlet)
    if be.size != bnodes.size - 1:
        return False
    uf = _UnionFind(space.n_nodes)
    for e in be:
        if not uf.union(int(space.edge_nodes[e, 0]), int(space.edge_nodes[e, 1])):
            return False
    roots = {uf.find(int(x)) for x in bnodes}
    return len(roots) == 1


def build_topology(space, primal_enabled=True):
    prob = space.prob
    subsets, nsub, wire, weight = classify_edges(space)
    tree = kruskal(space, weight)
    T = Topology()
    T.subsets, T.nsub, T.wire, T.weight, T.tree = subsets, nsub, wire, weight, tree
    T.dirichlet = space.dirichlet.copy()
    T.tree_consistent = dirichlet_tree_is_spanning(space, tree)
    free = (~space.dirichlet) & (~tree)
    T.free = free
    primal = free & (weight == 2) if primal_enabled else np.zeros_like(free)
    T.primal = primal
    T.primal_edges = np.flatnonzero(primal)
    T.n_gp = int(T.primal_edges.size)
    gp_index = -np.ones(space.n_edges, dtype=np.int64)
    gp_index[T.primal_edges] = np.arange(T.n_gp)
    T.gp_index = gp_index
    n_sub = prob.n_sub
    T.n_sub = n_sub
    # per-subdomain DOF lists
    T.sub_r, T.sub_p, T.sub_I = [], [], []
    for k in range(n_sub):
        member = np.any(subsets == k, axis=1) & free
        r = np.flatnonzero(member & ~primal)
        p = np.flatnonzero(member & primal)
        T.sub_r.append(r)
        T.sub_p.append(p)
        T.sub_I.append(nsub[r] >= 2)  # interface flag per local r DOF
    # multipliers
    mult_edges = np.flatnonzero(free & (~primal) & (nsub >= 2))
    if primal_enabled and np.any(nsub[mult_edges] > 2):
        raise AssertionError("a dual DOF is shared by more than two subdomains")
    rows = []
    loc_maps = [dict(zip(r.tolist(), range(len(r)))) for r in T.sub_r]
    for e in mult_edges:
        k, l = int(subsets[e, 0]), int(subsets[e, 1])
        rows.append((int(e), k, l, loc_maps[k][int(e)], loc_maps[l][int(e)]))
    T.mult = np.array(rows, dtype=np.int64).reshape(-1, 5)
    T.m_r = T.mult.shape[0]
    T.n_g = int(np.count_nonzero(free))
    return T
