"""Seeded greedy partitioner of a structured patch grid into subdomains.

The paper partitions the patch dual graph with METIS and assumes every
subdomain is connected and simply connected (Section 2); METIS itself cannot
guarantee the latter.  METIS is not available here, so workloads use a seeded
greedy region-growing partitioner instead and *reject and redraw* candidate
partitions that violate the paper's assumptions:

(a) every subdomain is face-connected (a union of patches glued along full
    patch-facets);
(b) every subdomain is simply connected: the first Betti number of the closed
    union of its patches is zero (Euler characteristic of the cubical complex
    plus the number of enclosed cavities);
(c) every subdomain is locally manifold: around each patch-line and each
    patch-vertex, the patches of one subdomain are face-connected among
    themselves (no two patches of a subdomain touch only along an edge or a
    corner there);
(d) the interface traces on the outer boundary (patch-lines on the boundary
    between boundary patch-facets of different subdomains) form one connected
    network.  This keeps the spanning tree's restriction to the Dirichlet
    boundary a tree (the consistency requirement of Section 3), because every
    interior wire-basket or interface path meets the boundary only on that
    network.

Only topology of the patch grid is used here; no solver arithmetic.
"""
from __future__ import annotations

import itertools

import numpy as np


def _neighbors6(c, P):
    i, j, k = c
    for d, s in ((0, -1), (0, 1), (1, -1), (1, 1), (2, -1), (2, 1)):
        n = [i, j, k]
        n[d] += s
        if 0 <= n[d] < P[d]:
            yield tuple(n)


def _betti1(cells):
    """First Betti number of the closed union of unit cubes at integer cells."""
    cells = set(cells)
    V, E, F = set(), set(), set()
    for (i, j, k) in cells:
        for dv in itertools.product((0, 1), repeat=3):
            V.add((i + dv[0], j + dv[1], k + dv[2]))
        # edges: along axis a, at offsets in the two other axes
        for a in range(3):
            o = [b for b in range(3) if b != a]
            for s0, s1 in itertools.product((0, 1), repeat=2):
                p = [i, j, k]
                p[o[0]] += s0
                p[o[1]] += s1
                E.add((a, p[0], p[1], p[2]))
        # faces: normal axis a at offset 0 or 1
        for a in range(3):
            for s in (0, 1):
                p = [i, j, k]
                p[a] += s
                F.add((a, p[0], p[1], p[2]))
    chi = len(V) - len(E) + len(F) - len(cells)
    # cavities: components of the complement inside a padded bounding box
    arr = np.array(sorted(cells))
    lo = arr.min(axis=0) - 1
    hi = arr.max(axis=0) + 1
    seen = set()
    ncomp = 0
    for c in itertools.product(*(range(lo[d], hi[d] + 1) for d in range(3))):
        if c in cells or c in seen:
            continue
        ncomp += 1
        stack = [c]
        seen.add(c)
        while stack:
            x = stack.pop()
            for d in range(3):
                for s in (-1, 1):
                    y = list(x)
                    y[d] += s
                    y = tuple(y)
                    if not (lo[d] <= y[d] <= hi[d]):
                        continue
                    if y in cells or y in seen:
                        continue
                    seen.add(y)
                    stack.append(y)
    b2 = ncomp - 1
    b0 = 1
    return b0 + b2 - chi


def _face_connected(cells):
    cells = list(cells)
    if not cells:
        return True
    s = set(cells)
    seen = {cells[0]}
    stack = [cells[0]]
    while stack:
        x = stack.pop()
        for d in range(3):
            for sgn in (-1, 1):
                y = list(x)
                y[d] += sgn
                y = tuple(y)
                if y in s and y not in seen:
                    seen.add(y)
                    stack.append(y)
    return len(seen) == len(s)


def _locally_manifold(owner, P):
    """Check (c): no edge or corner pinches inside any subdomain."""
    def own(c):
        if all(0 <= c[d] < P[d] for d in range(3)):
            return owner[c]
        return -1

    # patch-vertices (including boundary ones): 2x2x2 blocks
    for v in itertools.product(*(range(P[d] + 1) for d in range(3))):
        block = [tuple(v[d] - 1 + o[d] for d in range(3)) for o in itertools.product((0, 1), repeat=3)]
        subs = {}
        for c in block:
            s = own(c)
            if s >= 0:
                subs.setdefault(s, []).append(c)
        for s, cs in subs.items():
            if len(cs) > 1 and not _face_connected(cs):
                return False
    # patch-lines: 2x2 rings around lines along each axis
    for a in range(3):
        o = [b for b in range(3) if b != a]
        for seg in range(P[a]):
            for u in range(P[o[0]] + 1):
                for w in range(P[o[1]] + 1):
                    ring = []
                    for du, dw in itertools.product((0, 1), repeat=2):
                        c = [0, 0, 0]
                        c[a] = seg
                        c[o[0]] = u - 1 + du
                        c[o[1]] = w - 1 + dw
                        ring.append(tuple(c))
                    subs = {}
                    for c in ring:
                        s = own(c)
                        if s >= 0:
                            subs.setdefault(s, []).append(c)
                    for s, cs in subs.items():
                        if len(cs) > 1 and not _face_connected(cs):
                            return False
    return True


def _boundary_traces_connected(owner, P):
    """Check (d): interface traces on the box surface form one network."""
    parent = {}

    def find(x):
        while parent.setdefault(x, x) != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    def union(a, b):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb

    nodes = set()
    # a boundary patch-line lies on a domain face (normal axis n at 0 or P[n]);
    # it runs along axis a != n and separates two boundary patch-facets that
    # are adjacent along the third axis b.
    for n in range(3):
        for side in (0, P[n]):
            layer = 0 if side == 0 else P[n] - 1
            for a in range(3):
                if a == n:
                    continue
                b = 3 - n - a
                for seg in range(P[a]):
                    for cut in range(1, P[b]):
                        c1 = [0, 0, 0]
                        c1[n] = layer
                        c1[a] = seg
                        c1[b] = cut - 1
                        c2 = list(c1)
                        c2[b] = cut
                        if owner[tuple(c1)] != owner[tuple(c2)]:
                            v1 = [0, 0, 0]
                            v1[n] = side
                            v1[a] = seg
                            v1[b] = cut
                            v2 = list(v1)
                            v2[a] = seg + 1
                            v1, v2 = tuple(v1), tuple(v2)
                            nodes.add(v1)
                            nodes.add(v2)
                            union(v1, v2)
    roots = {find(x) for x in nodes}
    return len(roots) <= 1


def partition_is_admissible(patch_to_sub, P):
    """Return (ok, reason) for checks (a)-(d) on a box patch grid."""
    P = tuple(int(v) for v in P)
    owner = {}
    for idx, s in enumerate(np.asarray(patch_to_sub)):
        i = idx % P[0]
        j = (idx // P[0]) % P[1]
        k = idx // (P[0] * P[1])
        owner[(i, j, k)] = int(s)
    groups = {}
    for c, s in owner.items():
        groups.setdefault(s, []).append(c)
    if sorted(groups) != list(range(len(groups))):
        return False, "subdomain ids must be 0..N_sub-1"
    for s, cs in groups.items():
        if not _face_connected(cs):
            return False, f"subdomain {s} not face-connected"
        if _betti1(cs) != 0:
            return False, f"subdomain {s} not simply connected"
    if not _locally_manifold(owner, P):
        return False, "pinched subdomain (edge or corner contact only)"
    if len(groups) > 1 and not _boundary_traces_connected(owner, P):
        return False, "boundary interface traces disconnected"
    return True, "ok"


def _draw_sizes(n_patches, n_sub, rng, smin, smax):
    if n_sub is None:
        sizes = []
        left = n_patches
        while left > 0:
            s = int(rng.integers(smin, smax + 1))
            s = min(s, left)
            sizes.append(s)
            left -= s
        return sizes
    if not (n_sub * smin <= n_patches <= n_sub * smax):
        raise ValueError("infeasible subdomain count for the size range")
    sizes = [smin] * n_sub
    left = n_patches - smin * n_sub
    while left > 0:
        cand = [i for i in range(n_sub) if sizes[i] < smax]
        i = cand[int(rng.integers(len(cand)))]
        sizes[i] += 1
        left -= 1
    return sizes


def greedy_partition(P, n_sub, seed, smin=1, smax=8, max_attempts=20000):
    """Seeded greedy region growing with reject-and-redraw.

    Sizes are drawn in [smin, smax] (summing to the patch count; if ``n_sub``
    is None they are drawn one by one until the patches are used up).  Region
    s grows from the lowest-index unassigned patch; it repeatedly adds the
    unassigned face-neighbour with the most faces shared with the region
    (ties to the lowest patch index), which keeps regions compact and leaves
    no pockets behind the sweep.  A candidate is accepted only if
    :func:`partition_is_admissible` holds.

    Returns ``(patch_to_sub int32 array, attempts)``.
    """
    P = tuple(int(v) for v in P)
    rng = np.random.default_rng(seed)
    n_patches = int(np.prod(P))
    cells = [(idx % P[0], (idx // P[0]) % P[1], idx // (P[0] * P[1])) for idx in range(n_patches)]

    def lin(c):
        return c[0] + P[0] * (c[1] + P[1] * c[2])

    for attempt in range(1, max_attempts + 1):
        sizes = _draw_sizes(n_patches, n_sub, rng, smin, smax)
        owner = {}
        ok = True
        for s, size in enumerate(sizes):
            seed_cell = next((c for c in cells if c not in owner), None)
            if seed_cell is None:
                ok = False
                break
            region = {seed_cell}
            owner[seed_cell] = s
            while len(region) < size:
                frontier = {q for r in region for q in _neighbors6(r, P) if q not in owner}
                if not frontier:
                    break
                pick = min(frontier, key=lambda q: (-sum(1 for t in _neighbors6(q, P) if t in region), lin(q)))
                owner[pick] = s
                region.add(pick)
            if len(region) < size:
                ok = False
                break
        if not ok or len(owner) != n_patches:
            continue
        part = np.array([owner[c] for c in cells], dtype=np.int32)
        good, _ = partition_is_admissible(part, P)
        if good:
            return part, attempt
    raise RuntimeError("no admissible partition found")
