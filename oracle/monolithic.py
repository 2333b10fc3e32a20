"""Direct solve of the gauged global system (oracle, test infrastructure only).

Eq. discrMS restricted to the DOFs that are neither Dirichlet (n x A = 0,
Section 2) nor tree edges (the gauge of Section 3); the eliminated
coefficients are zero.  This is the plain definition the IETI-DP solution
must reproduce up to the PCG tolerance.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def global_matrix(mats):
    K = mats[0].copy()
    for M in mats[1:]:
        K = K + M
    return K.tocsr()


def solve_monolithic(space, topo, mats, loads):
    K = global_matrix(mats)
    j = space.global_load(loads)
    free = np.flatnonzero(topo.free)
    Kf = K[free][:, free].tocsc()
    lu = spla.splu(Kf, permc_spec="MMD_AT_PLUS_A")
    a = np.zeros(space.n_edges)
    a[free] = lu.solve(j[free])
    return a, K, j
