"""Plain FP64 CPU oracle for the tree-cotree gauged IETI-DP magnetostatics solver.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(the C-ABI library and its Python binding) never calls it and shares no code
with it.  Its only shared dependency is the input description in
``workloads`` (problem geometry, partition, reluctivity, source callables).

Everything here is slow and obvious on purpose: NumPy/SciPy in float64,
following the paper's steps in its order and notation:

* ``bspline``    1D B-splines (Cox-de Boor) and the derived degree-(p-1)
                 splines that carry the curl-conforming space.
* ``geometry``   patch maps F^(j) for boxes and the NURBS annulus.
* ``space``      the multipatch curl-conforming spline space, its global edge
                 numbering, and Galerkin assembly of K_g and j_g (Eq. discrMS).
* ``topology``   facets, wire basket, edge weights (Fig. weights), Kruskal's
                 spanning tree, primal selection (Section 3).
* ``ietidp``     dual-primal TI: K_rr, K_rp, K_pp, B_r, C_p, the coarse and
                 interface problems (Eqs. gloDP, intProb, coarseProb,
                 localProb), the Dirichlet preconditioner (Eq. DirPrec) and PCG.
* ``monolithic`` direct sparse solve of the gauged global system.
* ``post``       B = curl A at quadrature points and the error of Section 4.
* ``nn``         the warm-start network: forward pass, backpropagation and
                 Adam, in float64.

Parity-unpinned items are listed in the module docstrings where they occur.
"""
