"""Problem description shared by the oracle and the GPU library.

Conventions (the paper fixes none of them; both implementations follow these):

* Patches sit on a structured P0 x P1 x P2 grid.  Patch (i, j, k) has the
  linear index ``i + P0 * (j + P1 * k)``.
* ``geom_kind == 0``: an axis-aligned box ``[x0,x1] x [y0,y1] x [z0,z1]``
  split uniformly into patches; ``geom_params = [x0, x1, y0, y1, z0, z1]``.
* ``geom_kind == 1``: a NURBS annulus (solid ring).  Direction 0 is the
  azimuth (periodic, P0 equal sectors, each one rational quadratic arc),
  direction 1 the radius and direction 2 the height;
  ``geom_params = [z0, z1, r_0, r_1, ..., r_P1]``.
* The reluctivity is constant per patch; the source J is given as a callable
  mapping physical points ``(n, 3)`` to vectors ``(n, 3)``.
* Dirichlet data ``n x A = n x A_D`` on the whole boundary, with ``A_D`` a
  vector field (``dirichlet_A``); ``None`` means ``n x A = 0``, the setting
  the paper's derivation uses (Section 2).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

GEOM_BOX = 0
GEOM_ANNULUS = 1


def patch_index(i: int, j: int, k: int, P) -> int:
    return int(i + P[0] * (j + P[1] * k))


def patch_coords(idx: int, P):
    i = idx % P[0]
    j = (idx // P[0]) % P[1]
    k = idx // (P[0] * P[1])
    return int(i), int(j), int(k)


@dataclass
class Problem:
    name: str
    geom_kind: int
    patches: tuple
    periodic: tuple
    geom_params: np.ndarray
    degree: int
    n_el: int
    patch_to_sub: np.ndarray
    nu: np.ndarray
    source: Callable[[np.ndarray], np.ndarray]
    exact_A: Optional[Callable[[np.ndarray], np.ndarray]] = None
    exact_B: Optional[Callable[[np.ndarray], np.ndarray]] = None
    # Dirichlet data: n x A = n x dirichlet_A on the whole boundary (None: n x A = 0)
    dirichlet_A: Optional[Callable[[np.ndarray], np.ndarray]] = None
    seed: int = 0
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        self.patches = tuple(int(v) for v in self.patches)
        self.periodic = tuple(int(v) for v in self.periodic)
        self.geom_params = np.ascontiguousarray(self.geom_params, dtype=np.float64)
        self.patch_to_sub = np.ascontiguousarray(self.patch_to_sub, dtype=np.int32)
        self.nu = np.ascontiguousarray(self.nu, dtype=np.float64)
        n = self.n_patches
        if self.patch_to_sub.shape != (n,) or self.nu.shape != (n,):
            raise ValueError("patch_to_sub and nu must have one entry per patch")
        if self.degree < 1 or self.n_el < 1:
            raise ValueError("degree and n_el must be >= 1")
        if np.any(self.nu <= 0):
            raise ValueError("reluctivity must be positive")

    @property
    def n_patches(self) -> int:
        return int(np.prod(self.patches))

    @property
    def n_sub(self) -> int:
        return int(self.patch_to_sub.max()) + 1

    def with_partition(self, patch_to_sub, name=None) -> "Problem":
        return Problem(
            name=name or self.name,
            geom_kind=self.geom_kind,
            patches=self.patches,
            periodic=self.periodic,
            geom_params=self.geom_params.copy(),
            degree=self.degree,
            n_el=self.n_el,
            patch_to_sub=np.asarray(patch_to_sub, dtype=np.int32),
            nu=self.nu.copy(),
            source=self.source,
            exact_A=self.exact_A,
            exact_B=self.exact_B,
            seed=self.seed,
            meta=dict(self.meta),
        )

    def with_refinement(self, degree=None, n_el=None, name=None) -> "Problem":
        out = self.with_partition(self.patch_to_sub, name=name)
        if degree is not None:
            out.degree = int(degree)
        if n_el is not None:
            out.n_el = int(n_el)
        return out
