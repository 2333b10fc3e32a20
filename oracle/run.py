"""End-to-end oracle pipeline for one problem (test infrastructure only)."""
from __future__ import annotations

import time

import numpy as np

from .ietidp import IetiDP, lanczos_condition
from .monolithic import solve_monolithic
from .space import Space
from .topology import build_topology


class OracleRun:
    """Assemble, build topology, and (optionally) solve both ways."""

    def __init__(self, prob, primal_enabled=True):
        t0 = time.perf_counter()
        self.prob = prob
        self.space = Space(prob)
        self.mats, self.loads = self.space.assemble()
        # non-homogeneous Dirichlet data: prescribed boundary coefficients and lifted loads
        self.d_ids = np.zeros(0, dtype=np.int64)
        self.d_vals = np.zeros(0)
        if getattr(prob, "dirichlet_A", None) is not None:
            self.d_ids, self.d_vals = self.space.dirichlet_values()
            self.loads = self.space.lift_loads(self.mats, self.loads, self.d_ids, self.d_vals)
        t1 = time.perf_counter()
        self.topo = build_topology(self.space, primal_enabled=primal_enabled)
        t2 = time.perf_counter()
        self.timing = {"assemble_s": t1 - t0, "topology_s": t2 - t1}
        self._ieti = None

    @property
    def ieti(self):
        if self._ieti is None:
            t = time.perf_counter()
            self._ieti = IetiDP(self.space, self.topo, self.mats, self.loads)
            self.timing["ieti_setup_s"] = time.perf_counter() - t
        return self._ieti

    def monolithic(self):
        t = time.perf_counter()
        a, K, j = solve_monolithic(self.space, self.topo, self.mats, self.loads)
        a[self.d_ids] = self.d_vals
        self.timing["monolithic_s"] = time.perf_counter() - t
        self.K_g, self.j_g = K, j
        return a

    def solve_ieti(self, rtol=1e-8, maxit=1000, lam0=None):
        D = self.ieti
        t = time.perf_counter()
        lam, info = D.pcg(rtol=rtol, maxit=maxit, lam0=lam0)
        a = D.recover(lam)
        a[self.d_ids] = self.d_vals
        self.timing["pcg_s"] = time.perf_counter() - t
        info["kappa"] = lanczos_condition(info)
        return a, lam, info

    def sizes(self):
        T = self.topo
        return {
            "n_g": T.n_g,
            "sum_n_r": int(sum(len(r) for r in T.sub_r)),
            "m_r": T.m_r,
            "n_gp": T.n_gp,
            "n_sub": T.n_sub,
            "n_r": [int(len(r)) for r in T.sub_r],
            "n_I": [int(np.count_nonzero(i)) for i in T.sub_I],
        }
