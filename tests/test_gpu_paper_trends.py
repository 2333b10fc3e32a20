"""The trends of Section 4's two experiments, on the GPU path.

Problem: (0,3)^3 in 3x3x3 unit patches, nu = 1, the closed-form A_ana of
Section 4 with its tangential trace as Dirichlet data, PCG tolerance 1e-6
(relative to ||b||), seeded greedy partitions in place of METIS.

* First experiment (3 subdomains, p in {1,2,3}, h = 1/6, 1/12, 1/24 relative
  to the domain): the number of global primal DOFs does not depend on h or
  p; the B error converges as O(h^p); the condition number (Lanczos estimate
  from the recorded PCG coefficients) and the iteration count stay below the
  paper's bounding forms C (2 + log10(p^2/h))^2 and C~ (2 + log10(p^2/h)),
  here with C = 0.5 and C~ = 4 (the paper's fitted constants are about 0.3
  and 3.5 on its own partition).
* Second experiment (h = 1/12, N_sub = 2..12): the primal count grows at
  most linearly in N_sub, the B error does not depend on the decomposition
  (up to the PCG tolerance), the condition number and iteration counts stay
  inside the ranges of the paper's figures (8.5, here with 5% slack, and
  18); for p = 1 they equal the oracle's.

The constants are qualitative (the paper's partitions and data are not
available): parity unpinned beyond the oracle comparison.
"""
import numpy as np
import pytest

from oracle.post import b_error
from oracle.run import OracleRun
from workloads import configs

pytestmark = pytest.mark.gpu

RTOL = 1e-6


def _run(p, n_el, n_sub):
    from paper_2501_04340_amd import Solver
    prob = configs.paper_cube(degree=p, n_el=n_el, n_sub=n_sub)
    print(f"[paper-trends] p={p} n_el={n_el} n_sub={n_sub}", flush=True)
    S = Solver(prob)
    try:
        S.factor()
        S.record_pcg(1000)
        a, st = S.solve(rtol=RTOL, maxit=1000)
        lo, hi = S.condition()
        n_gp = S.n_gp
    finally:
        S.close()
    assert st["status"] == 0
    from oracle.space import Space
    err = b_error(Space(prob), a, b_ref=prob.exact_B)[0]
    row = dict(p=p, n_el=n_el, n_sub=n_sub, h=1.0 / (3 * n_el), n_gp=n_gp, iters=st["iters"], kappa=hi / lo,
               err=err, prob=prob)
    print(f"[paper-trends]   n_gp={n_gp} iters={st['iters']} kappa={hi / lo:.4f} eps_B={err:.4e}", flush=True)
    return row


def test_first_experiment_mesh_and_degree():
    rows = [_run(p, n_el, 3) for p in (1, 2, 3) for n_el in (2, 4, 8)]
    assert len({r["n_gp"] for r in rows}) == 1
    for p in (1, 2, 3):
        rp = [r for r in rows if r["p"] == p]
        rate = np.log2(rp[1]["err"] / rp[2]["err"])
        print(f"[paper-trends] p={p}: eps_B rate h=1/12 -> 1/24 = {rate:.3f}")
        assert rate >= p - 0.4
        for a, b in zip(rp[:-1], rp[1:]):
            assert b["kappa"] >= 0.99 * a["kappa"]
        for r in rp:
            g = 2.0 + np.log10(p * p / r["h"])
            assert r["kappa"] <= 0.5 * g * g
            assert r["iters"] <= 4.0 * g


def test_second_experiment_subdomain_count():
    for p in (1, 2, 3):
        rows = [_run(p, 4, k) for k in range(2, 13)]
        errs = np.array([r["err"] for r in rows])
        # the same discrete problem; the spread is the PCG tolerance's (visible at p = 3)
        assert errs.max() <= errs.min() * 1.05
        for r in rows:
            assert r["n_gp"] <= 2 * r["n_sub"]
            assert r["kappa"] <= 8.5 * 1.05 and r["iters"] <= 18
        if p == 1:
            for r in rows:
                O = OracleRun(r["prob"])
                _, _, info = O.solve_ieti(rtol=RTOL)
                lo, hi = info["kappa"]
                assert r["n_gp"] == O.topo.n_gp
                assert abs(r["iters"] - info["iters"]) <= 1
                assert abs(r["kappa"] - hi / lo) <= 1e-3 * hi / lo


def test_degree_three_rate_with_the_algebraic_error_removed():
    """At the paper's PCG tolerance (1e-6) the algebraic error is a visible
    part of eps_B for p = 3 on the finest mesh (the first experiment's rate
    comes out near 2.7); solved to rtol 1e-12 the B error converges at the
    discretisation's order, O(h^3)."""
    from paper_2501_04340_amd import Solver
    from oracle.space import Space
    errs = []
    for n_el in (4, 8):
        prob = configs.paper_cube(degree=3, n_el=n_el, n_sub=3)
        print(f"[paper-trends] p=3 n_el={n_el} rtol 1e-12", flush=True)
        S = Solver(prob)
        try:
            S.factor()
            a, st = S.solve(rtol=1e-12, maxit=3000)
        finally:
            S.close()
        assert st["status"] == 0
        errs.append(b_error(Space(prob), a, b_ref=prob.exact_B)[0])
    rate = np.log2(errs[0] / errs[1])
    print(f"[paper-trends] p=3 eps_B {errs} rate {rate:.3f}", flush=True)
    assert rate >= 2.85
