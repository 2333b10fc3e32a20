"""Pins of non-homogeneous Dirichlet data (n x A = n x A_D, Section 2):
boundary L2 projection of the tangential trace plus lifting of the loads.

* A field of the degree-2 spline space with a non-zero tangential trace is
  reproduced to round-off (monolithic and IETI-DP): the projection of an
  in-space trace is exact and the lifted problem has the field as solution.
* The paper's closed-form solution on (0,3)^3 (Section 4) converges in the
  flux density at the optimal rate O(h^p).
"""
import numpy as np
import pytest

from oracle.post import b_error
from oracle.run import OracleRun
from workloads import configs, sources


@pytest.mark.parametrize("P,part", [((2, 2, 2), np.arange(8, dtype=np.int32)),
                                    ((3, 2, 2), np.array([0, 0, 1, 2, 2, 1, 0, 3, 1, 2, 3, 3], dtype=np.int32))])
def test_in_space_field_with_trace_is_reproduced(P, part):
    prob = configs.box_problem(P, 2, 2, part, np.ones(int(np.prod(P))), sources.trace_J, exact_A=sources.trace_A,
                               exact_B=sources.trace_B)
    prob.dirichlet_A = sources.trace_A
    O = OracleRun(prob)
    assert len(O.d_ids) > 0 and np.all(O.space.dirichlet[O.d_ids])
    a = O.monolithic()
    assert b_error(O.space, a, b_ref=sources.trace_B)[1] <= 1e-12
    ai, lam, info = O.solve_ieti(rtol=1e-12)
    assert b_error(O.space, ai, b_ref=sources.trace_B)[1] <= 1e-10


@pytest.mark.parametrize("p,n_els,min_rate", [(1, (2, 4), 0.9), (2, (2, 4), 1.85), (3, (1, 2), 2.3)])
def test_paper_solution_converges_at_order_p(p, n_els, min_rate):
    errs = []
    for n_el in n_els:
        O = OracleRun(configs.paper_cube(degree=p, n_el=n_el, n_sub=3))
        errs.append(b_error(O.space, O.monolithic(), b_ref=sources.paper_B)[0])
    rate = np.log2(errs[0] / errs[1]) / np.log2(n_els[1] / n_els[0])
    assert rate >= min_rate, (errs, rate)
