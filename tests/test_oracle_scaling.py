"""Pins of the scaled Dirichlet preconditioner (rho-scaling, beyond the
paper's D_s = I): properties that FETI-DP theory fixes independently of
the implementation.

* delta_k + delta_l = 1 on every multiplier row (partition of unity).
* Multiplicity scaling (delta = 1/2) is exactly 1/4 of the unscaled
  preconditioner, so it leaves kappa unchanged.
* With a partition-of-unity scaling the smallest eigenvalue of M_D F is 1
  (bounded below by 1, attained).
* Coefficient robustness: on a checkerboard of reluctivity contrast c the
  stiffness-scaled kappa stays ~1 while the unscaled kappa grows with c.
* The scaling changes only the preconditioner: PCG reaches the same
  multipliers.
"""
import numpy as np
import pytest

from oracle.run import OracleRun
from workloads import configs


def _checker(c):
    nu = np.array([1.0, c, c, 1.0])
    prob = configs.small_cube(P=(2, 2, 1), part=np.arange(4, dtype=np.int32), degree=2, n_el=2, source="sine", nu=nu)
    return OracleRun(prob).ieti


def _eigs(D):
    F, M = D.dense_operators()
    return np.sort(np.linalg.eigvals(M @ F).real)


@pytest.fixture(scope="module")
def checker():
    return {c: _checker(c) for c in (1.0, 1e4)}


def test_partition_of_unity(checker):
    D = checker[1e4]
    D.set_scaling("stiffness")
    dk, dl = D.delta
    np.testing.assert_allclose(dk + dl, 1.0, rtol=0, atol=1e-15)
    assert np.all((dk > 0) & (dl > 0))
    D.set_scaling("identity")


def test_multiplicity_is_a_quarter_of_identity(checker):
    D = checker[1e4]
    r = np.random.default_rng(3).standard_normal(D.m_r)
    D.set_scaling("identity")
    z1 = D.apply_MD(r)
    D.set_scaling("multiplicity")
    z2 = D.apply_MD(r)
    D.set_scaling("identity")
    np.testing.assert_allclose(z2, 0.25 * z1, rtol=1e-14, atol=1e-14 * np.abs(z1).max())


def test_scaled_spectrum_is_bounded_below_by_one_and_robust(checker):
    kap = {}
    for c, D in checker.items():
        for kind in ("identity", "stiffness"):
            D.set_scaling(kind)
            w = _eigs(D)
            kap[(c, kind)] = w[-1] / w[0]
            if kind == "stiffness":
                assert abs(w[0] - 1.0) <= 1e-8
        D.set_scaling("identity")
    assert kap[(1e4, "stiffness")] <= 1.5 * kap[(1.0, "stiffness")]
    assert kap[(1e4, "identity")] >= 10.0 * kap[(1.0, "identity")]


def test_scaling_changes_only_the_preconditioner(checker):
    D = checker[1e4]
    D.set_scaling("identity")
    lam1, i1 = D.pcg(rtol=1e-12)
    D.set_scaling("stiffness")
    lam2, i2 = D.pcg(rtol=1e-12)
    D.set_scaling("identity")
    assert i2["iters"] < i1["iters"]
    np.testing.assert_allclose(lam2, lam1, rtol=0, atol=1e-9 * np.abs(lam1).max())
