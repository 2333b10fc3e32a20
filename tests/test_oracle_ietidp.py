"""Pins of the oracle's IETI-DP solver against the monolithic definition.

Section 2.1 (Eqs. gloDP-localProb) reaches exactly the gauged global
solution up to the PCG tolerance, which gives closed-form checks.
"""
import json
import os

import numpy as np
import pytest

from oracle.ietidp import IetiDP, SubdomainNotInvertible, lanczos_condition
from oracle.post import b_error
from oracle.run import OracleRun
from workloads import configs, sources


@pytest.fixture(scope="module")
def cube8_run():
    O = OracleRun(configs.cube8())
    a_mono = O.monolithic()
    a, lam, info = O.solve_ieti(rtol=1e-13)
    return O, a_mono, a, lam, info


def test_ieti_equals_monolithic(cube8_run):
    O, a_mono, a, lam, info = cube8_run
    assert info["converged"]
    assert np.abs(a - a_mono).max() <= 1e-10 * np.abs(a_mono).max()
    assert b_error(O.space, a, a_ref=a_mono)[1] < 1e-10
    assert b_error(O.space, a, b_ref=sources.poly_B)[1] < 1e-11


def test_lambda_closed_form_from_monolithic(cube8_run):
    """lambda_row = j_e^(k) - (K^(k) a^(k))_e for the +1 subdomain k of the row."""
    O, a_mono, a, lam, info = cube8_run
    prob = O.prob
    for k in range(O.topo.n_sub):
        pats = np.flatnonzero(prob.patch_to_sub == k)
        Kk = sum(O.mats[q] for q in pats)
        jk = np.zeros(O.space.n_edges)
        for q in pats:
            g, j = O.loads[q]
            np.add.at(jk, g, j)
        res = jk - Kk @ a_mono
        rows = np.flatnonzero(O.topo.mult[:, 1] == k)
        np.testing.assert_allclose(lam[rows], res[O.topo.mult[rows, 0]], atol=1e-10 * np.abs(lam).max())
        rows = np.flatnonzero(O.topo.mult[:, 2] == k)
        np.testing.assert_allclose(-lam[rows], res[O.topo.mult[rows, 0]], atol=1e-10 * np.abs(lam).max())


def test_dense_spectrum(cube8_run, golden_dir):
    O, *_ = cube8_run
    F, M = O.ieti.dense_operators()
    assert np.abs(F - F.T).max() < 1e-12 * np.abs(F).max()
    assert np.linalg.eigvalsh(F).min() > 0
    w = np.sort(np.linalg.eigvals(M @ F).real)
    # D_s = I with two subdomains per multiplier: M_D = 4x the multiplicity-scaled
    # preconditioner, whose spectrum is bounded below by 1 (FETI-DP theory).
    assert w[0] > 4.0 - 1e-8
    kappa = w[-1] / w[0]
    fits = json.load(open(os.path.join(golden_dir, "paper_fits.json")))
    lo, hi = fits["exp1_kappa_axis"]["min"], 8.5
    assert lo <= kappa <= hi
    # Lanczos estimate from the PCG coefficients agrees with the dense spectrum
    lmin, lmax = lanczos_condition(cube8_run[4])
    assert abs(lmax / lmin - kappa) < 1e-3 * kappa


def test_partition_independence_of_B():
    """Section 4: the multipatch problem (hence B) does not depend on the decomposition.

    Holds when the discrete load is compatible (orthogonal to discrete
    gradients): here the polynomial source, which Gauss quadrature integrates
    exactly.  With an inexactly integrated source each tree gauge picks a
    different representative and B changes at the level of the quadrature
    error, so GPU/oracle comparisons always use the identical tree.
    """
    base = configs.small_cube(P=(2, 2, 2), degree=2, n_el=2, source="poly")
    parts = [np.zeros(8, dtype=np.int32), np.array([0, 0, 0, 0, 1, 1, 1, 1]), np.arange(8)]
    sols = []
    for part in parts:
        O = OracleRun(base.with_partition(part))
        if O.topo.n_sub == 1:
            assert O.topo.m_r == 0
        a, lam, info = O.solve_ieti(rtol=1e-13)
        sols.append((O, a))
    ref_O, ref_a = sols[0]
    for O, a in sols[1:]:
        assert b_error(ref_O.space, a, a_ref=ref_a)[1] < 1e-10


def test_primal_dofs_are_needed():
    """Section 3: without the weight-2 primal DOFs some K_rr^(k) are singular."""
    with pytest.raises(SubdomainNotInvertible):
        O = OracleRun(configs.cube8(), primal_enabled=False)
        O.ieti


def test_warm_start_and_restart(cube8_run):
    O, a_mono, a, lam, info = cube8_run
    lam2, info2 = O.ieti.pcg(rtol=1e-8, lam0=lam)
    assert info2["iters"] == 0
    # checkpoint/resume: stop after 4 iterations, restart from there
    lam_k, _ = O.ieti.pcg(rtol=1e-8, maxit=4)
    lam_r, info_r = O.ieti.pcg(rtol=1e-10, lam0=lam_k)
    assert info_r["converged"]
    assert np.abs(lam_r - lam).max() < 1e-8 * np.abs(lam).max()


def test_heterogeneous_multipatch_subdomains():
    """Multi-patch uneven subdomains with nu contrast: IETI-DP still equals the monolithic solve."""
    part = np.array([0, 0, 1, 2, 2, 1, 0, 3, 1, 2, 3, 3], dtype=np.int32)
    prob = configs.small_cube(P=(3, 2, 2), part=part, degree=2, n_el=2, source="trig",
                              nu=np.where(np.arange(12) % 3 == 0, 1e-3, 1.0))
    O = OracleRun(prob)
    a_mono = O.monolithic()
    a, lam, info = O.solve_ieti(rtol=1e-13)
    assert O.topo.n_gp > 0
    assert b_error(O.space, a, a_ref=a_mono)[1] < 1e-9
