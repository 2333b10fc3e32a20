"""Pins of the oracle's discrete space and assembly (Section 2, Eq. discrMS)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.monolithic import global_matrix, solve_monolithic
from oracle.post import b_error
from oracle.space import Space
from oracle.topology import build_topology
from workloads import configs, sources


@pytest.fixture(scope="module")
def cube8_space():
    prob = configs.cube8()
    S = Space(prob)
    mats, loads = S.assemble()
    return prob, S, mats, loads


def test_curl_of_gradient_is_zero_exactly(cube8_space):
    _, S, _, _ = cube8_space
    C = S.curl_incidence()
    G = S.gradient_matrix()
    assert (C @ G).count_nonzero() == 0
    # every edge bounds at least one face and every face has 4 edges
    assert np.all(np.diff(C.indptr) == 4)


def test_stiffness_kernel_contains_gradients(cube8_space):
    _, S, mats, _ = cube8_space
    K = global_matrix(mats)
    G = S.gradient_matrix().astype(float)
    KG = K @ G
    assert abs(KG).max() <= 1e-12 * abs(K).max() * 2
    assert abs(K - K.T).max() <= 1e-15 * abs(K).max()


def test_curl_of_discrete_gradient_vanishes_pointwise(cube8_space):
    _, S, _, _ = cube8_space
    rng = np.random.default_rng(0)
    phi = rng.standard_normal(S.n_nodes)
    a = S.gradient_matrix() @ phi
    # B of a discrete gradient is zero at every quadrature point
    ed = S.element_data(0)
    for pidx in range(8):
        _, _, curl, _ = S.physical(pidx, ed)
        ae = a[S.patch_local_edges(pidx)][ed["loc"]]
        B = np.einsum("eqaf,ef->eqa", curl, ae)
        assert abs(B).max() < 1e-12 * abs(phi).max()


def test_discrete_kernel_dimension_tiny():
    """dim ker K (Dirichlet rows removed) = number of interior nodes (discrete de Rham)."""
    prob = configs.small_cube(P=(1, 1, 1), degree=2, n_el=2)
    S = Space(prob)
    K = global_matrix(S.assemble(with_load=False)[0]).toarray()
    free = ~S.dirichlet
    Kf = K[np.ix_(free, free)]
    ev = np.linalg.eigvalsh(Kf)
    n_kernel = int(np.sum(ev < 1e-10 * ev.max()))
    assert n_kernel == int(np.count_nonzero(~S.node_boundary))


def test_manufactured_polynomial_is_reproduced():
    """A in the p=2 space with n x A = 0: the Galerkin B equals curl A to round-off."""
    prob = configs.cube8()
    S = Space(prob)
    mats, loads = S.assemble()
    topo = build_topology(S)
    a, _, _ = solve_monolithic(S, topo, mats, loads)
    _, rel = b_error(S, a, b_ref=sources.poly_B)
    assert rel < 1e-12


def test_manufactured_fields_are_consistent():
    """The hand-expanded J and B of the workloads match finite differences of A."""
    rng = np.random.default_rng(1)
    x = rng.uniform(0.1, 0.9, size=(20, 3))
    h = 1e-5
    for A, B, J in ((sources.poly_A, sources.poly_B, sources.poly_J), (sources.sine_A, sources.sine_B, sources.sine_J)):
        def curl(f, x):
            g = np.zeros((x.shape[0], 3, 3))  # g[:, comp, dir]
            for d in range(3):
                e = np.zeros(3)
                e[d] = h
                g[:, :, d] = (f(x + e) - f(x - e)) / (2 * h)
            return np.stack([g[:, 2, 1] - g[:, 1, 2], g[:, 0, 2] - g[:, 2, 0], g[:, 1, 0] - g[:, 0, 1]], axis=1)
        np.testing.assert_allclose(curl(A, x), B(x), atol=1e-8)
        np.testing.assert_allclose(curl(B, x), J(x), atol=2e-6)


def test_trig_source_is_divergence_free():
    src = sources.TrigCurlSource(3)
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, size=(10, 3))
    h = 1e-5
    div = np.zeros(10)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        div += (src(x + e)[:, d] - src(x - e)[:, d]) / (2 * h)
    assert abs(div).max() < 1e-6 * abs(src(x)).max()


@pytest.mark.parametrize("p", [1, 2])
def test_optimal_convergence_order(p):
    """eps_B = O(h^p) for a smooth zero-trace field (Section 4 expects optimal order)."""
    errs = []
    for n_el in (2, 4):
        prob = configs.small_cube(P=(1, 1, 1), degree=p, n_el=n_el)
        S = Space(prob)
        mats, loads = S.assemble()
        topo = build_topology(S)
        a, _, _ = solve_monolithic(S, topo, mats, loads)
        errs.append(b_error(S, a, b_ref=sources.sine_B)[0])
    order = np.log2(errs[0] / errs[1])
    assert abs(order - p) < 0.35, (errs, order)


def test_annulus_map_is_exact_circle():
    prob = configs.ring576(n_theta=48)
    from oracle.geometry import patch_map
    xi = np.random.default_rng(0).uniform(0, 1, size=(50, 3))
    for pidx in (0, 17, 48 * 3 + 5):
        x, DF = patch_map(prob, pidx, xi)
        r = np.hypot(x[:, 0], x[:, 1])
        j = (pidx // 48) % 3
        radii = prob.geom_params[2:]
        np.testing.assert_allclose(r, radii[j] + xi[:, 1] * (radii[j + 1] - radii[j]), rtol=1e-14)
        # Jacobian against central differences
        h = 1e-6
        for b in range(3):
            e = np.zeros(3)
            e[b] = h
            fd = (patch_map(prob, pidx, xi + e)[0] - patch_map(prob, pidx, xi - e)[0]) / (2 * h)
            np.testing.assert_allclose(DF[:, :, b], fd, atol=1e-8)
