"""Pin of the oracle's push-forward on a non-affine patch map.

On the NURBS annulus the Jacobian DF of a patch map is not diagonal: its
columns are the azimuthal, radial and axial directions, rotated with the
angle.  The covariant Piola map w = DF^{-T} w_hat and the curl transform
curl w = DF curl_hat w_hat / det DF (Section 2, the curl-conforming
multipatch space of Eq. discrMS) then differ from their transposed
variants, which the box workloads (diagonal DF, DF^{-T} = DF^{-1}) cannot
tell apart.

Closed form used here (cylindrical coordinates r, theta, z, nu = 1): the
azimuthal field A = f(r) g(z) e_theta with f(r) = (r - 1)(1.75 - r) and
g(z) = z (1 - z) has n x A = 0 on the inner and outer cylinders (f = 0) and on
the two end planes (g = 0), so it solves the boundary value problem of
Section 2 with
    B = curl A = -f g' e_r + (f / r + f') g e_z,
    J = curl curl A = [-f g'' - (f'' + f' / r - f / r^2) g] e_theta,
which is divergence free (axisymmetric and azimuthal).  The annulus is a
solid torus, not simply connected, but its boundary is connected, so the
gauged problem still has a unique B.  The monolithic oracle solve must then
converge in B like h^p (Section 4's error slopes); a transposed DF in
either transform leaves an O(1) error that does not decrease.
"""
import numpy as np
import pytest

from oracle.post import b_error
from oracle.run import OracleRun
from workloads.problem import GEOM_ANNULUS, Problem

R_IN, R_OUT = 1.0, 1.75


def _cyl(x):
    r = np.hypot(x[:, 0], x[:, 1])
    e_t = np.stack([-x[:, 1] / r, x[:, 0] / r, np.zeros_like(r)], axis=1)
    e_r = np.stack([x[:, 0] / r, x[:, 1] / r, np.zeros_like(r)], axis=1)
    return r, x[:, 2], e_t, e_r


def _f(r):
    return (r - R_IN) * (R_OUT - r)


def _df(r):
    return R_IN + R_OUT - 2.0 * r


def _g(z):
    return z * (1.0 - z)


def _dg(z):
    return 1.0 - 2.0 * z


def field_A(x):
    r, z, e_t, _ = _cyl(x)
    return (_f(r) * _g(z))[:, None] * e_t


def field_B(x):
    r, z, _, e_r = _cyl(x)
    e_z = np.zeros_like(e_r)
    e_z[:, 2] = 1.0
    return (-_f(r) * _dg(z))[:, None] * e_r + ((_f(r) / r + _df(r)) * _g(z))[:, None] * e_z


def field_J(x):
    r, z, e_t, _ = _cyl(x)
    # f'' = -2, g'' = -2
    j_t = 2.0 * _f(r) - (-2.0 + _df(r) / r - _f(r) / r ** 2) * _g(z)
    return j_t[:, None] * e_t


def annulus(n_theta, degree, n_el):
    P = (n_theta, 3, 1)
    n = n_theta * 3
    return Problem(name=f"annulus_pin[{n_theta},{degree},{n_el}]", geom_kind=GEOM_ANNULUS, patches=P,
                   periodic=(1, 0, 0), geom_params=np.array([0.0, 1.0, 1.0, 1.25, 1.5, 1.75]), degree=degree,
                   n_el=n_el, patch_to_sub=(np.arange(n) % n_theta).astype(np.int32), nu=np.ones(n), source=field_J,
                   exact_A=field_A, exact_B=field_B)


def test_closed_form_is_consistent():
    """B and J above are the curl and curl curl of A (central differences)."""
    rng = np.random.default_rng(3)
    r = rng.uniform(1.1, 1.65, 20)
    th = rng.uniform(0, 2 * np.pi, 20)
    z = rng.uniform(0.1, 0.9, 20)
    x = np.stack([r * np.cos(th), r * np.sin(th), z], axis=1)

    def curl(F, x, h=1e-5):
        out = np.zeros_like(x)
        d = [np.zeros(3) for _ in range(3)]
        for a in range(3):
            d[a][a] = h
        D = [(F(x + d[a]) - F(x - d[a])) / (2 * h) for a in range(3)]  # D[a][:, c] = dF_c / dx_a
        out[:, 0] = D[1][:, 2] - D[2][:, 1]
        out[:, 1] = D[2][:, 0] - D[0][:, 2]
        out[:, 2] = D[0][:, 1] - D[1][:, 0]
        return out

    np.testing.assert_allclose(curl(field_A, x), field_B(x), atol=1e-8)
    np.testing.assert_allclose(curl(field_B, x, h=1e-4), field_J(x), atol=1e-6)
    # boundary: the tangential trace of A vanishes on every face
    xb = np.stack([R_IN * np.cos(th), R_IN * np.sin(th), z], axis=1)
    assert np.abs(field_A(xb)).max() == 0.0
    xb[:, 2] = 0.0
    assert np.abs(field_A(xb)).max() == 0.0


@pytest.mark.parametrize("degree", [1, 2])
def test_annulus_b_error_converges_like_h_to_the_p(degree):
    errs = []
    for n_el in (1, 2, 4):
        O = OracleRun(annulus(12, degree, n_el))
        a = O.monolithic()
        errs.append(b_error(O.space, a, b_ref=field_B)[1])
    errs = np.array(errs)
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(errs[1:] < errs[:-1]), errs
    # observed p = 1: 0.99, 1.00; p = 2: 2.005, 2.002
    assert orders[-1] > degree - 0.15, (errs, orders)
    assert errs[-1] < (0.02 if degree == 2 else 0.2), errs
