"""Host-side (no GPU) checks of multi-problem batches: the batch handle is
the exact concatenation of its problems (sizes, ranges, and every
subdomain's assembled system bit for bit)."""
import numpy as np
import pytest

from paper_2501_04340_amd import Solver
from workloads import configs


def _probs():
    part = np.array([0, 0, 1, 2, 2, 1, 0, 3, 1, 2, 3, 3], dtype=np.int32)
    return [
        configs.cube8(),
        configs.small_cube(P=(3, 2, 2), part=part, degree=2, n_el=2, source="trig",
                           nu=np.where(np.arange(12) % 3 == 0, 1e-3, 1.0)),
        configs.ring576(degree=2, n_el=1, n_theta=12),
    ]


@pytest.fixture(scope="module")
def batch(ietilib):
    probs = _probs()
    return probs, Solver(probs), [Solver(p) for p in probs]


def test_sizes_and_ranges_concatenate(batch):
    probs, B, singles = batch
    assert B.batch == 3
    for key in ["n_edges", "n_global", "m_r", "n_gp", "n_sub", "sum_n_r"]:
        assert getattr(B, key) == sum(getattr(S, key) for S in singles), key
    info = B.batch_info()
    acc = {"edge_base": 0, "mr_base": 0, "gp_base": 0, "sub_base": 0}
    for b, S in zip(info, singles):
        assert (b["n_edges"], b["m_r"], b["n_gp"], b["n_sub"]) == (S.n_edges, S.m_r, S.n_gp, S.n_sub)
        for k, n in [("edge_base", "n_edges"), ("mr_base", "m_r"), ("gp_base", "n_gp"), ("sub_base", "n_sub")]:
            assert b[k] == acc[k]
            acc[k] += b[n]


def test_subdomain_systems_are_bit_identical(batch):
    probs, B, singles = batch
    for b, S in zip(B.batch_info(), singles):
        for k in range(S.n_sub):
            K1, j1 = B.local_system(b["sub_base"] + k)
            K2, j2 = S.local_system(k)
            assert np.array_equal(K1.indptr, K2.indptr) and np.array_equal(K1.indices, K2.indices)
            assert np.array_equal(K1.data, K2.data) and np.array_equal(j1, j2)


def test_maps_are_per_problem(batch):
    probs, B, singles = batch
    with pytest.raises(Exception, match="STATE"):
        B.maps()


def test_batch_coefficient_update_matches_single(batch):
    probs, B, singles = batch
    nu = np.concatenate([np.asarray(p.nu, dtype=np.float64) for p in probs])
    scale = np.linspace(0.8, 1.2, len(nu))
    B.set_coefficients(nu * 1.5, scale)
    off = 0
    info = B.batch_info()
    for i, (p, S) in enumerate(zip(probs, singles)):
        n = len(p.nu)
        S.set_coefficients(nu[off:off + n] * 1.5, scale[off:off + n])
        for k in range(S.n_sub):
            K1, j1 = B.local_system(info[i]["sub_base"] + k)
            K2, j2 = S.local_system(k)
            assert np.array_equal(K1.data, K2.data) and np.array_equal(j1, j2)
        S.set_coefficients(nu[off:off + n], np.ones(n))
        off += n
    B.set_coefficients(nu, np.ones(len(nu)))


def test_batch_of_handles_equals_assembled_batch(batch):
    probs, B, singles = batch
    from paper_2501_04340_amd import Solver
    B2 = Solver.batch_of(singles)
    assert B2.batch == B.batch and B2.m_r == B.m_r and B2.n_edges == B.n_edges
    for k in range(B.n_sub):
        K1, j1 = B.local_system(k)
        K2, j2 = B2.local_system(k)
        assert np.array_equal(K1.data, K2.data) and np.array_equal(j1, j2)
    assert B2.batch_info() == B.batch_info()
