"""CPU tests of the C-ABI library: exports, host assembly and exact maps.

ieti_assemble runs on the host only, so its integer maps (weights, tree,
Dirichlet flags, primal DOFs, multiplier rows, local DOF lists) must equal
the oracle's bit for bit, and its assembled blocks must match to round-off.
"""
import os
import re

import numpy as np
import pytest

from oracle.run import OracleRun
from oracle.space import Space
from oracle.topology import build_topology
from workloads import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol(ietilib):
    header = open(os.path.join(ROOT, "include", "ietidp.h")).read()
    names = set(re.findall(r"\b(ieti_[A-Za-z_]+)\s*\(", header))
    names.discard("ieti_field_fn")
    assert len(names) >= 14
    for n in sorted(names):
        assert hasattr(ietilib, n), n


def _problems():
    part = np.array([0, 0, 1, 2, 2, 1, 0, 3, 1, 2, 3, 3], dtype=np.int32)
    return [
        ("cube8", configs.cube8()),
        ("uneven", configs.small_cube(P=(3, 2, 2), part=part, degree=2, n_el=2, source="trig",
                                      nu=np.where(np.arange(12) % 3 == 0, 1e-3, 1.0))),
        ("cube64_p1", configs.cube64(degree=1, n_el=2)),
        ("ring_coarse", configs.ring576(degree=2, n_el=1, n_theta=12)),
        # non-homogeneous Dirichlet data: the loads carry the lifting -K a_D
        ("paper_cube", configs.paper_cube(degree=2, n_el=2, n_sub=4)),
    ]


@pytest.mark.parametrize("name,prob", _problems(), ids=[n for n, _ in _problems()])
def test_maps_bit_exact_and_blocks_match_oracle(ietilib, name, prob):
    from paper_2501_04340_amd import Solver
    S = Solver(prob)
    O = OracleRun(prob)
    T = O.topo
    m = S.maps()
    assert np.array_equal(m["weight"], T.weight)
    assert np.array_equal(m["tree"], T.tree)
    assert np.array_equal(m["dirichlet"], T.dirichlet)
    assert np.array_equal(m["primal_edges"], T.primal_edges)
    assert np.array_equal(m["mult"], T.mult)
    assert all(np.array_equal(a, b) for a, b in zip(m["sub_r"], T.sub_r))
    sz = S.sizes()
    assert sz["n_g"] == T.n_g and sz["m_r"] == T.m_r and sz["n_gp"] == T.n_gp
    for k in range(T.n_sub):
        K, load = S.local_system(k)
        pats = np.flatnonzero(prob.patch_to_sub == k)
        Kk = sum(O.mats[q] for q in pats).tocsr()
        jk = np.zeros(O.space.n_edges)
        for q in pats:
            g, j = O.loads[q]
            np.add.at(jk, g, j)
        idx = np.concatenate([T.sub_r[k], T.sub_p[k]])
        Ko = Kk[idx][:, idx]
        assert abs(K - Ko).max() <= 1e-13 * abs(Ko).max()
        assert np.abs(load - jk[idx]).max() <= 1e-13 * max(np.abs(jk).max(), 1e-300)
    S.close()


def test_full_size_maps_bit_exact(ietilib):
    """The cube64 workload (123,201 DOFs): integer maps at full size."""
    from paper_2501_04340_amd import Solver
    prob = configs.cube64()
    # assembly is irrelevant for the maps; skip the expensive source evaluation
    prob.source = lambda x: np.zeros_like(x)
    S = Solver(prob)
    T = build_topology(Space(prob))
    m = S.maps()
    assert np.array_equal(m["weight"], T.weight)
    assert np.array_equal(m["tree"], T.tree)
    assert np.array_equal(m["primal_edges"], T.primal_edges)
    assert np.array_equal(m["mult"], T.mult)
    assert S.sizes()["n_g"] == 123201


def test_error_paths(ietilib):
    from paper_2501_04340_amd import Solver
    from paper_2501_04340_amd.ietidp import IetiError
    prob = configs.cube8()
    bad = prob.with_partition(np.array([0, 0, 0, 0, 2, 2, 2, 2], dtype=np.int32))
    with pytest.raises(IetiError) as e:
        Solver(bad)
    assert e.value.code == -2
    S = Solver(prob)
    with pytest.raises(IetiError) as e:
        S.solve()
    assert e.value.code == -8
    bad_deg = prob.with_refinement(degree=9)
    with pytest.raises(IetiError) as e:
        Solver(bad_deg)
    assert e.value.code == -1


def test_plan_accounts_for_every_tile(ietilib):
    from paper_2501_04340_amd import Solver
    S = Solver(configs.cube8())
    info = S.plan_info()
    assert info["tile"] == 64
    assert 0 < info["flops"] <= info["dense_flops"] * 1.0000001
    assert info["sum_nI2"] == 8 * 72 * 72


def test_network_file_is_checked_before_any_device_work(ietilib, tmp_path):
    """ieti_nn_load rejects a missing, foreign, inconsistent or truncated
    file from its header alone (no device allocation happens, so this runs
    without a GPU)."""
    import ctypes as C
    import struct
    lib = ietilib
    out = C.c_void_p()
    assert lib.ieti_nn_load(str(tmp_path / "missing.bin").encode(), C.byref(out)) == -1
    p = tmp_path / "foreign.bin"
    p.write_bytes(b"NOTANET!" + bytes(28))
    assert lib.ieti_nn_load(str(p).encode(), C.byref(out)) == -1
    # right tag, sizes of a 2x3x1 network (1 layer of 3, 1 coefficient, 2 outputs) but a wrong count
    good_n = 3 * (2 + 1) + 2 * (3 + 1)
    p.write_bytes(b"IETINN01" + struct.pack("<5iq", 2, 3, 1, 1, 2, good_n + 1) + bytes(4 * good_n))
    assert lib.ieti_nn_load(str(p).encode(), C.byref(out)) == -1
    # consistent header, parameters cut short
    p.write_bytes(b"IETINN01" + struct.pack("<5iq", 2, 3, 1, 1, 2, good_n) + bytes(4 * (good_n - 1)))
    assert lib.ieti_nn_load(str(p).encode(), C.byref(out)) == -1
    assert out.value is None


def test_schedule_parameters_are_validated(ietilib):
    """ieti_set_factor_params refuses thresholds and workgroup counts out of
    range (host-side checks, no GPU) and reads back what it accepted."""
    from paper_2501_04340_amd import Solver
    from paper_2501_04340_amd.ietidp import IetiError
    from workloads import configs

    S = Solver(configs.cube8())
    try:
        for bad in [(0, 4, 1024), (8, 0, 1024), (8, 4, 0), (100, 4, 1024)]:
            with pytest.raises(IetiError):
                S.set_factor_params(*bad)
        S.set_factor_params(12, 6, 512)
        params, log = S.factor_tuning()
        assert params == (12, 6, 512) and log.shape == (0, 4)
    finally:
        S.close()


def test_without_primal_dofs_maps_match_oracle(ietilib):
    """ieti_assemble_ex with primal = 0 (the singular local problems of
    Section 3): no primal DOFs, and the remaining DOFs and multiplier rows
    bit-exact against the oracle's topology without primal DOFs (an edge of
    three or more subdomains gets one row, between its first two)."""
    from paper_2501_04340_amd import Solver

    prob = configs.cube8()
    S = Solver(prob, primal=False)
    try:
        mp = S.maps()
        T = build_topology(Space(prob), primal_enabled=False)
        assert S.n_gp == 0 and T.n_gp == 0
        assert np.array_equal(mp["mult"], T.mult)
        for k in range(T.n_sub):
            assert np.array_equal(mp["sub_r"][k], T.sub_r[k])
    finally:
        S.close()
    # with the default assembly the same problem has the paper's primal DOFs
    S = Solver(prob)
    try:
        assert S.n_gp == 5
    finally:
        S.close()
