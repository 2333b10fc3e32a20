"""Admissibility of the patch-to-subdomain map in the library (Section 2:
subdomains are unions of patches, connected through patch interfaces, and
simply connected): IETI_ERR_PARTITION names the subdomain.  The library's
check is cross-checked against the workload partitioner's own
(independently written) face-connectivity and first-Betti-number tests on
random labelings."""
import numpy as np
import pytest

from paper_2501_04340_amd import Solver
from paper_2501_04340_amd.ietidp import IetiError
from workloads import configs, partition
from workloads.problem import GEOM_ANNULUS, Problem


def _box(P, part):
    n = int(np.prod(P))
    return configs.box_problem(P, 1, 1, np.asarray(part, dtype=np.int32), np.ones(n), lambda x: np.zeros_like(x))


def _code(prob):
    try:
        Solver(prob).close()
        return 0, ""
    except IetiError as e:
        return e.code, str(e)


def test_diagonal_patches_are_not_face_connected():
    # (0,0) and (1,1) touch along an edge only
    code, msg = _code(_box((2, 2, 1), [0, 1, 1, 0]))
    assert code == -2 and "subdomain 0" in msg and "patch faces" in msg


def test_ring_of_patches_is_not_simply_connected():
    part = np.zeros(9, dtype=np.int32)
    part[4] = 1  # the centre patch; subdomain 0 is a ring around it
    code, msg = _code(_box((3, 3, 1), part))
    assert code == -2 and "subdomain 0" in msg and "simply connected" in msg


def test_whole_annulus_as_one_subdomain_is_rejected():
    P = (3, 1, 1)
    prob = Problem(name="ring", geom_kind=GEOM_ANNULUS, patches=P, periodic=(1, 0, 0),
                   geom_params=np.array([0.0, 1.0, 1.0, 1.5]), degree=2, n_el=2,
                   patch_to_sub=np.zeros(3, dtype=np.int32), nu=np.ones(3), source=lambda x: np.zeros_like(x))
    code, msg = _code(prob)
    assert code == -2 and "simply connected" in msg
    # one sector per subdomain is admissible
    assert _code(prob.with_partition(np.arange(3)))[0] == 0


def test_empty_subdomain_is_rejected():
    code, msg = _code(_box((2, 1, 1), [0, 2]))
    assert code == -2 and "subdomain 1" in msg


def test_library_agrees_with_the_partitioner_on_random_labelings():
    rng = np.random.default_rng(2024)
    P = (3, 3, 2)
    seen = {"rejected": 0, "accepted": 0, "holes": 0}
    for _ in range(300):
        n_sub = int(rng.integers(2, 4))
        part = rng.integers(0, n_sub, size=int(np.prod(P)))
        if len(np.unique(part)) != n_sub:
            continue
        cells = {}
        for idx, s in enumerate(part):
            cells.setdefault(int(s), []).append((idx % P[0], (idx // P[0]) % P[1], idx // (P[0] * P[1])))
        ok = True
        hole = False
        for cs in cells.values():
            if not partition._face_connected(cs):
                ok = False
                break
            if partition._betti1(cs) != 0:
                ok, hole = False, True
                break
        code, _ = _code(_box(P, part))
        if ok:
            assert code != -2
            seen["accepted"] += 1
        else:
            assert code == -2
            seen["rejected"] += 1
            seen["holes"] += int(hole)
    assert seen["accepted"] > 0 and seen["rejected"] > 0, seen
