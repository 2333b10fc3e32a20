"""GPU tests of multi-problem batches: one handle, one set of launches for
all problems, per-problem PCG recurrences.

* With the same GEMV launch shape, a batch solve reproduces each problem's
  individual solve bit for bit (same reductions over the same per-problem
  ranges), including the per-problem iteration counts.
* Every problem's B field matches the oracle's monolithic solve (relative
  L2 error <= 1e-9 at rtol 1e-12).
* Mixed precision on a batch meets rtol on every problem's FP64 residual.
"""
import numpy as np
import pytest

from oracle.post import b_error
from oracle.run import OracleRun
from workloads import configs

pytestmark = pytest.mark.gpu


def _probs():
    part = np.array([0, 0, 1, 2, 2, 1, 0, 3, 1, 2, 3, 3], dtype=np.int32)
    return [
        configs.cube8(),
        configs.small_cube(P=(3, 2, 2), part=part, degree=2, n_el=2, source="trig",
                           nu=np.where(np.arange(12) % 3 == 0, 1e-3, 1.0)),
        configs.ring576(degree=2, n_el=1, n_theta=12),
        configs.paper_cube(degree=2, n_el=2, n_sub=4),  # prescribed boundary values at an edge offset
        configs.cube8(degree=3, n_el=4),
        configs.cube64(degree=2, n_el=2),
    ]


@pytest.fixture(scope="module")
def batch(ietilib):
    from paper_2501_04340_amd import Solver
    probs = _probs()
    print(f"[gpu-batch] {len(probs)} problems", flush=True)
    B = Solver(probs)
    singles = [Solver(p) for p in probs]
    return probs, B, singles


def test_batch_equals_individual_solves_bitwise(batch):
    probs, B, singles = batch
    B.factor(gemv_variant=5)
    a, st = B.solve(rtol=1e-10)
    parts = B.split(a)
    info = B.batch_info()
    lam = B.lambda_()
    for i, S in enumerate(singles):
        S.factor(gemv_variant=5)
        a_i, st_i = S.solve(rtol=1e-10)
        assert info[i]["iters"] == st_i["iters"], i
        assert np.array_equal(parts[i], a_i), i
        r0 = info[i]["mr_base"]
        assert np.array_equal(lam[r0:r0 + S.m_r], S.lambda_()), i
    assert st["iters"] == max(b["iters"] for b in info)


def test_batch_equals_individual_solves_bitwise_symmetric_gemv(batch):
    from paper_2501_04340_amd.ietidp import GEMV_SYM
    probs, B, singles = batch
    B.factor(gemv_variant=GEMV_SYM)
    a, st = B.solve(rtol=1e-10)
    parts = B.split(a)
    info = B.batch_info()
    for i, S in enumerate(singles):
        S.factor(gemv_variant=GEMV_SYM)
        a_i, st_i = S.solve(rtol=1e-10)
        assert info[i]["iters"] == st_i["iters"], i
        assert np.array_equal(parts[i], a_i), i


def test_batch_solution_matches_oracle(batch):
    probs, B, singles = batch
    B.factor()
    a, st = B.solve(rtol=1e-12, maxit=3000)
    assert st["status"] == 0 and st["rel_residual"] <= 1e-12
    for i, (p, ai) in enumerate(zip(probs, B.split(a))):
        O = OracleRun(p)
        rel = b_error(O.space, ai, a_ref=O.monolithic())[1]
        print(f"[gpu-batch] problem {i}: rel B error vs monolithic oracle = {rel:.3e}")
        assert rel <= 1e-9


def test_batch_mixed_precision(batch):
    from paper_2501_04340_amd.ietidp import PREC_FP64, PREC_MIXED
    probs, B, singles = batch
    B.factor(precision=PREC_MIXED)
    try:
        a, st = B.solve(rtol=1e-10, maxit=4000)
    finally:
        B.factor(precision=PREC_FP64)
    assert st["status"] == 0
    b = B.rhs()
    res = b - B.apply_F(B.lambda_())
    for info in B.batch_info():
        sl = slice(info["mr_base"], info["mr_base"] + info["m_r"])
        assert np.linalg.norm(res[sl]) <= 1e-10 * np.linalg.norm(b[sl])


def test_first_solve_does_not_read_stale_device_memory(ietilib):
    """Regression: the first PCG direction must not read the previous
    contents of its buffer (0 * NaN from reused device memory made the first
    p^T F p NaN).  Device memory is filled with NaN and released before the
    handle allocates its buffers."""
    import torch
    from paper_2501_04340_amd import Solver
    junk = torch.full((1 << 28,), float("nan"), dtype=torch.float64, device="cuda")
    del junk
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    S = Solver(configs.stream_problem(118))
    S.factor(gemv_variant=0)
    a, st = S.solve(rtol=1e-8)
    assert st["status"] == 0 and st["rel_residual"] <= 1e-8 and np.isfinite(a).all()
