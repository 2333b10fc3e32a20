"""The allocation-free operator application (ieti_apply_F_noalloc) against
ieti_apply_F, through the C ABI.

Both run the same kernels in the same order on the same factorisation, so
their results are compared bit for bit: first on a problem whose interface
blocks span several GEMV tasks per tile row (both the symmetric lower-tile
GEMV and a row-streaming shape), then on a smaller problem in the same
process, whose call reuses the device array the larger one left behind.
"""
import numpy as np
import pytest

from workloads import configs

pytestmark = pytest.mark.gpu


def _noalloc_apply(S, lam, stream=None):
    import torch

    d_lam = torch.from_numpy(lam).to("cuda")
    d_q = torch.full((S.m_r,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    S.apply_F_noalloc(d_lam.data_ptr(), d_q.data_ptr(), stream=stream)
    torch.cuda.synchronize()
    return d_q.cpu().numpy()


@pytest.mark.parametrize("variant", ["sym", 4])
def test_noalloc_matches_apply_F_then_a_smaller_problem(ietilib, variant):
    import torch

    from paper_2501_04340_amd import Solver
    from paper_2501_04340_amd.ietidp import GEMV_SYM

    torch.cuda.set_device(0)
    gv = GEMV_SYM if variant == "sym" else variant
    big = Solver(configs.cube64(degree=3, n_el=4))
    small = Solver(configs.cube8())
    print(f"noalloc: variant {variant}, m_r {big.m_r} then {small.m_r}", flush=True)
    try:
        rng = np.random.default_rng(7)
        for S in (big, small):
            S.factor(gemv_variant=gv)
            lam = rng.standard_normal(S.m_r)
            q_ref = S.apply_F(lam)
            q = _noalloc_apply(S, lam)
            assert np.all(np.isfinite(q))
            assert np.array_equal(q, q_ref), np.max(np.abs(q - q_ref))
        # on a caller's stream
        st = torch.cuda.Stream()
        lam = rng.standard_normal(small.m_r)
        with torch.cuda.stream(st):
            q = _noalloc_apply(small, lam, stream=st.cuda_stream)
        assert np.array_equal(q, small.apply_F(lam))
    finally:
        big.close()
        small.close()


def test_noalloc_rejects_unfactored_handle(ietilib):
    import torch

    from paper_2501_04340_amd import Solver
    from paper_2501_04340_amd.ietidp import IetiError

    torch.cuda.set_device(0)
    S = Solver(configs.cube8())
    try:
        d = torch.zeros(S.m_r, dtype=torch.float64, device="cuda")
        q = torch.zeros(S.m_r, dtype=torch.float64, device="cuda")
        with pytest.raises(IetiError):
            S.apply_F_noalloc(d.data_ptr(), q.data_ptr())
        S.factor()
        with pytest.raises(IetiError):
            S.apply_F_noalloc(d.data_ptr(), d.data_ptr())
    finally:
        S.close()
