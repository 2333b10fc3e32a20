"""Write the oracle's solution of the full cube64 workload (4x4x4 patches,
p=3, 8 elements per patch and direction, 16 uneven subdomains, 123,201
gauged DOFs) to ``cube64_oracle_a.npz``.

The stored vector is the oracle's reference IETI-DP (SuperLU local
factorisations, dense coarse Cholesky, PCG with the Dirichlet
preconditioner; Section 2.1) run to a relative residual of 1e-13, with the
same tree as every other implementation (Section 3).  The oracle's direct
solve of the gauged global system does not finish at this size; IETI-DP is
exact (Eqs. intProb, coarseProb and localProb reproduce the solution of
Eq. discrMS up to the PCG tolerance), and the oracle's IETI-DP is pinned
against its direct solve on smaller problems.

Only ``oracle/`` and the shared input description ``workloads/`` are used.
Run: ``python tests/golden/make_cube64_golden.py`` (about 10 minutes on one
core).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.monolithic import global_matrix  # noqa: E402
from oracle.run import OracleRun  # noqa: E402
from workloads import configs  # noqa: E402

RTOL = 1e-13
OUT = os.path.join(HERE, "cube64_oracle_a.npz")


def main():
    t0 = time.perf_counter()
    O = OracleRun(configs.cube64())
    a, lam, info = O.solve_ieti(rtol=RTOL, maxit=5000)
    T = O.topo
    K = global_matrix(O.mats)
    j = O.space.global_load(O.loads)
    res = float(np.linalg.norm((K @ a - j)[T.free]) / np.linalg.norm(j[T.free]))
    meta = {"workload": "cube64", "rtol": RTOL, "pcg_iters": int(info["iters"]),
            "rel_residual": float(info["hist"][-1] / np.linalg.norm(O.ieti.rhs)), "global_rel_residual": res,
            "n_edges": int(a.size), "n_g": int(T.n_g), "seconds": round(time.perf_counter() - t0, 1)}
    np.savez_compressed(OUT, a=a, meta=json.dumps(meta))
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
