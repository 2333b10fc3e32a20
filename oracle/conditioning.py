"""Condition numbers of the local systems of the IETI-DP method (analysis
for the precision choice of the local factorisations; test infrastructure
like the rest of the oracle).

For every subdomain k: kappa(K_rr^(k)) of the tree-gauged local stiffness
restricted to its remaining DOFs (Section 2.1, Eq. localProb: the matrix the
local factorisation works on), kappa(K_VV^(k)) of its interior block and
kappa(S_rIrI^(k)) of the Dirichlet Schur complement (Eq. DirPrec), each as
the ratio of the extreme eigenvalues of the symmetric positive definite
matrix: the largest by Lanczos on the matrix, the smallest by Lanczos on its
inverse (shift-invert about 0, SuperLU).

Usage: python -m oracle.conditioning cube64 | cube256 | stream [first] [count]
"""
from __future__ import annotations

import sys
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .run import OracleRun


def spd_extremes(A):
    """(lambda_min, lambda_max) of a sparse symmetric positive definite A."""
    n = A.shape[0]
    if n <= 400:
        w = np.linalg.eigvalsh(A.toarray())
        return float(w[0]), float(w[-1])
    hi = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False, tol=1e-6)[0]
    lo = spla.eigsh(A.tocsc(), k=1, sigma=0.0, which="LM", return_eigenvectors=False, tol=1e-6)[0]
    return float(lo), float(hi)


def schur_extremes(L):
    """(lambda_min, lambda_max) of S_rIrI through its action (dense for small n_I)."""
    nI = len(L.I)
    if nI == 0:
        return None
    S = np.column_stack([L.schur_I(e) for e in np.eye(nI)])
    w = np.linalg.eigvalsh(0.5 * (S + S.T))
    return float(w[0]), float(w[-1])


def local_conditioning(prob, schur=True):
    """Per subdomain: n_r, n_I and the three condition numbers."""
    O = OracleRun(prob)
    D = O.ieti
    out = []
    for L in D.locals:
        lo, hi = spd_extremes(L.K_rr)
        row = {"k": L.k, "n_r": int(L.K_rr.shape[0]), "n_I": int(len(L.I)), "kappa_Krr": hi / lo}
        # with the symmetric diagonal scaling D^{-1/2} K_rr D^{-1/2}, which bounds the
        # componentwise backward error of a Cholesky factorisation
        dsc = sp.diags(1.0 / np.sqrt(L.K_rr.diagonal()))
        slo, shi = spd_extremes((dsc @ L.K_rr @ dsc).tocsc())
        row["kappa_Krr_scaled"] = shi / slo
        if len(L.V):
            vlo, vhi = spd_extremes(L.K_VV)
            row["kappa_KVV"] = vhi / vlo
        if schur:
            e = schur_extremes(L)
            if e is not None:
                row["kappa_S"] = e[1] / e[0]
        out.append(row)
    return out


def _summary(name, rows):
    k = np.array([r["kappa_Krr"] for r in rows])
    kd = np.array([r["kappa_Krr_scaled"] for r in rows])
    kv = np.array([r.get("kappa_KVV", np.nan) for r in rows])
    ks = np.array([r.get("kappa_S", np.nan) for r in rows])
    eps32 = np.finfo(np.float32).eps
    print(f"{name}: {len(rows)} subdomains, kappa(K_rr) min {k.min():.3g} median {np.median(k):.3g} "
          f"max {k.max():.3g}; scaled kappa(D^-1/2 K_rr D^-1/2) min {kd.min():.3g} median {np.median(kd):.3g} "
          f"max {kd.max():.3g}; kappa(K_VV) max {np.nanmax(kv):.3g}; kappa(S_rIrI) max {np.nanmax(ks):.3g}; "
          f"eps32*kappa(K_rr) max {eps32 * k.max():.3g}, with scaling {eps32 * kd.max():.3g}", flush=True)


def main(argv):
    from workloads import configs

    which = argv[1] if len(argv) > 1 else "cube64"
    if which == "stream":
        first = int(argv[2]) if len(argv) > 2 else 0
        count = int(argv[3]) if len(argv) > 3 else 8
        allrows = []
        for i in range(first, first + count):
            t = time.perf_counter()
            rows = local_conditioning(configs.stream_problem(i), schur=False)
            allrows += rows
            _summary(f"stream problem {i} ({time.perf_counter() - t:.0f}s)", rows)
        _summary(f"stream problems {first}..{first + count - 1}", allrows)
        return
    prob = configs.make_config(which)
    rows = local_conditioning(prob, schur=(which != "cube64"))
    for r in rows:
        print(r, flush=True)
    _summary(which, rows)


if __name__ == "__main__":
    main(sys.argv)
