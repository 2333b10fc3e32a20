"""Reference dual-primal IETI solver (oracle).

TEST INFRASTRUCTURE ONLY.

Written in the paper's own notation and sign convention (Section 2.1,
Eqs. gloDP, recRem, intProb, coarseProb, localProb, DirPrec):

    F = C_p^T K_pr K_rr^{-1} K_rp C_p - C_p^T K_pp C_p       (n_gp x n_gp)
    G = B_r K_rr^{-1} K_rp C_p                               (m_r x n_gp)
    W = B_r K_rr^{-1} B_r^T                                  (m_r x m_r)
    d = C_p^T K_pr K_rr^{-1} j_r - C_p^T j_p
    e = B_r K_rr^{-1} j_r
    S lambda = (G F^{-1} G^T - W) lambda = G F^{-1} d - e     (intProb)
    a_p = C_p F^{-1} (d - G^T lambda)                         (coarseProb)
    a_r = K_rr^{-1} (j_r - K_rp a_p - B_r^T lambda)           (localProb)

As written F and S are negative definite; PCG is run on the equivalent
positive definite system (-S) lambda = e - G F^{-1} d.  The Dirichlet
preconditioner is M_D^{-1} = D_s B_rI S_rIrI B_rI^T D_s with D_s = I
(Eq. DirPrec; the paper's homogeneous-material choice), where
S_rIrI = K_rIrI - K_rIrV K_rVrV^{-1} K_rVrI and r_I are the remaining
DOFs on interface edges.  Optionally (beyond the paper, which keeps
D_s = I) the jump operator of the preconditioner is scaled, B_D = D B:
every multiplier row joins exactly two subdomains k (+1) and l (-1), and
its entries become +delta_k and -delta_l with delta_k = rho_l / (rho_k +
rho_l), delta_l = rho_k / (rho_k + rho_l) (a partition of unity, the
rho-scaling of Klawonn & Widlund 2002, Farhat et al. 2000).  Here rho_k of a
DOF is the diagonal entry of subdomain k's stiffness matrix there, which
carries the local reluctivity ("stiffness" scaling); "multiplicity" takes
delta = 1/2.

Every subdomain is factorised with SuperLU (scipy.sparse.linalg.splu);
everything else is plain NumPy in float64.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class SubdomainNotInvertible(RuntimeError):
    pass


class LocalProblem:
    """Blocks of one subdomain k."""

    def __init__(self, k, Kk, jk, r, p, isI, gp_index, m_r, mult):
        self.k = k
        self.r, self.p = r, p
        Kk = Kk.tocsr()
        Kr = Kk[r]
        self.K_rr = Kr[:, r].tocsc()
        self.K_rp = Kr[:, p].toarray()
        self.K_pp = Kk[p][:, p].toarray()
        self.j_r = jk[r]
        self.j_p = jk[p]
        n_gp = int(gp_index.max()) + 1 if gp_index.size and gp_index.max() >= 0 else 0
        self.C = np.zeros((len(p), n_gp))
        if len(p):
            self.C[np.arange(len(p)), gp_index[p]] = 1.0
        rows_k = mult[:, 1] == k
        rows_l = mult[:, 2] == k
        bi = np.concatenate([np.flatnonzero(rows_k), np.flatnonzero(rows_l)])
        bj = np.concatenate([mult[rows_k, 3], mult[rows_l, 4]])
        bv = np.concatenate([np.ones(rows_k.sum()), -np.ones(rows_l.sum())])
        self.B = sp.csr_matrix((bv, (bi, bj)), shape=(m_r, len(r)))
        self.isI = isI
        self.I = np.flatnonzero(isI)
        self.V = np.flatnonzero(~isI)
        if len(r):
            try:
                self.lu = spla.splu(self.K_rr, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                                    options={"SymmetricMode": True})
            except RuntimeError as exc:
                raise SubdomainNotInvertible(f"K_rr of subdomain {k} is singular") from exc
            d = self.lu.U.diagonal()
            if np.any(np.abs(d) <= 1e-13 * np.abs(self.K_rr.diagonal()).max()):
                raise SubdomainNotInvertible(f"K_rr of subdomain {k} is singular")
        else:
            self.lu = None
        Kc = self.K_rr.tocsr()
        self.K_II = Kc[self.I][:, self.I]
        self.K_IV = Kc[self.I][:, self.V]
        self.K_VV = Kc[self.V][:, self.V].tocsc()
        self.lu_VV = spla.splu(self.K_VV, permc_spec="MMD_AT_PLUS_A") if len(self.V) else None

    def solve(self, v):
        if self.lu is None:
            return np.zeros_like(v)
        return self.lu.solve(np.asarray(v, dtype=np.float64))

    def schur_I(self, u):
        """S_rIrI u = K_II u - K_IV K_VV^{-1} K_VI u (Eq. DirPrec)."""
        out = self.K_II @ u
        if self.lu_VV is not None:
            out = out - self.K_IV @ self.lu_VV.solve(self.K_IV.T @ u)
        return out


class IetiDP:
    def __init__(self, space, topo, mats, loads):
        self.space, self.topo = space, topo
        prob = space.prob
        n_sub = topo.n_sub
        self.locals = []
        ne = space.n_edges
        for k in range(n_sub):
            pats = np.flatnonzero(prob.patch_to_sub == k)
            Kk = sum(mats[q] for q in pats)
            jk = np.zeros(ne)
            for q in pats:
                g, j = loads[q]
                np.add.at(jk, g, j)
            self.locals.append(LocalProblem(k, Kk, jk, topo.sub_r[k], topo.sub_p[k], topo.sub_I[k],
                                            topo.gp_index, topo.m_r, topo.mult))
        self.m_r = topo.m_r
        self.n_gp = topo.n_gp
        self.scaling = "identity"
        self._coarse()

    def set_scaling(self, kind):
        """Scaling of the preconditioner's jump operator: identity (the
        paper's D_s = I), multiplicity or stiffness (see the module doc)."""
        if kind not in ("identity", "multiplicity", "stiffness"):
            raise ValueError(kind)
        self.scaling = kind
        mult = self.topo.mult
        if kind == "identity":
            dk = dl = np.ones(self.m_r)
        elif kind == "multiplicity":
            dk = dl = np.full(self.m_r, 0.5)
        else:
            rk = np.array([self.locals[k].K_rr.diagonal()[i] for k, i in zip(mult[:, 1], mult[:, 3])])
            rl = np.array([self.locals[l].K_rr.diagonal()[i] for l, i in zip(mult[:, 2], mult[:, 4])])
            dk, dl = rl / (rk + rl), rk / (rk + rl)
        self.delta = (dk, dl)
        for L in self.locals:
            rows_k = mult[:, 1] == L.k
            rows_l = mult[:, 2] == L.k
            bi = np.concatenate([np.flatnonzero(rows_k), np.flatnonzero(rows_l)])
            bj = np.concatenate([mult[rows_k, 3], mult[rows_l, 4]])
            bv = np.concatenate([dk[rows_k], -dl[rows_l]])
            L.BD = sp.csr_matrix((bv, (bi, bj)), shape=(self.m_r, len(L.r)))

    # ---------------------------------------------------------------- setup
    def _coarse(self):
        n_gp, m_r = self.n_gp, self.m_r
        F = np.zeros((n_gp, n_gp))
        G = np.zeros((m_r, n_gp))
        d = np.zeros(n_gp)
        e = np.zeros(m_r)
        for L in self.locals:
            if L.lu is None:
                continue
            KrpC = L.K_rp @ L.C
            X = np.column_stack([L.solve(KrpC[:, c]) for c in range(n_gp)]) if n_gp else np.zeros((len(L.r), 0))
            F += KrpC.T @ X - L.C.T @ L.K_pp @ L.C
            G += L.B @ X
            y = L.solve(L.j_r)
            d += KrpC.T @ y - L.C.T @ L.j_p
            e += L.B @ y
        self.F, self.G, self.d, self.e = F, G, d, e
        if n_gp:
            self.F_lu = sla.lu_factor(F)
            self.rhs = e - G @ sla.lu_solve(self.F_lu, d)  # = -(G F^{-1} d - e)
        else:
            self.F_lu = None
            self.rhs = e.copy()

    def Finv(self, v):
        return sla.lu_solve(self.F_lu, v) if self.F_lu is not None else np.zeros(0)

    # ---------------------------------------------------------------- operators
    def apply_W(self, lam):
        out = np.zeros(self.m_r)
        for L in self.locals:
            out += L.B @ L.solve(L.B.T @ lam)
        return out

    def apply_negS(self, lam):
        """-S lambda = W lambda - G F^{-1} G^T lambda (positive definite)."""
        out = self.apply_W(lam)
        if self.n_gp:
            out -= self.G @ self.Finv(self.G.T @ lam)
        return out

    def apply_MD(self, r):
        """M_D^{-1} r = B_D,rI S_rIrI B_D,rI^T r (B_D = B unless a scaling is set)."""
        out = np.zeros(self.m_r)
        for L in self.locals:
            Bk = L.B if self.scaling == "identity" else L.BD
            u = Bk.T @ r
            v = np.zeros_like(u)
            v[L.I] = L.schur_I(u[L.I])
            out += Bk @ v
        return out

    # ---------------------------------------------------------------- PCG
    def pcg(self, rtol=1e-8, maxit=1000, lam0=None, precondition=True):
        """Preconditioned CG on (-S) lambda = rhs; stops at ||r|| <= rtol ||rhs||."""
        b = self.rhs
        nb = np.linalg.norm(b)
        lam = np.zeros(self.m_r) if lam0 is None else np.array(lam0, dtype=np.float64)
        r = b - self.apply_negS(lam)
        hist = [np.linalg.norm(r)]
        alphas, betas = [], []
        if nb == 0.0 or hist[0] <= rtol * nb:
            return lam, {"iters": 0, "hist": hist, "alpha": alphas, "beta": betas, "converged": True}
        z = self.apply_MD(r) if precondition else r.copy()
        pdir = z.copy()
        rz = r @ z
        it = 0
        converged = False
        while it < maxit:
            q = self.apply_negS(pdir)
            pq = pdir @ q
            if pq <= 0:
                raise RuntimeError("PCG breakdown: p^T F p <= 0")
            alpha = rz / pq
            lam += alpha * pdir
            r -= alpha * q
            it += 1
            alphas.append(alpha)
            hist.append(np.linalg.norm(r))
            if hist[-1] <= rtol * nb:
                converged = True
                break
            z = self.apply_MD(r) if precondition else r.copy()
            rz_new = r @ z
            beta = rz_new / rz
            betas.append(beta)
            rz = rz_new
            pdir = z + beta * pdir
        return lam, {"iters": it, "hist": hist, "alpha": alphas, "beta": betas, "converged": converged}

    # ---------------------------------------------------------------- recovery
    def recover(self, lam):
        """a_p (Eq. coarseProb), a_r (Eq. localProb) and the global vector.

        A DOF shared by several subdomains takes the value of the
        lowest-index subdomain (equal up to the PCG tolerance).
        """
        a = np.zeros(self.space.n_edges)
        ap_glob = self.Finv(self.d - self.G.T @ lam) if self.n_gp else np.zeros(0)
        filled = np.zeros(self.space.n_edges, dtype=bool)
        for L in self.locals:
            a_p = L.C @ ap_glob
            a_r = L.solve(L.j_r - L.K_rp @ a_p - L.B.T @ lam)
            new = ~filled[L.r]
            a[L.r[new]] = a_r[new]
            filled[L.r] = True
        a[self.topo.primal_edges] = ap_glob
        return a

    # ---------------------------------------------------------------- dense (tiny cases)
    def dense_operators(self):
        I = np.eye(self.m_r)
        F = np.column_stack([self.apply_negS(I[:, i]) for i in range(self.m_r)])
        M = np.column_stack([self.apply_MD(I[:, i]) for i in range(self.m_r)])
        return F, M


def lanczos_condition(info):
    """Extreme eigenvalues of M^{-1}F from the PCG coefficients (Lanczos tridiagonal)."""
    a, b = info["alpha"], info["beta"]
    k = len(a)
    if k == 0:
        return 1.0, 1.0
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / a[i] + (b[i - 1] / a[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(b[i]) / a[i]
    ev = np.linalg.eigvalsh(T)
    return float(ev.min()), float(ev.max())
