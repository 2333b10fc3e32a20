"""Multipatch curl-conforming spline space and Galerkin assembly (oracle).

TEST INFRASTRUCTURE ONLY.

Discretisation of the weak form (Section 2, Eqs. weakMS and discrMS):
find a in W with K_g a_g = j_g,
    (K_g)_ij = int_Omega nu (curl w_j) . (curl w_i),
    (j_g)_i  = int_Omega J . w_i.

The space W is the curl-conforming multipatch IGA space.  On patch j the
reference basis functions are tensor products: component c uses the derived
splines D (degree p-1) along direction c and the B-splines N (degree p)
along the other two.  They are pushed forward by the covariant Piola map,
w = DF^{-T} w_hat o F^{-1}, so curl w = (det DF)^{-1} DF curl_hat w_hat.
Patches are glued conformingly: patch-local control points on a shared
patch-facet coincide, so each basis function belongs to one edge of the
global structured control mesh.

Reading of a point the paper leaves open:
* "degree p" is the degree of the H^1 (node) B-splines; curl components
  have degrees (p-1, p, p) and permutations.  p = 1 is the lowest order.
* Global numbering: control node (I,J,K) on an N0 x N1 x N2 grid with
  N_d = P_d (n-1) + 1 (or P_d (n-1) if direction d is periodic), n = n_el+p.
  Edge (d, I, J, K) joins node (I,J,K) to node (I,J,K)+e_d and is oriented
  along +e_d.  Global edge id = off_d + I + E_d0 (J + E_d1 K), where
  E_dc is the number of edge positions of direction-d edges along axis c,
  and off_0 < off_1 < off_2 stack the three directions.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads.problem import patch_coords

from .bspline import bspline_basis, bspline_deriv, dspline_basis, element_quadrature, open_knots
from .geometry import patch_map


class Space:
    def __init__(self, prob):
        self.prob = prob
        self.p = int(prob.degree)
        self.n_el = int(prob.n_el)
        self.n = self.n_el + self.p  # B-splines per patch and direction
        self.P = tuple(prob.patches)
        self.per = tuple(bool(v) for v in prob.periodic)
        self.N = tuple(self.P[d] * (self.n - 1) + (0 if self.per[d] else 1) for d in range(3))
        self.ext = []
        for d in range(3):
            self.ext.append(tuple(
                (self.N[c] - 1 if (c == d and not self.per[c]) else self.N[c]) for c in range(3)))
        counts = [int(np.prod(e)) for e in self.ext]
        self.off = (0, counts[0], counts[0] + counts[1])
        self.n_edges = int(sum(counts))
        self.n_nodes = int(np.prod(self.N))
        self._build_edge_arrays()
        self.knots = open_knots(self.p, self.n_el)
        self.nq = self.p + 1

    # ------------------------------------------------------------------ numbering
    def edge_id(self, d, I, J, K):
        e = self.ext[d]
        return self.off[d] + I + e[0] * (J + e[1] * K)

    def node_id(self, I, J, K):
        return I + self.N[0] * (J + self.N[1] * K)

    def _build_edge_arrays(self):
        dirs, co = [], []
        for d in range(3):
            e = self.ext[d]
            K, J, I = np.meshgrid(np.arange(e[2]), np.arange(e[1]), np.arange(e[0]), indexing="ij")
            c = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
            co.append(c)
            dirs.append(np.full(c.shape[0], d))
        self.edge_dir = np.concatenate(dirs)
        self.edge_coord = np.concatenate(co)  # (n_edges, 3)
        start = self.edge_coord.copy()
        end = self.edge_coord.copy()
        end[np.arange(self.n_edges), self.edge_dir] += 1
        for d in range(3):
            if self.per[d]:
                end[:, d] %= self.N[d]
        self.edge_nodes = np.stack([self.node_id(*start.T), self.node_id(*end.T)], axis=1)
        dirichlet = np.zeros(self.n_edges, dtype=bool)
        for c in range(3):
            if self.per[c]:
                continue
            transverse = self.edge_dir != c
            X = self.edge_coord[:, c]
            dirichlet |= transverse & ((X == 0) | (X == self.N[c] - 1))
        self.dirichlet = dirichlet
        nodes = np.stack(np.meshgrid(np.arange(self.N[0]), np.arange(self.N[1]), np.arange(self.N[2]), indexing="ij"), -1)
        nodes = nodes.reshape(-1, 3)
        bnode = np.zeros(nodes.shape[0], dtype=bool)
        for c in range(3):
            if not self.per[c]:
                bnode |= (nodes[:, c] == 0) | (nodes[:, c] == self.N[c] - 1)
        self.node_boundary = np.zeros(self.n_nodes, dtype=bool)
        self.node_boundary[self.node_id(*nodes.T)] = bnode

    def gradient_matrix(self):
        """Signed node-to-edge incidence G (n_edges x n_nodes): -1 at the start, +1 at the end."""
        rows = np.repeat(np.arange(self.n_edges), 2)
        cols = self.edge_nodes.ravel()
        vals = np.tile([-1, 1], self.n_edges)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.n_edges, self.n_nodes))

    def curl_incidence(self):
        """Signed edge-to-face incidence C (n_faces x n_edges) of the control mesh.

        A face with normal a and lower corner (I,J,K) is bounded by the edges
        along b and c = the other two axes (b < c cyclic order a->b->c):
        +edge_b(lo) + edge_c(lo+e_b) - edge_b(lo+e_c) - edge_c(lo).
        """
        rows, cols, vals = [], [], []
        fid = 0
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            ranges = []
            for t in range(3):
                if t == a:
                    ranges.append(np.arange(self.N[t]))
                else:
                    ranges.append(np.arange(self.ext[t][t]))
            grid = np.stack(np.meshgrid(*ranges, indexing="ij"), -1).reshape(-1, 3)
            nf = grid.shape[0]
            ids = np.arange(fid, fid + nf)
            fid += nf

            def eid(d, co):
                co = co.copy()
                for t in range(3):
                    if self.per[t]:
                        co[:, t] %= self.N[t]
                return self.edge_id(d, co[:, 0], co[:, 1], co[:, 2])

            eb = np.zeros(3, dtype=int)
            eb[b] = 1
            ec = np.zeros(3, dtype=int)
            ec[c] = 1
            for d, shift, s in ((b, 0 * eb, 1), (c, eb, 1), (b, ec, -1), (c, 0 * ec, -1)):
                rows.append(ids)
                cols.append(eid(d, grid + shift[None, :]))
                vals.append(np.full(nf, s))
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        vals = np.concatenate(vals)
        return sp.csr_matrix((vals, (rows, cols)), shape=(fid, self.n_edges))

    # ------------------------------------------------------------------ patches
    def patch_local_edges(self, pidx):
        """Global edge ids of patch-local functions, component-major, i fastest."""
        pc = patch_coords(pidx, self.P)
        n = self.n
        out = []
        for d in range(3):
            le = [n - 1 if c == d else n for c in range(3)]
            K, J, I = np.meshgrid(np.arange(le[2]), np.arange(le[1]), np.arange(le[0]), indexing="ij")
            co = [I.ravel() + pc[0] * (n - 1), J.ravel() + pc[1] * (n - 1), K.ravel() + pc[2] * (n - 1)]
            for c in range(3):
                if self.per[c]:
                    co[c] = co[c] % self.N[c]
            out.append(self.edge_id(d, *co))
        return np.concatenate(out)

    def _tables(self):
        xq, wq, el = element_quadrature(self.p, self.n_el, self.nq)
        N = bspline_basis(self.knots, self.p, xq)
        dN = bspline_deriv(self.knots, self.p, xq)
        D = dspline_basis(self.knots, self.p, xq)
        return xq, wq, N, dN, D

    def element_data(self, pidx):
        """Per-element reference data of one patch.

        Returns dict with
          xi   (E, Q, 3)  reference quadrature points
          w    (E, Q)     reference weights
          val  (E, Q, 3, nf) reference basis values w_hat (vector)
          curl (E, Q, 3, nf) reference curls curl_hat w_hat
          loc  (E, nf)    patch-local function indices (component-major)
        """
        p, n, ne, nq = self.p, self.n, self.n_el, self.nq
        xq, wq, N, dN, D = self._tables()
        Nr = N.reshape(ne, nq, n)
        dNr = dN.reshape(ne, nq, n)
        Dr = D.reshape(ne, nq, n - 1)
        e_idx = np.arange(ne)
        # active functions on element e: N -> e..e+p, D -> e..e+p-1
        aN = e_idx[:, None] + np.arange(p + 1)[None, :]
        aD = e_idx[:, None] + np.arange(p)[None, :]
        Na = np.take_along_axis(Nr, aN[:, None, :], axis=2)  # (ne, nq, p+1)
        dNa = np.take_along_axis(dNr, aN[:, None, :], axis=2)
        Da = np.take_along_axis(Dr, aD[:, None, :], axis=2)  # (ne, nq, p)
        E = ne ** 3
        Q = nq ** 3
        ee = np.stack(np.meshgrid(e_idx, e_idx, e_idx, indexing="ij"), -1).reshape(E, 3)  # (e0,e1,e2)
        qq = np.stack(np.meshgrid(np.arange(nq), np.arange(nq), np.arange(nq), indexing="ij"), -1).reshape(Q, 3)
        xr = xq.reshape(ne, nq)
        xi = np.stack([xr[ee[:, None, 0], qq[None, :, 0]], xr[ee[:, None, 1], qq[None, :, 1]], xr[ee[:, None, 2], qq[None, :, 2]]], -1)
        wr = wq.reshape(ne, nq)
        w = wr[ee[:, None, 0], qq[None, :, 0]] * wr[ee[:, None, 1], qq[None, :, 1]] * wr[ee[:, None, 2], qq[None, :, 2]]

        def tab(T, a):
            # T (ne, nq, m) -> (E, Q, m) for direction a
            return T[ee[:, None, a], qq[None, :, a], :]

        vals, curls, locs = [], [], []
        for c in range(3):
            f = [tab(Da if a == c else Na, a) for a in range(3)]
            g = [tab(Da if a == c else dNa, a) for a in range(3)]  # derivative tables (D never differentiated)
            m = [f[a].shape[2] for a in range(3)]
            # scalar w_hat_c = f0[i] f1[j] f2[k], index (i fastest) -> flat i + m0 (j + m1 k)
            def outer(a0, a1, a2):
                return (a2[:, :, :, None, None] * a1[:, :, None, :, None] * a0[:, :, None, None, :]).reshape(E, Q, -1)
            s = outer(f[0], f[1], f[2])
            v = np.zeros((E, Q, 3, s.shape[2]))
            v[:, :, c, :] = s
            cu = np.zeros_like(v)
            if c == 0:
                cu[:, :, 1, :] = outer(f[0], f[1], g[2])
                cu[:, :, 2, :] = -outer(f[0], g[1], f[2])
            elif c == 1:
                cu[:, :, 0, :] = -outer(f[0], f[1], g[2])
                cu[:, :, 2, :] = outer(g[0], f[1], f[2])
            else:
                cu[:, :, 0, :] = outer(f[0], g[1], f[2])
                cu[:, :, 1, :] = -outer(g[0], f[1], f[2])
            vals.append(v)
            curls.append(cu)
            # patch-local index of each active function
            le = [n - 1 if a == c else n for a in range(3)]
            base = sum(int(np.prod([n - 1 if a == cc else n for a in range(3)])) for cc in range(c))
            act = [aD[ee[:, a]] if a == c else aN[ee[:, a]] for a in range(3)]  # (E, m_a)
            li = (act[0][:, None, None, :] + le[0] * (act[1][:, None, :, None] + le[1] * act[2][:, :, None, None]))
            locs.append(base + li.reshape(E, -1))
        return {
            "xi": xi,
            "w": w,
            "val": np.concatenate(vals, axis=3),
            "curl": np.concatenate(curls, axis=3),
            "loc": np.concatenate(locs, axis=1),
        }

    def n_local(self):
        n = self.n
        return 3 * (n - 1) * n * n

    def physical(self, pidx, ed):
        """Push reference data forward: physical points, |det DF| w, curl w, w."""
        E, Q = ed["w"].shape
        x, DF = patch_map(self.prob, pidx, ed["xi"].reshape(-1, 3))
        det = np.linalg.det(DF)
        x = x.reshape(E, Q, 3)
        DF = DF.reshape(E, Q, 3, 3)
        det = det.reshape(E, Q)
        curl = np.einsum("eqab,eqbf->eqaf", DF, ed["curl"]) / det[:, :, None, None]
        DFinvT = np.linalg.inv(DF).transpose(0, 1, 3, 2)
        val = np.einsum("eqab,eqbf->eqaf", DFinvT, ed["val"])
        return x, np.abs(det) * ed["w"], curl, val

    def assemble_patch(self, pidx, with_load=True, ed=None):
        """Patch stiffness (nu = 1) and load, in patch-local numbering.

        Returns (K_loc dense (nloc, nloc), j_loc (nloc,)).
        """
        if ed is None:
            ed = self.element_data(pidx)
        x, wdet, curl, val = self.physical(pidx, ed)
        E, Q = wdet.shape
        nf = curl.shape[3]
        Cw = (curl * np.sqrt(wdet)[:, :, None, None]).reshape(E, Q * 3, nf)
        Ke = np.matmul(Cw.transpose(0, 2, 1), Cw)  # (E, nf, nf)
        nloc = self.n_local()
        loc = ed["loc"]
        flat = (loc[:, :, None] * nloc + loc[:, None, :]).ravel()
        K = np.bincount(flat, weights=Ke.ravel(), minlength=nloc * nloc).reshape(nloc, nloc)
        j = None
        if with_load:
            Jv = self.prob.source(x.reshape(-1, 3)).reshape(E, Q, 3)
            je = np.einsum("eqa,eqaf,eq->ef", Jv, val, wdet)
            j = np.bincount(loc.ravel(), weights=je.ravel(), minlength=nloc)
        return K, j

    def assemble(self, with_load=True):
        """Per-patch stiffness and loads in global edge ids.

        Returns (list of sparse patch matrices with nu applied (global ids),
                 list of patch loads as (global ids, values)).
        The global system of Eq. discrMS is the sum over patches.
        """
        mats, loads = [], []
        ed = self.element_data(0)  # reference data is identical for every patch
        for pidx in range(int(np.prod(self.P))):
            K, j = self.assemble_patch(pidx, with_load, ed=ed)
            g = self.patch_local_edges(pidx)
            r, c = np.nonzero(K)
            nu = self.prob.nu[pidx]
            mats.append(sp.csr_matrix((nu * K[r, c], (g[r], g[c])), shape=(self.n_edges, self.n_edges)))
            loads.append((g, j if with_load else np.zeros(g.size)))
        return mats, loads

    def dirichlet_values(self):
        """Boundary DOFs of n x A = n x A_D: the L2 projection of the
        tangential trace of A_D onto the tangential traces of the boundary
        basis functions, over every patch face on the boundary of the
        domain.  Only functions of the two tangential components whose index
        across the face is the first (or last) one have a tangential trace
        there (open knot vectors); the normal component's push-forward is
        normal to the face.  Returns (edge ids, values)."""
        A_D = self.prob.dirichlet_A
        p, n = self.p, self.n
        xq, wq, N, dN, D = self._tables()
        M = len(xq)
        rows, cols, vals = [], [], []
        rhs = np.zeros(self.n_edges)
        P = self.P
        for pidx in range(int(np.prod(P))):
            pc = (pidx % P[0], (pidx // P[0]) % P[1], pidx // (P[0] * P[1]))
            g = self.patch_local_edges(pidx)
            for d in range(3):
                if self.per[d]:
                    continue
                for side in (0, 1):
                    if pc[d] != (0 if side == 0 else P[d] - 1):
                        continue
                    a, b = [x for x in range(3) if x != d]
                    # face quadrature grid: xi_a fastest
                    ia, ib = np.meshgrid(np.arange(M), np.arange(M), indexing="xy")
                    ia, ib = ia.ravel(), ib.ravel()
                    xi = np.zeros((ia.size, 3))
                    xi[:, a], xi[:, b], xi[:, d] = xq[ia], xq[ib], float(side)
                    W = wq[ia] * wq[ib]
                    x, DF = patch_map(self.prob, pidx, xi)
                    DFinvT = np.linalg.inv(DF).transpose(0, 2, 1)
                    det = np.abs(np.linalg.det(DF))
                    nvec = DFinvT[:, :, d]
                    nn = np.linalg.norm(nvec, axis=1)
                    nhat = nvec / nn[:, None]
                    dS = W * det * nn
                    fun_vals, fun_ids = [], []
                    for c in (a, b):
                        le = [n - 1 if q == c else n for q in range(3)]
                        base = sum(int(np.prod([n - 1 if q == cc else n for q in range(3)])) for cc in range(c))
                        ta = D if a == c else N       # (M, le[a])
                        tb = D if b == c else N
                        s_ab = (tb[ib][:, :, None] * ta[ia][:, None, :]).reshape(ia.size, -1)  # index i_a fastest
                        ii_a, ii_b = np.meshgrid(np.arange(le[a]), np.arange(le[b]), indexing="xy")
                        ii_a, ii_b = ii_a.ravel(), ii_b.ravel()
                        idx = [None, None, None]
                        idx[a], idx[b], idx[d] = ii_a, ii_b, np.full(ii_a.size, 0 if side == 0 else le[d] - 1)
                        loc = base + idx[0] + le[0] * (idx[1] + le[1] * idx[2])
                        w = DFinvT[:, :, c][:, :, None] * s_ab[:, None, :]          # (Q, 3, nf)
                        wt = w - np.einsum("qa,qaf->qf", nhat, w)[:, None, :] * nhat[:, :, None]
                        fun_vals.append(wt)
                        fun_ids.append(g[loc])
                    wt = np.concatenate(fun_vals, axis=2)
                    ids = np.concatenate(fun_ids)
                    Mf = np.einsum("qaf,qag,q->fg", wt, wt, dS)
                    bf = np.einsum("qa,qaf,q->f", A_D(x), wt, dS)
                    r, cc = np.meshgrid(ids, ids, indexing="ij")
                    rows.append(r.ravel())
                    cols.append(cc.ravel())
                    vals.append(Mf.ravel())
                    np.add.at(rhs, ids, bf)
        rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
        ids = np.unique(rows)
        if not np.all(self.dirichlet[ids]):
            raise RuntimeError("a boundary function is not a Dirichlet DOF")
        pos = np.full(self.n_edges, -1)
        pos[ids] = np.arange(ids.size)
        Mg = sp.csr_matrix((vals, (pos[rows], pos[cols])), shape=(ids.size, ids.size)).tocsc()
        return ids, spla.spsolve(Mg, rhs[ids])

    def lift_loads(self, mats, loads, d_ids, d_vals):
        """Loads minus the coupling to the prescribed Dirichlet coefficients:
        j - K a_D per patch (the Dirichlet rows themselves are never used)."""
        aD = np.zeros(self.n_edges)
        aD[d_ids] = d_vals
        return [(g, j - (K @ aD)[g]) for K, (g, j) in zip(mats, loads)]

    def global_load(self, loads):
        jg = np.zeros(self.n_edges)
        for g, j in loads:
            np.add.at(jg, g, j)
        return jg
