"""Learned warm start for the annulus (ring) workload.

One network row per interface facet.  Facet f is the plane of control nodes
at azimuthal node index f (n_el + p - 1), between sector f-1 (below) and
sector f (above).  The row's features are the log reluctivities of the
patches of the 2w sectors around the facet.  Its coefficients are the coil
currents of the axial rings: the multipliers are linear in the source, and
the network's output groups carry the response to each ring.  The outputs
are the facet's multipliers in increasing edge id, signed so that +1 means
the lower sector.  Every facet of the ring has the same multiplier pattern
(checked here), so one set of weights serves all facets.

The library does the data generation (assembly with new coefficients,
factorisation, solve, and the network rows: log-reluctivity features,
coefficients, signed multiplier targets), the normalisation of the rows,
the seeded initial weights, the training (forward, backward and Adam
kernels) and the inference inside ``ieti_solve``.  This module only builds
the layout (which patches feed a facet's row, which multiplier rows it
predicts) from the problem's numbering and marshals arrays.
"""
from __future__ import annotations

import time

import numpy as np

from .ietidp import NN, train_file


def decode_edges(edge_ids, patches, periodic, degree, n_el):
    """(direction, I, J, K) of global edge ids under the library's numbering."""
    n = n_el + degree
    N = [patches[d] * (n - 1) + (0 if periodic[d] else 1) for d in range(3)]
    E = []
    for d in range(3):
        e = list(N)
        if not periodic[d]:
            e[d] -= 1
        E.append(e)
    off = np.cumsum([0] + [e[0] * e[1] * e[2] for e in E])
    edge_ids = np.asarray(edge_ids, dtype=np.int64)
    d = np.searchsorted(off, edge_ids, side="right") - 1
    loc = edge_ids - off[d]
    e0 = np.array([E[x][0] for x in range(3)])[d]
    e1 = np.array([E[x][1] for x in range(3)])[d]
    return d, loc % e0, (loc // e0) % e1, loc // (e0 * e1)


class RingWarmStart:
    """Layout, solver-generated data, training and attachment for a ring."""

    def __init__(self, solver, prob, window=2, hidden=256, layers=2):
        P = prob.patches
        if not (prob.periodic[0] and prob.geom_kind == 1):
            raise ValueError("the ring layout needs the periodic annulus")
        self.solver, self.prob, self.window = solver, prob, int(window)
        self.P0, self.P1, self.P2 = P
        self.hidden, self.layers = int(hidden), int(layers)
        part = np.asarray(prob.patch_to_sub)
        if not np.array_equal(part, np.arange(int(np.prod(P))) % P[0]):
            raise ValueError("the ring layout needs one subdomain per azimuthal sector")
        mult = solver.maps()["mult"]
        d, I, J, K = decode_edges(mult[:, 0], P, prob.periodic, prob.degree, prob.n_el)
        step = prob.n_el + prob.degree - 1
        if np.any(I % step):
            raise ValueError("a multiplier lies off the sector planes")
        facet = I // step
        keys = None
        self.out_row = np.full((self.P0, 0), -1, np.int32)
        rows, signs = [], []
        for f in range(self.P0):
            sel = np.flatnonzero(facet == f)
            order = np.lexsort((K[sel], J[sel], d[sel]))
            sel = sel[order]
            kf = list(zip(d[sel], J[sel], K[sel]))
            if keys is None:
                keys = kf
            elif kf != keys:
                raise ValueError("facets differ in their multiplier pattern")
            lower = (f - 1) % self.P0
            k = mult[sel, 1]
            if not np.all((k == lower) | (k == f)):
                raise ValueError("multiplier rows of a facet must join its two sectors")
            rows.append(sel)
            signs.append(np.where(k == lower, 1, -1))
        self.out_row = np.array(rows, dtype=np.int32)
        self.out_sign = np.array(signs, dtype=np.int8)
        self.n_out = self.out_row.shape[1]
        # features: patches of sectors f-w .. f+w-1, in (sector, radial, axial) order
        w = self.window
        fp = []
        for f in range(self.P0):
            idx = []
            for s in range(f - w, f + w):
                for j in range(self.P1):
                    for kk in range(self.P2):
                        idx.append((s % self.P0) + self.P0 * (j + self.P1 * kk))
            fp.append(idx)
        self.feat_patch = np.array(fp, dtype=np.int32)
        self.n_feat = self.feat_patch.shape[1]
        # coefficients: the coil patch of each axial ring in the facet's upper sector
        coil = self.P1 - 1
        self.comb_patch = np.array([[f + self.P0 * (coil + self.P1 * kk) for kk in range(self.P2)]
                                    for f in range(self.P0)], dtype=np.int32)
        self.n_comb = self.P2
        self.net = None

    def layout(self):
        return self.feat_patch, self.comb_patch, self.out_row, self.out_sign

    # ---- data from the solver itself
    def generate(self, draws, rtol=1e-10, log=None, dataset=None):
        """Solve every (nu, load_scale) draw; returns the network rows
        (features, coefficients, targets) built by the library from each
        solve, and the solve statistics.  With ``dataset`` the rows are also
        appended to that dataset file."""
        X, Cc, T, stats = [], [], [], []
        t0 = time.perf_counter()
        for i, (nu, scale) in enumerate(draws):
            self.solver.set_coefficients(nu, scale)
            self.solver.factor()
            _, st = self.solver.solve(rtol=rtol, maxit=5000)
            x, c, y = self.solver.warm_rows(*self.layout())
            if dataset is not None:
                self.solver.warm_append(dataset, *self.layout())
            X.append(x)
            Cc.append(c)
            T.append(y)
            stats.append(st)
            if log and (i + 1) % 32 == 0:
                log(f"generated {i + 1}/{len(draws)} solves ({time.perf_counter() - t0:.1f}s)")
        return np.array(X), np.array(Cc), np.array(T), stats

    # ---- training
    def arch(self):
        return (self.n_feat, self.hidden, self.layers, self.n_comb, self.n_out)

    def fit(self, X, Cc, T, epochs=200, lr=1e-3, batch=256, seed=0):
        """Seeded initial weights, normalisation fitted to the rows, Adam on
        the GPU (all in the library); returns the epoch losses."""
        Xf = np.asarray(X, dtype=np.float32).reshape(-1, self.n_feat)
        Cf = np.asarray(Cc, dtype=np.float32).reshape(-1, self.n_comb)
        Tf = np.asarray(T, dtype=np.float32).reshape(-1, self.n_out)
        self.net = NN(*self.arch())
        self.net.init_params(seed)
        self.net.fit_normalisation(Xf, Tf)
        self.net.set_data(Xf, Cf, Tf)
        return self.net.train(epochs, lr, batch=batch, seed=seed)

    def fit_file(self, dataset, model_out, epochs=200, lr=1e-3, batch=256, seed=0):
        """The same training from a dataset file written by ``generate``;
        the trained network is written to ``model_out`` and loaded."""
        losses = train_file(dataset, self.arch(), model_out, epochs, lr, batch=batch, seed=seed)
        self.net = NN.load(model_out)
        return losses

    # ---- persistence
    def save(self, prefix):
        """The trained network with its normalisation (``prefix + '.net'``,
        the library's file) and the layout parameters (``prefix + '.npz'``);
        the facet layout itself follows from the problem and is rebuilt on
        load."""
        self.net.save(str(prefix) + ".net")
        np.savez(str(prefix) + ".npz", window=self.window, hidden=self.hidden, layers=self.layers)

    @classmethod
    def load(cls, solver, prob, prefix):
        """A warm start saved by ``save`` for the same ring layout."""
        z = np.load(str(prefix) + ".npz", allow_pickle=False)
        self = cls(solver, prob, window=int(z["window"]), hidden=int(z["hidden"]), layers=int(z["layers"]))
        net = NN.load(str(prefix) + ".net")
        if net.arch != self.arch():
            raise ValueError("the saved network does not fit this problem's layout")
        self.net = net
        return self

    def attach(self, solver=None):
        (solver or self.solver).set_warm_start(self.net, *self.layout())

    def predict_lambda(self, solver=None):
        """The multipliers the attached network predicts for the solver's
        current coefficients (host copy, ``ieti_warm_predict``), for tests."""
        return (solver or self.solver).warm_predict()
