"""Source current densities J (and manufactured exact fields) for workloads.

All fields are vectorised callables ``f(xyz: (n,3)) -> (n,3)``.  They are
inputs to the solver, written out by hand from the stated formulas; they are
not part of the solver's arithmetic.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Manufactured polynomial field that lies in the degree-2 curl-conforming
# spline space on the unit cube and has zero tangential trace:
#   A = (f(y) f(z) (1+2x), f(x) f(z) (2-y), f(x) f(y) (1+z)),  f(t) = t(1-t).
# With nu = 1:  J = curl curl A = grad div A - Laplace A  (expanded by hand).
# ---------------------------------------------------------------------------
def _f(t):
    return t * (1.0 - t)


def _df(t):
    return 1.0 - 2.0 * t


def poly_A(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return np.stack([_f(y) * _f(z) * (1 + 2 * x), _f(x) * _f(z) * (2 - y), _f(x) * _f(y) * (1 + z)], axis=1)


def poly_B(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    bx = _f(x) * _df(y) * (1 + z) - _f(x) * (2 - y) * _df(z)
    by = (1 + 2 * x) * _f(y) * _df(z) - _df(x) * _f(y) * (1 + z)
    bz = _df(x) * (2 - y) * _f(z) - (1 + 2 * x) * _df(y) * _f(z)
    return np.stack([bx, by, bz], axis=1)


def poly_J(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    fx, fy, fz = _f(x), _f(y), _f(z)
    jx = _df(x) * (fy - fz) + 2 * (1 + 2 * x) * (fy + fz)
    jy = _df(y) * (2 * fz + fx) + 2 * (2 - y) * (fx + fz)
    jz = _df(z) * (2 * fy - fx) + 2 * (1 + z) * (fx + fy)
    return np.stack([jx, jy, jz], axis=1)


# ---------------------------------------------------------------------------
# Smooth zero-trace field on the unit cube (not in any spline space):
#   A = (sin(pi y) sin(pi z), sin(pi x) sin(pi z), sin(pi x) sin(pi y)),
# div A = 0, so J = curl curl A = 2 pi^2 A (nu = 1).
# ---------------------------------------------------------------------------
def sine_A(xyz):
    s = np.sin(np.pi * xyz)
    return np.stack([s[:, 1] * s[:, 2], s[:, 0] * s[:, 2], s[:, 0] * s[:, 1]], axis=1)


def sine_B(xyz):
    s = np.sin(np.pi * xyz)
    c = np.cos(np.pi * xyz)
    pi = np.pi
    bx = pi * s[:, 0] * c[:, 1] - pi * s[:, 0] * c[:, 2]
    by = pi * s[:, 1] * c[:, 2] - pi * c[:, 0] * s[:, 1]
    bz = pi * c[:, 0] * s[:, 2] - pi * c[:, 1] * s[:, 2]
    return np.stack([bx, by, bz], axis=1)


def sine_J(xyz):
    return 2.0 * np.pi ** 2 * sine_A(xyz)


# ---------------------------------------------------------------------------
# Random smooth divergence-free source: J = curl T with
#   T_d(x) = sum_{k in {1..m}^3} a_{d,k} prod_i sin(pi k_i x_i + th_{d,k,i}),
#   a ~ N(0,1)/|k|^2, th ~ U(0, 2 pi).
# ---------------------------------------------------------------------------
class TrigCurlSource:
    def __init__(self, seed, modes=4):
        rng = np.random.default_rng(seed)
        ks = np.array(list(np.ndindex(modes, modes, modes)), dtype=np.float64) + 1.0  # (M,3)
        self.k = ks
        self.amp = rng.standard_normal((3, ks.shape[0])) / np.sum(ks * ks, axis=1)[None, :]
        self.phase = rng.uniform(0.0, 2.0 * np.pi, size=(3, ks.shape[0], 3))

    def T_and_grad(self, xyz):
        """T_d and dT_d/dx_j at points: returns (n,3), (n,3,3) [d, j].

        sin(pi k x + th) and cos(pi k x + th) are formed from the per-axis
        tables sin(pi k x), cos(pi k x) by the angle-addition identities.
        """
        n = xyz.shape[0]
        T = np.zeros((n, 3))
        dT = np.zeros((n, 3, 3))
        pk = np.pi * self.k  # (M,3)
        ki = self.k.astype(np.int64) - 1  # (M,3) table index
        kmax = int(self.k.max())
        ang = np.pi * xyz[:, :, None] * np.arange(1, kmax + 1)[None, None, :]  # (n,3,K)
        st, ct = np.sin(ang), np.cos(ang)
        s_ax = [st[:, i, :][:, ki[:, i]] for i in range(3)]  # (n,M)
        c_ax = [ct[:, i, :][:, ki[:, i]] for i in range(3)]
        for d in range(3):
            cth = np.cos(self.phase[d])  # (M,3)
            sth = np.sin(self.phase[d])
            S = [s_ax[i] * cth[None, :, i] + c_ax[i] * sth[None, :, i] for i in range(3)]
            Cc = [c_ax[i] * cth[None, :, i] - s_ax[i] * sth[None, :, i] for i in range(3)]
            a = self.amp[d][None, :]
            T[:, d] = np.sum(a * S[0] * S[1] * S[2], axis=1)
            dT[:, d, 0] = np.sum(a * pk[None, :, 0] * Cc[0] * S[1] * S[2], axis=1)
            dT[:, d, 1] = np.sum(a * pk[None, :, 1] * S[0] * Cc[1] * S[2], axis=1)
            dT[:, d, 2] = np.sum(a * pk[None, :, 2] * S[0] * S[1] * Cc[2], axis=1)
        return T, dT

    def curl_numpy(self, xyz):
        xyz = np.asarray(xyz, dtype=np.float64)
        out = np.empty((xyz.shape[0], 3))
        step = 20000
        for s in range(0, xyz.shape[0], step):
            _, dT = self.T_and_grad(xyz[s:s + step])
            out[s:s + step, 0] = dT[:, 2, 1] - dT[:, 1, 2]
            out[s:s + step, 1] = dT[:, 0, 2] - dT[:, 2, 0]
            out[s:s + step, 2] = dT[:, 1, 0] - dT[:, 0, 1]
        return out

    def _derivative_tensors(self):
        """W[p] (2K x 2K x 2K) for the six derivatives dT_d/dx_j, d != j, in
        the order of PAIRS: by angle addition every factor
        sin(pi k_i x_i + th) is cos(th) sin(pi k_i x_i) + sin(th) cos(pi k_i x_i),
        and its x_i-derivative pi k_i (cos(th) cos(pi k_i x_i) - sin(th) sin(pi k_i x_i)),
        so each derivative is a trilinear form in the per-axis vectors
        g_i = [sin(pi k x_i), cos(pi k x_i)]_{k=1..K}."""
        if getattr(self, "_W", None) is not None:
            return self._W
        K = int(self.k.max())
        W = np.zeros((len(self.PAIRS), 2 * K, 2 * K, 2 * K))
        for q, (d, j) in enumerate(self.PAIRS):
            for m in range(self.k.shape[0]):
                e = []
                for i in range(3):
                    v = np.zeros(2 * K)
                    ki = int(self.k[m, i]) - 1
                    ct, st = np.cos(self.phase[d, m, i]), np.sin(self.phase[d, m, i])
                    if i == j:
                        f = np.pi * self.k[m, i]
                        v[ki], v[K + ki] = -f * st, f * ct
                    else:
                        v[ki], v[K + ki] = ct, st
                    e.append(v)
                W[q] += self.amp[d, m] * np.einsum("a,b,c->abc", e[0], e[1], e[2])
        self._W = W
        return W

    # (d, j) of dT_d/dx_j needed by curl T
    PAIRS = ((2, 1), (1, 2), (0, 2), (2, 0), (1, 0), (0, 1))

    def __call__(self, xyz):
        xyz = np.asarray(xyz, dtype=np.float64)
        W = self._derivative_tensors()
        P, K2 = W.shape[0], W.shape[1]
        K = K2 // 2
        Wf = W.reshape(P * K2 * K2, K2)                    # [(q, a, b), c]
        kr = np.arange(1, K + 1, dtype=np.float64)
        out = np.empty((xyz.shape[0], 3))
        step = 32768
        for s in range(0, xyz.shape[0], step):
            x = xyz[s:s + step]
            n = x.shape[0]
            ang = np.pi * x[:, :, None] * kr[None, None, :]   # (n,3,K)
            g = np.concatenate([np.sin(ang), np.cos(ang)], axis=2)  # (n,3,2K)
            Y = g[:, 2, :] @ Wf.T                              # (n, P*2K*2K): contract axis 2
            Y = np.matmul(Y.reshape(n, P * K2, K2), g[:, 1, :, None])[..., 0]   # axis 1
            D = np.matmul(Y.reshape(n, P, K2), g[:, 0, :, None])[..., 0]       # axis 0 -> (n, P)
            out[s:s + step, 0] = D[:, 0] - D[:, 1]
            out[s:s + step, 1] = D[:, 2] - D[:, 3]
            out[s:s + step, 2] = D[:, 4] - D[:, 5]
        return out


# ---------------------------------------------------------------------------
# Azimuthal coil current for the annulus workload: J = c(z) e_theta inside
# r in [r_in, r_out], zero elsewhere; c(z) is piecewise constant per axial
# ring of patches.
# ---------------------------------------------------------------------------
class CoilSource:
    def __init__(self, r_in, r_out, z_edges, ring_current):
        self.r_in = float(r_in)
        self.r_out = float(r_out)
        self.z_edges = np.asarray(z_edges, dtype=np.float64)
        self.ring_current = np.asarray(ring_current, dtype=np.float64)

    def __call__(self, xyz):
        xyz = np.asarray(xyz, dtype=np.float64)
        r = np.hypot(xyz[:, 0], xyz[:, 1])
        ring = np.clip(np.searchsorted(self.z_edges, xyz[:, 2], side="right") - 1, 0, len(self.ring_current) - 1)
        c = self.ring_current[ring] * ((r > self.r_in) & (r < self.r_out))
        out = np.zeros_like(xyz)
        rs = np.where(r > 0, r, 1.0)
        out[:, 0] = -c * xyz[:, 1] / rs
        out[:, 1] = c * xyz[:, 0] / rs
        return out


# ---------------------------------------------------------------------------
# Closed-form solution of the paper's numerical experiments on (0,3)^3
# (Section 4), nu = 1: A is divergence free, so J = curl curl A = -Laplace A
# = 3 A; B = curl A.
# ---------------------------------------------------------------------------
def paper_A(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return np.stack([np.cos(y) * np.cos(z) * np.sin(x), -2.0 * np.cos(x) * np.cos(z) * np.sin(y),
                     np.cos(x) * np.cos(y) * np.sin(z)], axis=1)


def paper_B(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return np.stack([-3.0 * np.cos(x) * np.sin(y) * np.sin(z), np.zeros_like(x),
                     3.0 * np.cos(z) * np.sin(x) * np.sin(y)], axis=1)


def paper_J(xyz):
    return 3.0 * paper_A(xyz)


# ---------------------------------------------------------------------------
# A field of the degree-2 curl-conforming spline space with a non-zero
# tangential trace: A = (y^2 z, x z^2, x^2 y) (each component has degree <= 1
# along its own direction and <= 2 along the others), div A = 0, so with
# nu = 1: J = -Laplace A = -2 (z, x, y), B = curl A.
# ---------------------------------------------------------------------------
def trace_A(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return np.stack([y * y * z, x * z * z, x * x * y], axis=1)


def trace_B(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return np.stack([x * x - 2 * x * z, y * y - 2 * x * y, z * z - 2 * y * z], axis=1)


def trace_J(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return -2.0 * np.stack([z, x, y], axis=1)
