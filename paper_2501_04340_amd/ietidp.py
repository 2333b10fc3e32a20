"""Thin ctypes binding of the C ABI in ``include/ietidp.h``.

Argument marshalling only: every step of assembly, factorisation and solve
runs inside ``lib/libietidp.so``.  Loading fails loudly if the library has not
been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libietidp.so")
_lib = None

ABI_VERSION = 2
GEMV_SHAPES = 13   # interface GEMV launch shapes: 0..11 row streaming, 12 symmetric (lower tiles)
GEMV_SYM = 12
PREC_FP64, PREC_MIXED = 0, 1
SCALE_IDENTITY, SCALE_STIFFNESS, SCALE_MULTIPLICITY = 0, 1, 2
ERRORS = {
    -1: "INVALID_ARG", -2: "PARTITION", -3: "TREE", -4: "NOT_SPD", -5: "BREAKDOWN",
    -6: "NOT_CONVERGED", -7: "HIP", -8: "STATE",
}

FIELD_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_double), C.c_void_p)


class Problem(C.Structure):
    _fields_ = [
        ("version", C.c_int32),
        ("geom_kind", C.c_int32),
        ("patches", C.c_int32 * 3),
        ("periodic", C.c_int32 * 3),
        ("geom_params", C.c_double * 16),
        ("degree_p", C.c_int32),
        ("n_el", C.c_int32),
        ("patch_to_subdomain", C.POINTER(C.c_int32)),
        ("nu_per_patch", C.POINTER(C.c_double)),
        ("J", FIELD_FN),
        ("J_user", C.c_void_p),
        ("A_D", FIELD_FN),
        ("A_D_user", C.c_void_p),
    ]


class FactorOpts(C.Structure):
    _fields_ = [
        ("precision", C.c_int32),
        ("tile", C.c_int32),
        ("ordering", C.c_int32),
        ("gemv_variant", C.c_int32),
        ("scaling", C.c_int32),
        ("factor_tune", C.c_int32),
        ("hip_stream", C.c_void_p),
    ]


class SolveOpts(C.Structure):
    _fields_ = [
        ("rtol", C.c_double),
        ("maxit", C.c_int32),
        ("check_every", C.c_int32),
        ("lambda0", C.POINTER(C.c_double)),
        ("use_graph", C.c_int32),
        ("warm_start", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("n_global", C.c_int64),
        ("n_multipliers", C.c_int64),
        ("n_primal", C.c_int64),
        ("n_sub", C.c_int64),
        ("iters", C.c_int32),
        ("outer_iters", C.c_int32),
        ("status", C.c_int32),
        ("f_applies", C.c_int32),
        ("rel_residual", C.c_double),
        ("t_factor_s", C.c_double),
        ("t_solve_s", C.c_double),
        ("t_pcg_s", C.c_double),
        ("factor_flops", C.c_double),
        ("rel_residual0", C.c_double),
        ("warm_start", C.c_int32),
        ("reserved", C.c_int32),
        ("pcg_bytes", C.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ProblemStats(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("outer_iters", C.c_int32), ("status", C.c_int32), ("warm_start", C.c_int32),
        ("f_applies", C.c_int32 * 2), ("m_applies", C.c_int32 * 2),
        ("rel_residual", C.c_double), ("rel_residual0", C.c_double), ("block_entries", C.c_double),
        ("bytes_F", C.c_double * 2), ("bytes_M", C.c_double * 2), ("pcg_bytes", C.c_double),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class NNArch(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hidden", C.c_int32), ("n_layers", C.c_int32), ("n_comb", C.c_int32),
                ("n_out", C.c_int32)]


class NNTrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64)]


class AssembleOpts(C.Structure):
    _fields_ = [("version", C.c_int32), ("primal", C.c_int32), ("reserved", C.c_int32 * 6)]


class WarmLayout(C.Structure):
    _fields_ = [
        ("n_facets", C.c_int32), ("n_feat", C.c_int32), ("n_comb", C.c_int32), ("n_out", C.c_int32),
        ("feat_patch", C.POINTER(C.c_int32)), ("comb_patch", C.POINTER(C.c_int32)),
        ("out_row", C.POINTER(C.c_int32)), ("out_sign", C.POINTER(C.c_int8)),
    ]


EXPORTS = [
    "ieti_assemble", "ieti_factor", "ieti_solve", "ieti_solve_device", "ieti_get_sizes", "ieti_get_maps",
    "ieti_get_local_system", "ieti_get_schur", "ieti_apply_F", "ieti_apply_M", "ieti_get_rhs",
    "ieti_get_lambda", "ieti_get_plan_info", "ieti_set_profiling", "ieti_get_kernel_times", "ieti_destroy",
    "ieti_last_error", "ieti_set_coefficients", "ieti_set_warm_start", "ieti_nn_create", "ieti_nn_num_params",
    "ieti_nn_set_params", "ieti_nn_get_params", "ieti_nn_set_data", "ieti_nn_loss_grad", "ieti_nn_train",
    "ieti_nn_predict", "ieti_nn_destroy", "ieti_get_gemv_tuning", "ieti_assemble_batch", "ieti_get_batch_info",
    "ieti_batch_of", "ieti_record_pcg", "ieti_get_pcg_coefficients", "ieti_nn_save", "ieti_nn_load",
    "ieti_get_problem_stats", "ieti_nn_init_params", "ieti_nn_set_normalisation", "ieti_nn_fit_normalisation",
    "ieti_nn_get_normalisation", "ieti_nn_dataset_append", "ieti_nn_train_file", "ieti_warm_rows",
    "ieti_warm_append", "ieti_warm_load", "ieti_warm_predict", "ieti_get_condition", "ieti_apply_F_noalloc",
    "ieti_set_factor_params", "ieti_get_factor_tuning", "ieti_assemble_ex",
]


class IetiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def library_path():
    return _LIB_PATH


def load_library():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with `python -m paper_2501_04340_amd.build`")
    try:  # load torch's HIP runtime first so the process holds exactly one runtime
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER
    lib.ieti_assemble.argtypes = [P(Problem), P(C.c_void_p)]
    lib.ieti_factor.argtypes = [C.c_void_p, P(FactorOpts)]
    lib.ieti_solve.argtypes = [C.c_void_p, P(SolveOpts), P(C.c_double), P(Stats)]
    lib.ieti_solve_device.argtypes = [C.c_void_p, P(SolveOpts), C.c_void_p, P(Stats)]
    lib.ieti_get_sizes.argtypes = [C.c_void_p, P(C.c_int64)]
    lib.ieti_get_maps.argtypes = [C.c_void_p, P(C.c_uint8), P(C.c_uint8), P(C.c_uint8), P(C.c_int64),
                                  P(C.c_int64), P(C.c_int64), P(C.c_int64)]
    lib.ieti_get_local_system.argtypes = [C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_int64), P(C.c_int64),
                                          P(C.c_int32), P(C.c_double), P(C.c_double)]
    lib.ieti_get_schur.argtypes = [C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_double), P(C.c_double)]
    lib.ieti_apply_F.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    lib.ieti_apply_M.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    lib.ieti_apply_F_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.ieti_set_factor_params.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
    lib.ieti_assemble_ex.argtypes = [P(Problem), P(AssembleOpts), P(C.c_void_p)]
    lib.ieti_get_factor_tuning.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_double), P(C.c_int32)]
    lib.ieti_get_rhs.argtypes = [C.c_void_p, P(C.c_double)]
    lib.ieti_get_lambda.argtypes = [C.c_void_p, P(C.c_double)]
    lib.ieti_get_plan_info.argtypes = [C.c_void_p, P(C.c_double)]
    lib.ieti_set_profiling.argtypes = [C.c_void_p, C.c_int32]
    lib.ieti_get_kernel_times.argtypes = [C.c_void_p, P(C.c_double)]
    lib.ieti_destroy.argtypes = [C.c_void_p]
    lib.ieti_destroy.restype = None
    lib.ieti_last_error.restype = C.c_char_p
    lib.ieti_assemble_batch.argtypes = [P(Problem), C.c_int32, P(C.c_void_p)]
    lib.ieti_batch_of.argtypes = [P(C.c_void_p), C.c_int32, P(C.c_void_p)]
    lib.ieti_record_pcg.argtypes = [C.c_void_p, C.c_int32]
    lib.ieti_nn_save.argtypes = [C.c_void_p, C.c_char_p]
    lib.ieti_nn_load.argtypes = [C.c_char_p, P(C.c_void_p)]
    lib.ieti_get_pcg_coefficients.argtypes = [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double), P(C.c_int32)]
    lib.ieti_get_batch_info.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int32), P(C.c_double)]
    lib.ieti_get_problem_stats.argtypes = [C.c_void_p, C.c_int32, P(ProblemStats)]
    lib.ieti_get_gemv_tuning.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_float)]
    lib.ieti_set_coefficients.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    lib.ieti_set_warm_start.argtypes = [C.c_void_p, C.c_void_p, P(WarmLayout)]
    lib.ieti_nn_create.argtypes = [P(NNArch), P(C.c_void_p)]
    lib.ieti_nn_num_params.argtypes = [C.c_void_p, P(C.c_int64)]
    lib.ieti_nn_set_params.argtypes = [C.c_void_p, P(C.c_float)]
    lib.ieti_nn_get_params.argtypes = [C.c_void_p, P(C.c_float)]
    lib.ieti_nn_set_data.argtypes = [C.c_void_p, P(C.c_float), P(C.c_float), P(C.c_float), C.c_int64]
    lib.ieti_nn_loss_grad.argtypes = [C.c_void_p, C.c_int64, C.c_int64, P(C.c_double), P(C.c_float)]
    lib.ieti_nn_train.argtypes = [C.c_void_p, P(NNTrainOpts), P(C.c_double)]
    lib.ieti_nn_predict.argtypes = [C.c_void_p, P(C.c_float), P(C.c_float), C.c_int64, P(C.c_float)]
    lib.ieti_nn_destroy.argtypes = [C.c_void_p]
    lib.ieti_nn_destroy.restype = None
    lib.ieti_nn_init_params.argtypes = [C.c_void_p, C.c_uint64]
    lib.ieti_nn_set_normalisation.argtypes = [C.c_void_p, P(C.c_float), P(C.c_float), C.c_double]
    lib.ieti_nn_fit_normalisation.argtypes = [C.c_void_p, P(C.c_float), P(C.c_float), C.c_int64]
    lib.ieti_nn_get_normalisation.argtypes = [C.c_void_p, P(C.c_float), P(C.c_float), P(C.c_double)]
    lib.ieti_nn_dataset_append.argtypes = [C.c_char_p, P(C.c_float), P(C.c_float), P(C.c_float), C.c_int64,
                                           C.c_int32, C.c_int32, C.c_int32]
    lib.ieti_nn_train_file.argtypes = [C.c_char_p, P(NNArch), P(NNTrainOpts), C.c_char_p, P(C.c_double)]
    lib.ieti_warm_rows.argtypes = [C.c_void_p, P(WarmLayout), P(C.c_float), P(C.c_float), P(C.c_float)]
    lib.ieti_warm_append.argtypes = [C.c_void_p, P(WarmLayout), C.c_char_p]
    lib.ieti_warm_load.argtypes = [C.c_void_p, C.c_char_p, P(WarmLayout)]
    lib.ieti_warm_predict.argtypes = [C.c_void_p, P(C.c_double)]
    lib.ieti_get_condition.argtypes = [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double)]
    for name in EXPORTS:
        if name not in ("ieti_destroy", "ieti_last_error", "ieti_nn_destroy"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _check(lib, rc):
    if rc != 0:
        raise IetiError(rc, lib.ieti_last_error().decode())


def _problem_struct(prob, keep):
    """ctypes problem statement of a ``workloads.Problem``; arrays and the
    source callback are appended to ``keep`` (they must outlive assembly)."""
    part = np.ascontiguousarray(prob.patch_to_sub, dtype=np.int32)
    nu = np.ascontiguousarray(prob.nu, dtype=np.float64)
    src = prob.source

    def _field(xyz, npts, out, user):
        X = np.ctypeslib.as_array(xyz, shape=(int(npts), 3))
        O = np.ctypeslib.as_array(out, shape=(int(npts), 3))
        O[:] = src(np.array(X))

    cb = FIELD_FN(_field)
    keep.extend([part, nu, cb])
    dirichlet = getattr(prob, "dirichlet_A", None)
    if dirichlet is not None:
        def _dfield(xyz, npts, out, user):
            X = np.ctypeslib.as_array(xyz, shape=(int(npts), 3))
            O = np.ctypeslib.as_array(out, shape=(int(npts), 3))
            O[:] = dirichlet(np.array(X))

        dcb = FIELD_FN(_dfield)
        keep.append(dcb)
    pr = Problem()
    pr.version = ABI_VERSION
    pr.geom_kind = int(prob.geom_kind)
    for d in range(3):
        pr.patches[d] = int(prob.patches[d])
        pr.periodic[d] = int(prob.periodic[d])
    gp = np.zeros(16)
    gp[:len(prob.geom_params)] = prob.geom_params
    for i in range(16):
        pr.geom_params[i] = float(gp[i])
    pr.degree_p = int(prob.degree)
    pr.n_el = int(prob.n_el)
    pr.patch_to_subdomain = _ptr(part, C.c_int32)
    pr.nu_per_patch = _ptr(nu, C.c_double)
    pr.J = cb
    pr.J_user = None
    if dirichlet is not None:
        pr.A_D = dcb
    pr.A_D_user = None
    return pr


class Solver:
    """One assembled problem, or a batch of independent problems (a list),
    on the current HIP device."""

    def __init__(self, prob, primal=True):
        """primal=False (one problem only): no primal DOFs, the singular local
        problems of Section 3 (``ieti_assemble_ex``), for checking that."""
        self.lib = load_library()
        probs = list(prob) if isinstance(prob, (list, tuple)) else [prob]
        self.prob = prob
        self.batch = len(probs)
        keep = []
        arr = (Problem * len(probs))(*[_problem_struct(p, keep) for p in probs])
        self._part = np.concatenate([np.asarray(p.patch_to_sub) for p in probs]).astype(np.int32)
        h = C.c_void_p()
        if primal:
            _check(self.lib, self.lib.ieti_assemble_batch(arr, len(probs), C.byref(h)))
        else:
            if len(probs) != 1:
                raise ValueError("primal=False takes one problem")
            o = AssembleOpts()
            o.version = ABI_VERSION
            o.primal = 0
            _check(self.lib, self.lib.ieti_assemble_ex(arr, C.byref(o), C.byref(h)))
        self.h = h
        s = np.zeros(8, dtype=np.int64)
        _check(self.lib, self.lib.ieti_get_sizes(self.h, _ptr(s, C.c_int64)))
        self.n_edges, self.n_global, self.sum_n_r, self.m_r, self.n_gp, self.n_sub, self.n_nodes, self.max_n_I = map(int, s)

    @classmethod
    def batch_of(cls, solvers):
        """Batch handle from single-problem solvers (their systems are copied)."""
        self = cls.__new__(cls)
        self.lib = load_library()
        self.prob = [S.prob for S in solvers]
        self.batch = len(solvers)
        self._part = np.concatenate([S._part for S in solvers]).astype(np.int32)
        arr = (C.c_void_p * len(solvers))(*[S.h.value for S in solvers])
        h = C.c_void_p()
        _check(self.lib, self.lib.ieti_batch_of(arr, len(solvers), C.byref(h)))
        self.h = h
        s = np.zeros(8, dtype=np.int64)
        _check(self.lib, self.lib.ieti_get_sizes(self.h, _ptr(s, C.c_int64)))
        self.n_edges, self.n_global, self.sum_n_r, self.m_r, self.n_gp, self.n_sub, self.n_nodes, self.max_n_I = map(int, s)
        return self

    def batch_info(self):
        """Per problem: ranges (edge, m_r, primal, subdomain offsets and counts), last iterations and residuals."""
        n = self.batch
        rg = np.zeros((n, 8), np.int64)
        it = np.zeros(n, np.int32)
        rr = np.zeros(n)
        _check(self.lib, self.lib.ieti_get_batch_info(self.h, _ptr(rg, C.c_int64), _ptr(it, C.c_int32),
                                                      _ptr(rr, C.c_double)))
        keys = ["edge_base", "n_edges", "mr_base", "m_r", "gp_base", "n_gp", "sub_base", "n_sub"]
        return [dict(zip(keys, map(int, r)), iters=int(i), rel_residual=float(x)) for r, i, x in zip(rg, it, rr)]

    def split(self, a):
        """Per-problem coefficient vectors of a batch output."""
        return [a[b["edge_base"]:b["edge_base"] + b["n_edges"]] for b in self.batch_info()]

    def close(self):
        if getattr(self, "h", None):
            self.lib.ieti_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self):
        return {"n_edges": self.n_edges, "n_g": self.n_global, "sum_n_r": self.sum_n_r, "m_r": self.m_r,
                "n_gp": self.n_gp, "n_sub": self.n_sub, "n_nodes": self.n_nodes, "max_n_I": self.max_n_I}

    def maps(self):
        ne = self.n_edges
        weight = np.zeros(ne, np.uint8)
        tree = np.zeros(ne, np.uint8)
        dirichlet = np.zeros(ne, np.uint8)
        primal = np.zeros(max(self.n_gp, 1), np.int64)
        mult = np.zeros(max(self.m_r, 1) * 5, np.int64)
        offs = np.zeros(self.n_sub + 1, np.int64)
        redges = np.zeros(max(self.sum_n_r, 1), np.int64)
        _check(self.lib, self.lib.ieti_get_maps(self.h, _ptr(weight, C.c_uint8), _ptr(tree, C.c_uint8),
                                                _ptr(dirichlet, C.c_uint8), _ptr(primal, C.c_int64),
                                                _ptr(mult, C.c_int64), _ptr(offs, C.c_int64),
                                                _ptr(redges, C.c_int64)))
        return {
            "weight": weight, "tree": tree.astype(bool), "dirichlet": dirichlet.astype(bool),
            "primal_edges": primal[:self.n_gp], "mult": mult[:self.m_r * 5].reshape(-1, 5),
            "sub_r": [redges[offs[k]:offs[k + 1]] for k in range(self.n_sub)],
        }

    def local_system(self, k):
        n = C.c_int64()
        nnz = C.c_int64()
        _check(self.lib, self.lib.ieti_get_local_system(self.h, k, C.byref(n), C.byref(nnz), None, None, None, None))
        indptr = np.zeros(n.value + 1, np.int64)
        indices = np.zeros(max(nnz.value, 1), np.int32)
        values = np.zeros(max(nnz.value, 1), np.float64)
        load = np.zeros(max(n.value, 1), np.float64)
        _check(self.lib, self.lib.ieti_get_local_system(self.h, k, C.byref(n), C.byref(nnz), _ptr(indptr, C.c_int64),
                                                        _ptr(indices, C.c_int32), _ptr(values, C.c_double),
                                                        _ptr(load, C.c_double)))
        import scipy.sparse as sp
        K = sp.csr_matrix((values[:nnz.value], indices[:nnz.value], indptr), shape=(n.value, n.value))
        return K, load[:n.value]

    def factor(self, precision=PREC_FP64, ordering=0, stream=None, gemv_variant=None, scaling=SCALE_IDENTITY,
               tune=False):
        o = FactorOpts()
        o.precision = precision
        o.scaling = int(scaling)
        o.factor_tune = 1 if tune else 0
        o.tile = 0
        o.ordering = ordering
        o.gemv_variant = 0 if gemv_variant is None else int(gemv_variant) + 1
        o.hip_stream = stream
        _check(self.lib, self.lib.ieti_factor(self.h, C.byref(o)))

    def set_coefficients(self, nu=None, load_scale=None):
        """New per-patch reluctivity and load scales (no re-assembly); factor() again before solving."""
        self._coef = [None if v is None else np.ascontiguousarray(v, dtype=np.float64) for v in (nu, load_scale)]
        for v in self._coef:
            if v is not None and v.shape != (len(self._part),):
                raise ValueError("one value per patch expected")
        args = [None if v is None else _ptr(v, C.c_double) for v in self._coef]
        _check(self.lib, self.lib.ieti_set_coefficients(self.h, *args))

    def _layout(self, feat_patch, comb_patch, out_row, out_sign):
        fp = np.ascontiguousarray(feat_patch, dtype=np.int32)
        cp = np.ascontiguousarray(comb_patch, dtype=np.int32)
        orow = np.ascontiguousarray(out_row, dtype=np.int32)
        osg = np.ascontiguousarray(out_sign, dtype=np.int8)
        if fp.ndim != 2 or cp.ndim != 2 or orow.ndim != 2:
            raise ValueError("layout arrays are [n_facets, k]")
        if cp.shape[0] != fp.shape[0] or orow.shape != osg.shape or orow.shape[0] != fp.shape[0]:
            raise ValueError("layout arrays disagree in the number of facets")
        L = WarmLayout()
        L.n_facets, L.n_feat = fp.shape
        L.n_comb = cp.shape[1]
        L.n_out = orow.shape[1]
        L.feat_patch, L.comb_patch = _ptr(fp, C.c_int32), _ptr(cp, C.c_int32)
        L.out_row, L.out_sign = _ptr(orow, C.c_int32), _ptr(osg, C.c_int8)
        L._keep = (fp, cp, orow, osg)
        return L

    def set_warm_start(self, net, feat_patch, comb_patch, out_row, out_sign):
        """Attach a copy of ``net`` (an NN, with its normalisation) and the row layout of the warm start."""
        L = self._layout(feat_patch, comb_patch, out_row, out_sign)
        _check(self.lib, self.lib.ieti_set_warm_start(self.h, net.h, C.byref(L)))

    def warm_rows(self, feat_patch, comb_patch, out_row, out_sign, targets=True):
        """(X, C, Y) network rows of the current coefficients and, with
        ``targets``, of the last solve's multipliers (``ieti_warm_rows``)."""
        L = self._layout(feat_patch, comb_patch, out_row, out_sign)
        X = np.zeros((L.n_facets, L.n_feat), np.float32)
        Cc = np.zeros((L.n_facets, L.n_comb), np.float32)
        Y = np.zeros((L.n_facets, L.n_out), np.float32)
        _check(self.lib, self.lib.ieti_warm_rows(self.h, C.byref(L), _ptr(X, C.c_float), _ptr(Cc, C.c_float),
                                                 _ptr(Y, C.c_float) if targets else None))
        return X, Cc, (Y if targets else None)

    def warm_append(self, path, feat_patch, comb_patch, out_row, out_sign):
        """Append the last solve's rows to a dataset file (``ieti_warm_append``)."""
        L = self._layout(feat_patch, comb_patch, out_row, out_sign)
        _check(self.lib, self.lib.ieti_warm_append(self.h, C.byref(L), os.fsencode(path)))

    def warm_load(self, model_path, feat_patch, comb_patch, out_row, out_sign):
        """Load a network file and attach it (``ieti_warm_load``)."""
        L = self._layout(feat_patch, comb_patch, out_row, out_sign)
        _check(self.lib, self.lib.ieti_warm_load(self.h, os.fsencode(model_path), C.byref(L)))

    def warm_predict(self):
        """The attached network's lambda_0 for the current coefficients (``ieti_warm_predict``)."""
        lam = np.zeros(self.m_r)
        _check(self.lib, self.lib.ieti_warm_predict(self.h, _ptr(lam, C.c_double)))
        return lam

    def _solve_opts(self, rtol, maxit, lambda0, check_every, use_graph=True, warm_start=False):
        o = SolveOpts()
        o.rtol = rtol
        o.maxit = maxit
        o.check_every = check_every
        o.use_graph = 1 if use_graph else 0
        o.warm_start = 1 if warm_start else 0
        self._lam0 = None
        if lambda0 is not None:
            self._lam0 = np.ascontiguousarray(lambda0, dtype=np.float64)
            o.lambda0 = _ptr(self._lam0, C.c_double)
        return o

    def solve(self, rtol=1e-8, maxit=1000, lambda0=None, check_every=8, raise_on_nonconv=True, use_graph=True,
              warm_start=False):
        o = self._solve_opts(rtol, maxit, lambda0, check_every, use_graph, warm_start)
        a = np.zeros(self.n_edges)
        st = Stats()
        rc = self.lib.ieti_solve(self.h, C.byref(o), _ptr(a, C.c_double), C.byref(st))
        if rc != 0 and not (rc == -6 and not raise_on_nonconv):
            _check(self.lib, rc)
        return a, st.as_dict()

    def solve_device(self, out_ptr, rtol=1e-8, maxit=1000, lambda0=None, check_every=8):
        o = self._solve_opts(rtol, maxit, lambda0, check_every)
        st = Stats()
        _check(self.lib, self.lib.ieti_solve_device(self.h, C.byref(o), C.c_void_p(out_ptr), C.byref(st)))
        return st.as_dict()

    def schur(self, k):
        n = C.c_int64()
        _check(self.lib, self.lib.ieti_get_schur(self.h, k, C.byref(n), None, None))
        S = np.zeros((n.value, n.value))
        Sinv = np.zeros((n.value, n.value))
        _check(self.lib, self.lib.ieti_get_schur(self.h, k, C.byref(n), _ptr(S, C.c_double), _ptr(Sinv, C.c_double)))
        return S, Sinv

    def apply_F(self, lam):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        q = np.zeros(self.m_r)
        _check(self.lib, self.lib.ieti_apply_F(self.h, _ptr(lam, C.c_double), _ptr(q, C.c_double)))
        return q

    def apply_F_noalloc(self, d_lam, d_q, stream=None):
        """q = F lambda on device vectors (addresses of m_r doubles) without
        any allocation, on `stream` (a HIP stream handle, None = the
        handle's stream); asynchronous."""
        _check(self.lib, self.lib.ieti_apply_F_noalloc(self.h, C.c_void_p(d_lam), C.c_void_p(d_q),
                                                       C.c_void_p(stream) if stream else None))

    def apply_M(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros(self.m_r)
        _check(self.lib, self.lib.ieti_apply_M(self.h, _ptr(r, C.c_double), _ptr(z, C.c_double)))
        return z

    def rhs(self):
        b = np.zeros(self.m_r)
        _check(self.lib, self.lib.ieti_get_rhs(self.h, _ptr(b, C.c_double)))
        return b

    def plan_info(self):
        v = np.zeros(12)
        _check(self.lib, self.lib.ieti_get_plan_info(self.h, _ptr(v, C.c_double)))
        keys = ["pool_elems", "S_elems", "flops", "dense_flops", "n_steps", "n_update_tasks", "sum_nI2",
                "I_total", "max_ld", "tile", "flops_scalar_rr", "flops_scalar_aug"]
        return dict(zip(keys, v.tolist()))

    def set_factor_params(self, defer, defer_tail, update_wgs):
        _check(self.lib, self.lib.ieti_set_factor_params(self.h, int(defer), int(defer_tail), int(update_wgs)))

    def factor_tuning(self):
        """(defer, defer_tail, update_wgs) in use and the autotuner's record
        [n, 4] = (defer, defer_tail, update_wgs, ms per local factorisation)."""
        prm = np.zeros(3, np.int32)
        n = C.c_int32(0)
        _check(self.lib, self.lib.ieti_get_factor_tuning(self.h, _ptr(prm, C.c_int32), None, C.byref(n)))
        log = np.zeros(max(n.value, 1) * 4)
        _check(self.lib, self.lib.ieti_get_factor_tuning(self.h, None, _ptr(log, C.c_double), None))
        return tuple(int(x) for x in prm), log[:n.value * 4].reshape(-1, 4)

    def gemv_tuning(self):
        """(chosen shape for FP64 and FP32 blocks, ms per shape [2, GEMV_SHAPES]) of the GEMV autotuner."""
        v = np.zeros(2, np.int32)
        ms = np.zeros(2 * GEMV_SHAPES, np.float32)
        _check(self.lib, self.lib.ieti_get_gemv_tuning(self.h, _ptr(v, C.c_int32), _ptr(ms, C.c_float)))
        return v.tolist(), ms.reshape(2, GEMV_SHAPES)

    def set_profiling(self, enable=True):
        _check(self.lib, self.lib.ieti_set_profiling(self.h, 1 if enable else 0))

    def kernel_times(self):
        v = np.zeros(12)
        _check(self.lib, self.lib.ieti_get_kernel_times(self.h, _ptr(v, C.c_double)))
        keys = ["gemv_launches", "gemv_ms", "update_launches", "update_ms", "update_tasks", "gemv_bytes",
                "gemv_bytes_full", "gemv_bytes_lower", "gemv_bytes_alg", "gemv32_launches", "gemv32_ms"]
        return dict(zip(keys, v.tolist()))

    def problem_stats(self, prob=0):
        """Per-problem results of the last solve (``ieti_get_problem_stats``)."""
        st = ProblemStats()
        _check(self.lib, self.lib.ieti_get_problem_stats(self.h, int(prob), C.byref(st)))
        return st.as_dict()

    def lambda_(self):
        lam = np.zeros(self.m_r)
        _check(self.lib, self.lib.ieti_get_lambda(self.h, _ptr(lam, C.c_double)))
        return lam

    def record_pcg(self, cap):
        """Record alpha/beta of the first ``cap`` PCG iterations (0 = off)."""
        _check(self.lib, self.lib.ieti_record_pcg(self.h, int(cap)))

    def pcg_coefficients(self, prob=0):
        """(alpha, beta) of problem ``prob``'s last PCG run."""
        n = C.c_int32()
        _check(self.lib, self.lib.ieti_get_pcg_coefficients(self.h, int(prob), None, None, C.byref(n)))
        a, b = np.zeros(n.value), np.zeros(n.value)
        if n.value:
            _check(self.lib, self.lib.ieti_get_pcg_coefficients(self.h, int(prob), _ptr(a, C.c_double),
                                                                _ptr(b, C.c_double), C.byref(n)))
        return a, b

    def condition(self, prob=0):
        """(lambda_min, lambda_max) of the Lanczos tridiagonal of the recorded
        PCG run: extreme eigenvalues of the preconditioned interface operator
        (``ieti_get_condition``)."""
        lo, hi = C.c_double(), C.c_double()
        _check(self.lib, self.lib.ieti_get_condition(self.h, int(prob), C.byref(lo), C.byref(hi)))
        return float(lo.value), float(hi.value)


class NN:
    """The warm-start network on the current HIP device (see ``ieti_nn_*``)."""

    def __init__(self, n_in, n_hidden, n_layers, n_comb, n_out):
        self.lib = load_library()
        a = NNArch(n_in, n_hidden, n_layers, n_comb, n_out)
        self.arch = (n_in, n_hidden, n_layers, n_comb, n_out)
        h = C.c_void_p()
        _check(self.lib, self.lib.ieti_nn_create(C.byref(a), C.byref(h)))
        self.h = h
        n = C.c_int64()
        _check(self.lib, self.lib.ieti_nn_num_params(self.h, C.byref(n)))
        self.n_params = int(n.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.ieti_nn_destroy(self.h)
            self.h = None

    def save(self, path):
        """Architecture and parameters to a file (``ieti_nn_save``)."""
        _check(self.lib, self.lib.ieti_nn_save(self.h, os.fsencode(path)))

    @classmethod
    def load(cls, path):
        """Network on the current device from a file written by ``save``."""
        self = cls.__new__(cls)
        self.lib = load_library()
        h = C.c_void_p()
        _check(self.lib, self.lib.ieti_nn_load(os.fsencode(path), C.byref(h)))
        self.h = h
        a = np.zeros(5, np.int32)
        with open(path, "rb") as f:
            f.seek(8)
            a[:] = np.frombuffer(f.read(20), dtype=np.int32)
        self.arch = tuple(int(x) for x in a)
        n = C.c_int64()
        _check(self.lib, self.lib.ieti_nn_num_params(self.h, C.byref(n)))
        self.n_params = int(n.value)
        return self

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_params(self, seed):
        """Seeded Glorot-uniform weights and zero biases (``ieti_nn_init_params``)."""
        _check(self.lib, self.lib.ieti_nn_init_params(self.h, int(seed)))

    def set_normalisation(self, shift=None, scale=None, out_scale=1.0):
        n_in = self.arch[0]
        self._norm = [None if v is None else np.ascontiguousarray(v, dtype=np.float32).reshape(n_in)
                      for v in (shift, scale)]
        args = [None if v is None else _ptr(v, C.c_float) for v in self._norm]
        _check(self.lib, self.lib.ieti_nn_set_normalisation(self.h, *args, float(out_scale)))

    def fit_normalisation(self, X, Y):
        """Feature means / inverse deviations and output RMS of the rows (``ieti_nn_fit_normalisation``)."""
        n_in, _, _, _, n_out = self.arch
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, n_in)
        Y = np.ascontiguousarray(Y, dtype=np.float32).reshape(X.shape[0], n_out)
        _check(self.lib, self.lib.ieti_nn_fit_normalisation(self.h, _ptr(X, C.c_float), _ptr(Y, C.c_float),
                                                            X.shape[0]))

    def normalisation(self):
        n_in = self.arch[0]
        sh, sc, o = np.zeros(n_in, np.float32), np.zeros(n_in, np.float32), C.c_double()
        _check(self.lib, self.lib.ieti_nn_get_normalisation(self.h, _ptr(sh, C.c_float), _ptr(sc, C.c_float),
                                                            C.byref(o)))
        return sh, sc, float(o.value)

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        if theta.shape != (self.n_params,):
            raise ValueError(f"{self.n_params} parameters expected")
        _check(self.lib, self.lib.ieti_nn_set_params(self.h, _ptr(theta, C.c_float)))

    def params(self):
        theta = np.zeros(self.n_params, np.float32)
        _check(self.lib, self.lib.ieti_nn_get_params(self.h, _ptr(theta, C.c_float)))
        return theta

    def set_data(self, X, Cc, Y):
        n_in, _, _, n_comb, n_out = self.arch
        self._X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, n_in)
        n = self._X.shape[0]
        self._C = np.ascontiguousarray(Cc, dtype=np.float32).reshape(n, n_comb)
        self._Y = np.ascontiguousarray(Y, dtype=np.float32).reshape(n, n_out)
        _check(self.lib, self.lib.ieti_nn_set_data(self.h, _ptr(self._X, C.c_float), _ptr(self._C, C.c_float),
                                                   _ptr(self._Y, C.c_float), n))
        self.n_data = n

    def loss_grad(self, row0=0, nrows=None):
        nrows = self.n_data - row0 if nrows is None else nrows
        loss = C.c_double()
        g = np.zeros(self.n_params, np.float32)
        _check(self.lib, self.lib.ieti_nn_loss_grad(self.h, row0, nrows, C.byref(loss), _ptr(g, C.c_float)))
        return float(loss.value), g

    def train(self, epochs, lr, batch=256, seed=0, beta1=0.9, beta2=0.999, eps=1e-8):
        o = NNTrainOpts(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps), int(seed))
        losses = np.zeros(max(int(epochs), 1))
        _check(self.lib, self.lib.ieti_nn_train(self.h, C.byref(o), _ptr(losses, C.c_double)))
        return losses[:int(epochs)]

    def predict(self, X, Cc):
        n_in, _, _, n_comb, n_out = self.arch
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, n_in)
        n = X.shape[0]
        Cc = np.ascontiguousarray(Cc, dtype=np.float32).reshape(n, n_comb)
        out = np.zeros((n, n_out), np.float32)
        _check(self.lib, self.lib.ieti_nn_predict(self.h, _ptr(X, C.c_float), _ptr(Cc, C.c_float), n,
                                                  _ptr(out, C.c_float)))
        return out


def dataset_append(path, X, Cc, Y):
    """Append rows to a dataset file (``ieti_nn_dataset_append``)."""
    lib = load_library()
    X = np.ascontiguousarray(X, dtype=np.float32)
    n = X.shape[0]
    Cc = np.ascontiguousarray(Cc, dtype=np.float32).reshape(n, -1)
    Y = np.ascontiguousarray(Y, dtype=np.float32).reshape(n, -1)
    _check(lib, lib.ieti_nn_dataset_append(os.fsencode(path), _ptr(X, C.c_float), _ptr(Cc, C.c_float),
                                           _ptr(Y, C.c_float), n, X.shape[1], Cc.shape[1], Y.shape[1]))


def train_file(dataset_path, arch, model_out, epochs, lr, batch=256, seed=0, beta1=0.9, beta2=0.999, eps=1e-8):
    """Train a network of ``arch`` = (n_in, n_hidden, n_layers, n_comb, n_out)
    on a dataset file and write it to ``model_out`` (``ieti_nn_train_file``);
    returns the epoch losses."""
    lib = load_library()
    a = NNArch(*[int(v) for v in arch])
    o = NNTrainOpts(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps), int(seed))
    losses = np.zeros(max(int(epochs), 1))
    _check(lib, lib.ieti_nn_train_file(os.fsencode(dataset_path), C.byref(a), C.byref(o), os.fsencode(model_out),
                                       _ptr(losses, C.c_double)))
    return losses[:int(epochs)]
