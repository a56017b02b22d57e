"""Thin ctypes binding of ``libmfmg.so`` (include/mfmg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Vectors are torch tensors on the GPU (``torch`` provides device memory and the
current HIP stream); the library is required, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfmg.so")

MFMG_OK = 0
ERRORS = {-1: "INVALID_ARG", -2: "UNSUPPORTED", -3: "HIP_ERROR", -4: "OOM", -5: "NOT_CONVERGED",
          -6: "BREAKDOWN", -7: "NET_REJECTED"}
(ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_OOM, ERR_NOT_CONVERGED, ERR_BREAKDOWN,
 ERR_NET_REJECTED) = -1, -2, -3, -4, -5, -6, -7
F64, F32, BF16 = 0, 1, 2
SCHEME_H, SCHEME_P_THEN_H, SCHEME_H_THEN_P, SCHEME_LS, SCHEME_LS_THEN_P, SCHEME_HP = 0, 1, 2, 3, 4, 5
LEVEL_ACTIVE = -1  # the leaves (the outer solver's mesh)
RHS_CONST, RHS_GAUSS, RHS_SINE = 0, 1, 2
COARSE_EXACT, COARSE_LEARNED, COARSE_ZERO = 0, 1, 2
MAX_STEPS, MAX_LEVELS = 16, 32


class MfmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mfmg error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("n0", C.c_int), ("lo", C.c_double), ("hi", C.c_double), ("n_global", C.c_int),
                ("n_steps", C.c_int), ("kind", C.c_int * MAX_STEPS),
                ("params", (C.c_double * 8) * MAX_STEPS)]


class LevelDesc(C.Structure):
    _fields_ = [("degree", C.c_int), ("scheme", C.c_int), ("dirichlet", C.c_int),
                ("n_level_dtype", C.c_int), ("level_dtype", C.c_int * MAX_LEVELS),
                ("cheb_degree", C.c_int), ("smoothing_range", C.c_double), ("eig_safety", C.c_double),
                ("eig_iterations", C.c_int), ("max_rhs", C.c_int), ("drop_coarse", C.c_int),
                ("coef_kind", C.c_int), ("coef_params", C.c_double * 8), ("graph_vcycle", C.c_int),
                ("fmg_start", C.c_int), ("geom_kind", C.c_int), ("geom_params", C.c_double * 8),
                ("deterministic", C.c_int)]


class NetTrainDesc(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch_rows", C.c_int), ("lr", C.c_double), ("init_seed", C.c_uint64),
                ("shuffle_seed", C.c_uint64)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("initial_residual", C.c_double),
                ("final_residual", C.c_double), ("residual_history", C.c_double * 256),
                ("time_ms", C.c_double), ("coarse_fallbacks", C.c_int), ("coarse_accepted", C.c_int)]


_lib = None
_P = C.c_void_p
_I = C.c_int
_I64P = C.POINTER(C.c_int64)

_SIGS = {
    "mfmg_setup_mesh": (_I, [C.POINTER(MeshDesc), C.POINTER(_P)]),
    "mfmg_mesh_info": (_I, [_P, C.POINTER(_I), _I64P, _I64P]),
    "mfmg_host_level_matrix": (_I, [_P, _I, _I, _I, _I64P, _I64P, C.POINTER(C.c_double)]),
    "mfmg_host_ls_level": (_I, [_P, _I, _I, _I64P, _I64P, _I64P, C.POINTER(C.c_uint8), C.POINTER(C.c_double),
                                C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "mfmg_setup_levels": (_I, [_P, C.POINTER(LevelDesc), _P, C.POINTER(_P)]),
    "mfmg_n_levels": (_I, [_P, C.POINTER(_I)]),
    "mfmg_level_info": (_I, [_P, _I, _I64P, _I64P, C.POINTER(_I), C.POINTER(_I), _I64P]),
    "mfmg_level_dof_codes": (_I, [_P, _I, _I64P]),
    "mfmg_smoother_range": (_I, [_P, _I, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mfmg_vmult": (_I, [_P, _I, _I, _I, _P, _P, _P]),
    "mfmg_vmult_noalloc": (_I, [_P, _I, _I, _I, _P, _P, _P]),
    "mfmg_diagonal": (_I, [_P, _I, _I, _P, _P]),
    "mfmg_smooth": (_I, [_P, _I, _I, _I, _P, _P, _I, C.POINTER(C.c_double), _P]),
    "mfmg_residual": (_I, [_P, _I, _I, _I, _P, _P, _P, _P]),
    "mfmg_prolongate_add": (_I, [_P, _I, _I, _I, _P, _P, _P]),
    "mfmg_restrict_add": (_I, [_P, _I, _I, _I, _P, _P, _P]),
    "mfmg_coarse_solve": (_I, [_P, _I, _I, _P, _P, _P]),
    "mfmg_vcycle": (_I, [_P, _I, _P, _P, _P]),
    "mfmg_fmg": (_I, [_P, _I, _P, _P, _I, _P]),
    "mfmg_copy_to_mg": (_I, [_P, _I, _I, _P, _P, _P]),
    "mfmg_copy_from_mg": (_I, [_P, _I, _I, _P, _P, _P]),
    "mfmg_level_edge": (_I, [_P, _I, _I64P, C.POINTER(C.c_uint8)]),
    "mfmg_solve": (_I, [_P, _I, _P, _P, C.c_double, _I, _I, C.POINTER(SolveStats), _P]),
    "mfmg_rhs": (_I, [_P, _I, _I, C.POINTER(C.c_double), _I, _I, _P, _P]),
    "mfmg_distribute": (_I, [_P, _I, _P, _P, _P]),
    "mfmg_level_cells": (_I, [_P, _I, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "mfmg_set_coefficient": (_I, [_P, _P, _P]),
    "mfmg_net_n_params": (_I, [_P, C.POINTER(_I)]),
    "mfmg_net_record": (_I, [_P, _I]),
    "mfmg_net_n_recorded": (_I, [_P, C.POINTER(_I)]),
    "mfmg_net_set_params": (_I, [_P, C.POINTER(C.c_float), _I]),
    "mfmg_net_get_params": (_I, [_P, C.POINTER(C.c_float), _I]),
    "mfmg_net_loss_grad": (_I, [_P, _I, _P, _P, _P, C.POINTER(C.c_float)]),
    "mfmg_net_train": (_I, [_P, C.POINTER(NetTrainDesc), C.POINTER(C.c_float)]),
    "mfmg_net_infer": (_I, [_P, _I, _P, _P, _P]),
    "mfmg_net_mode": (_I, [_P, _I, C.c_double]),
    "mfmg_net_counts": (_I, [_P, C.POINTER(_I), C.POINTER(_I), C.POINTER(C.c_double)]),
    "mfmg_destroy_ctx": (None, [_P]),
    "mfmg_destroy_mesh": (None, [_P]),
    "mfmg_last_error": (C.c_char_p, []),
}


def lib():
    """Load ``libmfmg.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2203_12292_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != MFMG_OK:
        raise MfmgError(code, lib().mfmg_last_error().decode())
    return code


def mesh_desc(d):
    """ctypes descriptor from a ``synth`` mesh descriptor dict."""
    m = MeshDesc()
    m.n0, m.lo, m.hi, m.n_global = d["n0"], d["lo"], d["hi"], d["n_global"]
    m.n_steps = len(d["steps"])
    for s, (kind, params) in enumerate(d["steps"]):
        m.kind[s] = kind
        for q, p in enumerate(params):
            m.params[s][q] = p
    return m


def _dtype_code(t):
    import torch
    return {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[t.dtype]


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _vec(t, numel, name, dtype=None, like=None, device=True):
    """Check a vector argument before it becomes a raw device pointer: a
    contiguous torch tensor of exactly `numel` elements, of torch dtype
    `dtype` (or of the dtype of tensor `like`), on the GPU.  The C ABI cannot
    check the size of device memory, so every wrapper calls this first."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    want = like.dtype if like is not None else dtype
    if want is not None and t.dtype != want:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {want}")
    if t.dtype not in (torch.float64, torch.float32, torch.bfloat16):
        raise TypeError(f"{name}: unsupported dtype {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if device and not t.is_cuda:
        raise ValueError(f"{name}: tensor must be on the GPU")
    return t


def _vecs(*args):
    """_vec for several arguments: first every argument's size, dtype and
    layout, then every argument's device."""
    for a in args:
        _vec(*a, device=False)
    for a in args:
        _vec(*a)


def _f64(name):
    """torch.float64 (the FP64 vectors of the outer solver), imported lazily"""
    import torch
    return torch.float64


class Mesh:
    def __init__(self, desc):
        self.handle = C.c_void_p()
        self._desc = mesh_desc(desc) if isinstance(desc, dict) else desc
        _check(lib().mfmg_setup_mesh(C.byref(self._desc), C.byref(self.handle)))

    def info(self):
        n = C.c_int()
        _check(lib().mfmg_mesh_info(self.handle, C.byref(n), None, None))
        cells = (C.c_int64 * n.value)()
        nh = C.c_int64()
        _check(lib().mfmg_mesh_info(self.handle, None, cells, C.byref(nh)))
        return list(cells), nh.value

    def host_level(self, mesh_index, degree, dirichlet=True, dense=False):
        """(codes (n,3) int64, dense matrix or None) from the host set-up."""
        n = C.c_int64()
        _check(lib().mfmg_host_level_matrix(self.handle, mesh_index, degree, int(dirichlet), C.byref(n),
                                            None, None))
        codes = np.zeros((n.value, 3), dtype=np.int64)
        A = np.zeros((n.value, n.value)) if dense else None
        _check(lib().mfmg_host_level_matrix(
            self.handle, mesh_index, degree, int(dirichlet), C.byref(n),
            codes.ctypes.data_as(_I64P),
            A.ctypes.data_as(C.POINTER(C.c_double)) if dense else None))
        return codes, A

    def host_ls_level(self, level, degree, dense=False):
        """Local-smoothing level from the host set-up: dict of codes (n,3),
        edge flags, dense matrix (or None), and the copy map (level DoFs,
        active DoFs)."""
        n, m = C.c_int64(), C.c_int64()
        _check(lib().mfmg_host_ls_level(self.handle, level, degree, C.byref(n), C.byref(m), None, None, None, None,
                                        None))
        codes = np.zeros((n.value, 3), dtype=np.int64)
        edge = np.zeros(n.value, dtype=np.uint8)
        A = np.zeros((n.value, n.value)) if dense else None
        cl = np.zeros(m.value, dtype=np.int32)
        ca = np.zeros(m.value, dtype=np.int32)
        _check(lib().mfmg_host_ls_level(
            self.handle, level, degree, C.byref(n), C.byref(m), codes.ctypes.data_as(_I64P),
            edge.ctypes.data_as(C.POINTER(C.c_uint8)),
            A.ctypes.data_as(C.POINTER(C.c_double)) if dense else None,
            cl.ctypes.data_as(C.POINTER(C.c_int32)), ca.ctypes.data_as(C.POINTER(C.c_int32))))
        return {"codes": codes, "edge": edge.astype(bool), "dense": A, "copy_level": cl, "copy_active": ca}

    def close(self):
        if self.handle:
            lib().mfmg_destroy_mesh(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """Multigrid levels on the GPU (``mfmg_setup_levels``) and the hot-path calls."""

    def __init__(self, mesh, degree, scheme=SCHEME_H, level_dtypes=None, dirichlet=True, cheb_degree=3,
                 max_rhs=1, smoothing_range=20.0, eig_safety=1.2, eig_iterations=15, drop_coarse=0,
                 coef=None, graph_vcycle=False, fmg_start=False, geometry=None, deterministic=False):
        d = LevelDesc()
        d.degree, d.scheme, d.dirichlet = degree, scheme, int(dirichlet)
        level_dtypes = list(level_dtypes or [])
        d.n_level_dtype = len(level_dtypes)
        for i, t in enumerate(level_dtypes):
            d.level_dtype[i] = t
        d.cheb_degree, d.smoothing_range, d.eig_safety = cheb_degree, smoothing_range, eig_safety
        d.eig_iterations, d.max_rhs, d.drop_coarse = eig_iterations, max_rhs, drop_coarse
        d.graph_vcycle, d.fmg_start = int(graph_vcycle), int(fmg_start)
        d.deterministic = int(deterministic)
        if coef is not None:  # a synth coefficient descriptor {"kind": k, "params": [...]}
            d.coef_kind = coef["kind"]
            for i, v in enumerate(coef["params"]):
                d.coef_params[i] = v
        if geometry is not None:  # a synth geometry descriptor {"kind": k, "params": [...]}
            d.geom_kind = geometry["kind"]
            for i, v in enumerate(geometry["params"]):
                d.geom_params[i] = v
        self.desc = d
        self.handle = C.c_void_p()
        self.mesh = mesh
        _check(lib().mfmg_setup_levels(mesh.handle, C.byref(d), _stream(), C.byref(self.handle)))
        n = C.c_int()
        _check(lib().mfmg_n_levels(self.handle, C.byref(n)))
        self.n_levels = n.value
        self._nd = {}

    # -- information -----------------------------------------------------------
    def level_info(self, level):
        nd, nc, nh = C.c_int64(), C.c_int64(), C.c_int64()
        k, dt = C.c_int(), C.c_int()
        _check(lib().mfmg_level_info(self.handle, level, C.byref(nd), C.byref(nc), C.byref(k), C.byref(dt),
                                     C.byref(nh)))
        return {"n_dofs": nd.value, "n_cells": nc.value, "degree": k.value, "dtype": dt.value,
                "n_hanging_cells": nh.value}

    def n_dofs(self, level=LEVEL_ACTIVE):
        return self.level_info(level)["n_dofs"]

    def level_edge(self, level):
        """(number of refinement-edge DoFs, uint8 flag per DoF) of a level."""
        n = C.c_int64()
        flags = np.zeros(self.n_dofs(level), dtype=np.uint8)
        _check(lib().mfmg_level_edge(self.handle, level, C.byref(n), flags.ctypes.data_as(C.POINTER(C.c_uint8))))
        return n.value, flags

    def dof_codes(self, level):
        n = self.n_dofs(level)
        codes = np.zeros((n, 3), dtype=np.int64)
        _check(lib().mfmg_level_dof_codes(self.handle, level, codes.ctypes.data_as(_I64P)))
        return codes

    def smoother_range(self, level):
        a, b = C.c_double(), C.c_double()
        _check(lib().mfmg_smoother_range(self.handle, level, C.byref(a), C.byref(b)))
        return a.value, b.value

    # -- hot path (torch tensors on the GPU) -------------------------------------
    def _n(self, level):
        if level not in self._nd:
            self._nd[level] = self.level_info(level)["n_dofs"]
        return self._nd[level]

    def _nv(self, n_vec):
        if not 1 <= n_vec <= 8:
            raise ValueError(f"n_vec must be in [1, 8], got {n_vec}")
        return n_vec

    def vmult(self, level, dst, src, n_vec=1):
        n = self._n(level) * self._nv(n_vec)
        _vecs((src, n, "src", None, None), (dst, n, "dst", None, src))
        _check(lib().mfmg_vmult(self.handle, level, _dtype_code(src), n_vec, _ptr(dst), _ptr(src), _stream()))
        return dst

    def vmult_noalloc(self, level, dst, src, n_vec=1):
        """dst = A src through the allocation-free entry point (fixed work space)."""
        n = self._n(level) * self._nv(n_vec)
        _vecs((src, n, "src", None, None), (dst, n, "dst", None, src))
        _check(lib().mfmg_vmult_noalloc(self.handle, level, _dtype_code(src), n_vec, _ptr(dst), _ptr(src),
                                        _stream()))
        return dst

    def diagonal(self, level, diag):
        _vecs((diag, self._n(level), "diag", None, None))
        _check(lib().mfmg_diagonal(self.handle, level, _dtype_code(diag), _ptr(diag), _stream()))
        return diag

    def smooth(self, level, x, b, x_is_zero=False, lam=None, n_vec=1):
        n = self._n(level) * self._nv(n_vec)
        _vecs((x, n, "x", None, None), (b, n, "b", None, x))
        lp = (C.c_double * 2)(*lam) if lam is not None else None
        _check(lib().mfmg_smooth(self.handle, level, _dtype_code(x), n_vec, _ptr(x), _ptr(b), int(x_is_zero),
                                 lp, _stream()))
        return x

    def residual(self, level, r, b, x, n_vec=1):
        n = self._n(level) * self._nv(n_vec)
        _vecs((r, n, "r", None, None), (b, n, "b", None, r), (x, n, "x", None, r))
        _check(lib().mfmg_residual(self.handle, level, _dtype_code(r), n_vec, _ptr(r), _ptr(b), _ptr(x),
                                   _stream()))
        return r

    def prolongate_add(self, fine_level, dst_fine, src_coarse, n_vec=1):
        nv = self._nv(n_vec)
        _vecs((dst_fine, self._n(fine_level) * nv, "dst_fine", None, None),
              (src_coarse, self._n(fine_level - 1) * nv, "src_coarse", None, dst_fine))
        _check(lib().mfmg_prolongate_add(self.handle, fine_level, _dtype_code(dst_fine), n_vec, _ptr(dst_fine),
                                         _ptr(src_coarse), _stream()))
        return dst_fine

    def restrict_add(self, fine_level, dst_coarse, src_fine, n_vec=1):
        nv = self._nv(n_vec)
        _vecs((dst_coarse, self._n(fine_level - 1) * nv, "dst_coarse", None, None),
              (src_fine, self._n(fine_level) * nv, "src_fine", None, dst_coarse))
        _check(lib().mfmg_restrict_add(self.handle, fine_level, _dtype_code(dst_coarse), n_vec,
                                       _ptr(dst_coarse), _ptr(src_fine), _stream()))
        return dst_coarse

    def coarse_solve(self, x, b, n_vec=1):
        n = self._n(0) * self._nv(n_vec)
        _vecs((x, n, "x", None, None), (b, n, "b", None, x))
        _check(lib().mfmg_coarse_solve(self.handle, _dtype_code(x), n_vec, _ptr(x), _ptr(b), _stream()))
        return x

    def fmg(self, x, b, cycles=1, n_vec=1):
        n = self._n(LEVEL_ACTIVE) * self._nv(n_vec)
        _vecs((x, n, "x", _f64("x"), None), (b, n, "b", _f64("b"), None))
        _check(lib().mfmg_fmg(self.handle, n_vec, _ptr(x), _ptr(b), cycles, _stream()))
        return x

    def copy_to_mg(self, level, dst, src, n_vec=1):
        nv = self._nv(n_vec)
        _vecs((dst, self._n(level) * nv, "dst", None, None),
              (src, self._n(LEVEL_ACTIVE) * nv, "src", _f64("src"), None))
        _check(lib().mfmg_copy_to_mg(self.handle, level, n_vec, _ptr(dst), _ptr(src), _stream()))
        return dst

    def copy_from_mg(self, level, dst, src, n_vec=1):
        nv = self._nv(n_vec)
        _vecs((dst, self._n(LEVEL_ACTIVE) * nv, "dst", _f64("dst"), None),
              (src, self._n(level) * nv, "src", None, None))
        _check(lib().mfmg_copy_from_mg(self.handle, level, n_vec, _ptr(dst), _ptr(src), _stream()))
        return dst

    def vcycle(self, x, b, n_vec=1):
        n = self._n(LEVEL_ACTIVE) * self._nv(n_vec)
        _vecs((x, n, "x", _f64("x"), None), (b, n, "b", _f64("b"), None))
        _check(lib().mfmg_vcycle(self.handle, n_vec, _ptr(x), _ptr(b), _stream()))
        return x

    def solve(self, x, b, rtol=1e-10, max_it=100, flexible=False, n_vec=1, raise_on_fail=True):
        n = self._n(LEVEL_ACTIVE) * self._nv(n_vec)
        _vecs((x, n, "x", _f64("x"), None), (b, n, "b", _f64("b"), None))
        st = SolveStats()
        code = lib().mfmg_solve(self.handle, n_vec, _ptr(x), _ptr(b), rtol, max_it, int(flexible), C.byref(st),
                                _stream())
        if raise_on_fail:
            _check(code)
        hist = [st.residual_history[i] for i in range(min(st.iterations + 1, 256))]
        return {"code": code, "iterations": st.iterations, "converged": bool(st.converged),
                "initial_residual": st.initial_residual, "final_residual": st.final_residual,
                "time_ms": st.time_ms, "history": hist, "coarse_fallbacks": st.coarse_fallbacks,
                "coarse_accepted": st.coarse_accepted}

    def rhs(self, b, kind=RHS_CONST, params=(1.0,), n_terms=0, n_vec=1, level=LEVEL_ACTIVE):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).ravel())
        nv = self._nv(n_vec)
        need = {RHS_CONST: 1, RHS_SINE: 2}.get(kind, 5 * n_terms * nv)
        if kind == RHS_GAUSS and n_terms < 1:
            raise ValueError("n_terms must be >= 1 for Gaussian sums")
        if p.size < need:
            raise ValueError(f"params: {p.size} values, the load of kind {kind} reads {need}")
        _vecs((b, self._n(level) * nv, "b", _f64("b"), None))
        _check(lib().mfmg_rhs(self.handle, level, kind, p.ctypes.data_as(C.POINTER(C.c_double)), n_terms, n_vec,
                              _ptr(b), _stream()))
        return b

    def distribute(self, x, out, level=LEVEL_ACTIVE):
        info = self.level_info(level)
        _vecs((x, info["n_dofs"], "x", _f64("x"), None),
              (out, info["n_cells"] * (info["degree"] + 1) ** 3, "out", _f64("out"), None))
        _check(lib().mfmg_distribute(self.handle, level, _ptr(x), _ptr(out), _stream()))
        return out

    def level_cells(self, level):
        nc = self.level_info(level)["n_cells"]
        lv = np.zeros(nc, dtype=np.int32)
        ijk = np.zeros((nc, 3), dtype=np.int32)
        _check(lib().mfmg_level_cells(self.handle, level, lv.ctypes.data_as(C.POINTER(C.c_int32)),
                                      ijk.ctypes.data_as(C.POINTER(C.c_int32))))
        return lv, ijk

    def set_coefficient(self, c):
        """New cellwise-constant diffusion coefficient from the finest level's
        cell values (float64 device tensor in the order of level_cells of the
        finest level); every level, diagonal, Chebyshev interval and the
        coarse solver follow (a set-up call)."""
        n = self.level_info(self.n_levels - 1)["n_cells"]
        _vecs((c, n, "c", _f64("c"), None))
        _check(lib().mfmg_set_coefficient(self.handle, _ptr(c), _stream()))

    # -- learned coarse correction ------------------------------------------------
    def net_n_params(self):
        n = C.c_int()
        _check(lib().mfmg_net_n_params(self.handle, C.byref(n)))
        return n.value

    def net_record(self, capacity):
        _check(lib().mfmg_net_record(self.handle, capacity))

    def net_n_recorded(self):
        n = C.c_int()
        _check(lib().mfmg_net_n_recorded(self.handle, C.byref(n)))
        return n.value

    def net_set_params(self, theta):
        t = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
        _check(lib().mfmg_net_set_params(self.handle, t.ctypes.data_as(C.POINTER(C.c_float)), t.size))

    def net_get_params(self):
        t = np.zeros(self.net_n_params(), dtype=np.float32)
        _check(lib().mfmg_net_get_params(self.handle, t.ctypes.data_as(C.POINTER(C.c_float)), t.size))
        return t

    def net_loss_grad(self, X, T, grad):
        import torch
        n = self.net_n_params()
        nq = (n - 4416) // 129  # n = (nq + 3) 64 + 64 + 64 64 + 64 + 64 nq + nq
        nin = nq + 3
        if X.dim() != 2 or X.shape[1] != nin:
            raise ValueError(f"X: expected shape (rows, {nin}), got {tuple(X.shape)}")
        _vecs((X, X.shape[0] * nin, "X", torch.float32, None),
              (T, X.shape[0] * nq, "T", torch.float32, None),
              (grad, n, "grad", torch.float32, None))
        loss = C.c_float()
        _check(lib().mfmg_net_loss_grad(self.handle, X.shape[0], _ptr(X), _ptr(T), _ptr(grad), C.byref(loss)))
        return loss.value

    def net_train(self, epochs, batch_rows=4096, lr=1e-3, init_seed=1, shuffle_seed=2):
        d = NetTrainDesc(epochs, batch_rows, lr, init_seed, shuffle_seed)
        hist = (C.c_float * epochs)()
        _check(lib().mfmg_net_train(self.handle, C.byref(d), hist))
        return list(hist)

    def net_infer(self, y, b):
        """y = the network's coarse correction of the level-0 right-hand side b
        (no residual check); y and b of one dtype."""
        n = self._n(0)
        _vecs((b, n, "b", None, None), (y, n, "y", None, b))
        _check(lib().mfmg_net_infer(self.handle, _dtype_code(b), _ptr(y), _ptr(b), _stream()))
        return y

    def net_mode(self, mode, tau=0.5):
        _check(lib().mfmg_net_mode(self.handle, mode, tau))

    def net_counts(self):
        """(accepted, rejected, mean relative coarse residual of the predictions)"""
        a, r, m = C.c_int(), C.c_int(), C.c_double()
        _check(lib().mfmg_net_counts(self.handle, C.byref(a), C.byref(r), C.byref(m)))
        return a.value, r.value, m.value

    def close(self):
        if self.handle:
            lib().mfmg_destroy_ctx(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exported_names():
    """Function names declared in include/mfmg.h."""
    import re
    hdr = open(os.path.join(os.path.dirname(_HERE), "include", "mfmg.h")).read()
    return sorted(set(re.findall(r"\b(mfmg_[a-z0-9_]+)\s*\(", hdr)))
