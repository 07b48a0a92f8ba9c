"""ctypes binding of libbem.so (argument marshalling only).

Every computation runs in the library's HIP kernels; torch tensors provide
device memory (``data_ptr()``) and the HIP stream (``cuda_stream``).  The
library must be built (``python -m paper_2104_04609_amd.build``); importing
this module fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2104_04609_amd.build` (hipcc, gfx950)")

lib = ctypes.CDLL(LIB_PATH)

BEM_FP64, BEM_FP32, BEM_FP32_DENSE, BEM_FP64_DENSE, BEM_FP32_HMAT = 0, 1, 2, 3, 4
_PREC = {"fp64": BEM_FP64, "fp32": BEM_FP32, "fp32_dense": BEM_FP32_DENSE,
         "fp64_dense": BEM_FP64_DENSE, "fp32_hmat": BEM_FP32_HMAT, BEM_FP64: BEM_FP64,
         BEM_FP32: BEM_FP32, BEM_FP32_DENSE: BEM_FP32_DENSE, BEM_FP64_DENSE: BEM_FP64_DENSE,
         BEM_FP32_HMAT: BEM_FP32_HMAT}
ERRORS = {1: "BEM_W_NOT_CONVERGED", 2: "BEM_W_PENDING", 3: "BEM_W_DEFAULT", -1: "BEM_E_INVAL", -2: "BEM_E_BAD_MESH",
          -3: "BEM_E_NOMEM", -4: "BEM_E_DEVICE", -5: "BEM_E_NAN",
          -6: "BEM_E_UNSUPPORTED"}


class c64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


def _c(z) -> c64:
    z = complex(z)
    return c64(z.real, z.imag)


class SolveOpts(ctypes.Structure):
    _fields_ = [("pade_terms", ctypes.c_int), ("theta", ctypes.c_double),
                ("osrc_interior", ctypes.c_int), ("R", ctypes.c_double),
                ("precision", ctypes.c_int), ("maxiter", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("path", ctypes.c_int), ("formulation", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("outer_steps", ctypes.c_int),
                ("fp64_matvecs", ctypes.c_int), ("fp32_matvecs", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TuneEntry(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("multi", ctypes.c_int), ("gemm_min", ctypes.c_int),
                ("skinny_min", ctypes.c_int), ("path", ctypes.c_int),
                ("t_matrix_free", ctypes.c_double),
                ("t_assembled", ctypes.c_double), ("t_assembly", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class HMatStats(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_int64), ("lowrank_bytes", ctypes.c_int64),
                ("dense_bytes", ctypes.c_int64), ("n_clusters", ctypes.c_int32),
                ("n_admissible", ctypes.c_int32), ("n_dense", ctypes.c_int32),
                ("max_rank", ctypes.c_int32), ("split_blocks", ctypes.c_int32),
                ("leaf", ctypes.c_int32), ("kmax", ctypes.c_int32),
                ("mean_rank", ctypes.c_double), ("admissible_fraction", ctypes.c_double),
                ("eta", ctypes.c_double), ("tol", ctypes.c_double),
                ("setup_seconds", ctypes.c_double), ("alpha", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class OsrcStats(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("pade_terms", ctypes.c_int32),
                ("n_factors", ctypes.c_int32), ("solves_per_apply", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("nnz_l", ctypes.c_int64),
                ("nnz_offblock", ctypes.c_int64), ("dense_entries", ctypes.c_int64),
                ("mass_nnz", ctypes.c_int64), ("factor_bytes", ctypes.c_int64),
                ("bytes_per_apply", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved0"}


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("workers", ctypes.c_int),
                ("max_replicas", ctypes.c_int), ("dense_max_bytes", ctypes.c_int64)]


class RequestStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("path", ctypes.c_int), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_end", ctypes.c_double),
                ("footprint", ctypes.c_int64), ("replica", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_int64), ("resident_bytes", ctypes.c_int64),
                ("reserved_bytes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("inflight", ctypes.c_int), ("peak_inflight", ctypes.c_int),
                ("queued", ctypes.c_int), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("krylov_growth_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
lib.bem_mesh_create.argtypes = [_vp, _i64, _vp, _i64, _vp, ctypes.POINTER(_vp)]
lib.bem_mesh_destroy.argtypes = [_vp]
lib.bem_mesh_destroy.restype = None
lib.bem_mesh_info.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_i64)]
lib.pmchwt_matvec.argtypes = [_vp, c64, c64, ctypes.c_double, _vp, _vp,
                              ctypes.c_int, ctypes.c_int, _vp]
lib.pmchwt_matvec_multi.argtypes = [_vp, c64, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]
lib.pmchwt_solve_multi.argtypes = [_vp, c64, _vp, _vp, _vp, ctypes.c_int, ctypes.c_double,
                                   ctypes.POINTER(SolveOpts), _vp, _vp, _vp]
lib.pmchwt_field_multi.argtypes = [_vp, c64, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp]
lib.muller_matvec.argtypes = [_vp, c64, c64, ctypes.c_double, _vp, _vp,
                              ctypes.c_int, ctypes.c_int, _vp]
lib.osrc_apply.argtypes = [_vp, ctypes.c_int, ctypes.c_double, c64, c64, _vp, _vp,
                           ctypes.c_int, _vp]
lib.osrc_apply_noalloc.argtypes = [_vp, ctypes.c_int, ctypes.c_double, c64, c64, _vp, _vp,
                                   ctypes.c_int, _vp]
lib.pmchwt_rhs.argtypes = [_vp, c64, _vp, ctypes.c_int, _vp, _vp]
lib.bem_solve_opts_default.argtypes = [ctypes.POINTER(SolveOpts)]
lib.bem_solve_opts_default.restype = None
lib.pmchwt_solve.argtypes = [_vp, c64, c64, ctypes.c_double, _vp, ctypes.c_int,
                             ctypes.c_double, ctypes.POINTER(SolveOpts), _vp, _vp, _vp]
lib.bem_far_field.argtypes = [_vp, c64, _vp, _vp, ctypes.c_int, _vp, _vp]
lib.pmchwt_field.argtypes = [_vp, c64, c64, ctypes.c_double, _vp, _vp, _vp, _i64, _vp, _vp, _vp]
lib.bem_profile_enable.argtypes = [ctypes.c_int]
lib.bem_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(_i64)]
lib.bem_valu_rates.argtypes = [_vp, _vp]
lib.bem_tune_set.argtypes = [ctypes.c_char_p, _i64]
lib.bem_hmat_info.argtypes = [_vp, c64, c64, ctypes.c_double, ctypes.POINTER(HMatStats), _vp]
lib.bem_osrc_info.argtypes = [_vp, ctypes.c_int, ctypes.c_double, c64, c64,
                              ctypes.POINTER(OsrcStats), _vp]
lib.bem_autotune.argtypes = [_vp, c64, c64, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                             ctypes.POINTER(TuneEntry), _vp]
lib.bem_tune_cache_load.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]
lib.bem_tune_lookup.argtypes = [_i64, ctypes.c_int, ctypes.POINTER(TuneEntry)]
lib.bem_tune_clear.argtypes = []
lib.bem_tune_clear.restype = None
lib.bem_tune_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(_i64)]
lib.bem_server_opts_default.argtypes = [ctypes.POINTER(ServerOpts)]
lib.bem_server_opts_default.restype = None
lib.bem_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp)]
lib.bem_server_destroy.argtypes = [_vp]
lib.bem_server_destroy.restype = None
lib.bem_server_add_mesh.argtypes = [_vp, _vp, _i64, _vp, _i64, _vp, ctypes.POINTER(ctypes.c_int)]
lib.bem_server_submit.argtypes = [_vp, ctypes.c_int, c64, c64, ctypes.c_double, _vp, ctypes.c_int,
                                  ctypes.c_double, ctypes.POINTER(SolveOpts), _vp, _vp,
                                  ctypes.POINTER(_i64)]
lib.bem_server_submit_multi.argtypes = [_vp, ctypes.c_int, c64, _vp, _vp, _vp, ctypes.c_int,
                                        ctypes.c_double, ctypes.POINTER(SolveOpts), _vp, _vp,
                                        ctypes.POINTER(_i64)]
lib.bem_server_wait.argtypes = [_vp, _i64, ctypes.c_double, ctypes.POINTER(RequestStats)]
lib.bem_server_stats_get.argtypes = [_vp, ctypes.POINTER(ServerStats)]
lib.bem_last_error.restype = ctypes.c_char_p
lib.bem_last_error.argtypes = []


class BemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(rc: int) -> int:
    if rc < 0:
        raise BemError(rc, lib.bem_last_error().decode())
    return rc


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(_vp)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def _dev_c128(t, n2: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.complex128 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous complex128")
    if t.numel() % n2 != 0:
        raise ValueError(f"{name} has {t.numel()} entries, not a multiple of 2N={n2}")
    return t.numel() // n2


class Mesh:
    """Device-resident mesh handle (bem_mesh_create / bem_mesh_destroy)."""

    def __init__(self, vertices, triangles, object_id=None):
        P = np.ascontiguousarray(vertices, dtype=np.float64)
        T = np.ascontiguousarray(triangles, dtype=np.int32)
        O = None if object_id is None else np.ascontiguousarray(object_id, np.int32)
        if P.ndim != 2 or P.shape[1] != 3 or T.ndim != 2 or T.shape[1] != 3:
            raise ValueError("vertices [N,3] and triangles [T,3] expected")
        if O is not None and O.shape != (T.shape[0],):
            raise ValueError("object_id must have one entry per triangle")
        h = _vp()
        self._h = None
        _check(lib.bem_mesh_create(_np_ptr(P), P.shape[0], _np_ptr(T), T.shape[0],
                                   _np_ptr(O) if O is not None else None,
                                   ctypes.byref(h)))
        self._h = h
        self.n_vertices = P.shape[0]
        self.n_triangles = T.shape[0]
        self.n_objects = int(O.max()) + 1 if O is not None and O.size else 1

    @classmethod
    def from_inputs(cls, m):
        return cls(m.vertices, m.triangles, m.object_id)

    @property
    def handle(self):
        return self._h

    def info(self):
        nv, nt, by = _i64(), _i64(), _i64()
        no = ctypes.c_int32()
        _check(lib.bem_mesh_info(self._h, ctypes.byref(nv), ctypes.byref(nt),
                                 ctypes.byref(no), ctypes.byref(by)))
        return dict(n_vertices=nv.value, n_triangles=nt.value, n_objects=no.value,
                    device_bytes=by.value)

    def __del__(self):
        if getattr(self, "_h", None):
            lib.bem_mesh_destroy(self._h)
            self._h = None


def _operator_matvec(fn, mesh, k_ext, k_int, rho, x, y, precision, stream):
    import torch
    n2 = 2 * mesh.n_vertices
    n_rhs = _dev_c128(x, n2, "x")
    if y is None:
        y = torch.empty_like(x)
    _dev_c128(y, n2, "y")
    _check(fn(mesh.handle, _c(k_ext), _c(k_int), float(rho), _vp(x.data_ptr()),
              _vp(y.data_ptr()), n_rhs, _PREC[precision], _stream(stream)))
    return y


def pmchwt_matvec(mesh: Mesh, k_ext, k_int, rho: float, x, y=None,
                  precision="fp64", stream=None):
    """y = B x (weak-form permuted PMCHWT); x, y complex128 [n_rhs, 2N] on device."""
    return _operator_matvec(lib.pmchwt_matvec, mesh, k_ext, k_int, rho, x, y, precision, stream)


def _materials(mesh: Mesh, k_int, rho):
    """Host arrays (c64 [n_objects], float64 [n_objects]) of per-object materials."""
    k = np.atleast_1d(np.asarray(k_int, dtype=np.complex128))
    r = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    n = mesh.n_objects
    if k.shape != (n,) or r.shape != (n,):
        raise ValueError(f"k_int and rho need one entry per object ({n})")
    kc = (c64 * n)(*[c64(complex(v).real, complex(v).imag) for v in k])
    rc = np.ascontiguousarray(r)
    return kc, rc


def pmchwt_matvec_multi(mesh: Mesh, k_ext, k_int, rho, x, y=None, precision="fp64",
                        stream=None):
    """y = B x with object m's interior material (k_int[m], rho[m])."""
    import torch
    kc, rc = _materials(mesh, k_int, rho)
    n2 = 2 * mesh.n_vertices
    n_rhs = _dev_c128(x, n2, "x")
    if y is None:
        y = torch.empty_like(x)
    _dev_c128(y, n2, "y")
    _check(lib.pmchwt_matvec_multi(mesh.handle, _c(k_ext), ctypes.cast(kc, _vp), _np_ptr(rc),
                                   _vp(x.data_ptr()), _vp(y.data_ptr()), n_rhs,
                                   _PREC[precision], _stream(stream)))
    return y


def muller_matvec(mesh: Mesh, k_ext, k_int, rho: float, x, y=None,
                  precision="fp64", stream=None):
    """y = B_M x (weak-form Mueller operator on the permuted unknowns [psi; phi]);
    x, y complex128 [n_rhs, 2N] on device."""
    return _operator_matvec(lib.muller_matvec, mesh, k_ext, k_int, rho, x, y, precision, stream)


def osrc_apply(mesh: Mesh, pade_terms: int, theta: float, k, k_eps, x, y=None,
               stream=None):
    """y = diag(L_DtN, L_NtD) x (strong form); complex128 [n_rhs, 2N] on device."""
    import torch
    n2 = 2 * mesh.n_vertices
    n_rhs = _dev_c128(x, n2, "x")
    if y is None:
        y = torch.empty_like(x)
    _dev_c128(y, n2, "y")
    _check(lib.osrc_apply(mesh.handle, int(pade_terms), float(theta), _c(k), _c(k_eps),
                          _vp(x.data_ptr()), _vp(y.data_ptr()), n_rhs, _stream(stream)))
    return y


def osrc_info(mesh: Mesh, pade_terms: int, theta: float, k, k_eps, stream=None) -> dict:
    """bem_osrc_info: OSRC factor sizes and the algorithmic bytes of one
    single-vector apply (factors created and cached when absent)."""
    st = OsrcStats()
    _check(lib.bem_osrc_info(mesh.handle, int(pade_terms), float(theta), _c(k), _c(k_eps),
                             ctypes.byref(st), _stream(stream)))
    return st.as_dict()


def osrc_apply_noalloc(mesh: Mesh, pade_terms: int, theta: float, k, k_eps, x, y,
                       stream=None):
    """osrc_apply into a caller-allocated y, without device allocation in the
    library (the factors must be resident: call osrc_apply once first)."""
    n2 = 2 * mesh.n_vertices
    n_rhs = _dev_c128(x, n2, "x")
    if _dev_c128(y, n2, "y") != n_rhs:
        raise ValueError("x and y hold different numbers of vectors")
    _check(lib.osrc_apply_noalloc(mesh.handle, int(pade_terms), float(theta), _c(k),
                                  _c(k_eps), _vp(x.data_ptr()), _vp(y.data_ptr()), n_rhs,
                                  _stream(stream)))
    return y


def pmchwt_rhs(mesh: Mesh, k_ext, directions, stream=None):
    """Weak right-hand sides [f_D; f_N] for plane waves: complex128 [n_waves, 2N]."""
    import torch
    d = np.ascontiguousarray(np.atleast_2d(directions), dtype=np.float64)
    f = torch.empty((d.shape[0], 2 * mesh.n_vertices), dtype=torch.complex128,
                    device="cuda")
    _check(lib.pmchwt_rhs(mesh.handle, _c(k_ext), _np_ptr(d), d.shape[0],
                          _vp(f.data_ptr()), _stream(stream)))
    return f


def default_opts() -> SolveOpts:
    o = SolveOpts()
    lib.bem_solve_opts_default(ctypes.byref(o))
    return o


# formulations (BEM_FORM_*)
FORMULATIONS = {"osrc": 0, "pmchwt": 1, "calderon": 2, "muller": 3}


def pmchwt_solve(mesh: Mesh, k_ext, k_int, rho: float, directions, tol: float,
                 opts: Optional[SolveOpts] = None, stream=None, **overrides):
    """Strong-form solve of formulation "osrc" (default), "pmchwt",
    "calderon" or "muller"; returns (solution [n_waves, 2N] as [psi; phi],
    infos, rc)."""
    import torch
    d = np.ascontiguousarray(np.atleast_2d(directions), dtype=np.float64)
    o = default_opts() if opts is None else opts
    for k, v in overrides.items():
        if k == "precision":
            v = _PREC[v]
        if k == "formulation" and isinstance(v, str):
            v = FORMULATIONS[v]
        setattr(o, k, v)
    sol = torch.empty((d.shape[0], 2 * mesh.n_vertices), dtype=torch.complex128,
                      device="cuda")
    infos = (SolveInfo * d.shape[0])()
    rc = _check(lib.pmchwt_solve(mesh.handle, _c(k_ext), _c(k_int), float(rho),
                                 _np_ptr(d), d.shape[0], float(tol), ctypes.byref(o),
                                 _vp(sol.data_ptr()), ctypes.cast(infos, _vp),
                                 _stream(stream)))
    return sol, [i.as_dict() for i in infos], rc


def pmchwt_solve_multi(mesh: Mesh, k_ext, k_int, rho, directions, tol: float,
                       opts: Optional[SolveOpts] = None, stream=None, **overrides):
    """pmchwt_solve with object m's interior material (k_int[m], rho[m])."""
    import torch
    kc, rc = _materials(mesh, k_int, rho)
    d = np.ascontiguousarray(np.atleast_2d(directions), dtype=np.float64)
    o = default_opts() if opts is None else opts
    for k, v in overrides.items():
        if k == "precision":
            v = _PREC[v]
        if k == "formulation" and isinstance(v, str):
            v = FORMULATIONS[v]
        setattr(o, k, v)
    sol = torch.empty((d.shape[0], 2 * mesh.n_vertices), dtype=torch.complex128,
                      device="cuda")
    infos = (SolveInfo * d.shape[0])()
    rc_ = _check(lib.pmchwt_solve_multi(mesh.handle, _c(k_ext), ctypes.cast(kc, _vp),
                                        _np_ptr(rc), _np_ptr(d), d.shape[0], float(tol),
                                        ctypes.byref(o), _vp(sol.data_ptr()),
                                        ctypes.cast(infos, _vp), _stream(stream)))
    return sol, [i.as_dict() for i in infos], rc_


def far_field(mesh: Mesh, k_ext, solution, dirs, stream=None) -> np.ndarray:
    d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
    _dev_c128(solution, 2 * mesh.n_vertices, "solution")
    out = np.zeros(d.shape[0], np.complex128)
    _check(lib.bem_far_field(mesh.handle, _c(k_ext), _vp(solution.data_ptr()),
                             _np_ptr(d), d.shape[0], _np_ptr(out), _stream(stream)))
    return out


def pmchwt_field(mesh: Mesh, k_ext, k_int, rho, direction, solution, points,
                 stream=None):
    """Total field at points off the surface (device float64 [n, 3]) for the
    solution [psi; phi] of the plane wave along `direction`; returns
    (field complex128 [n], region int32 [n]: 0 outside, m + 1 inside object m),
    both on the device.  k_int and rho: one material for every object, or
    sequences with one per object (pmchwt_field_multi)."""
    import torch
    multi = np.ndim(k_int) > 0 or np.ndim(rho) > 0
    if multi:
        kc, rc = _materials(mesh, k_int, rho)
    if _dev_c128(solution, 2 * mesh.n_vertices, "solution") != 1:
        raise ValueError("solution must hold one vector [psi; phi] of 2N entries")
    if not (points.is_cuda and points.dtype == torch.float64 and points.is_contiguous()
            and points.dim() == 2 and points.shape[1] == 3):
        raise ValueError("points must be a contiguous float64 [n, 3] device tensor")
    n = points.shape[0]
    d = np.ascontiguousarray(direction, dtype=np.float64).reshape(3)
    out = torch.empty(n, dtype=torch.complex128, device=points.device)
    reg = torch.empty(n, dtype=torch.int32, device=points.device)
    if multi:
        _check(lib.pmchwt_field_multi(mesh.handle, _c(k_ext), ctypes.cast(kc, _vp), _np_ptr(rc),
                                      _np_ptr(d), _vp(solution.data_ptr()),
                                      _vp(points.data_ptr()), n, _vp(out.data_ptr()),
                                      _vp(reg.data_ptr()), _stream(stream)))
    else:
        _check(lib.pmchwt_field(mesh.handle, _c(k_ext), _c(k_int), float(rho), _np_ptr(d),
                                _vp(solution.data_ptr()), _vp(points.data_ptr()), n,
                                _vp(out.data_ptr()), _vp(reg.data_ptr()), _stream(stream)))
    return out, reg


class Server:
    """Serving loop (bem_server_*): queued solves on worker streams with
    device-memory admission and resident per-mesh state."""

    def __init__(self, hbm_budget: int = 0, workers: int = 4, max_replicas: int = 0,
                 dense_max_bytes: int = -1):
        o = ServerOpts()
        lib.bem_server_opts_default(ctypes.byref(o))
        o.hbm_budget, o.workers = int(hbm_budget), int(workers)
        o.max_replicas, o.dense_max_bytes = int(max_replicas), int(dense_max_bytes)
        h = _vp()
        self._h = None
        _check(lib.bem_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._meshes = {}      # mesh id -> number of vertices
        self._pending = {}     # request id -> (solution tensor, info array)

    def add_mesh(self, vertices, triangles, object_id=None) -> int:
        P = np.ascontiguousarray(vertices, dtype=np.float64)
        T = np.ascontiguousarray(triangles, dtype=np.int32)
        O = None if object_id is None else np.ascontiguousarray(object_id, np.int32)
        if P.ndim != 2 or P.shape[1] != 3 or T.ndim != 2 or T.shape[1] != 3:
            raise ValueError("vertices [N,3] and triangles [T,3] expected")
        mid = ctypes.c_int()
        _check(lib.bem_server_add_mesh(self._h, _np_ptr(P), P.shape[0], _np_ptr(T), T.shape[0],
                                       _np_ptr(O) if O is not None else None, ctypes.byref(mid)))
        self._meshes[mid.value] = P.shape[0]
        return mid.value

    def submit(self, mesh_id: int, k_ext, k_int, rho: float, directions, tol: float,
               opts: Optional[SolveOpts] = None, **overrides) -> int:
        import torch
        d = np.ascontiguousarray(np.atleast_2d(directions), dtype=np.float64)
        o = default_opts() if opts is None else opts
        for k, v in overrides.items():
            if k == "precision":
                v = _PREC[v]
            if k == "formulation" and isinstance(v, str):
                v = FORMULATIONS[v]
            setattr(o, k, v)
        n = self._meshes.get(mesh_id, 1)   # an unknown id is rejected by the library
        sol = torch.empty((d.shape[0], 2 * n), dtype=torch.complex128, device="cuda")
        infos = (SolveInfo * d.shape[0])()
        rid = _i64()
        if np.ndim(k_int) > 0 or np.ndim(rho) > 0:   # a material per object
            k = np.atleast_1d(np.asarray(k_int, dtype=np.complex128))
            kc = (c64 * len(k))(*[c64(v.real, v.imag) for v in k])
            rc = np.ascontiguousarray(np.atleast_1d(rho), dtype=np.float64)
            if len(k) != len(rc):
                raise ValueError("k_int and rho need one entry per object")
            _check(lib.bem_server_submit_multi(self._h, int(mesh_id), _c(k_ext),
                                               ctypes.cast(kc, _vp), _np_ptr(rc), _np_ptr(d),
                                               d.shape[0], float(tol), ctypes.byref(o),
                                               _vp(sol.data_ptr()), ctypes.cast(infos, _vp),
                                               ctypes.byref(rid)))
        else:
            _check(lib.bem_server_submit(self._h, int(mesh_id), _c(k_ext), _c(k_int), float(rho),
                                         _np_ptr(d), d.shape[0], float(tol), ctypes.byref(o),
                                         _vp(sol.data_ptr()), ctypes.cast(infos, _vp),
                                         ctypes.byref(rid)))
        self._pending[rid.value] = (sol, infos)
        return rid.value

    def wait(self, request_id: int, timeout: float = -1.0):
        """(solution, infos, stats) when done, None on time-out."""
        st = RequestStats()
        rc = _check(lib.bem_server_wait(self._h, int(request_id), float(timeout),
                                        ctypes.byref(st)))
        if rc == 2:
            return None
        sol, infos = self._pending.pop(request_id)
        stats = st.as_dict()
        if st.status < 0:
            stats["error"] = f"{ERRORS.get(st.status, st.status)}: {lib.bem_last_error().decode()}"
        return sol, [i.as_dict() for i in infos], stats

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib.bem_server_stats_get(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib.bem_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def profile_enable(on: bool = True):
    _check(lib.bem_profile_enable(1 if on else 0))


def profile_read(kernel: str):
    ms, n = ctypes.c_double(), _i64()
    _check(lib.bem_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def autotune(mesh: Mesh, k_ext, k_int, rho: float, n_rhs: int = 1,
             expected_matvecs: int = 50, stream=None) -> dict:
    """Time the launch choices on the device; the result is used from now on
    for this mesh size and right-hand-side bucket."""
    e = TuneEntry()
    _check(lib.bem_autotune(mesh.handle, _c(k_ext), _c(k_int), float(rho), int(n_rhs),
                            int(expected_matvecs), ctypes.byref(e), _stream(stream)))
    return e.as_dict()


def tune_cache_load(path: str, arch: Optional[str] = None) -> int:
    n = ctypes.c_int()
    _check(lib.bem_tune_cache_load(path.encode(), arch.encode() if arch else None,
                                   ctypes.byref(n)))
    return n.value


def tune_lookup(n_triangles: int, n_rhs: int = 1):
    """(entry, tuned): the autotuned entry, or the defaults with tuned False."""
    e = TuneEntry()
    rc = _check(lib.bem_tune_lookup(int(n_triangles), int(n_rhs), ctypes.byref(e)))
    return e.as_dict(), rc == 0


def tune_clear():
    lib.bem_tune_clear()


def hmat_info(mesh: Mesh, k_ext, k_int, rho: float, stream=None) -> dict:
    """Size and set-up time of the compressed operator (precision
    "fp32_hmat") of a wavenumber pair; builds it if needed."""
    st = HMatStats()
    _check(lib.bem_hmat_info(mesh.handle, _c(k_ext), _c(k_int), float(rho), ctypes.byref(st),
                             _stream(stream)))
    return st.as_dict()


def tune_set(key: str, value: int):
    _check(lib.bem_tune_set(key.encode(), int(value)))


def tune_get(key: str) -> int:
    v = _i64()
    _check(lib.bem_tune_get(key.encode(), ctypes.byref(v)))
    return v.value


def valu_rates(stream=None) -> dict:
    """Measured issue rates (lane operations/s over the device)."""
    r = np.zeros(5, np.float64)
    _check(lib.bem_valu_rates(_np_ptr(r), _stream(stream)))
    return dict(zip(("fma_f32", "sin_f32", "cos_f32", "rsq_f32", "fma_f64"), r.tolist()))


def exported_symbols(names: Sequence[str]):
    """Names among `names` that the loaded library does not export."""
    missing = []
    for n in names:
        try:
            getattr(lib, n)
        except AttributeError:
            missing.append(n)
    return missing
