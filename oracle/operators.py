"""Dense Galerkin P1 operators and the permuted PMCHWT matrix (oracle only).

Permuted PMCHWT, single scatterer, unknowns [psi; phi] with
psi = exterior Neumann trace, phi = Dirichlet trace of the total field
(Sec. 2.2, unique pair of traces; Sec. 2.7, permuted formulation):

    B = [[ V_0 + rho V_1 ,  -(K_0 + K_1)        ],
         [ K'_0 + K'_1   ,   D_0 + D_1 / rho    ]],   rho = rho_int / rho_ext,

right-hand side [gamma_D u_inc; gamma_N u_inc].  The Mueller operator
(Sec. 2.2) is built on the same unknowns by muller_matrix.  Exterior operators (index 0)
couple all triangles; interior ones (index 1) act within each object only
(Sec. 2.7, multiple scattering).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import quadrature as Q
from .build import LIB, build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        _lib = ctypes.CDLL(LIB)
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Rules:
    def __init__(self, n_ss: int = 4):
        bary, w = Q.dunavant6()
        self.reg = np.ascontiguousarray(np.hstack([bary, w[:, None]]))
        self.tabs = [np.ascontiguousarray(t) for t in Q.singular_rules(n_ss)]


_RULES = {}


def rules(n_ss: int = 4) -> Rules:
    if n_ss not in _RULES:
        _RULES[n_ss] = Rules(n_ss)
    return _RULES[n_ss]


def _mesh_args(mesh):
    P = np.ascontiguousarray(mesh.vertices, dtype=np.float64)
    T = np.ascontiguousarray(mesh.triangles, dtype=np.int32)
    obj = None if mesh.object_id is None else \
        np.ascontiguousarray(mesh.object_id, dtype=np.int32)
    return P, T, obj


def assemble(mesh, k, interior=False, n_ss=4):
    """Dense V, K, K', D at wavenumber k: dict of complex [N, N]."""
    lib = _load()
    R = rules(n_ss)
    P, T, obj = _mesh_args(mesh)
    nv, nt = P.shape[0], T.shape[0]
    outs = [np.zeros((nv, nv), np.complex128) for _ in range(4)]
    k = complex(k)
    lib.oracle_assemble_dense(
        _ptr(P), ctypes.c_int(nv), _ptr(T), ctypes.c_int(nt),
        _ptr(obj) if obj is not None else None, ctypes.c_int(int(interior)),
        ctypes.c_double(k.real), ctypes.c_double(k.imag), _ptr(R.reg),
        _ptr(R.tabs[0]), ctypes.c_int(len(R.tabs[0])),
        _ptr(R.tabs[1]), ctypes.c_int(len(R.tabs[1])),
        _ptr(R.tabs[2]), ctypes.c_int(len(R.tabs[2])),
        *[_ptr(o) for o in outs])
    return dict(V=outs[0], K=outs[1], Kp=outs[2], D=outs[3])


def pmchwt_blocks(ops0, ops1, rho):
    """Combine exterior (ops0) and interior (ops1) operators into B."""
    B11 = ops0["V"] + rho * ops1["V"]
    B12 = -(ops0["K"] + ops1["K"])
    B21 = ops0["Kp"] + ops1["Kp"]
    B22 = ops0["D"] + ops1["D"] / rho
    return np.block([[B11, B12], [B21, B22]])


def pmchwt_matrix(mesh, k_ext, k_int, rho, n_ss=4):
    """Weak-form permuted PMCHWT matrix, complex [2N, 2N]."""
    ops0 = assemble(mesh, k_ext, interior=False, n_ss=n_ss)
    ops1 = assemble(mesh, k_int, interior=True, n_ss=n_ss)
    return pmchwt_blocks(ops0, ops1, rho)


def vertex_objects(mesh):
    """Object of each vertex (objects are disjoint closed surfaces)."""
    v = np.zeros(mesh.n_vertices, int)
    if mesh.object_id is not None:
        for o in range(mesh.n_objects()):
            v[np.unique(mesh.triangles[mesh.object_id == o])] = o
    return v


def pmchwt_matrix_multi(mesh, k_ext, k_int, rho, n_ss=4):
    """Permuted PMCHWT matrix with object m's own interior material
    (k_int[m], rho[m]) (Sec. 2.7, several scatterers): the exterior operators
    couple all objects, the interior operators of object m are taken at
    k_int[m] and weighted by rho[m] and 1/rho[m]."""
    ops0 = assemble(mesh, k_ext, interior=False, n_ss=n_ss)
    B11, B12 = ops0["V"].copy(), -ops0["K"]
    B21, B22 = ops0["Kp"].copy(), ops0["D"].copy()
    vobj = vertex_objects(mesh)
    for m in range(mesh.n_objects()):
        ops1 = assemble(mesh, k_int[m], interior=True, n_ss=n_ss)
        sel = vobj == m
        mask = np.outer(sel, sel)
        B11 = B11 + rho[m] * ops1["V"] * mask
        B12 = B12 - ops1["K"] * mask
        B21 = B21 + ops1["Kp"] * mask
        B22 = B22 + ops1["D"] / rho[m] * mask
    return np.block([[B11, B12], [B21, B22]])


def muller_blocks(ops0, ops1, rho, M):
    """Combine exterior (ops0) and interior (ops1) operators and the P1 mass
    matrix M into the weak Mueller operator (I + A_0 - A^_1) of Sec. 2.2 on the
    permuted unknowns [psi; phi] of B: the interior terms enter with the
    opposite sign, and the identity, tested in both trace rows against P1
    functions, is M acting on the row's own trace (phi in the first row, psi
    in the second), i.e. on the off-diagonal blocks after the permutation."""
    B11 = ops0["V"] - rho * ops1["V"]
    B12 = M - (ops0["K"] - ops1["K"])
    B21 = M + (ops0["Kp"] - ops1["Kp"])
    B22 = ops0["D"] - ops1["D"] / rho
    return np.block([[B11, B12], [B21, B22]])


def muller_matrix(mesh, k_ext, k_int, rho, n_ss=4):
    """Weak-form Mueller matrix on the permuted unknowns, complex [2N, 2N].
    k_int, rho: one material, or one per object (object m's interior terms at
    k_int[m] with rho[m])."""
    from .osrc import mass_matrix
    M = mass_matrix(mesh).toarray()
    ops0 = assemble(mesh, k_ext, interior=False, n_ss=n_ss)
    if np.ndim(k_int) == 0 and np.ndim(rho) == 0:
        ops1 = assemble(mesh, k_int, interior=True, n_ss=n_ss)
        return muller_blocks(ops0, ops1, rho, M)
    B11, B12 = ops0["V"].copy(), M - ops0["K"]
    B21, B22 = M + ops0["Kp"], ops0["D"].copy()
    vobj = vertex_objects(mesh)
    for m in range(mesh.n_objects()):
        ops1 = assemble(mesh, k_int[m], interior=True, n_ss=n_ss)
        sel = vobj == m
        mask = np.outer(sel, sel)
        B11 = B11 - rho[m] * ops1["V"] * mask
        B12 = B12 + ops1["K"] * mask
        B21 = B21 - ops1["Kp"] * mask
        B22 = B22 - ops1["D"] / rho[m] * mask
    return np.block([[B11, B12], [B21, B22]])


def _matvec_tris(mesh, k, interior, test, xs, n_ss=4):
    lib = _load()
    R = rules(n_ss)
    P, T, obj = _mesh_args(mesh)
    test = np.ascontiguousarray(test, dtype=np.int32)
    xs = [np.ascontiguousarray(x, dtype=np.complex128) for x in xs]
    out = np.zeros((len(test), 4, 3), np.complex128)
    k = complex(k)
    lib.oracle_matvec_tris(
        _ptr(P), ctypes.c_int(P.shape[0]), _ptr(T), ctypes.c_int(T.shape[0]),
        _ptr(obj) if obj is not None else None, ctypes.c_int(int(interior)),
        ctypes.c_double(k.real), ctypes.c_double(k.imag), _ptr(R.reg),
        _ptr(R.tabs[0]), ctypes.c_int(len(R.tabs[0])),
        _ptr(R.tabs[1]), ctypes.c_int(len(R.tabs[1])),
        _ptr(R.tabs[2]), ctypes.c_int(len(R.tabs[2])),
        _ptr(test), ctypes.c_int(len(test)), *[_ptr(x) for x in xs],
        _ptr(out))
    return out


def pmchwt_matvec_rows(mesh, k_ext, k_int, rho, x, rows, n_ss=4):
    """Rows `rows` (vertex indices) of both block rows of y = B x, matrix-free.

    x = [psi; phi] complex [2N].  Returns (y1[rows], y2[rows]).  k_int, rho:
    one material, or one per object (a test triangle's interior terms at its
    object's k_int[m], rho[m]).
    """
    N = mesh.n_vertices
    psi, phi = x[:N], x[N:]
    rows = np.asarray(rows)
    T = mesh.triangles
    mask = np.isin(T, rows).any(axis=1)
    test = np.nonzero(mask)[0]
    o0 = _matvec_tris(mesh, k_ext, False, test, (psi, phi, psi, phi), n_ss)
    if np.ndim(k_int) == 0 and np.ndim(rho) == 0:
        o1 = _matvec_tris(mesh, k_int, True, test, (psi, phi, psi, phi), n_ss)
        rt = np.full(len(test), float(rho))
    else:
        obj = mesh.object_id[test]
        o1 = np.zeros_like(o0)
        for m in np.unique(obj):
            sel = obj == m
            o1[sel] = _matvec_tris(mesh, k_int[m], True, test[sel], (psi, phi, psi, phi), n_ss)
        rt = np.asarray(rho, float)[obj]
    r1 = (o0[:, 0] + rt[:, None] * o1[:, 0]) - (o0[:, 1] + o1[:, 1])
    r2 = (o0[:, 2] + o1[:, 2]) + (o0[:, 3] + o1[:, 3] / rt[:, None])
    y1 = np.zeros(N, np.complex128)
    y2 = np.zeros(N, np.complex128)
    tv = T[test]
    for a in range(3):
        np.add.at(y1, tv[:, a], r1[:, a])
        np.add.at(y2, tv[:, a], r2[:, a])
    return y1[rows], y2[rows]


def pair_kernel_integral(vx, vy, which, px, py, k, power, n_ss=4):
    """Singular-rule integral of exp(ikr)/r^power over one triangle pair."""
    lib = _load()
    tab = np.ascontiguousarray(Q.singular_rules(n_ss)[which])
    res = np.zeros(2)
    lib.oracle_pair_kernel(
        _ptr(np.ascontiguousarray(vx, np.float64)),
        _ptr(np.ascontiguousarray(vy, np.float64)), ctypes.c_int(which),
        _ptr(tab), ctypes.c_int(len(tab)),
        _ptr(np.ascontiguousarray(px, np.int32)),
        _ptr(np.ascontiguousarray(py, np.int32)),
        ctypes.c_double(complex(k).real), ctypes.c_double(complex(k).imag),
        ctypes.c_int(power), _ptr(res))
    return res[0] + 1j * res[1]


def muller_matvec_rows(mesh, k_ext, k_int, rho, x, rows, n_ss=4):
    """Rows `rows` of both block rows of y = B_M x (Mueller operator of
    muller_blocks), matrix-free: interior terms with the opposite sign, plus
    the P1 mass matrix applied to the row's own trace (phi in the first row,
    psi in the second).  x = [psi; phi] complex [2N].  Returns (y1[rows],
    y2[rows])."""
    from .osrc import mass_matrix
    N = mesh.n_vertices
    psi, phi = x[:N], x[N:]
    rows = np.asarray(rows)
    T = mesh.triangles
    mask = np.isin(T, rows).any(axis=1)
    test = np.nonzero(mask)[0]
    o0 = _matvec_tris(mesh, k_ext, False, test, (psi, phi, psi, phi), n_ss)
    o1 = _matvec_tris(mesh, k_int, True, test, (psi, phi, psi, phi), n_ss)
    r1 = (o0[:, 0] - rho * o1[:, 0]) - (o0[:, 1] - o1[:, 1])
    r2 = (o0[:, 2] - o1[:, 2]) + (o0[:, 3] - o1[:, 3] / rho)
    y1 = np.zeros(N, np.complex128)
    y2 = np.zeros(N, np.complex128)
    tv = T[test]
    for a in range(3):
        np.add.at(y1, tv[:, a], r1[:, a])
        np.add.at(y2, tv[:, a], r2[:, a])
    M = mass_matrix(mesh)
    return y1[rows] + M[rows] @ phi, y2[rows] + M[rows] @ psi
