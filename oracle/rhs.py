"""Plane-wave right-hand side and far field (oracle only).

Incident plane wave of unit amplitude u_inc = exp(i k_ext d . x) (Sec. 2.1).
Weak right-hand side of the permuted PMCHWT (Sec. 2.7):
    f_D,i = int u_inc phi_i,     f_N,i = int (d/dn) u_inc phi_i
          = int i k_ext (d . n) exp(i k_ext d . x) phi_i,
both with the 6-point triangle rule.

Far field: with the exterior representation formula (Sec. 2.2) and the
surface potentials psi~+ = -psi, phi~+ = -phi (psi, phi = exterior traces of
the total field), u_sca(x) ~ F(x^) exp(i k r)/r with
    F(x^) = 1/(4 pi) int exp(-i k x^ . y) [ -psi(y) - i k (x^ . n_y) phi(y) ] dy.
"""
from __future__ import annotations

import numpy as np

from .osrc import triangle_geometry
from .quadrature import dunavant6


def _points(mesh):
    bary, w = dunavant6()
    P, T = mesh.vertices, mesh.triangles
    X = np.einsum("qa,tac->tqc", bary, P[T])       # [T, 6, 3]
    return bary, w, X


def plane_wave_rhs(mesh, k_ext, d):
    """Weak [f_D; f_N] (complex [2N]) for unit direction d."""
    d = np.asarray(d, float)
    area, n = triangle_geometry(mesh)
    bary, w, X = _points(mesh)
    T = mesh.triangles
    N = mesh.n_vertices
    u = np.exp(1j * k_ext * X @ d)                  # [T, 6]
    dn = 1j * k_ext * (n @ d)                       # [T]
    fD = np.zeros(N, np.complex128)
    fN = np.zeros(N, np.complex128)
    for a in range(3):
        cD = area * np.einsum("q,tq->t", w * bary[:, a], u)
        np.add.at(fD, T[:, a], cD)
        np.add.at(fN, T[:, a], cD * dn)
    return np.concatenate([fD, fN])


def far_field(mesh, k_ext, x, dirs):
    """F(x^) for unit directions dirs [m, 3]; x = [psi; phi] coefficients."""
    area, n = triangle_geometry(mesh)
    bary, w, X = _points(mesh)
    T = mesh.triangles
    N = mesh.n_vertices
    psi = bary @ x[:N][T].T                          # [6, T]
    phi = bary @ x[N:][T].T
    out = []
    for xh in np.atleast_2d(dirs):
        e = np.exp(-1j * k_ext * (X @ xh))          # [T, 6]
        integ = -psi.T - 1j * k_ext * (n @ xh)[:, None] * phi.T
        out.append(np.sum(area[:, None] * w[None, :] * e * integ) / (4 * np.pi))
    return np.array(out)
