"""Field off the surface from a boundary solution (oracle only; test
infrastructure, not part of the product path).

Representation formulas (Sec. 2.2) with the surface potentials of the total
field, psi~+ = -psi, phi~+ = -phi on the exterior side and psi~- = rho psi,
phi~- = phi on the interior side (psi = exterior Neumann trace, phi =
Dirichlet trace; the interior Neumann trace is rho_int/rho_ext times the
exterior one):

    outside every object:  u = u_inc + sum over all triangles of
        int [ -G_0(p, y) psi(y) + (n_y . grad_y G_0(p, y)) phi(y) ] dy
    inside object m:       u = int over object m's surface of
        [ rho G_m(p, y) psi(y) - (n_y . grad_y G_m(p, y)) phi(y) ] dy

with n_y . grad_y G(p, y) = ((y - p) . n_y) G(r) (i k r - 1) / r^2 and
G = e^{ikr} / (4 pi r).  psi, phi are the P1 functions of the coefficients;
the 6-point rule per triangle is used.

A point lies inside object m when the solid angle that m's closed surface
subtends at it is 4 pi (0 outside).  Solid angle of a flat triangle with
vertices a, b, c seen from the origin (Van Oosterom and Strackee, 1983):
    tan(Omega / 2) = a . (b x c) / (|a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|).
"""
from __future__ import annotations

import numpy as np

from .osrc import triangle_geometry
from .quadrature import dunavant6


def solid_angles(mesh, points):
    """[n_points, n_objects] solid angle of each object's surface, / 4 pi."""
    P, T = mesh.vertices, mesh.triangles
    obj = np.zeros(len(T), int) if mesh.object_id is None else mesh.object_id
    nobj = mesh.n_objects()
    out = np.zeros((len(points), nobj))
    for i, p in enumerate(np.atleast_2d(points)):
        a, b, c = P[T[:, 0]] - p, P[T[:, 1]] - p, P[T[:, 2]] - p
        la, lb, lc = (np.linalg.norm(v, axis=1) for v in (a, b, c))
        num = np.einsum("ij,ij->i", a, np.cross(b, c))
        den = (la * lb * lc + np.einsum("ij,ij->i", a, b) * lc +
               np.einsum("ij,ij->i", a, c) * lb + np.einsum("ij,ij->i", b, c) * la)
        om = 2.0 * np.arctan2(num, den)
        for o in range(nobj):
            out[i, o] = om[obj == o].sum() / (4 * np.pi)
    return out


def regions(mesh, points):
    """0 outside every object, m + 1 inside object m."""
    w = np.abs(solid_angles(mesh, points))
    r = np.zeros(len(w), int)
    inside = w.max(axis=1) > 0.5
    r[inside] = np.argmax(w[inside], axis=1) + 1
    return r


def _sources(mesh, x):
    """Quadrature points [T, 6, 3], w |tau| psi_h and w |tau| phi_h [T, 6]."""
    bary, w = dunavant6()
    P, T = mesh.vertices, mesh.triangles
    N = mesh.n_vertices
    area, n = triangle_geometry(mesh)
    Y = np.einsum("qa,tac->tqc", bary, P[T])
    wa = area[:, None] * w[None, :]
    psi = wa * (x[:N][T] @ bary.T)
    phi = wa * (x[N:][T] @ bary.T)
    return Y, n, psi, phi


def layer_potentials(mesh, k, x, points, tri_mask=None):
    """(S psi, D phi) at points: single layer int G psi and double layer
    int (n_y . grad_y G) phi over the triangles in tri_mask (all if None)."""
    Y, n, psi, phi = _sources(mesh, x)
    if tri_mask is not None:
        Y, n, psi, phi = Y[tri_mask], n[tri_mask], psi[tri_mask], phi[tri_mask]
    S = np.zeros(len(points), np.complex128)
    D = np.zeros(len(points), np.complex128)
    for i, p in enumerate(np.atleast_2d(points)):
        d = Y - p                                     # y - p  [T, 6, 3]
        r = np.linalg.norm(d, axis=2)
        G = np.exp(1j * k * r) / (4 * np.pi * r)
        dG = np.einsum("tqc,tc->tq", d, n) * G * (1j * k * r - 1) / r ** 2
        S[i] = np.sum(G * psi)
        D[i] = np.sum(dG * phi)
    return S, D


def field(mesh, k_ext, k_int, rho, x, d, points):
    """Total field at points for the solution x = [psi; phi] of the plane
    wave exp(i k_ext d . p).  k_int, rho: one material, or one per object."""
    points = np.atleast_2d(np.asarray(points, float))
    d = np.asarray(d, float)
    reg = regions(mesh, points)
    obj = np.zeros(mesh.n_triangles, int) if mesh.object_id is None else mesh.object_id
    u = np.zeros(len(points), np.complex128)
    ext = reg == 0
    if ext.any():
        S, D = layer_potentials(mesh, k_ext, x, points[ext])
        u[ext] = np.exp(1j * k_ext * points[ext] @ d) - S + D
    nobj = mesh.n_objects()
    ks = np.broadcast_to(np.asarray(k_int, np.complex128), (nobj,))
    rs = np.broadcast_to(np.asarray(rho, float), (nobj,))
    for m in range(nobj):
        sel = reg == m + 1
        if sel.any():
            S, D = layer_potentials(mesh, ks[m], x, points[sel], tri_mask=obj == m)
            u[sel] = rs[m] * S - D
    return u, reg
