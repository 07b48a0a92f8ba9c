"""Series solution of plane-wave transmission through a penetrable sphere.

Used as the end-to-end pin (the paper compares with the analytic solution of
a sphere, Sec. 3.2).  Sphere of radius a at the origin, incident
u_inc = exp(i k0 z) = sum i^n (2n+1) j_n(k0 r) P_n(cos t),
u_sca = sum i^n (2n+1) A_n h_n(k0 r) P_n,  u_int = sum i^n (2n+1) B_n j_n(k1 r) P_n.
The transmission conditions of the Helmholtz system (Sec. 2.1): continuity of
u and of (1/rho) du/dr at r = a.  With g = k1 rho0 / (k0 rho1):
    A_n = [g j_n(k0a) j_n'(k1a) - j_n'(k0a) j_n(k1a)]
          / [h_n'(k0a) j_n(k1a) - g h_n(k0a) j_n'(k1a)],
    B_n = [j_n(k0a) + A_n h_n(k0a)] / j_n(k1a).
Far field (u_sca ~ F exp(i k0 r)/r): F(t) = (-i/k0) sum (2n+1) A_n P_n(cos t).
Total field at a point: u_inc + u_sca outside, u_int inside.
"""
from __future__ import annotations

import numpy as np
from scipy.special import eval_legendre, spherical_jn, spherical_yn


def _h(n, x, derivative=False):
    return spherical_jn(n, x, derivative) + 1j * spherical_yn(n, x, derivative)


def n_terms(k0, k1, a):
    ka = max(abs(k0), abs(k1)) * a
    return int(ka + 4.0 * ka ** (1.0 / 3.0) + 10)


def coefficients(k0, k1, rho, a=1.0, nmax=None):
    """(A_n, B_n) for n = 0..nmax; rho = rho_int / rho_ext."""
    nmax = n_terms(k0, k1, a) if nmax is None else nmax
    n = np.arange(nmax + 1)
    x0, x1 = k0 * a, k1 * a
    g = k1 / (k0 * rho)
    j0, dj0 = spherical_jn(n, x0), spherical_jn(n, x0, True)
    h0, dh0 = _h(n, x0), _h(n, x0, True)
    j1, dj1 = spherical_jn(n, x1), spherical_jn(n, x1, True)
    A = (g * j0 * dj1 - dj0 * j1) / (dh0 * j1 - g * h0 * dj1)
    B = (j0 + A * h0) / j1
    return A, B


def far_field(k0, k1, rho, theta, a=1.0):
    A, _ = coefficients(k0, k1, rho, a)
    n = np.arange(len(A))
    c = np.cos(np.atleast_1d(theta))
    P = np.array([eval_legendre(m, c) for m in n])  # [n, m]
    return (-1j / k0) * ((2 * n + 1) * A) @ P


def surface_traces(k0, k1, rho, cos_t, a=1.0):
    """(phi, psi) on r = a: Dirichlet trace and exterior Neumann trace."""
    A, B = coefficients(k0, k1, rho, a)
    n = np.arange(len(A))
    P = np.array([eval_legendre(m, np.asarray(cos_t)) for m in n])
    c = (1j ** n) * (2 * n + 1)
    phi = (c * B * spherical_jn(n, k1 * a)) @ P
    psi = k0 * (c * (spherical_jn(n, k0 * a, True) + A * _h(n, k0 * a, True))) @ P
    return phi, psi


def total_field(k0, k1, rho, points, a=1.0):
    """Total field at points [m, 3] (sphere at the origin, wave along +z)."""
    p = np.atleast_2d(np.asarray(points, float))
    r = np.linalg.norm(p, axis=1)
    ct = np.where(r > 0, p[:, 2] / np.where(r > 0, r, 1.0), 1.0)
    A, B = coefficients(k0, k1, rho, a)
    n = np.arange(len(A))
    c = (1j ** n) * (2 * n + 1)
    P = np.array([eval_legendre(m, ct) for m in n])          # [n, m]
    out = np.empty(len(p), np.complex128)
    ext = r >= a
    for sel, inside in ((ext, False), (~ext, True)):
        if not sel.any():
            continue
        rs = r[sel][None, :]
        nn = n[:, None]
        if inside:
            out[sel] = np.sum(c[:, None] * B[:, None] * spherical_jn(nn, k1 * rs) * P[:, sel],
                              axis=0)
        else:
            # the incident wave in closed form (its series needs ~k0 r terms)
            us = np.sum(c[:, None] * A[:, None] * _h(nn, k0 * rs) * P[:, sel], axis=0)
            out[sel] = np.exp(1j * k0 * p[sel, 2]) + us
    return out
