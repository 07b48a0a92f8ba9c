"""Closed-form potential of a uniformly charged flat triangle (test helper).

Phi(x) = int_T 1/|x - y| dS_y, from the edge decomposition of the Laplace
potential of a planar polygon (Wilton, Rao, Glisson, Schaubert, Al-Bundak,
Butler, IEEE TAP 1984, eq. for constant sources):  for edges i with endpoints
p-, p+, unit direction l, in-plane outward unit normal u = l x n,
  P0 = (p - rho) . u,   l+- = (p+- - rho) . l,   R+- = |x - p+-|,
  R0^2 = P0^2 + d^2,  d = (x - p) . n,  rho = projection of x on the plane,
Phi = sum_i P0 ln((R+ + l+)/(R- + l-))
      - |d| sum_i [atan(P0 l+ / (R0^2 + |d| R+)) - atan(P0 l- / (R0^2 + |d| R-))].
"""
import numpy as np


def triangle_potential(tri, x):
    tri = np.asarray(tri, float)
    x = np.asarray(x, float)
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n /= np.linalg.norm(n)
    d = np.dot(x - tri[0], n)
    rho = x - d * n
    ad = abs(d)
    total = 0.0
    for i in range(3):
        pm, pp = tri[i], tri[(i + 1) % 3]
        L = pp - pm
        l = L / np.linalg.norm(L)
        u = np.cross(l, n)
        P0 = np.dot(pm - rho, u)
        lm = np.dot(pm - rho, l)
        lp = np.dot(pp - rho, l)
        Rm = np.linalg.norm(x - pm)
        Rp = np.linalg.norm(x - pp)
        R02 = P0 * P0 + d * d
        if abs(P0) > 1e-300:
            total += P0 * np.log((Rp + lp) / (Rm + lm))
        if ad > 0:
            total -= ad * (np.arctan(P0 * lp / (R02 + ad * Rp)) -
                           np.arctan(P0 * lm / (R02 + ad * Rm)))
    return total


def triangle_rule(tri, n):
    """Collapsed-square Gauss rule on a triangle: points [m,3], weights [m]."""
    t, w = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (t + 1)
    w = 0.5 * w
    tri = np.asarray(tri, float)
    area = 0.5 * np.linalg.norm(np.cross(tri[1] - tri[0], tri[2] - tri[0]))
    pts, wts = [], []
    for s, ws in zip(t, w):
        for r, wr in zip(t, w):
            # x = A + s (B - A) + s r (C - B), Jacobian 2|T| s
            p = tri[0] + s * (tri[1] - tri[0]) + s * r * (tri[2] - tri[1])
            pts.append(p)
            wts.append(ws * wr * s * 2 * area)
    return np.array(pts), np.array(wts)
