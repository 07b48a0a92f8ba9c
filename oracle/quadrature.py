"""Quadrature rules of the oracle (test infrastructure only).

Reference triangle used for singular rules:  K = {(x1, x2): 0 <= x2 <= x1 <= 1}
with vertices (0,0)->A, (1,0)->B, (1,1)->C, map  chi(x) = A + x1 (B-A) + x2 (C-B)
(|det D chi| = 2|tau|) and barycentric coordinates
(lambda_A, lambda_B, lambda_C) = (1 - x1, x1 - x2, x2).

Singular rules integrate f over K x K.  Their weights sum to |K|^2 = 1/4; a
physical pair integral is 4 |tau| |sigma| times the rule's sum.  All three
rules are tensor Gauss-Legendre rules on [0,1]^4 composed with maps that make
the integrand smooth (Sauter & Schwab, Boundary Element Methods, Sec. 5.2, as
the paper's Galerkin discretisation (Sec. 2.3) requires for weakly singular
kernels).  The maps are derived from relative coordinates:

  coincident  (6 regions):  z = y - x runs over the hexagon K - K, cut into the
      six sectors on which g(z) = max(0,z1) + max(0,-z2) + max(0,z2-z1) is
      linear; z = xi * (v_i + eta (v_{i+1} - v_i)); for fixed z the admissible
      x form the triangle K n (K - z), a copy of K scaled by s = 1 - xi.
      Weight  xi (1-xi)^2 alpha.
  common edge (4 regions): shared edge = reference edge A-B of both triangles;
      w = (y1 - x1, x2, y2) is blown up radially with respect to the gauge
      m(w) = max(z1 + x2, y2) (z1 >= 0, two faces) and its mirror (z1 < 0);
      the remaining coordinate runs over an interval of length 1 - xi.
      Weights  xi^2 (1-xi)  and  xi^2 (1-xi) u.
  common vertex (2 regions): shared vertex = A of both; x = x1 (1, u),
      y = y1 (1, v), split at x1 = y1.  Weight  xi^3 eta.

In every region the distance |chi_tau(x) - chi_sigma(y)| is xi times a
smooth positive function, so 1/r, the double-layer kernels and the Maue-form
hypersingular kernel become smooth integrands.
"""
from __future__ import annotations

import numpy as np

# Dunavant (1985) symmetric 6-point rule of degree 4, barycentric orbits
# (1-2a, a, a); weights sum to 1.
_DUN_A1 = 0.44594849091596488631832925388305
_DUN_W1 = 0.22338158967801146569500700843312
_DUN_A2 = 0.091576213509770743459571463402202
_DUN_W2 = 0.10995174365532186763832632490021


def dunavant6():
    """(bary [6,3], weights [6]) with sum(weights) = 1."""
    pts, wts = [], []
    for a, w in ((_DUN_A1, _DUN_W1), (_DUN_A2, _DUN_W2)):
        b = 1.0 - 2.0 * a
        for p in ((b, a, a), (a, b, a), (a, a, b)):
            pts.append(p)
            wts.append(w)
    return np.array(pts), np.array(wts)


def gauss01(n: int):
    """Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _grid4(n):
    t, w = gauss01(n)
    a, b, c, d = np.meshgrid(t, t, t, t, indexing="ij")
    wa, wb, wc, wd = np.meshgrid(w, w, w, w, indexing="ij")
    return (a.ravel(), b.ravel(), c.ravel(), d.ravel(),
            (wa * wb * wc * wd).ravel())


_HEX = np.array([(1, 0), (1, 1), (0, 1), (-1, 0), (-1, -1), (0, -1)], float)


def rule_coincident(n: int = 4):
    """Rows (x1, x2, y1, y2, w) for tau == sigma (same vertex order A,B,C)."""
    xi, eta, al, be, w4 = _grid4(n)
    rows = []
    for i in range(6):
        v0, v1 = _HEX[i], _HEX[(i + 1) % 6]
        jac = abs(v0[0] * (v1[1] - v0[1]) - v0[1] * (v1[0] - v0[0]))
        z1 = xi * (v0[0] + eta * (v1[0] - v0[0]))
        z2 = xi * (v0[1] + eta * (v1[1] - v0[1]))
        a = np.maximum(0.0, -z2)
        b = np.maximum(0.0, z2 - z1)
        s = 1.0 - xi
        P = al * be
        Q = al * (1.0 - be)
        x2 = a + s * P
        x1 = x2 + b + s * Q
        rows.append(np.stack([x1, x2, x1 + z1, x2 + z2,
                              w4 * jac * xi * s * s * al], axis=1))
    return np.vstack(rows)


def rule_edge(n: int = 4):
    """Rows (x1, x2, y1, y2, w): shared edge is A-B (x2 = 0, y2 = 0) of both."""
    xi, t, u, v, w4 = _grid4(n)
    L = 1.0 - xi
    y1 = 1.0 - L * t
    # face z1 + x2 = 1 of the gauge ball
    z1 = xi * (1.0 - u)
    r1 = np.stack([y1 - z1, xi * u, y1, xi * v, w4 * xi * xi * L], axis=1)
    # face y2 = 1
    z1 = xi * u * (1.0 - v)
    r2 = np.stack([y1 - z1, xi * u * v, y1, xi, w4 * xi * xi * L * u], axis=1)
    # mirrors (y1 < x1): exchange the roles of x and y
    r3 = r1[:, [2, 3, 0, 1, 4]]
    r4 = r2[:, [2, 3, 0, 1, 4]]
    return np.vstack([r1, r2, r3, r4])


def rule_vertex(n: int = 4):
    """Rows (x1, x2, y1, y2, w): shared vertex is A = (0,0) of both."""
    xi, eta, u, v, w4 = _grid4(n)
    r1 = np.stack([xi, xi * u, xi * eta, xi * eta * v, w4 * xi ** 3 * eta],
                  axis=1)
    r2 = r1[:, [2, 3, 0, 1, 4]]
    return np.vstack([r1, r2])


def singular_rules(n: int = 4):
    return rule_coincident(n), rule_edge(n), rule_vertex(n)
