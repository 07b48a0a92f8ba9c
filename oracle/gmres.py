"""Unrestarted GMRES with modified Gram-Schmidt Arnoldi (oracle only).

The paper runs GMRES without restart and stops on the preconditioned
residual (Sec. 3.1).  Start vector x_0 = 0; stop when the least-squares
residual |g_{j+1}| <= tol * ||b||.

Complex Givens rotation for a pair (a, c): with d = sqrt(|a|^2 + |c|^2),
c_j = a / d, s_j = c / d and Omega_j = [[conj(c_j), conj(s_j)], [-s_j, c_j]],
Omega_j (a, c)^T = (d, 0)^T.
"""
from __future__ import annotations

import numpy as np


def _rotate(c, s, u, v):
    return np.conj(c) * u + np.conj(s) * v, -s * u + c * v


def gmres(apply, b, tol=1e-8, maxiter=500):
    """Solve apply(x) = b.  Returns (x, iterations, residual history)."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros_like(b), 0, [0.0]
    V = np.zeros((maxiter + 1, n), np.complex128)
    H = np.zeros((maxiter + 1, maxiter), np.complex128)
    cs = np.zeros(maxiter, np.complex128)
    sn = np.zeros(maxiter, np.complex128)
    g = np.zeros(maxiter + 1, np.complex128)
    g[0] = beta
    V[0] = b / beta
    hist = [1.0]
    j = 0
    for j in range(maxiter):
        w = apply(V[j])
        for i in range(j + 1):            # modified Gram-Schmidt
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] != 0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):                # previous rotations
            H[i, j], H[i + 1, j] = _rotate(cs[i], sn[i], H[i, j], H[i + 1, j])
        d = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
        cs[j] = H[j, j] / d
        sn[j] = H[j + 1, j] / d
        H[j, j], H[j + 1, j] = _rotate(cs[j], sn[j], H[j, j], H[j + 1, j])
        g[j], g[j + 1] = _rotate(cs[j], sn[j], g[j], 0.0)
        res = abs(g[j + 1]) / beta
        hist.append(res)
        if res <= tol:
            break
    m = j + 1
    y = np.linalg.solve(np.triu(H[:m, :m]), g[:m])
    x = V[:m].T @ y
    return x, m, hist
