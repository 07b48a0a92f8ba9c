"""OSRC preconditioner and P1 mass/stiffness matrices (oracle only).

OSRC operators (Sec. 2.6):  L_NtD = (1/ik) (I + Delta_Gamma / k_eps^2)^(-1/2),
L_DtN = ik (I + Delta_Gamma / k_eps^2)^(1/2), damped wavenumber
k_eps = k (1 + 0.4 i (k R)^(-2/3)).  The square root is localised by a Pade
series of N_p terms with branch-cut rotation theta (Sec. 2.7, last paragraph);
the paper gives no formulas for it, so this follows the rotated Pade
approximant it cites (Milinazzo-Zala-Brooke coefficients with the
Antoine-Darbas rotation):

  a_j = 2/(2N_p+1) sin^2(j pi/(2N_p+1)),  b_j = cos^2(j pi/(2N_p+1)),
  C_0 = e^{i theta/2} [1 + sum_j a_j (e^{-i theta} - 1)/(1 + b_j (e^{-i theta} - 1))],
  A_j = e^{-i theta/2} a_j / (1 + b_j (e^{-i theta} - 1))^2,
  B_j = e^{-i theta} b_j / (1 + b_j (e^{-i theta} - 1)),
  sqrt(1 + z) ~ R(z) = C_0 + sum_j A_j z / (1 + B_j z).

Discretisation with P1 mass M and stiffness S (weak Laplace-Beltrami, so the
discrete Delta_Gamma / k_eps^2 is X = -M^{-1} S / k_eps^2):

  R(X) u = M^{-1} [ C_0 M u - (1/k_eps^2) S sum_j A_j (M - beta_j S)^{-1} M u ],
  beta_j = B_j / k_eps^2,
  L_DtN u = ik R(X) u,     L_NtD u = (1/ik) R(X) (M - S/k_eps^2)^{-1} M u.

All shifted systems are solved with a sparse LU computed once (Sec. 2.7).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def triangle_geometry(mesh):
    P = mesh.vertices
    T = mesh.triangles
    e1 = P[T[:, 1]] - P[T[:, 0]]
    e2 = P[T[:, 2]] - P[T[:, 0]]
    nrm = np.cross(e1, e2)
    area = 0.5 * np.linalg.norm(nrm, axis=1)
    n = nrm / (2.0 * area[:, None])
    return area, n


def p1_gradients(mesh):
    """grad phi_a on each triangle: [T, 3 (a), 3 (xyz)]."""
    P = mesh.vertices
    T = mesh.triangles
    area, n = triangle_geometry(mesh)
    g = np.zeros((len(T), 3, 3))
    for a in range(3):
        e = P[T[:, (a + 2) % 3]] - P[T[:, (a + 1) % 3]]
        g[:, a] = np.cross(n, e) / (2.0 * area[:, None])
    return g


def mass_matrix(mesh):
    area, _ = triangle_geometry(mesh)
    T = mesh.triangles
    N = mesh.n_vertices
    loc = np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]], float) / 12.0
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            rows.append(T[:, a])
            cols.append(T[:, b])
            vals.append(area * loc[a, b])
    return sp.csr_matrix((np.concatenate(vals),
                          (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def stiffness_matrix(mesh):
    area, _ = triangle_geometry(mesh)
    g = p1_gradients(mesh)
    T = mesh.triangles
    N = mesh.n_vertices
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            rows.append(T[:, a])
            cols.append(T[:, b])
            vals.append(area * np.einsum("ij,ij->i", g[:, a], g[:, b]))
    return sp.csr_matrix((np.concatenate(vals),
                          (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def pade_unrotated(n_p):
    j = np.arange(1, n_p + 1)
    a = 2.0 / (2 * n_p + 1) * np.sin(j * np.pi / (2 * n_p + 1)) ** 2
    b = np.cos(j * np.pi / (2 * n_p + 1)) ** 2
    return a, b


def pade_coefficients(n_p, theta):
    """(C0, A[n_p], B[n_p]) of the rotated Pade approximant of sqrt(1+z)."""
    a, b = pade_unrotated(n_p)
    e = np.exp(-1j * theta)
    den = 1.0 + b * (e - 1.0)
    C0 = np.exp(1j * theta / 2) * (1.0 + np.sum(a * (e - 1.0) / den))
    A = np.exp(-1j * theta / 2) * a / den ** 2
    B = e * b / den
    return C0, A, B


def pade_eval(z, n_p, theta):
    C0, A, B = pade_coefficients(n_p, theta)
    z = np.asarray(z, dtype=np.complex128)
    out = np.full(z.shape, C0, dtype=np.complex128)
    for Aj, Bj in zip(A, B):
        out = out + Aj * z / (1.0 + Bj * z)
    return out


def damped_wavenumber(k, R):
    """k_eps = k (1 + 0.4 i (k R)^(-2/3)), principal branch (Sec. 2.6)."""
    k = complex(k)
    return k * (1.0 + 0.4j * (k * R) ** (-2.0 / 3.0))


def object_radius(mesh, obj):
    """Circumradius of object `obj` about its vertex centroid."""
    T = mesh.triangles
    if mesh.object_id is None:
        vid = np.arange(mesh.n_vertices)
    else:
        vid = np.unique(T[mesh.object_id == obj])
    P = mesh.vertices[vid]
    return float(np.linalg.norm(P - P.mean(axis=0), axis=1).max())


class OSRC:
    """diag(L_DtN, L_NtD) in strong form, per-vertex wavenumber k (one value,
    or that of each vertex's object) and per-vertex k_eps."""

    def __init__(self, mesh, k, k_eps, n_p=4, theta=np.pi / 3):
        self.N = mesh.n_vertices
        # the operators are block diagonal by object: the factor ik of each
        # object's L_DtN (1/ik of L_NtD) scales that object's rows
        self.k = np.broadcast_to(np.asarray(k, np.complex128), (self.N,))
        keps = np.broadcast_to(np.asarray(k_eps, np.complex128), (self.N,))
        self.M = mass_matrix(mesh).tocsc()
        self.S = stiffness_matrix(mesh).tocsc()
        self.C0, self.A, self.B = pade_coefficients(n_p, theta)
        # row scaling by 1/k_eps^2 of the vertex's object: S is block
        # diagonal by object, so diag(c) S == the per-object operator
        self.inv_k2 = sp.diags(1.0 / keps ** 2).tocsc()
        self.Sk = (self.inv_k2 @ self.S).tocsc()
        self.lu_M = spla.splu(self.M.astype(np.complex128))
        self.lu_shift = [spla.splu((self.M - Bj * self.Sk).tocsc())
                         for Bj in self.B]
        self.lu_first = spla.splu((self.M - self.Sk).tocsc())

    def _R_weak(self, m):
        """C_0 m - (1/k_eps^2) S sum_j A_j (M - beta_j S)^{-1} m."""
        acc = np.zeros_like(m)
        for Aj, lu in zip(self.A, self.lu_shift):
            acc = acc + Aj * lu.solve(m)
        return self.C0 * m - self.Sk @ acc

    def dtn(self, u):
        m = self.M @ u
        return 1j * self.k * self.lu_M.solve(self._R_weak(m))

    def ntd(self, u):
        v = self.lu_first.solve(self.M @ u)
        return self.lu_M.solve(self._R_weak(self.M @ v)) / (1j * self.k)

    def apply(self, x):
        """x = [psi; phi] (strong coefficients) -> [L_DtN psi; L_NtD phi]."""
        N = self.N
        return np.concatenate([self.dtn(x[:N]), self.ntd(x[N:])])

    def mass_solve(self, y):
        return self.lu_M.solve(y)
