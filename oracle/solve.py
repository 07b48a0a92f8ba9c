"""Preconditioned solves (oracle only; test infrastructure, not part of the
product path): the OSRC-preconditioned permuted PMCHWT (Sec. 2.7) and the
formulations it is compared with (Sec. 3.1): standard PMCHWT and Mueller in
strong form (Sec. 2.2, 2.4) and the block-diagonal Calderon preconditioner
(Sec. 2.5).

Preconditioned strong-form system (Sec. 2.4 mass preconditioning, Sec. 2.7
OSRC-preconditioned PMCHWT):
    L M^{-1} B x = L M^{-1} f,   L = diag(L_DtN, L_NtD) per object,
with M^{-1} applied to each N-block, the OSRC wavenumber the interior one by
default (Sec. 3.1), k_eps from R = one tenth of the object's radius (Sec. 3.1;
radius = circumradius about the object's vertex centroid), and unrestarted
GMRES (Sec. 3.1).
"""
from __future__ import annotations

import numpy as np

from .gmres import gmres
from .operators import muller_matrix, pmchwt_matrix, pmchwt_matrix_multi, vertex_objects
from .osrc import OSRC, damped_wavenumber, object_radius
from .rhs import plane_wave_rhs


def osrc_keps_per_vertex(mesh, k, R=None):
    """Per-vertex damped wavenumber: each object's k_eps from its own R (and
    its own k when k is a sequence with one entry per object)."""
    N = mesh.n_vertices
    keps = np.empty(N, np.complex128)
    nobj = mesh.n_objects()
    ks = np.broadcast_to(np.asarray(k, np.complex128), (nobj,))
    for o in range(nobj):
        Ro = 0.1 * object_radius(mesh, o) if R is None else R
        if mesh.object_id is None:
            vid = np.arange(N)
        else:
            vid = np.unique(mesh.triangles[mesh.object_id == o])
        keps[vid] = damped_wavenumber(ks[o], Ro)
    return keps


class PreconditionedSystem:
    """k_int and rho: one material for every object, or sequences with one
    entry per object (Sec. 2.7, several scatterers)."""

    def __init__(self, mesh, k_ext, k_int, rho, n_p=4, theta=np.pi / 3,
                 osrc_interior=True, R=None, B=None):
        self.mesh = mesh
        self.N = mesh.n_vertices
        self.k_ext, self.k_int, self.rho = k_ext, k_int, rho
        multi = np.ndim(k_int) > 0 or np.ndim(rho) > 0
        if B is None:
            B = (pmchwt_matrix_multi(mesh, k_ext, k_int, rho) if multi
                 else pmchwt_matrix(mesh, k_ext, k_int, rho))
        self.B = B
        nobj = mesh.n_objects()
        k_obj = np.broadcast_to(np.asarray(k_int if osrc_interior else k_ext, np.complex128),
                                (nobj,))
        k_vert = k_obj[vertex_objects(mesh)]
        self.osrc = OSRC(mesh, k_vert, osrc_keps_per_vertex(mesh, k_obj, R), n_p, theta)

    def strong(self, y):
        N = self.N
        return np.concatenate([self.osrc.mass_solve(y[:N]),
                               self.osrc.mass_solve(y[N:])])

    def apply(self, x):
        return self.osrc.apply(self.strong(self.B @ x))

    def rhs(self, d):
        return self.osrc.apply(self.strong(plane_wave_rhs(self.mesh,
                                                          self.k_ext, d)))

    def solve(self, d, tol=1e-8, maxiter=500):
        b = self.rhs(d)
        x, it, hist = gmres(self.apply, b, tol=tol, maxiter=maxiter)
        return x, it, hist


class _PaperOrderingSystem(PreconditionedSystem):
    """Base of the formulations iterated on the paper's ordering
    u = [phi; psi] (Sec. 2.2): Bu = B[:, perm] with Bu u = B x for
    x = [psi; phi]; the solution is returned in the permuted ordering x."""

    def __init__(self, mesh, k_ext, k_int, rho, **kw):
        super().__init__(mesh, k_ext, k_int, rho, **kw)
        N = self.N
        perm = np.concatenate([np.arange(N, 2 * N), np.arange(N)])   # [phi; psi] -> [psi; phi]
        self.Bu = self.B[:, perm]

    def solve(self, d, tol=1e-8, maxiter=500):
        u, it, hist = gmres(self.apply, self.rhs(d), tol=tol, maxiter=maxiter)
        N = self.N
        return np.concatenate([u[N:], u[:N]]), it, hist


class PMCHWTSystem(_PaperOrderingSystem):
    """Standard PMCHWT formulation in strong form (Sec. 2.2, mass
    preconditioning Sec. 2.4): M^{-1} Bu u = M^{-1} f on u = [phi; psi],
    M^{-1} applied to each N-block.  Same discrete system B x = f as the
    OSRC-preconditioned one."""

    def apply(self, u):
        return self.strong(self.Bu @ u)

    def rhs(self, d):
        return self.strong(plane_wave_rhs(self.mesh, self.k_ext, d))


class MullerSystem(PMCHWTSystem):
    """Mueller formulation in strong form (Sec. 2.2, Sec. 2.4):
    M^{-1} (I + A_0 - A^_1) u = M^{-1} f on u = [phi; psi], the weak operator
    from muller_matrix (B holds it here, in the permuted ordering)."""

    def __init__(self, mesh, k_ext, k_int, rho, B=None, **kw):
        if B is None:
            B = muller_matrix(mesh, k_ext, k_int, rho)
        super().__init__(mesh, k_ext, k_int, rho, B=B, **kw)


class CalderonPreconditionedSystem(_PaperOrderingSystem):
    """PMCHWT with the block-diagonal Calderon preconditioner (Sec. 2.5):
    M^{-1} C M^{-1} Bu u = M^{-1} C M^{-1} f with Bu = A_0 + A^_1 acting on
    u = [phi; psi] (the paper's ordering) and C = diag_m(A_{0,mm} + A^_m), the
    self-interaction blocks of each object (with one object C = Bu).  The
    solution is returned in the permuted ordering x = [psi; phi] of B."""

    def __init__(self, mesh, k_ext, k_int, rho, **kw):
        super().__init__(mesh, k_ext, k_int, rho, **kw)
        N = self.N
        C = self.Bu.copy()
        if mesh.n_objects() > 1:
            # drop the exterior coupling between different objects (the
            # interior operators act within one object already)
            vobj = np.full(N, -1)
            for o in range(mesh.n_objects()):
                vobj[np.unique(mesh.triangles[mesh.object_id == o])] = o
            same = vobj[:, None] == vobj[None, :]
            mask = np.block([[same, same], [same, same]])
            C = np.where(mask, C, 0.0)
        self.C = C

    def apply(self, u):
        return self.strong(self.C @ self.strong(self.Bu @ u))

    def rhs(self, d):
        return self.strong(self.C @ self.strong(plane_wave_rhs(self.mesh, self.k_ext, d)))
