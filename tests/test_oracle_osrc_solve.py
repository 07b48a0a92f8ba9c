"""Pins of the oracle's OSRC preconditioner, GMRES and end-to-end solve.

* Pade: theta = 0 gives the unrotated coefficients; N_p = 1 gives
  (4 + 3z)/(4 + z); R_{N_p}(z) -> sqrt(1 + z) away from the rotated cut.
* Mass and stiffness: M 1 = vertex areas, 1^T M 1 = surface area, S 1 = 0,
  Rayleigh quotients of M^{-1} S on degree-n harmonics -> n(n+1)/a^2.
* OSRC on generalised eigenpairs S v = mu M v (dense, tiny mesh):
  L_DtN v = ik R(-mu/k_eps^2) v and L_NtD v = R(-mu/k_eps^2)/(ik (1 - mu/k_eps^2)) v.
* GMRES against a dense direct solve.
* End to end: the OSRC-preconditioned PMCHWT solution converges to the Mie
  series of a penetrable sphere under refinement (far field and traces).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from bem_inputs import ellipsoid, icosphere, two_spheres
from oracle import mie
from oracle.gmres import gmres
from oracle.osrc import (OSRC, damped_wavenumber, mass_matrix, object_radius,
                         pade_coefficients, pade_eval, pade_unrotated, stiffness_matrix,
                         triangle_geometry)
from oracle.rhs import far_field
from oracle.solve import PreconditionedSystem, osrc_keps_per_vertex


def test_pade_theta_zero_reduces_to_unrotated():
    for n_p in (1, 4, 8):
        C0, A, B = pade_coefficients(n_p, 0.0)
        a, b = pade_unrotated(n_p)
        assert abs(C0 - 1.0) < 1e-15
        assert np.allclose(A, a, atol=1e-15) and np.allclose(B, b, atol=1e-15)


def test_pade_single_term_closed_form():
    z = np.array([0.3, -0.5, 2.0 + 1j, -0.2 - 0.7j])
    assert np.allclose(pade_eval(z, 1, 0.0), (4 + 3 * z) / (4 + z), atol=1e-15)


def test_pade_converges_to_sqrt():
    theta = np.pi / 3
    z = np.array([0.5, -0.5, 3.0, 2j, -0.9 + 0.3j, -4.0 + 0.5j])
    exact = np.exp(1j * theta / 2) * np.sqrt((1 + z) * np.exp(-1j * theta))
    e4 = abs(pade_eval(z, 4, theta) - exact)
    e8 = abs(pade_eval(z, 8, theta) - exact)
    e16 = abs(pade_eval(z, 16, theta) - exact)
    assert np.all(e8 <= e4 + 1e-15) and np.all(e16 < 1e-3)


def test_damped_wavenumber_matches_alternative_algebra():
    for k in (10.0, 30 + 1.5j):
        R = 0.1
        alt = k + 0.4j * k ** (1 / 3) * R ** (-2 / 3)
        assert abs(damped_wavenumber(k, R) - alt) < 1e-12 * abs(k)


def test_object_radius_closed_forms():
    """R of k_eps (Sec. 2.6, 3.1) is read as the circumradius of each object
    about its own vertex centroid: a sphere of radius a gives a wherever it
    sits (an origin-based or diameter-based reading gives 8.6 or 5 here), two
    unit spheres give 1 each (one radius for both objects would be 2.5), and
    the (1, 0.6, 0.4) ellipsoid gives its largest semi-axis, since subdivision
    places vertices at (+-1, 0, 0)."""
    assert abs(object_radius(icosphere(3), 0) - 1.0) < 1e-12
    moved = icosphere(2, radius=2.5, centre=(3.0, -2.0, 5.0))
    assert abs(object_radius(moved, 0) - 2.5) < 1e-12
    two = two_spheres(2, offset=1.5)
    for o in (0, 1):
        assert abs(object_radius(two, o) - 1.0) < 1e-12
    assert abs(object_radius(ellipsoid(icosphere(3)), 0) - 1.0) < 1e-12


def test_keps_per_vertex_closed_form():
    """Each object's vertices carry k_eps = k (1 + 0.4 i (k R)^(-2/3)) with its
    own k and R = 0.1 (one tenth of the unit radius, Sec. 3.1): k = 10 gives
    10 + 4i exactly; k = 30 + 1.5i the principal-branch value."""
    two = two_spheres(2, offset=1.5)
    k = [10.0, 30.0 + 1.5j]
    ke = osrc_keps_per_vertex(two, k)
    nv = two.n_vertices // 2
    k1 = 30.0 + 1.5j
    z = (k1 * 0.1) ** (-2.0 / 3.0)
    z_ref = abs(k1 * 0.1) ** (-2.0 / 3.0) * np.exp(-2.0j / 3.0 * np.angle(k1 * 0.1))
    assert abs(z - z_ref) < 1e-14
    assert np.allclose(ke[:nv], 10.0 + 4.0j, rtol=0, atol=1e-12)
    assert np.allclose(ke[nv:], k1 * (1 + 0.4j * z_ref), rtol=0, atol=1e-12)
    # an explicit R overrides the radius
    assert np.allclose(osrc_keps_per_vertex(two, 10.0, R=1.0), 10.0 * (1 + 0.4j * 10.0 ** (-2 / 3)))


def test_mass_and_stiffness_closed_forms():
    m = icosphere(3)
    M = mass_matrix(m)
    S = stiffness_matrix(m)
    area, _ = triangle_geometry(m)
    vert_area = np.zeros(m.n_vertices)
    for a in range(3):
        np.add.at(vert_area, m.triangles[:, a], area / 3.0)
    one = np.ones(m.n_vertices)
    assert np.allclose(M @ one, vert_area, rtol=1e-14)
    assert abs(one @ M @ one - area.sum()) < 1e-13
    assert abs(S @ one).max() < 1e-12
    assert abs(S - S.T).max() < 1e-14


def test_laplace_beltrami_eigenvalues():
    errs = []
    for L in (2, 3):
        m = icosphere(L)
        M = mass_matrix(m).toarray()
        S = stiffness_matrix(m).toarray()
        z = m.vertices[:, 2]
        e = []
        for n, f in ((1, z), (2, 0.5 * (3 * z * z - 1))):
            e.append(abs((f @ S @ f) / (f @ M @ f) - n * (n + 1)))
        errs.append(e)
    assert errs[1][0] < errs[0][0] / 3 and errs[1][1] < errs[0][1] / 3
    assert errs[1][1] < 0.05 * 6


def test_osrc_on_generalised_eigenpairs():
    m = icosphere(1)
    k = 3.0
    keps = damped_wavenumber(k, 0.1)
    op = OSRC(m, k, keps, n_p=4, theta=np.pi / 3)
    M = mass_matrix(m).toarray()
    S = stiffness_matrix(m).toarray()
    mu, V = sla.eigh(S, M)
    for i in (0, 3, 10, 25, 41):
        v = V[:, i].astype(np.complex128)
        Rv = pade_eval(-mu[i] / keps ** 2, 4, np.pi / 3)
        dtn = op.dtn(v)
        ntd = op.ntd(v)
        assert np.linalg.norm(dtn - 1j * k * Rv * v) < 1e-12 * abs(k * Rv)
        lam = Rv / (1j * k * (1 - mu[i] / keps ** 2))
        assert np.linalg.norm(ntd - lam * v) < 1e-12 * abs(lam) + 1e-14


def test_gmres_matches_direct_solve():
    rng = np.random.default_rng(3)
    n = 60
    A = np.eye(n) * 4 + (rng.standard_normal((n, n)) +
                         1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist = gmres(lambda v: A @ v, b, tol=1e-12, maxiter=n)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10
    assert it <= n and hist[-1] <= 1e-12
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) < 1e-11


def test_preconditioned_gmres_matches_dense_solve(oracle_lib):
    m = icosphere(2)
    S = PreconditionedSystem(m, 2.0, 3.0, 1.5)
    b = S.rhs([0, 0, 1])
    x, it, hist = S.solve([0, 0, 1], tol=1e-10)
    n = 2 * m.n_vertices
    P = np.stack([S.apply(e) for e in np.eye(n, dtype=np.complex128)], axis=1)
    xd = np.linalg.solve(P, b)
    cond = np.linalg.cond(P)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10 * cond * 10
    assert it < 60


@pytest.mark.slow
def test_mie_convergence(oracle_lib):
    k0, k1, rho = 2.0, 3.0, 1.5
    th = np.linspace(0, np.pi, 181)
    dirs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    Fm = mie.far_field(k0, k1, rho, th)
    errs, terr = [], []
    for L in (2, 3):
        m = icosphere(L)
        S = PreconditionedSystem(m, k0, k1, rho)
        x, it, _ = S.solve([0, 0, 1], tol=1e-8)
        F = far_field(m, k0, x, dirs)
        errs.append(np.linalg.norm(F - Fm) / np.linalg.norm(Fm))
        N = m.n_vertices
        ct = m.vertices[:, 2] / np.linalg.norm(m.vertices, axis=1)
        phi, psi = mie.surface_traces(k0, k1, rho, ct)
        terr.append(np.linalg.norm(x[N:] - phi) / np.linalg.norm(phi) +
                    np.linalg.norm(x[:N] - psi) / np.linalg.norm(psi))
    assert errs[1] < errs[0] / 3 and errs[1] < 1.5e-2
    assert terr[1] < terr[0] / 3
    # the sign of the density ratio matters: rho -> 1/rho is far off
    m = icosphere(3)
    S = PreconditionedSystem(m, k0, k1, 1 / rho)
    x, _, _ = S.solve([0, 0, 1], tol=1e-8)
    F = far_field(m, k0, x, dirs)
    assert np.linalg.norm(F - Fm) / np.linalg.norm(Fm) > 0.1
