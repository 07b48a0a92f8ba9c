"""Pins of the oracle's Galerkin operators (no GPU).

Closed forms used (sphere of radius a, spherical harmonics of degree n are
eigenfunctions; h_n = j_n + i y_n):
  V: i k a^2 j_n(ka) h_n(ka)          K = K': i k^2 a^2 j_n(ka) h_n'(ka) + 1/2
  D: -i k^3 a^2 j_n'(ka) h_n'(ka)     with K^2 + V D = 1/4 (Calderon projector).
Laplace limits: V 1 = a, K 1 = -1/2.  Galerkin symmetries V = V^T, D = D^T,
K' = K^T.  Calderon identities (Sec. 2.2): (-1/2 I + A) applied to the
Cauchy data of an interior solution vanishes, (1/2 I + A) applied to those
of a radiating solution vanishes, with A = [[-K, V], [D, K']].
"""
import numpy as np
import pytest
from scipy.special import spherical_jn, spherical_yn

from bem_inputs import icosphere, Mesh
from oracle.operators import assemble
from oracle.osrc import mass_matrix, triangle_geometry
from oracle.rhs import _points


def _h(n, x, d=False):
    return spherical_jn(n, x, d) + 1j * spherical_yn(n, x, d)


def sphere_eigs(n, k, a=1.0):
    ka = k * a
    lv = 1j * k * a * a * spherical_jn(n, ka) * _h(n, ka)
    lk = 1j * k * k * a * a * spherical_jn(n, ka) * _h(n, ka, True) + 0.5
    ld = -1j * k ** 3 * a * a * spherical_jn(n, ka, True) * _h(n, ka, True)
    return dict(V=lv, K=lk, Kp=lk, D=ld)


_CACHE = {}


def ops(level, k):
    key = (level, complex(k))
    if key not in _CACHE:
        m = icosphere(level)
        _CACHE[key] = (m, assemble(m, k), mass_matrix(m).toarray())
    return _CACHE[key]


def test_closed_form_identity():
    for n in range(4):
        e = sphere_eigs(n, 2.0)
        assert abs(e["K"] ** 2 + e["V"] * e["D"] - 0.25) < 1e-12


@pytest.mark.parametrize("k", [2.0, 3.0 + 0.4j])
def test_symmetries(oracle_lib, k):
    _, A, _ = ops(2, k)
    s = max(abs(A["V"]).max(), abs(A["D"]).max())
    assert abs(A["V"] - A["V"].T).max() < 1e-14 * s
    assert abs(A["D"] - A["D"].T).max() < 1e-14 * s
    assert abs(A["Kp"] - A["K"].T).max() < 1e-14 * s


def test_flat_coincident_double_layer_vanishes(oracle_lib):
    tri = Mesh(np.array([[0, 0, 0], [1, 0, 0], [0.2, 0.9, 0]], float),
               np.array([[0, 1, 2]], np.int32))
    A = assemble(tri, 2.5)
    assert np.all(A["K"] == 0) and np.all(A["Kp"] == 0)
    assert abs(A["V"]).min() > 0


def test_laplace_limits(oracle_lib):
    m, A, M = ops(3, 1e-9)
    one = np.ones(m.n_vertices)
    v1 = np.linalg.solve(M, A["V"] @ one).real
    k1 = np.linalg.solve(M, A["K"] @ one).real
    # the polyhedron is inscribed in the unit sphere: V 1 ~ a up to O(h^2)
    assert np.all(abs(v1 - 1.0) < 1e-2)
    # K 1 = -1/2 holds exactly on a closed polyhedron (Gauss' solid angle);
    # what remains is quadrature error
    assert np.all(abs(k1 + 0.5) < 2e-5)


@pytest.mark.parametrize("n", [1, 2])
def test_sphere_eigenvalues_converge(oracle_lib, n):
    k = 2.0
    ex = sphere_eigs(n, k)
    errs = {}
    for L in (2, 3):
        m, A, M = ops(L, k)
        z = m.vertices[:, 2]
        f = z if n == 1 else 0.5 * (3 * z * z - 1)
        den = f @ M @ f
        errs[L] = {op: abs((f @ A[op] @ f) / den - ex[op]) for op in A}
    for op in ("V", "K", "Kp", "D"):
        assert errs[3][op] < errs[2][op] / 3.0, op    # O(h^2)
        assert errs[3][op] < 0.08 * abs(ex[op]) + 1e-3, op


def _cauchy_data(m, k, u, grad_u):
    """P1 coefficients: phi = interpolant, psi = L2 projection of du/dn."""
    area, nrm = triangle_geometry(m)
    bary, w, X = _points(m)
    T = m.triangles
    N = m.n_vertices
    phi = u(m.vertices)
    fN = np.zeros(N, np.complex128)
    dn = np.einsum("tqc,tc->tq", grad_u(X.reshape(-1, 3)).reshape(X.shape), nrm)
    for a in range(3):
        np.add.at(fN, T[:, a], area * ((w * bary[:, a])[None, :] * dn).sum(1))
    M = mass_matrix(m).toarray()
    return phi, np.linalg.solve(M, fN), M


def _calderon_residual(level, k, sign, u, gu):
    m, A, M = ops(level, k)
    phi, psi, _ = _cauchy_data(m, k, u, gu)
    r1 = sign * 0.5 * M @ phi - A["K"] @ phi + A["V"] @ psi
    r2 = A["D"] @ phi + sign * 0.5 * M @ psi + A["Kp"] @ psi
    ref = np.linalg.norm(M @ phi) + np.linalg.norm(M @ psi)
    return (np.linalg.norm(r1) + np.linalg.norm(r2)) / ref


def test_calderon_interior_plane_wave(oracle_lib):
    k, d = 2.0, np.array([0.0, 0.6, 0.8])
    u = lambda x: np.exp(1j * k * x @ d)
    gu = lambda x: (1j * k * np.exp(1j * k * x @ d))[:, None] * d[None, :]
    r2 = _calderon_residual(2, k, -1.0, u, gu)
    r3 = _calderon_residual(3, k, -1.0, u, gu)
    assert r3 < r2 / 2.5 and r3 < 0.02


def test_calderon_exterior_point_source(oracle_lib):
    k, s = 2.0, np.array([0.1, -0.2, 0.15])

    def u(x):
        r = np.linalg.norm(x - s, axis=-1)
        return np.exp(1j * k * r) / (4 * np.pi * r)

    def gu(x):
        dvec = x - s
        r = np.linalg.norm(dvec, axis=-1)
        g = np.exp(1j * k * r) / (4 * np.pi * r)
        return (g * (1j * k * r - 1) / r ** 2)[:, None] * dvec

    r2 = _calderon_residual(2, k, +1.0, u, gu)
    r3 = _calderon_residual(3, k, +1.0, u, gu)
    assert r3 < r2 / 2.5 and r3 < 0.02
    # the interior identity must NOT hold for radiating data (sign check)
    assert _calderon_residual(3, k, -1.0, u, gu) > 0.3


def test_calderon_square_is_quarter_identity(oracle_lib):
    # (M^-1 A)^2 ~ 1/4 I on smooth data (A is twice a projector minus I)
    m, A, M = ops(3, 2.0)
    N = m.n_vertices
    Z = np.zeros((N, N))
    Mi = np.linalg.inv(M)
    Ah = np.block([[-Mi @ A["K"], Mi @ A["V"]], [Mi @ A["D"], Mi @ A["Kp"]]])
    z = m.vertices[:, 2]
    x = np.concatenate([z, 0.7 * z]).astype(np.complex128)
    y = Ah @ (Ah @ x)
    assert np.linalg.norm(y - 0.25 * x) / np.linalg.norm(0.25 * x) < 0.05
    del Z
