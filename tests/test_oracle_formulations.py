"""Oracle pins of the formulations compared with the OSRC-preconditioned
PMCHWT (Sec. 3.1).

* Standard PMCHWT in strong form (Sec. 2.2, 2.4) and the Calderon
  preconditioner (Sec. 2.5) precondition the same discrete system B x = f as
  the OSRC-preconditioned one (Sec. 2.7), so all three return the same x up
  to the GMRES tolerance; the Calderon system is built on the paper's
  [phi; psi] ordering and its block-diagonal C drops exactly the exterior
  coupling of different objects.
* Mueller (Sec. 2.2) is another discrete system.  With the same material on
  both sides (k_int = k_ext, rho = 1) the interior Calderon operator equals
  the exterior one, so I + A_0 - A^_1 is the identity: the weak matrix is the
  P1 mass matrix on the row's own trace and the solution is the L2
  projection of the incident traces.  With a contrast, its far field
  converges to the series solution of the sphere (Sec. 3.2) at the rate of
  the PMCHWT one."""
import numpy as np
import pytest

from bem_inputs import icosphere, two_spheres
from oracle import mie
from oracle.operators import muller_matrix
from oracle.osrc import mass_matrix
from oracle.rhs import far_field, plane_wave_rhs
from oracle.solve import (CalderonPreconditionedSystem, MullerSystem, PMCHWTSystem,
                          PreconditionedSystem)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("k0,k1,rho", [(2.0, 3.0, 1.5), (1.5, 2.5 + 0.2j, 1.9)])
def test_formulations_solve_the_same_system(k0, k1, rho):
    mesh = icosphere(2)
    d = np.array([0.0, 0.0, 1.0])
    ref, it_o, _ = PreconditionedSystem(mesh, k0, k1, rho).solve(d, tol=1e-11)
    S_m = PMCHWTSystem(mesh, k0, k1, rho)
    x_m, it_m, _ = S_m.solve(d, tol=1e-11)
    S_c = CalderonPreconditionedSystem(mesh, k0, k1, rho, B=S_m.B)
    x_c, it_c, _ = S_c.solve(d, tol=1e-11)
    print(it_o, it_m, it_c, _rel(x_m, ref), _rel(x_c, ref))
    assert _rel(x_m, ref) < 1e-8 and _rel(x_c, ref) < 1e-8
    # and x solves the weak system itself
    f = plane_wave_rhs(mesh, k0, d)
    assert _rel(S_m.B @ x_c, f) < 1e-8


def test_calderon_one_object_uses_the_full_operator():
    mesh = icosphere(1)
    S = CalderonPreconditionedSystem(mesh, 2.0, 3.0, 1.5)
    assert np.array_equal(S.C, S.Bu)
    N = mesh.n_vertices
    # Bu u with u = [phi; psi] equals B x with x = [psi; phi]
    rng = np.random.default_rng(0)
    x = rng.standard_normal(2 * N) + 1j * rng.standard_normal(2 * N)
    u = np.concatenate([x[N:], x[:N]])
    assert np.allclose(S.Bu @ u, S.B @ x, rtol=0, atol=1e-13 * np.abs(S.B @ x).max())


def test_calderon_two_objects_drops_cross_coupling():
    mesh = two_spheres(1, offset=1.5)
    S = CalderonPreconditionedSystem(mesh, 2.0, 3.0, 1.5)
    N = mesh.n_vertices
    h = N // 2   # vertices of the two objects are contiguous halves
    D = S.Bu - S.C
    # only the blocks coupling vertices of different objects differ
    for bi in range(2):
        for bj in range(2):
            blk = D[bi * N:(bi + 1) * N, bj * N:(bj + 1) * N]
            assert np.all(blk[:h, :h] == 0) and np.all(blk[h:, h:] == 0)
            assert np.abs(blk[:h, h:]).max() > 0 and np.abs(blk[h:, :h]).max() > 0


def test_muller_same_material_is_the_identity():
    mesh = icosphere(2)
    N = mesh.n_vertices
    k = 2.0 + 0.1j
    Bm = muller_matrix(mesh, k, k, 1.0)
    M = mass_matrix(mesh).toarray()
    Z = np.zeros((N, N))
    assert np.abs(Bm - np.block([[Z, M], [M, Z]])).max() <= 1e-14 * np.abs(M).max()
    d = np.array([0.6, 0.0, 0.8])
    x, it, _ = MullerSystem(mesh, k, k, 1.0, B=Bm).solve(d, tol=1e-12)
    f = plane_wave_rhs(mesh, k, d)
    # no scatterer: phi, psi are the L2 projections of the incident traces
    assert it <= 1
    assert _rel(x[N:], np.linalg.solve(M, f[:N])) < 1e-12
    assert _rel(x[:N], np.linalg.solve(M, f[N:])) < 1e-12


@pytest.mark.slow
def test_muller_mie_convergence(oracle_lib):
    k0, k1, rho = 2.0, 3.0, 1.5
    th = np.linspace(0, np.pi, 91)
    dirs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    Fm = mie.far_field(k0, k1, rho, th)
    errs = []
    for L in (2, 3):
        m = icosphere(L)
        x, it, _ = MullerSystem(m, k0, k1, rho).solve([0, 0, 1], tol=1e-8)
        F = far_field(m, k0, x, dirs)
        errs.append(np.linalg.norm(F - Fm) / np.linalg.norm(Fm))
    print(errs)
    assert errs[1] < errs[0] / 3 and errs[1] < 1.5e-2
    # the sign of the interior terms matters: the PMCHWT matrix with the
    # Mueller identity added is far off
    m = icosphere(3)
    from oracle.operators import pmchwt_matrix
    N = m.n_vertices
    M = mass_matrix(m).toarray()
    Z = np.zeros((N, N))
    Bw = pmchwt_matrix(m, k0, k1, rho) + np.block([[Z, M], [M, Z]])
    x, _, _ = MullerSystem(m, k0, k1, rho, B=Bw).solve([0, 0, 1], tol=1e-8)
    F = far_field(m, k0, x, dirs)
    assert np.linalg.norm(F - Fm) / np.linalg.norm(Fm) > 0.1


def test_muller_rows_match_matrix():
    """The matrix-free Mueller rows (used at full size) against the dense
    Mueller matrix, on a mesh with two objects."""
    from oracle.operators import muller_matvec_rows
    mesh = two_spheres(1, offset=1.5)
    N = mesh.n_vertices
    k0, k1, rho = 2.0, 3.5 + 0.2j, 1.3
    rng = np.random.default_rng(7)
    x = rng.standard_normal(2 * N) + 1j * rng.standard_normal(2 * N)
    y = muller_matrix(mesh, k0, k1, rho) @ x
    rows = np.array([0, 5, N // 2, N - 1])
    r1, r2 = muller_matvec_rows(mesh, k0, k1, rho, x, rows)
    assert _rel(r1, y[rows]) < 1e-12 and _rel(r2, y[N + rows]) < 1e-12
