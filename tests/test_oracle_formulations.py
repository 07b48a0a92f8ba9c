"""Oracle pins of the mass- and Calderon-preconditioned PMCHWT solves
(Sec. 2.4, 2.5): both precondition the same discrete system B x = f as the
OSRC-preconditioned one (Sec. 2.7), so all three must return the same x up to
the GMRES tolerance; the Calderon system is built on the paper's [phi; psi]
ordering and its block-diagonal C drops exactly the exterior coupling of
different objects."""
import numpy as np
import pytest

from bem_inputs import icosphere, two_spheres
from oracle.solve import (CalderonPreconditionedSystem, MassPreconditionedSystem,
                          PreconditionedSystem)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("k0,k1,rho", [(2.0, 3.0, 1.5), (1.5, 2.5 + 0.2j, 1.9)])
def test_formulations_solve_the_same_system(k0, k1, rho):
    mesh = icosphere(2)
    d = np.array([0.0, 0.0, 1.0])
    ref, it_o, _ = PreconditionedSystem(mesh, k0, k1, rho).solve(d, tol=1e-11)
    S_m = MassPreconditionedSystem(mesh, k0, k1, rho)
    x_m, it_m, _ = S_m.solve(d, tol=1e-11)
    S_c = CalderonPreconditionedSystem(mesh, k0, k1, rho, B=S_m.B)
    x_c, it_c, _ = S_c.solve(d, tol=1e-11)
    print(it_o, it_m, it_c, _rel(x_m, ref), _rel(x_c, ref))
    assert _rel(x_m, ref) < 1e-8 and _rel(x_c, ref) < 1e-8
    # and x solves the weak system itself
    from oracle.rhs import plane_wave_rhs
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
