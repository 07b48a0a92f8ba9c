"""Pins of the oracle's PMCHWT matrix and solve with a material per object
(Sec. 2.7, several scatterers; the paper's four-sphere test mixes fat and
bone):

* with the same material everywhere it is the PMCHWT matrix;
* the block of object m equals the PMCHWT matrix of that sphere assembled
  alone with its own (k_m, rho_m), and the blocks coupling two objects hold
  the exterior operators only;
* the OSRC-preconditioned GMRES solution (OSRC wavenumber and damping per
  object) solves B x = f;
* the Mueller matrix with a material per object has the single-sphere
  Mueller matrices as its object blocks.
"""
import numpy as np

from bem_inputs import icosphere, two_spheres
from oracle.operators import pmchwt_matrix, pmchwt_matrix_multi
from oracle.rhs import plane_wave_rhs
from oracle.solve import PreconditionedSystem

K0 = 2.0
KS = [3.0, 4.5 + 0.2j]
RHOS = [1.5, 0.8]


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_same_material_is_pmchwt():
    m = two_spheres(1, offset=1.5)
    B1 = pmchwt_matrix_multi(m, K0, [3.0, 3.0], [1.5, 1.5])
    B0 = pmchwt_matrix(m, K0, 3.0, 1.5)
    assert _rel(B1, B0) < 1e-14


def test_object_blocks_are_the_single_sphere_operators():
    m = two_spheres(1, offset=1.5)
    N = m.n_vertices
    h = N // 2
    B = pmchwt_matrix_multi(m, K0, KS, RHOS)
    for o, c in enumerate([(0.0, -1.5, 0.0), (0.0, 1.5, 0.0)]):
        s = icosphere(1, 1.0, centre=c)
        Bs = pmchwt_matrix(s, K0, KS[o], RHOS[o])
        idx = np.concatenate([np.arange(o * h, (o + 1) * h), N + np.arange(o * h, (o + 1) * h)])
        assert _rel(B[np.ix_(idx, idx)], Bs) < 1e-13
    # coupling blocks: exterior operators only (any interior material gives them)
    Bx = pmchwt_matrix(m, K0, 1.0, 1.0)
    r0 = np.concatenate([np.arange(h), N + np.arange(h)])
    r1 = np.concatenate([np.arange(h, N), N + np.arange(h, N)])
    for a, b in ((r0, r1), (r1, r0)):
        assert _rel(B[np.ix_(a, b)], Bx[np.ix_(a, b)]) < 1e-14


def test_multi_material_solve_solves_the_weak_system():
    m = two_spheres(1, offset=1.5)
    S = PreconditionedSystem(m, K0, KS, RHOS)
    x, it, _ = S.solve([0.0, 0.6, 0.8], tol=1e-11)
    f = plane_wave_rhs(m, K0, [0.0, 0.6, 0.8])
    xd = np.linalg.solve(S.B, f)
    print(it, _rel(x, xd))
    assert _rel(x, xd) < 1e-8 and it < 100


def test_muller_per_object_blocks():
    """Mueller with a material per object: each object's block is that
    sphere's Mueller matrix assembled alone; one material reduces to
    muller_matrix."""
    from oracle.operators import muller_matrix
    m = two_spheres(1, offset=1.5)
    N = m.n_vertices
    h = N // 2
    B = muller_matrix(m, K0, KS, RHOS)
    assert _rel(muller_matrix(m, K0, [3.0, 3.0], [1.5, 1.5]), muller_matrix(m, K0, 3.0, 1.5)) < 1e-14
    for o, c in enumerate([(0.0, -1.5, 0.0), (0.0, 1.5, 0.0)]):
        Bs = muller_matrix(icosphere(1, 1.0, centre=c), K0, KS[o], RHOS[o])
        idx = np.concatenate([np.arange(o * h, (o + 1) * h), N + np.arange(o * h, (o + 1) * h)])
        assert _rel(B[np.ix_(idx, idx)], Bs) < 1e-13


def test_matrix_free_rows_per_object_materials():
    """The matrix-free rows with a material per object (used at full size)
    against the dense matrix."""
    from oracle.operators import pmchwt_matvec_rows
    m = two_spheres(1, offset=1.5)
    N = m.n_vertices
    rng = np.random.default_rng(3)
    x = rng.standard_normal(2 * N) + 1j * rng.standard_normal(2 * N)
    y = pmchwt_matrix_multi(m, K0, KS, RHOS) @ x
    rows = np.array([0, 7, N // 2 + 3, N - 1])
    r1, r2 = pmchwt_matvec_rows(m, K0, KS, RHOS, x, rows)
    assert _rel(r1, y[rows]) < 1e-12 and _rel(r2, y[N + rows]) < 1e-12
