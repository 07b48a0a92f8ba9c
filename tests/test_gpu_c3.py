"""Precision-form workload: ellipsoid with semi-axes (1, 0.6, 0.4) from an
icosphere of level 6 (40 962 vertices, 81 920 triangles), k_ext = 20,
k_int = 30 + 1.5i (lossy interior), rho = 1.9, OSRC with 8 Pade terms,
theta = pi/3, k_eps from the damped-wavenumber formula with R = 0.1 x the
circumradius.

* matvec FP64 and FP32 on 512 seed-sampled rows (seed 1) of both block rows
  against the oracle's matrix-free rows (<= 1e-10 / <= 1e-5), stored by
  tests/golden/make_c3_rows.py;
* osrc_apply (strong form, both blocks) against the oracle (<= 1e-10);
* solves to 1e-6: FP32 + refinement on the assembled operator and on the
  matrix-free pair kernel, FP64 GMRES on the matrix-free pair kernel.  Each
  solution is checked by the oracle's weak residual f - B x on 128
  seed-sampled vertex rows of both block rows (the oracle's rows of B x for
  the GPU's x; a dense oracle solve at this size is out of reach), which must
  equal the GPU's FP64 rows of the same product to 1e-10 and be small, and the
  three solutions must agree with each other.
"""
import numpy as np
import pytest

from bem_inputs import complex_normal, ellipsoid, icosphere, sample_rows

pytestmark = pytest.mark.gpu

K_EXT, K_INT, RHO = 20.0, 30.0 + 1.5j, 1.9


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2104_04609_amd as P
    return P


@pytest.fixture(scope="module")
def c3():
    mesh = ellipsoid(icosphere(6))
    assert mesh.n_vertices == 40962 and mesh.n_triangles == 81920
    return mesh


@pytest.fixture(scope="module")
def handle(P, c3):
    return P.Mesh.from_inputs(c3)


def oracle_rows(mesh):
    """512 oracle rows written by tests/golden/make_c3_rows.py (oracle only)."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "c3_rows.npz"))
    assert complex(g["k_int"]) == K_INT and float(g["rho"]) == RHO
    x = complex_normal(2 * mesh.n_vertices, seed=int(g["seed_x"]))
    rows = sample_rows(mesh.n_vertices, 512, seed=int(g["seed_rows"]))
    assert np.array_equal(rows, g["rows"])
    return x, rows, (g["r1"], g["r2"])


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_c3_matvec_sampled_rows(P, c3, handle, precision, tol):
    import torch
    x, rows, (r1, r2) = oracle_rows(c3)
    N = c3.n_vertices
    print(f"C3 matvec {precision}", flush=True)
    y = P.pmchwt_matvec(handle, K_EXT, K_INT, RHO, torch.from_numpy(x).cuda(),
                        precision=precision).cpu().numpy()
    e1 = np.linalg.norm(y[rows] - r1) / np.linalg.norm(r1)
    e2 = np.linalg.norm(y[N + rows] - r2) / np.linalg.norm(r2)
    print(precision, e1, e2)
    assert e1 <= tol and e2 <= tol


def test_c3_osrc_apply(P, c3, handle):
    import torch
    from oracle.osrc import OSRC, damped_wavenumber, object_radius
    keps = damped_wavenumber(K_INT, 0.1 * object_radius(c3, 0))
    N = c3.n_vertices
    x = complex_normal(2 * N, seed=12)
    print("C3 oracle OSRC", flush=True)
    ref = OSRC(c3, K_INT, keps, 8, np.pi / 3).apply(x)
    y = P.osrc_apply(handle, 8, np.pi / 3, K_INT, keps, torch.from_numpy(x).cuda()).cpu().numpy()
    for sl in (slice(0, N), slice(N, 2 * N)):
        err = np.linalg.norm(y[sl] - ref[sl]) / np.linalg.norm(ref[sl])
        print("osrc", err)
        assert err <= 1e-10


_C3_SOLUTIONS = {}


def _weak_residual_rows(P, c3, handle, sol):
    """Oracle rows of f - B x on 128 sampled rows (seed 4) of both block rows,
    checked against the GPU's FP64 rows of B x; returns the relative residual
    on those rows and the GPU's residual over all rows."""
    from oracle.operators import pmchwt_matvec_rows
    from oracle.rhs import plane_wave_rhs
    N = c3.n_vertices
    x = sol.cpu().numpy()
    f = plane_wave_rhs(c3, K_EXT, [0.0, 0.0, 1.0])
    y = P.pmchwt_matvec(handle, K_EXT, K_INT, RHO, sol, precision="fp64").cpu().numpy()
    rows = sample_rows(N, 128, seed=4)
    print("C3 oracle rows of B x", flush=True)
    r1, r2 = pmchwt_matvec_rows(c3, K_EXT, K_INT, RHO, x, rows)
    for got, ref in ((y[rows], r1), (y[N + rows], r2)):
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
    idx = np.concatenate([rows, N + rows])
    ro = np.concatenate([r1, r2])
    rel_rows = np.linalg.norm(f[idx] - ro) / np.linalg.norm(f[idx])
    rel_all = np.linalg.norm(f - y) / np.linalg.norm(f)
    return rel_rows, rel_all


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,path", [("fp32", 1), ("fp32", 0), ("fp64", 0), ("fp32", 3)])
def test_c3_solve(P, c3, handle, precision, path):
    print(f"C3 solve {precision} path {path}", flush=True)
    sol, info, rc = P.pmchwt_solve(handle, K_EXT, K_INT, RHO, [[0.0, 0.0, 1.0]], 1e-6,
                                   precision=precision, path=path, pade_terms=8)
    print(info)
    assert rc == 0 and info[0]["rel_residual"] <= 1e-6
    assert np.isfinite(sol.cpu().numpy()).all()
    rel_rows, rel_all = _weak_residual_rows(P, c3, handle, sol[0].contiguous())
    print("weak residual: oracle rows", rel_rows, "GPU all rows", rel_all)
    assert rel_rows <= 1e-3 and rel_all <= 1e-3
    x = sol.cpu().numpy()[0]
    for key, other in _C3_SOLUTIONS.items():
        d = np.linalg.norm(x - other) / np.linalg.norm(other)
        print("vs", key, d)
        assert d <= 1e-4
    _C3_SOLUTIONS[(precision, path)] = x
