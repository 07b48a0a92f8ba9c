"""Precision-form workload: ellipsoid with semi-axes (1, 0.6, 0.4) from an
icosphere of level 6 (40 962 vertices, 81 920 triangles), k_ext = 20,
k_int = 30 + 1.5i (lossy interior), rho = 1.9, OSRC with 8 Pade terms,
theta = pi/3, k_eps from the damped-wavenumber formula with R = 0.1 x the
circumradius.

* matvec FP64 and FP32 on 512 seed-sampled rows (seed 1) of both block rows
  against the oracle's matrix-free rows (<= 1e-10 / <= 1e-5), stored by
  tests/golden/make_c3_rows.py;
* osrc_apply (strong form, both blocks) against the oracle (<= 1e-10);
* the FP32 + refinement solve on the assembled operator reaches 1e-6.
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


def test_c3_solve_fp32_assembled(P, handle):
    print("C3 solve", flush=True)
    sol, info, rc = P.pmchwt_solve(handle, K_EXT, K_INT, RHO, [[0.0, 0.0, 1.0]], 1e-6,
                                   precision="fp32", path=1, pade_terms=8)
    print(info)
    assert rc == 0 and info[0]["rel_residual"] <= 1e-6
    assert np.isfinite(sol.cpu().numpy()).all()
