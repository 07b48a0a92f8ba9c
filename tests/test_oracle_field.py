"""Pins of the oracle's field evaluation off the surface (representation
formulas of Sec. 2.2) and of the sphere series field it is compared with
(Sec. 3.2), against facts fixed by the mathematics:

* the series total field: its scattered part tends to the series far field,
  and it is continuous across the sphere, where it equals the series
  Dirichlet trace;
* the solid angle of a closed surface is 4 pi at points inside, 0 outside;
* Green's representation: the interior formula reproduces a plane wave from
  its own traces, the exterior one a point source at the centre (both at the
  O(h^2) rate of the P1 interpolated traces);
* end to end: the field of the BEM solution converges to the series field.
"""
import numpy as np
import pytest

from bem_inputs import icosphere, two_spheres
from oracle import mie
from oracle.field import field, layer_potentials, regions, solid_angles


def test_series_field_far_limit_and_continuity():
    k0, k1, rho = 2.0, 3.0 + 0.1j, 1.5
    th = np.array([0.3, 1.0, 2.5])
    F = mie.far_field(k0, k1, rho, th)
    errs = []
    for R in (300.0, 3000.0):
        p = np.stack([R * np.sin(th), 0 * th, R * np.cos(th)], 1)
        us = mie.total_field(k0, k1, rho, p) - np.exp(1j * k0 * p[:, 2])
        errs.append(np.abs(us * R * np.exp(-1j * k0 * R) - F).max())
    assert errs[0] < 1e-2 * np.abs(F).max() and errs[1] < errs[0] / 5
    ct = np.array([-0.9, 0.1, 0.7])
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st, 0 * ct, ct], 1)
    ui = mie.total_field(k0, k1, rho, d * (1 - 1e-10))
    ue = mie.total_field(k0, k1, rho, d * (1 + 1e-10))
    phi, _ = mie.surface_traces(k0, k1, rho, ct)
    assert np.abs(ui - ue).max() < 1e-8 and np.abs(ue - phi).max() < 1e-8


def test_solid_angles_classify_points():
    m = icosphere(2)
    w = solid_angles(m, [[0.1, -0.2, 0.3], [0, 0, 0], [1.3, 0, 0], [0, 5, 1]])[:, 0]
    assert np.allclose(w, [1, 1, 0, 0], atol=1e-12)
    m2 = two_spheres(1, offset=1.5)
    p = np.array([[0, 0, 0.], [0, 1.5, 0], [0, -1.5, 0], [0, 3.0, 0], [0.3, -1.2, 0.2]])
    assert np.allclose(solid_angles(m2, p), [[0, 0], [0, 1], [1, 0], [0, 0], [1, 0]],
                       atol=1e-12)
    assert list(regions(m2, p)) == [0, 2, 1, 0, 1]


def test_green_representation_interior_and_exterior():
    k = 2.5 + 0.1j
    d = np.array([0.6, 0, 0.8])
    p_in = np.array([[0.1, 0.2, -0.3], [0.0, 0.0, 0.5], [-0.4, 0.1, 0.2]])
    p_out = np.array([[1.5, 0.2, -0.3], [0.0, 0.0, 2.0], [-1.2, 1.1, 0.2]])
    ro = np.linalg.norm(p_out, axis=1)
    e_in, e_out = [], []
    for L in (2, 3):
        m = icosphere(L)
        V = m.vertices
        r = np.linalg.norm(V, axis=1)
        nv = V / r[:, None]
        # plane wave (regular inside): interior formula with rho = 1 gives it back
        v = np.exp(1j * k * V @ d)
        S, D = layer_potentials(m, k, np.concatenate([1j * k * (nv @ d) * v, v]), p_in)
        e_in.append(np.abs(S - D - np.exp(1j * k * p_in @ d)).max())
        # point source at the centre (radiating): exterior formula gives it back
        g = np.exp(1j * k * r) / (4 * np.pi * r)
        S, D = layer_potentials(m, k, np.concatenate([(1j * k - 1 / r) * g, g]), p_out)
        e_out.append(np.abs(-S + D - np.exp(1j * k * ro) / (4 * np.pi * ro)).max())
    print(e_in, e_out)
    assert e_in[1] < e_in[0] / 3 and e_in[1] < 1.5e-2
    assert e_out[1] < e_out[0] / 3 and e_out[1] < 5e-4


@pytest.mark.slow
def test_field_of_solution_converges_to_series(oracle_lib):
    from oracle.solve import PreconditionedSystem
    k0, k1, rho = 2.0, 3.0, 1.5
    g = np.linspace(-1.5, 1.5, 21)
    X, Z = np.meshgrid(g, g)
    pts = np.stack([X.ravel(), 0 * X.ravel(), Z.ravel()], 1)
    um = mie.total_field(k0, k1, rho, pts)
    rr = np.linalg.norm(pts, axis=1)
    band = np.abs(rr - 1) > 0.15   # the 6-point rule is coarse next to the surface
    errs = []
    for L in (2, 3):
        m = icosphere(L)
        x, _, _ = PreconditionedSystem(m, k0, k1, rho).solve([0, 0, 1], tol=1e-8)
        u, reg = field(m, k0, k1, rho, x, [0, 0, 1], pts)
        assert np.array_equal(reg > 0, rr < 1)
        errs.append(np.linalg.norm((u - um)[band]) / np.linalg.norm(um[band]))
    print(errs)
    assert errs[1] < errs[0] / 3 and errs[1] < 1e-2
