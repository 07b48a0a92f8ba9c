"""C-ABI library checks that need no GPU: the shared library loads, exports
every function include/bem.h declares, and host-side mesh validation rejects
malformed surfaces with the documented error codes before any device call."""
import os
import re

import numpy as np
import pytest

from bem_inputs import icosphere, two_spheres

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_][a-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def P():
    import paper_2104_04609_amd as P
    return P


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("bem_mesh_create", "bem_mesh_destroy", "pmchwt_matvec", "osrc_apply",
              "pmchwt_rhs", "pmchwt_solve", "bem_last_error", "bem_far_field"):
        assert n in names


def test_library_exports_every_declared_symbol(P):
    from paper_2104_04609_amd._binding import exported_symbols
    assert exported_symbols(declared_functions()) == []


def test_default_options(P):
    o = P.default_opts()
    assert o.pade_terms == 4 and abs(o.theta - np.pi / 3) < 1e-15
    assert o.osrc_interior == 1 and o.precision == P.BEM_FP64


def _bad(P, vertices, triangles, object_id=None, code=-2):
    with pytest.raises(P.BemError) as e:
        P.Mesh(vertices, triangles, object_id)
    assert e.value.code == code, str(e.value)


def test_open_mesh_rejected(P):
    m = icosphere(1)
    _bad(P, m.vertices, m.triangles[:-1])


def test_inconsistent_orientation_rejected(P):
    m = icosphere(1)
    T = m.triangles.copy()
    T[5] = T[5][[0, 2, 1]]
    _bad(P, m.vertices, T)


def test_inward_normals_rejected(P):
    m = icosphere(1)
    _bad(P, m.vertices, m.triangles[:, [0, 2, 1]])


def test_degenerate_triangle_rejected(P):
    m = icosphere(1)
    V = m.vertices.copy()
    a, b, c = m.triangles[0]
    V[c] = 0.5 * (V[a] + V[b])
    _bad(P, V, m.triangles)


def test_index_out_of_range_rejected(P):
    m = icosphere(1)
    T = m.triangles.copy()
    T[0, 0] = m.n_vertices
    _bad(P, m.vertices, T, code=-1)


def test_objects_must_not_share_vertices(P):
    m = two_spheres(1)
    oid = m.object_id.copy()
    oid[0] = 1   # a triangle of object 0 labelled as object 1
    _bad(P, m.vertices, m.triangles, oid)


def test_objects_must_have_contiguous_vertices(P):
    m = two_spheres(1)
    # swap object labels so that the vertex blocks are in decreasing order
    _bad(P, m.vertices, m.triangles, 1 - m.object_id)
