"""The synthetic Menger sponge surface (stand-in for the paper's Gmsh mesh
of the level-2 sponge) is a closed, consistently oriented triangle surface
enclosing exactly the sponge: checked against the sponge's own volume
(400 of 729 voxels) and area (1056 voxel faces), and its Euler
characteristic does not depend on the subdivision."""
import numpy as np
import pytest

from bem_inputs import menger_sponge


def _geometry(m):
    P, T = m.vertices, m.triangles
    a, b, c = P[T[:, 0]], P[T[:, 1]], P[T[:, 2]]
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1).sum()
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0   # divergence theorem
    return area, vol


@pytest.mark.parametrize("k", [1, 3])
def test_sponge_closed_oriented_volume_area(k):
    m = menger_sponge(2, k, edge=10.0)
    T = m.triangles
    directed = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    keys = directed[:, 0].astype(np.int64) * m.n_vertices + directed[:, 1]
    rev = directed[:, 1].astype(np.int64) * m.n_vertices + directed[:, 0]
    assert len(np.unique(keys)) == len(keys)          # each directed edge once
    assert np.array_equal(np.sort(keys), np.sort(rev))  # and its reverse once
    area, vol = _geometry(m)
    h = 10.0 / 9
    assert area == pytest.approx(1056 * h * h, rel=1e-12)
    assert vol == pytest.approx(400 * h ** 3, rel=1e-12)   # positive: normals outward
    E = len(keys) // 2
    assert m.n_vertices - E + m.n_triangles == -160        # genus 81, any k
