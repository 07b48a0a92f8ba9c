"""Closed, outward-oriented triangle meshes of spheres and ellipsoids.

Constructions:
  * icosphere(L): the regular icosahedron refined L times by edge-midpoint
    subdivision (each triangle -> 4), every new vertex pushed radially onto the
    sphere at the level where it is created.  Vertex count 10*4^L + 2.
  * geodesic_sphere(n): every icosahedron face cut into n^2 triangles on its
    barycentric grid, then all vertices pushed radially onto the sphere.
    Vertex count 10*n^2 + 2.
  * ellipsoid(base, axes): a sphere mesh scaled per axis (orientation kept).
  * two_spheres(L, centres): two disjoint icospheres, vertices of each object
    contiguous, with a per-triangle object id.

Triangles are 0-based vertex triples ordered counter-clockwise when seen from
outside, i.e. (v1-v0) x (v2-v0) points away from the enclosed volume.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import combinations
from typing import Optional, Tuple

import numpy as np


@dataclass
class Mesh:
    vertices: np.ndarray            # float64 [N, 3]
    triangles: np.ndarray           # int32 [T, 3]
    object_id: Optional[np.ndarray] = None   # int32 [T] or None (one object)
    name: str = ""
    radius: float = 1.0             # circumradius about the object's centroid
    meta: dict = field(default_factory=dict)

    @property
    def n_vertices(self) -> int:
        return int(self.vertices.shape[0])

    @property
    def n_triangles(self) -> int:
        return int(self.triangles.shape[0])

    def n_objects(self) -> int:
        return 1 if self.object_id is None else int(self.object_id.max()) + 1


def mesh_counts(level: int) -> Tuple[int, int]:
    """(vertices, triangles) of an icosphere of the given subdivision level."""
    return 10 * 4 ** level + 2, 20 * 4 ** level


def _icosahedron() -> Tuple[np.ndarray, np.ndarray]:
    g = (1.0 + 5.0 ** 0.5) / 2.0
    pts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            pts.append((0.0, s1, s2 * g))
            pts.append((s1, s2 * g, 0.0))
            pts.append((s2 * g, 0.0, s1))
    v = np.array(pts, dtype=np.float64)
    # faces are the vertex triples with all three edges of length 2
    faces = []
    for a, b, c in combinations(range(12), 3):
        if (abs(np.linalg.norm(v[a] - v[b]) - 2.0) < 1e-9 and
                abs(np.linalg.norm(v[b] - v[c]) - 2.0) < 1e-9 and
                abs(np.linalg.norm(v[a] - v[c]) - 2.0) < 1e-9):
            nrm = np.cross(v[b] - v[a], v[c] - v[a])
            if np.dot(nrm, v[a] + v[b] + v[c]) < 0:
                b, c = c, b
            faces.append((a, b, c))
    assert len(faces) == 20
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, np.array(faces, dtype=np.int64)


def icosphere(level: int, radius: float = 1.0,
              centre=(0.0, 0.0, 0.0)) -> Mesh:
    v, f = _icosahedron()
    verts = [tuple(p) for p in v]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = np.array(verts[a]) + np.array(verts[b])
                p /= np.linalg.norm(p)
                idx = len(verts)
                verts.append(tuple(p))
                cache[key] = idx
            return idx

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int64)
    vert = np.array(verts, dtype=np.float64) * radius + np.asarray(centre)
    m = Mesh(vert, f.astype(np.int32), None, name=f"icosphere{level}",
             radius=float(radius))
    return m


def geodesic_sphere(n: int, radius: float = 1.0) -> Mesh:
    v, f = _icosahedron()
    keys = {}
    pts = []

    def point(face, i, j):
        a, b, c = face
        w = {}
        for vid, wt in ((a, n - i - j), (b, i), (c, j)):
            if wt > 0:
                w[vid] = w.get(vid, 0) + wt
        key = tuple(sorted(w.items()))
        idx = keys.get(key)
        if idx is None:
            p = sum(wt * v[vid] for vid, wt in w.items()) / n
            p = p / np.linalg.norm(p)
            idx = len(pts)
            pts.append(p)
            keys[key] = idx
        return idx

    tris = []
    for face in f:
        grid = {}
        for i in range(n + 1):
            for j in range(n + 1 - i):
                grid[(i, j)] = point(face, i, j)
        for i in range(n):
            for j in range(n - i):
                tris.append((grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]))
                if i + j < n - 1:
                    tris.append((grid[(i + 1, j)], grid[(i + 1, j + 1)],
                                 grid[(i, j + 1)]))
    P = np.array(pts, dtype=np.float64)
    T = np.array(tris, dtype=np.int64)
    # orient outward (the sphere is convex about the origin)
    nrm = np.cross(P[T[:, 1]] - P[T[:, 0]], P[T[:, 2]] - P[T[:, 0]])
    flip = np.einsum("ij,ij->i", nrm, P[T].sum(axis=1)) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return Mesh(P * radius, T.astype(np.int32), None, name=f"geodesic{n}",
                radius=float(radius))


def ellipsoid(base: Mesh, axes=(1.0, 0.6, 0.4)) -> Mesh:
    ax = np.asarray(axes, dtype=np.float64)
    P = base.vertices * ax
    c = P.mean(axis=0)
    return Mesh(P, base.triangles.copy(), None,
                name=f"ellipsoid({base.name};{axes})",
                radius=float(np.linalg.norm(P - c, axis=1).max()))


def two_spheres(level: int = 4, offset: float = 1.5,
                radius: float = 1.0) -> Mesh:
    a = icosphere(level, radius, centre=(0.0, -offset, 0.0))
    b = icosphere(level, radius, centre=(0.0, offset, 0.0))
    P = np.vstack([a.vertices, b.vertices])
    T = np.vstack([a.triangles, b.triangles + a.n_vertices]).astype(np.int32)
    oid = np.concatenate([np.zeros(a.n_triangles, np.int32),
                          np.ones(b.n_triangles, np.int32)])
    return Mesh(P, T, oid, name=f"two_spheres{level}", radius=float(radius))


def four_spheres(level: int = 2, radius: float = 1.0, geodesic: int = 0) -> Mesh:
    """Four disjoint spheres of the given radius with centres at
    (+-3, +-1.5, 0) radii: the layout of the paper's multiple-scattering test
    (radius 5 mm, centres (+-15, +-7.5, 0) mm) in units of the radius.
    Objects 0..3 in the order (-3,-1.5), (3,-1.5), (-3,1.5), (3,1.5).  Each
    sphere is an icosphere of the given level, or with geodesic > 0 a
    geodesic sphere of 10 geodesic^2 + 2 vertices."""
    centres = [(sx * 3.0 * radius, sy * 1.5 * radius, 0.0) for sy in (-1, 1) for sx in (-1, 1)]
    if geodesic > 0:
        g = geodesic_sphere(geodesic, radius)
        parts = [Mesh(g.vertices + np.asarray(c), g.triangles.copy(), None, name=g.name,
                      radius=float(radius)) for c in centres]
    else:
        parts = [icosphere(level, radius, centre=c) for c in centres]
    P, T, oid, off = [], [], [], 0
    for o, p in enumerate(parts):
        P.append(p.vertices)
        T.append(p.triangles + off)
        oid.append(np.full(p.n_triangles, o, np.int32))
        off += p.n_vertices
    return Mesh(np.vstack(P), np.vstack(T).astype(np.int32), np.concatenate(oid),
                name=f"four_spheres{level}" if geodesic <= 0 else f"four_spheres_g{geodesic}",
                radius=float(radius))
