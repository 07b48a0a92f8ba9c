"""Seeded, synthetic inputs shared by the HIP path's tests/bench and by the oracle.

This package holds no arithmetic of the boundary element method itself: it only
builds triangle meshes (vertex coordinates and connectivity), holds the media
table of the paper's benchmarks, and draws seeded random vectors, plane-wave
directions and request streams.  Both the GPU path
and the CPU oracle consume what it produces; neither shares any other code.
"""
from .meshes import (icosphere, geodesic_sphere, ellipsoid, two_spheres,
                     four_spheres, mesh_counts, Mesh)
from .materials import MEDIA, wavenumber, density_ratio
from .vectors import (complex_normal, wave_directions, request_stream,
                      sample_rows)

__all__ = ["icosphere", "geodesic_sphere", "ellipsoid", "two_spheres", "four_spheres",
           "MEDIA", "wavenumber", "density_ratio",
           "mesh_counts", "Mesh", "complex_normal", "wave_directions",
           "request_stream", "sample_rows"]
