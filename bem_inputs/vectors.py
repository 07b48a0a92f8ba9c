"""Seeded random vectors, wave directions, sampled row sets and request streams."""
from __future__ import annotations

import numpy as np


def complex_normal(shape, seed: int = 0) -> np.ndarray:
    """Complex128 array with independent standard-normal real and imaginary parts."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im).astype(np.complex128)


def wave_directions(n: int, seed: int = 2104) -> np.ndarray:
    """n unit vectors, uniform on the sphere (normalised Gaussian draws)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def sample_rows(n_rows: int, count: int, seed: int = 1) -> np.ndarray:
    """Sorted sample of distinct row indices (without replacement)."""
    rng = np.random.default_rng(seed)
    count = min(count, n_rows)
    return np.sort(rng.choice(n_rows, size=count, replace=False)).astype(np.int64)


def request_stream(n_requests: int = 256, seed: int = 5, rate: float = 1.0,
                   mesh_names=("ico3", "ico4", "ico5", "ellipsoid45",
                               "two_spheres4")):
    """Poisson arrivals of solve requests with random meshes and materials.

    Each request: arrival time (s), mesh name, k_ext ~ U[1, 20],
    k_int / k_ext ~ U[1.3, 1.9], rho ~ U[1.2, 2.0], 1-8 plane waves with
    uniformly random directions.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        mesh = mesh_names[int(rng.integers(len(mesh_names)))]
        k_ext = float(rng.uniform(1.0, 20.0))
        ratio = float(rng.uniform(1.3, 1.9))
        rho = float(rng.uniform(1.2, 2.0))
        nw = int(rng.integers(1, 9))
        d = rng.standard_normal((nw, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        out.append(dict(id=i, arrival=t, mesh=mesh, k_ext=k_ext,
                        k_int=k_ext * ratio, rho=rho, directions=d))
    return out
