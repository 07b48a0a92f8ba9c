"""Writes c3_rows.npz: oracle rows of y = B x for the precision-form workload
(ellipsoid (1, 0.6, 0.4) from icosphere level 6, k_ext = 20,
k_int = 30 + 1.5i, rho = 1.9), x = complex standard normal (seed 0), 512
vertex rows sampled with seed 1.  Calls only the oracle.

    python tests/golden/make_c3_rows.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from bem_inputs import complex_normal, ellipsoid, icosphere, sample_rows  # noqa: E402
from oracle.operators import pmchwt_matvec_rows  # noqa: E402


def main():
    mesh = ellipsoid(icosphere(6))
    N = mesh.n_vertices
    x = complex_normal(2 * N, seed=0)
    rows = sample_rows(N, 512, seed=1)
    r1, r2 = pmchwt_matvec_rows(mesh, 20.0, 30.0 + 1.5j, 1.9, x, rows)
    np.savez(os.path.join(HERE, "c3_rows.npz"), rows=rows, r1=r1, r2=r2,
             k_ext=20.0, k_int=30.0 + 1.5j, rho=1.9, seed_x=0, seed_rows=1)


if __name__ == "__main__":
    main()
