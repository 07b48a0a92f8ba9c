"""Writes c2_solution.npz: the oracle's solution of the OSRC-preconditioned
permuted PMCHWT system for the metric workload (unit sphere as icosphere
level 5, 10 242 vertices, k_ext = 10, k_int = 15, rho = 1.5, plane wave along
+z, 4 Pade terms, theta = pi/3, OSRC at the interior wavenumber), GMRES to a
relative preconditioned residual of 1e-10, plus its far field on 181 polar
angles of the x-z plane and that far field's relative L2 error against the
series solution.  Calls only the oracle (dense complex128 assembly, SciPy
sparse LU for the OSRC systems, MGS GMRES): about 10 minutes on 8 cores and
20 GB of memory.

    python tests/golden/make_c2_solution.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from bem_inputs import icosphere  # noqa: E402
from oracle import mie  # noqa: E402
from oracle.rhs import far_field  # noqa: E402
from oracle.solve import PreconditionedSystem  # noqa: E402

K_EXT, K_INT, RHO, TOL = 10.0, 15.0, 1.5, 1e-10


def main():
    t0 = time.time()
    mesh = icosphere(5)
    assert mesh.n_vertices == 10242
    S = PreconditionedSystem(mesh, K_EXT, K_INT, RHO)
    print(f"assembled in {time.time() - t0:.0f} s", flush=True)
    x, it, hist = S.solve([0.0, 0.0, 1.0], tol=TOL, maxiter=400)
    print(f"GMRES: {it} iterations, residual {hist[-1]:.2e}, {time.time() - t0:.0f} s",
          flush=True)
    b = S.rhs([0.0, 0.0, 1.0])
    res = np.linalg.norm(S.apply(x) - b) / np.linalg.norm(b)
    th = np.linspace(0.0, np.pi, 181)
    dirs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    Fo = far_field(mesh, K_EXT, x, dirs)
    Fm = mie.far_field(K_EXT, K_INT, RHO, th)
    e = np.linalg.norm(Fo - Fm) / np.linalg.norm(Fm)
    print(f"true residual {res:.2e}, far-field error vs series {e:.3e}", flush=True)
    np.savez_compressed(os.path.join(HERE, "c2_solution.npz"), x=x, iterations=it,
                        residual=res, far_field=Fo, mie_error=e, k_ext=K_EXT, k_int=K_INT,
                        rho=RHO, tol=TOL, direction=np.array([0.0, 0.0, 1.0]))


if __name__ == "__main__":
    main()
