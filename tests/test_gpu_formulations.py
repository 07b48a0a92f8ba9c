"""GPU tests of the mass- and Calderon-preconditioned PMCHWT solves
(Sec. 2.4, 2.5) through pmchwt_solve, against the oracle's solves of the same
preconditioned systems and against the OSRC-preconditioned solution (all
three solve the same B x = f)."""
import numpy as np
import pytest

from bem_inputs import icosphere, two_spheres

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2104_04609_amd as P
    return P


CASES = {
    "C1_ico3": (lambda: icosphere(3), 2.0, 3.0, 1.5),
    "ico2_lossy": (lambda: icosphere(2), 2.5, 4.0 + 0.3j, 1.9),
}
SYSTEMS = {"mass": "MassPreconditionedSystem", "calderon": "CalderonPreconditionedSystem"}


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("form", sorted(SYSTEMS))
@pytest.mark.parametrize("case", sorted(CASES))
def test_formulation_fp64_matches_oracle(P, case, form):
    import oracle.solve as OS
    make, k0, k1, rho = CASES[case]
    mesh = make()
    print(f"{form} {case}", flush=True)
    S = getattr(OS, SYSTEMS[form])(mesh, k0, k1, rho)
    xo, it_o, _ = S.solve([0.0, 0.0, 1.0], tol=1e-10)
    M = P.Mesh.from_inputs(mesh)
    sol, info, rc = P.pmchwt_solve(M, k0, k1, rho, [[0.0, 0.0, 1.0]], 1e-10, formulation=form)
    x = sol.cpu().numpy()[0]
    ref, _, _ = P.pmchwt_solve(M, k0, k1, rho, [[0.0, 0.0, 1.0]], 1e-10)
    print(case, form, "err", _rel(x, xo), "vs osrc", _rel(x, ref.cpu().numpy()[0]),
          "iters gpu", info[0]["iterations"], "oracle", it_o)
    assert rc == 0
    assert _rel(x, xo) <= 1e-8
    assert abs(info[0]["iterations"] - it_o) <= 3
    assert info[0]["rel_residual"] <= 1e-10 * 1.01
    assert _rel(x, ref.cpu().numpy()[0]) <= 1e-8


@pytest.mark.parametrize("path", [0, 1])
def test_calderon_fp32_refinement(P, path):
    make, k0, k1, rho = CASES["C1_ico3"]
    mesh = make()
    M = P.Mesh.from_inputs(mesh)
    d = [[0.0, 0.0, 1.0], [0.6, 0.0, 0.8]]
    sol, info, rc = P.pmchwt_solve(M, k0, k1, rho, d, 1e-8, precision="fp32", path=path,
                                   formulation="calderon")
    ref, _, _ = P.pmchwt_solve(M, k0, k1, rho, d, 1e-10)
    print(path, info)
    assert rc == 0
    for w in range(2):
        assert info[w]["rel_residual"] <= 1e-8
        assert _rel(sol[w].cpu().numpy(), ref[w].cpu().numpy()) <= 1e-6


def test_formulation_errors(P):
    m2 = two_spheres(1, offset=1.5)
    M2 = P.Mesh.from_inputs(m2)
    with pytest.raises(P.BemError):
        P.pmchwt_solve(M2, 2.0, 3.0, 1.5, [[0, 0, 1.0]], 1e-6, formulation="calderon")
    M = P.Mesh.from_inputs(icosphere(1))
    with pytest.raises(P.BemError):
        P.pmchwt_solve(M, 2.0, 3.0, 1.5, [[0, 0, 1.0]], 1e-6, formulation=7)
