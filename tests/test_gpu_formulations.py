"""GPU tests of the formulations compared with the OSRC-preconditioned
PMCHWT (Sec. 3.1) through pmchwt_solve: standard PMCHWT and Mueller in strong
form (Sec. 2.2, 2.4) and the Calderon-preconditioned PMCHWT (Sec. 2.5),
against the oracle's solves of the same systems (solution and iteration
count: GMRES on the paper's ordering) and, for PMCHWT and Calderon, against
the OSRC-preconditioned solution (the same discrete system B x = f)."""
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
SYSTEMS = {"pmchwt": "PMCHWTSystem", "calderon": "CalderonPreconditionedSystem",
           "muller": "MullerSystem"}


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
    if form != "muller":
        assert _rel(x, ref.cpu().numpy()[0]) <= 1e-8


@pytest.mark.parametrize("form", ["calderon", "muller"])
@pytest.mark.parametrize("path", [0, 1])
def test_fp32_refinement(P, path, form):
    make, k0, k1, rho = CASES["C1_ico3"]
    mesh = make()
    M = P.Mesh.from_inputs(mesh)
    d = [[0.0, 0.0, 1.0], [0.6, 0.0, 0.8]]
    sol, info, rc = P.pmchwt_solve(M, k0, k1, rho, d, 1e-8, precision="fp32", path=path,
                                   formulation=form)
    ref, _, _ = P.pmchwt_solve(M, k0, k1, rho, d, 1e-10, formulation=form)
    print(path, info)
    assert rc == 0
    for w in range(2):
        assert info[w]["rel_residual"] <= 1e-8
        assert _rel(sol[w].cpu().numpy(), ref[w].cpu().numpy()) <= 1e-6


def test_calderon_several_objects_matches_oracle(P):
    """Block-diagonal C with several objects (Sec. 2.5): each object's own
    operator, applied through a mesh of each object; two spheres with one
    material and four spheres of fat and bone (a material per object)."""
    import oracle.solve as OS
    from bem_inputs import density_ratio, four_spheres, wavenumber
    f, a = 5e5, 5e-3
    tissue = ["fat", "bone", "bone", "fat"]
    cases = [(two_spheres(1, offset=1.5), 2.0, 3.5 + 0.2j, 1.3),
             (four_spheres(1), wavenumber("water", f, a), [wavenumber(t, f, a) for t in tissue],
              [density_ratio(t) for t in tissue])]
    for mesh, k0, k1, rho in cases:
        d = [0.0, 0.6, 0.8]
        xo, it_o, _ = OS.CalderonPreconditionedSystem(mesh, k0, k1, rho).solve(d, tol=1e-10)
        M = P.Mesh.from_inputs(mesh)
        multi = np.ndim(k1) > 0
        for prec, path in (("fp64", 0), ("fp32", 1)):
            print(f"calderon {mesh.name} {prec}", flush=True)
            fn = P.pmchwt_solve_multi if multi else P.pmchwt_solve
            sol, info, rc = fn(M, k0, k1, rho, [d], 1e-10 if prec == "fp64" else 1e-9,
                               formulation="calderon", precision=prec, path=path)
            x = sol.cpu().numpy()[0]
            print(mesh.name, prec, _rel(x, xo), info[0]["iterations"], it_o)
            assert rc == 0
            assert _rel(x, xo) <= (1e-8 if prec == "fp64" else 1e-7)
            if prec == "fp64":
                assert abs(info[0]["iterations"] - it_o) <= 3


def test_formulation_errors(P):
    M = P.Mesh.from_inputs(icosphere(1))
    with pytest.raises(P.BemError):
        P.pmchwt_solve(M, 2.0, 3.0, 1.5, [[0, 0, 1.0]], 1e-6, formulation=7)


def test_muller_two_objects_matches_oracle(P):
    """Mueller couples the objects through the exterior operators only
    (Sec. 2.2): two spheres against the oracle's Mueller solve."""
    import oracle.solve as OS
    mesh = two_spheres(1, offset=1.5)
    k0, k1, rho = 2.0, 3.5 + 0.2j, 1.3
    xo, it_o, _ = OS.MullerSystem(mesh, k0, k1, rho).solve([0.0, 0.0, 1.0], tol=1e-10)
    M = P.Mesh.from_inputs(mesh)
    sol, info, rc = P.pmchwt_solve(M, k0, k1, rho, [[0.0, 0.0, 1.0]], 1e-10, formulation="muller")
    x = sol.cpu().numpy()[0]
    print("two spheres muller", _rel(x, xo), info[0]["iterations"], it_o)
    assert rc == 0 and _rel(x, xo) <= 1e-8
    assert abs(info[0]["iterations"] - it_o) <= 3
