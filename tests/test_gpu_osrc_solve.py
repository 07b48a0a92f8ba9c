"""GPU parity of the OSRC preconditioner and the preconditioned GMRES solve
against the FP64 oracle, through the C ABI.

* osrc_apply (strong form, diag(L_DtN, L_NtD)) element by element, <= 1e-10,
  for N_p = 1, 4, 8, 16 (both operators' solves in one batch; 16 is the
  largest such batch) and 20 (two stages), real and lossy wavenumbers, one
  and two objects.
* pmchwt_solve FP64: the solution agrees with the oracle's GMRES solution to
  the accuracy both solves reach; iteration counts agree within 2 (several
  solutions of the rounding are valid; the discrete solution is unique).
* pmchwt_solve FP32 + refinement: the true FP64 residual reaches tol and the
  solution agrees with the FP64 one.
* far field against the Mie series: |e_GPU - e_oracle| <= 1e-3.
"""
import numpy as np
import pytest

from bem_inputs import complex_normal, icosphere, two_spheres

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2104_04609_amd as P
    return P


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


OSRC_CASES = {
    "ico3_np4": (lambda: icosphere(3), 3.0, 4, np.pi / 3, 0.1),
    "ico2_np8_lossy": (lambda: icosphere(2), 6.0 + 0.3j, 8, np.pi / 3, 0.1),
    "ico2_np1_theta0": (lambda: icosphere(2), 2.0, 1, 0.0, 0.5),
    "two_spheres2": (lambda: two_spheres(2, offset=1.5), 4.0, 4, np.pi / 3, 0.1),
    "ico5_np4": (lambda: icosphere(5), 15.0, 4, np.pi / 3, 0.1),
    "ico3_np16_lossy": (lambda: icosphere(3), 5.0 + 0.2j, 16, np.pi / 3, 0.1),
    "ico3_np20_two_stages": (lambda: icosphere(3), 5.0, 20, np.pi / 4, 0.1),
}


@pytest.mark.parametrize("case", sorted(OSRC_CASES))
def test_osrc_apply_matches_oracle(P, case):
    from oracle.osrc import OSRC, damped_wavenumber
    make, k, n_p, theta, R = OSRC_CASES[case]
    mesh = make()
    N = mesh.n_vertices
    keps = damped_wavenumber(k, R)
    print(f"osrc {case} N={N} k={k} keps={keps}", flush=True)
    ref_op = OSRC(mesh, k, keps, n_p, theta)
    x = complex_normal(2 * N, seed=11)
    ref = ref_op.apply(x)
    M = P.Mesh.from_inputs(mesh)
    y = P.osrc_apply(M, n_p, theta, k, keps, _dev(x)).cpu().numpy()
    for sl in (slice(0, N), slice(N, 2 * N)):
        err = np.linalg.norm(y[sl] - ref[sl]) / np.linalg.norm(ref[sl])
        print(case, err)
        assert err <= 1e-10, err


# schedules of the block solves:
# (osrc.split, osrc.sub_rows, osrc.top_single_work, osrc.bottom_rows)
SCHEDULES = {
    "levels": (0, 0, 300000, 1024),            # one launch per dissection level
    "auto": (1, 0, 300000, 1024),              # the default: bottom subtrees, plan per batch
    "split_default": (2, 0, 300000, 1024),     # two-part with partial sums of the top rows
    "split_top_single": (2, 512, 1 << 30, 1024),  # many subtrees, big top in one workgroup
    "split_top_levels": (2, 512, 0, 1024),        # many subtrees, top level by level
    "split_tiny": (2, 64, 1 << 30, 1024),
    "bottom_1024": (3, 0, 300000, 1024),       # one bottom-subtree plan, top by level kernels
    "bottom_tiny": (3, 0, 300000, 64),
    "bottom_large": (3, 0, 300000, 4096),
}


@pytest.fixture
def osrc_schedule(P):
    keys = ("osrc.split", "osrc.sub_rows", "osrc.top_single_work", "osrc.bottom_rows")
    old = [P.tune_get(k) for k in keys]

    def set_(vals):
        for k, v in zip(keys, vals):
            P.tune_set(k, v)
    yield set_
    set_(old)


@pytest.mark.parametrize("mesh_name", ["ico4", "two_spheres3"])
@pytest.mark.parametrize("schedule", sorted(SCHEDULES))
def test_osrc_apply_schedules(P, osrc_schedule, schedule, mesh_name):
    """Every schedule of the block solves (fresh mesh handles, since the
    schedule is fixed when a handle builds its OSRC state) against the oracle,
    4 vectors with 8 Pade terms and a lossy wavenumber."""
    from oracle.osrc import OSRC, damped_wavenumber
    mesh = icosphere(4) if mesh_name == "ico4" else two_spheres(3, offset=1.5)
    N = mesh.n_vertices
    k = 9.0 + 0.4j
    keps = damped_wavenumber(k, 0.1)
    osrc_schedule(SCHEDULES[schedule])
    M = P.Mesh.from_inputs(mesh)
    X = complex_normal((4, 2 * N), seed=17)
    print(f"osrc schedule {schedule} {mesh_name}", flush=True)
    Y = P.osrc_apply(M, 8, np.pi / 3, k, keps, _dev(X)).cpu().numpy()
    op = OSRC(mesh, k, keps, 8, np.pi / 3)
    for r in range(4):
        ref = op.apply(X[r])
        for sl in (slice(0, N), slice(N, 2 * N)):
            err = np.linalg.norm(Y[r][sl] - ref[sl]) / np.linalg.norm(ref[sl])
            assert err <= 1e-10, (schedule, r, err)


def test_osrc_apply_batched_rhs(P):
    import torch
    mesh = icosphere(2)
    N = mesh.n_vertices
    M = P.Mesh.from_inputs(mesh)
    X = _dev(complex_normal((3, 2 * N), seed=5))
    Y = P.osrc_apply(M, 4, np.pi / 3, 3.0, 3.3 + 0.9j, X)
    for r in range(3):
        yr = P.osrc_apply(M, 4, np.pi / 3, 3.0, 3.3 + 0.9j, X[r].contiguous())
        assert torch.equal(yr, Y[r])


@pytest.mark.parametrize("level", [3, 4])
def test_osrc_info_sizes(P, level):
    """bem_osrc_info: the P1 mass pattern of a closed genus-0 triangulation
    holds the diagonal and both directions of every edge, N + 2 (3N - 6)
    entries (Euler: E = 3N - 6); N_p + 2 factors, 2 N_p + 2 block solves per
    apply, the factor bytes of their stored parts."""
    mesh = icosphere(level)
    N = mesh.n_vertices
    M = P.Mesh.from_inputs(mesh)
    st = P.osrc_info(M, 4, np.pi / 3, 15.0, 15.0 + 2.0j)
    print(st)
    assert st["n_vertices"] == N
    assert st["mass_nnz"] == 7 * N - 12
    assert st["n_factors"] == 6 and st["solves_per_apply"] == 10
    assert 0 < st["nnz_offblock"] <= st["nnz_l"]
    assert st["factor_bytes"] == 16 * 6 * (N + 2 * st["nnz_l"] + 2 * st["dense_entries"])
    assert st["bytes_per_apply"] > 10 * 16 * 2 * N
    with pytest.raises(P.BemError):
        P.osrc_info(M, 0, np.pi / 3, 15.0, 15.0 + 2.0j)


_SOLVES = {}


def oracle_solve(mesh, k0, k1, rho, tol):
    from oracle.solve import PreconditionedSystem
    key = (mesh.name, k0, k1, rho, tol)
    if key not in _SOLVES:
        S = PreconditionedSystem(mesh, k0, k1, rho)
        x, it, hist = S.solve([0, 0, 1], tol=tol)
        _SOLVES[key] = (S, x, it)
    return _SOLVES[key]


SOLVE_CASES = {
    "C1_ico3": (lambda: icosphere(3), 2.0, 3.0, 1.5),
    "two_spheres2": (lambda: two_spheres(2, offset=1.5), 2.0, 3.0 + 0.2j, 1.3),
}


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("case", sorted(SOLVE_CASES))
def test_solve_fp64_matches_oracle(P, case, path):
    """FP64 GMRES on the matrix-free operator (path 0) and on the assembled
    complex128 operator (path 1)."""
    make, k0, k1, rho = SOLVE_CASES[case]
    mesh = make()
    print(f"solve {case} path {path}", flush=True)
    S, xo, it_o = oracle_solve(mesh, k0, k1, rho, 1e-10)
    M = P.Mesh.from_inputs(mesh)
    sol, info, rc = P.pmchwt_solve(M, k0, k1, rho, [[0.0, 0.0, 1.0]], 1e-10, path=path)
    x = sol.cpu().numpy()[0]
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(case, "err", err, "iters gpu", info[0]["iterations"], "oracle", it_o, info[0])
    assert rc == 0
    assert err <= 1e-8
    assert abs(info[0]["iterations"] - it_o) <= 2
    assert info[0]["rel_residual"] <= 1e-10 * 1.01
    # the oracle's own residual of the GPU solution
    b = S.rhs([0, 0, 1])
    assert np.linalg.norm(S.apply(x) - b) / np.linalg.norm(b) <= 2e-10


def test_auto_path_fp64_uses_assembled_operator(P):
    """path 2 (the default) with FP64 on a mesh whose complex128 operator fits:
    the same operator as path 1, so the same solution bit for bit (fixed
    reduction order); the matrix-free path 0 agrees within the solve accuracy.
    The server resolves the request the same way and reports path 1."""
    import torch
    P.tune_clear()   # no autotuned preference for the matrix-free path
    mesh = icosphere(3)
    M = P.Mesh.from_inputs(mesh)
    d = [[0.0, 0.0, 1.0]]
    print("auto path fp64 ico3", flush=True)
    s2, i2, rc2 = P.pmchwt_solve(M, 2.0, 3.0, 1.5, d, 1e-10, precision="fp64", path=2)
    s1, i1, rc1 = P.pmchwt_solve(M, 2.0, 3.0, 1.5, d, 1e-10, precision="fp64", path=1)
    s0, i0, rc0 = P.pmchwt_solve(M, 2.0, 3.0, 1.5, d, 1e-10, precision="fp64", path=0)
    assert rc0 == rc1 == rc2 == 0
    assert torch.equal(s1, s2) and i1[0]["iterations"] == i2[0]["iterations"]
    assert (torch.linalg.norm(s0 - s2) / torch.linalg.norm(s0)).item() <= 1e-8
    srv = P.Server(workers=1)
    try:
        mid = srv.add_mesh(mesh.vertices, mesh.triangles)
        rid = srv.submit(mid, 2.0, 3.0, 1.5, d, 1e-10, precision="fp64", path=2)
        sol, info, st = srv.wait(rid)
    finally:
        srv.close()
    assert st["status"] == 0 and st["path"] == 1
    assert torch.equal(sol.to(s2.device), s2)


@pytest.mark.parametrize("path", [0, 1])
def test_solve_fp32_refinement(P, path):
    """path 0: FP32 matrix-free pair kernel; path 1: assembled complex64."""
    mesh = icosphere(3)
    M = P.Mesh.from_inputs(mesh)
    S, xo, _ = oracle_solve(mesh, 2.0, 3.0, 1.5, 1e-10)
    sol, info, rc = P.pmchwt_solve(M, 2.0, 3.0, 1.5, [[0.0, 0.0, 1.0]], 1e-6,
                                   precision="fp32", path=path)
    x = sol.cpu().numpy()[0]
    print(info[0])
    assert rc == 0 and info[0]["rel_residual"] <= 1e-6
    assert info[0]["fp32_matvecs"] >= info[0]["iterations"]
    b = S.rhs([0, 0, 1])
    assert np.linalg.norm(S.apply(x) - b) / np.linalg.norm(b) <= 1.5e-6
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-4


def test_far_field_against_mie(P):
    from oracle import mie
    from oracle.rhs import far_field
    mesh = icosphere(3)
    k0, k1, rho = 2.0, 3.0, 1.5
    _, xo, _ = oracle_solve(mesh, k0, k1, rho, 1e-10)
    M = P.Mesh.from_inputs(mesh)
    sol, info, rc = P.pmchwt_solve(M, k0, k1, rho, [[0.0, 0.0, 1.0]], 1e-8)
    th = np.linspace(0, np.pi, 181)
    dirs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    Fm = mie.far_field(k0, k1, rho, th)
    Fg = P.far_field(M, k0, sol[0].contiguous(), dirs)
    Fo = far_field(mesh, k0, xo, dirs)
    eg = np.linalg.norm(Fg - Fm) / np.linalg.norm(Fm)
    eo = np.linalg.norm(Fo - Fm) / np.linalg.norm(Fm)
    print("mie errors", eg, eo)
    assert abs(eg - eo) <= 1e-3 and eg < 1.5e-2


def test_solve_not_converged_returns_best_iterate(P):
    mesh = icosphere(2)
    M = P.Mesh.from_inputs(mesh)
    sol, info, rc = P.pmchwt_solve(M, 2.0, 3.0, 1.5, [[0.0, 0.0, 1.0]], 1e-10, maxiter=3)
    assert rc == 1   # BEM_W_NOT_CONVERGED
    assert info[0]["iterations"] == 3
    assert 0 < info[0]["rel_residual"] < 1.0
    assert np.isfinite(sol.cpu().numpy()).all()


@pytest.mark.parametrize("precision,path", [("fp64", 0), ("fp64", 1), ("fp32", 0)])
def test_solve_reports_nan(P, precision, path):
    """A density ratio whose reciprocal overflows (rho = 1e-320 > 0 passes the
    argument checks, 1/rho = inf): the operator holds Inf, the first Arnoldi
    step meets NaN, and the solve returns BEM_E_NAN instead of iterating."""
    mesh = icosphere(1)
    M = P.Mesh.from_inputs(mesh)
    assert 1.0 / 1e-320 == float("inf")
    with pytest.raises(P.BemError) as e:
        P.pmchwt_solve(M, 2.0, 3.0, 1e-320, [[0.0, 0.0, 1.0]], 1e-8, precision=precision,
                       path=path)
    assert e.value.code == -5, e.value
    # the handle stays usable
    sol, info, rc = P.pmchwt_solve(M, 2.0, 3.0, 1.5, [[0.0, 0.0, 1.0]], 1e-8,
                                   precision=precision, path=path)
    assert rc == 0 and info[0]["rel_residual"] <= 1e-8


def test_solve_multiple_waves(P):
    """FP64: waves solved in one lockstep group (pair kernel shared by two
    vectors, summed in another order) against each wave alone, both to 1e-9;
    the discrete solution is unique, so they agree to the solve accuracy."""
    from bem_inputs import wave_directions
    mesh = icosphere(2)
    M = P.Mesh.from_inputs(mesh)
    d = wave_directions(3, seed=2)
    sol, info, rc = P.pmchwt_solve(M, 2.0, 3.0, 1.5, d, 1e-9)
    assert rc == 0
    for w in range(3):
        one, i1, _ = P.pmchwt_solve(M, 2.0, 3.0, 1.5, d[w:w + 1], 1e-9)
        a, b = sol.cpu().numpy()[w], one.cpu().numpy()[0]
        assert info[w]["rel_residual"] <= 1e-9 and i1[0]["rel_residual"] <= 1e-9
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-8, w


def test_solve_lockstep_groups_fp64(P):
    """18 waves: a full lockstep group of 16 (every wave orthogonalised in one
    launch per step) and a group of 2, against waves solved alone."""
    from bem_inputs import wave_directions
    mesh = icosphere(2)
    M = P.Mesh.from_inputs(mesh)
    d = wave_directions(18, seed=4)
    sol, info, rc = P.pmchwt_solve(M, 2.5, 3.5, 1.4, d, 1e-10, precision="fp64", path=1)
    assert rc == 0
    X = sol.cpu().numpy()
    for w in (0, 7, 15, 16, 17):
        one, i1, rc1 = P.pmchwt_solve(M, 2.5, 3.5, 1.4, d[w:w + 1], 1e-10, precision="fp64", path=1)
        assert rc1 == 0 and info[w]["rel_residual"] <= 1e-10 and i1[0]["rel_residual"] <= 1e-10
        b = one.cpu().numpy()[0]
        assert np.linalg.norm(X[w] - b) / np.linalg.norm(b) < 1e-8, w
        assert abs(info[w]["iterations"] - i1[0]["iterations"]) <= 1, w


def test_solve_lockstep_waves_fp32_dense(P):
    """Waves solved in one lockstep group (multi-vector dense product, batched
    OSRC) against each wave solved alone; both to 1e-9."""
    from bem_inputs import wave_directions
    mesh = icosphere(3)
    M = P.Mesh.from_inputs(mesh)
    d = wave_directions(5, seed=8)
    sol, info, rc = P.pmchwt_solve(M, 3.0, 4.5, 1.6, d, 1e-9, precision="fp32", path=1)
    assert rc == 0
    for w in range(5):
        one, i1, _ = P.pmchwt_solve(M, 3.0, 4.5, 1.6, d[w:w + 1], 1e-9, precision="fp32", path=1)
        a, b = sol.cpu().numpy()[w], one.cpu().numpy()[0]
        assert info[w]["rel_residual"] <= 1e-9 and i1[0]["rel_residual"] <= 1e-9
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-7, w
