"""GPU parity of the permuted PMCHWT matvec, RHS and far field against the
FP64 oracle (element by element), through the C ABI.

Bar: relative L2 error <= 1e-10 for the FP64 path and <= 1e-5 for the FP32
path, per block row (the V-row and the D-row differ in scale) and overall.
Sizes: icosphere L3 (C1, all rows, dense oracle), L2 and a geodesic sphere
(ragged triangle counts), two objects, lossy wavenumbers, and the full
icosphere L5 workload on seed-sampled rows.
"""
import numpy as np
import pytest

from bem_inputs import (complex_normal, geodesic_sphere, icosphere, sample_rows,
                        two_spheres, wave_directions)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "fp32_dense": 1e-5, "fp64_dense": 1e-10}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2104_04609_amd as P
    return P


_DENSE = {}


def dense(mesh, k0, k1, rho):
    from oracle.operators import pmchwt_matrix
    key = (mesh.name, complex(k0), complex(k1), rho)
    if key not in _DENSE:
        _DENSE[key] = pmchwt_matrix(mesh, k0, k1, rho)
    return _DENSE[key]


def rel_blocks(y, ref, N):
    out = {}
    for name, sl in (("row1", slice(0, N)), ("row2", slice(N, 2 * N)),
                     ("all", slice(0, 2 * N))):
        out[name] = np.linalg.norm(y[sl] - ref[sl]) / np.linalg.norm(ref[sl])
    return out


def gpu_matvec(P, mesh, k0, k1, rho, x, precision):
    import torch
    M = P.Mesh.from_inputs(mesh)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    y = P.pmchwt_matvec(M, k0, k1, rho, xt, precision=precision)
    torch.cuda.synchronize()
    return y.cpu().numpy()


CASES = {
    "C1_ico3": (lambda: icosphere(3), 2.0, 3.0, 1.5),
    "ico2_lossy": (lambda: icosphere(2), 2.5 + 0.3j, 4.0 + 0.6j, 1.9),
    "geodesic3_ragged": (lambda: geodesic_sphere(3), 1.5, 2.2, 0.7),
    "two_spheres1": (lambda: two_spheres(1, offset=1.5), 2.0, 3.5 + 0.2j, 1.3),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_dense", "fp64_dense"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_matvec_matches_dense_oracle(P, case, precision):
    make, k0, k1, rho = CASES[case]
    mesh = make()
    print(f"case {case} N={mesh.n_vertices} T={mesh.n_triangles} {precision}", flush=True)
    N = mesh.n_vertices
    x = complex_normal(2 * N, seed=0)
    ref = dense(mesh, k0, k1, rho) @ x
    y = gpu_matvec(P, mesh, k0, k1, rho, x, precision)
    err = rel_blocks(y, ref, N)
    print(case, precision, err)
    for v in err.values():
        assert v <= TOL[precision], err


def _relabelled(mesh, seed):
    """The same surface with its vertices numbered in a seeded random order
    (within each object's range: the vertices of an object stay contiguous)."""
    from bem_inputs import Mesh
    rng = np.random.default_rng(seed)
    vobj = np.zeros(mesh.n_vertices, dtype=np.int64)
    if mesh.object_id is not None:
        vobj[mesh.triangles.ravel()] = np.repeat(mesh.object_id, 3)
    perm = np.arange(mesh.n_vertices)
    for o in np.unique(vobj):
        idx = np.flatnonzero(vobj == o)
        perm[idx] = rng.permutation(idx)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(mesh.n_vertices)
    return Mesh(vertices=mesh.vertices[perm], triangles=inv[mesh.triangles].astype(np.int32),
                object_id=mesh.object_id, name=mesh.name + f"_relabel{seed}",
                radius=mesh.radius)


@pytest.mark.parametrize("precision", ["fp32_dense", "fp64_dense"])
@pytest.mark.parametrize("operator", ["pmchwt", "pmchwt_multi", "muller"])
def test_assembled_operator_any_vertex_numbering(P, operator, precision):
    """The assembled operators evaluate the entries with rank(i) <= rank(j)
    (vertex ranks in a spatial order) and mirror the others: parity with the
    oracle on meshes whose vertex numbering is a random permutation (one and
    two objects, one material per object), so that ranks and indices are
    unrelated."""
    import torch
    from oracle.operators import muller_matrix, pmchwt_matrix, pmchwt_matrix_multi
    if operator == "pmchwt":
        mesh, k0, k1, rho = _relabelled(icosphere(3), 7), 2.0, 3.0 + 0.1j, 1.5
        A = pmchwt_matrix(mesh, k0, k1, rho)
    elif operator == "pmchwt_multi":
        mesh = _relabelled(two_spheres(1, offset=1.5), 8)
        k0, k1, rho = 2.0, [3.5 + 0.2j, 2.5], [1.3, 0.8]
        A = pmchwt_matrix_multi(mesh, k0, k1, rho)
    else:
        mesh, k0, k1, rho = _relabelled(geodesic_sphere(3), 9), 1.5, 2.2, 0.7
        A = muller_matrix(mesh, k0, k1, rho)
    print(f"relabelled {operator} N={mesh.n_vertices} {precision}", flush=True)
    N = mesh.n_vertices
    x = complex_normal(2 * N, seed=11)
    M = P.Mesh.from_inputs(mesh)
    xt = torch.from_numpy(x[None, :].copy()).cuda()
    if operator == "pmchwt":
        y = P.pmchwt_matvec(M, k0, k1, rho, xt, precision=precision)
    elif operator == "pmchwt_multi":
        y = P.pmchwt_matvec_multi(M, k0, k1, rho, xt, precision=precision)
    else:
        y = P.muller_matvec(M, k0, k1, rho, xt, precision=precision)
    torch.cuda.synchronize()
    err = rel_blocks(y.cpu().numpy()[0], A @ x, N)
    print(operator, precision, err)
    for v in err.values():
        assert v <= TOL[precision], err


def test_matvec_smooth_input_fp32(P):
    # a converged-solution-like smooth input (low-order harmonics)
    mesh = icosphere(3)
    N = mesh.n_vertices
    z = mesh.vertices[:, 2]
    x = np.concatenate([np.exp(2j * z), (0.3 + 0.1j) * z ** 2]).astype(np.complex128)
    ref = dense(mesh, 2.0, 3.0, 1.5) @ x
    y = gpu_matvec(P, mesh, 2.0, 3.0, 1.5, x, "fp32")
    err = rel_blocks(y, ref, N)
    assert max(err.values()) <= TOL["fp32"], err


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_dense", "fp64_dense"])
def test_matvec_full_size_sampled_rows(P, precision):
    """Icosphere L5 (10 242 vertices), k_ext = 10, k_int = 15, rho = 1.5, in
    the launch configuration used for timing; 40 seed-sampled rows of each
    block row against the oracle's matrix-free rows."""
    from oracle.operators import pmchwt_matvec_rows
    mesh = icosphere(5)
    N = mesh.n_vertices
    x = complex_normal(2 * N, seed=0)
    rows = sample_rows(N, 40, seed=1)
    print(f"ico5 sampled rows {precision}", flush=True)
    r1, r2 = pmchwt_matvec_rows(mesh, 10.0, 15.0, 1.5, x, rows)
    y = gpu_matvec(P, mesh, 10.0, 15.0, 1.5, x, precision)
    e1 = np.linalg.norm(y[rows] - r1) / np.linalg.norm(r1)
    e2 = np.linalg.norm(y[N + rows] - r2) / np.linalg.norm(r2)
    print(precision, e1, e2)
    assert e1 <= TOL[precision] and e2 <= TOL[precision], (e1, e2)


def test_matvec_deterministic_and_batched(P):
    import torch
    mesh = icosphere(3)
    N = mesh.n_vertices
    M = P.Mesh.from_inputs(mesh)
    X = torch.from_numpy(complex_normal((3, 2 * N), seed=4)).cuda()
    for prec in ("fp64", "fp32", "fp32_dense"):
        ys = [P.pmchwt_matvec(M, 2.0, 3.0, 1.5, X, precision=prec) for _ in range(3)]
        torch.cuda.synchronize()
        assert torch.equal(ys[0], ys[1]) and torch.equal(ys[0], ys[2])
        for r in range(3):
            yr = P.pmchwt_matvec(M, 2.0, 3.0, 1.5, X[r].contiguous(), precision=prec)
            # multi-vector kernels (pair kernel, skinny MFMA product) sum in
            # another order than the single-vector ones
            rel = (torch.linalg.norm(yr - ys[0][r]) / torch.linalg.norm(yr)).item()
            assert rel < (1e-13 if prec == "fp64" else 2e-6), (prec, r, rel)


def test_rhs_matches_oracle(P):
    from oracle.rhs import plane_wave_rhs
    mesh = geodesic_sphere(4)
    M = P.Mesh.from_inputs(mesh)
    d = wave_directions(3, seed=7)
    f = P.pmchwt_rhs(M, 3.0 + 0.1j, d).cpu().numpy()
    for w in range(3):
        ref = plane_wave_rhs(mesh, 3.0 + 0.1j, d[w])
        assert np.linalg.norm(f[w] - ref) / np.linalg.norm(ref) < 1e-13


def test_far_field_matches_oracle(P):
    import torch
    from oracle.rhs import far_field
    mesh = icosphere(2)
    M = P.Mesh.from_inputs(mesh)
    x = complex_normal(2 * mesh.n_vertices, seed=9)
    dirs = wave_directions(17, seed=3)
    out = P.far_field(M, 2.0, torch.from_numpy(x).cuda(), dirs)
    ref = far_field(mesh, 2.0, x, dirs)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-13


def test_invalid_arguments_raise(P):
    import torch
    mesh = icosphere(1)
    M = P.Mesh.from_inputs(mesh)
    x = torch.zeros(2 * mesh.n_vertices, dtype=torch.complex128, device="cuda")
    with pytest.raises(P.BemError):
        P.pmchwt_matvec(M, 2.0, 3.0, -1.0, x)
    with pytest.raises(P.BemError):
        P.pmchwt_matvec(M, 2.0 - 0.5j, 3.0, 1.0, x)
    with pytest.raises(ValueError):
        P.pmchwt_matvec(M, 2.0, 3.0, 1.0, x[:-1].contiguous())


@pytest.fixture
def dense_paths(P):
    keys = ("dense.gemm_min_rhs", "dense.skinny_min_rhs")
    old = {k: P.tune_get(k) for k in keys}
    yield lambda k, v: P.tune_set(k, v)
    for k, v in old.items():
        P.tune_set(k, v)


@pytest.mark.parametrize("n_rhs", [16, 67])
def test_dense_mfma_gemm_matches_gemv_and_oracle(P, dense_paths, n_rhs):
    """Multi-RHS product on MFMA (from 16 vectors here, ragged column tile at
    67) against per-column dense GEMVs and the oracle's dense matrix."""
    import torch
    dense_paths("dense.gemm_min_rhs", 16)
    mesh = icosphere(3)
    N = mesh.n_vertices
    M = P.Mesh.from_inputs(mesh)
    X = torch.from_numpy(complex_normal((n_rhs, 2 * N), seed=21)).cuda()
    Y = P.pmchwt_matvec(M, 2.0, 3.0, 1.5, X, precision="fp32_dense").cpu().numpy()
    B = dense(mesh, 2.0, 3.0, 1.5)
    Xn = X.cpu().numpy()
    for r in (0, n_rhs // 2, n_rhs - 1):
        g = P.pmchwt_matvec(M, 2.0, 3.0, 1.5, X[r].contiguous(),
                            precision="fp32_dense").cpu().numpy()
        ref = B @ Xn[r]
        assert np.linalg.norm(Y[r] - g) / np.linalg.norm(g) < 2e-6
        err = rel_blocks(Y[r], ref, N)
        assert max(err.values()) <= 1e-5, err


@pytest.mark.parametrize("skinny", [True, False])
@pytest.mark.parametrize("n_rhs", [2, 5, 8, 11, 20])
def test_dense_multi_vector_product(P, dense_paths, n_rhs, skinny):
    """Skinny MFMA product (16 columns per pass; from 5 vectors here) and the
    multi-vector GEMV (8 vectors per pass, ragged last group at 11 and 20)
    against single-vector products and the oracle's dense matrix."""
    import torch
    dense_paths("dense.gemm_min_rhs", 24)
    dense_paths("dense.skinny_min_rhs", 5 if skinny else 24)
    mesh = icosphere(3)
    N = mesh.n_vertices
    M = P.Mesh.from_inputs(mesh)
    X = torch.from_numpy(complex_normal((n_rhs, 2 * N), seed=31)).cuda()
    Y = P.pmchwt_matvec(M, 2.0, 3.0, 1.5, X, precision="fp32_dense").cpu().numpy()
    B = dense(mesh, 2.0, 3.0, 1.5)
    Xn = X.cpu().numpy()
    for r in range(n_rhs):
        g = P.pmchwt_matvec(M, 2.0, 3.0, 1.5, X[r].contiguous(),
                            precision="fp32_dense").cpu().numpy()
        assert np.linalg.norm(Y[r] - g) / np.linalg.norm(g) < 2e-6
        err = rel_blocks(Y[r], B @ Xn[r], N)
        assert max(err.values()) <= 1e-5, err


@pytest.fixture
def multi_max(P):
    old = P.tune_get("farfield.multi_max")
    yield lambda v: P.tune_set("farfield.multi_max", v)
    P.tune_set("farfield.multi_max", old)


@pytest.mark.parametrize("case", ["C1_ico3", "ico2_lossy", "two_spheres1"])
def test_matvec_multi_rhs_fp64(P, multi_max, case):
    """FP64 pair kernel shared by 2 right-hand sides (3 vectors: one pair
    launch plus a single-vector launch) against the oracle's dense matrix."""
    import torch
    make, k0, k1, rho = CASES[case]
    mesh = make()
    N = mesh.n_vertices
    M = P.Mesh.from_inputs(mesh)
    X = torch.from_numpy(complex_normal((3, 2 * N), seed=43)).cuda()
    multi_max(2)
    Y = P.pmchwt_matvec(M, k0, k1, rho, X, precision="fp64").cpu().numpy()
    B = dense(mesh, k0, k1, rho)
    Xn = X.cpu().numpy()
    for r in range(3):
        err = rel_blocks(Y[r], B @ Xn[r], N)
        print(case, r, err)
        assert max(err.values()) <= TOL["fp64"], err


@pytest.mark.parametrize("mm", [2, 4])
@pytest.mark.parametrize("case", ["C1_ico3", "ico2_lossy", "two_spheres1"])
def test_matvec_multi_rhs_fp32(P, multi_max, case, mm):
    """Pair kernel shared by 2 or 4 right-hand sides (5 vectors: a multi
    launch plus single-vector remainder) against the oracle's dense matrix."""
    import torch
    make, k0, k1, rho = CASES[case]
    mesh = make()
    N = mesh.n_vertices
    M = P.Mesh.from_inputs(mesh)
    X = torch.from_numpy(complex_normal((5, 2 * N), seed=41)).cuda()
    multi_max(mm)
    Y = P.pmchwt_matvec(M, k0, k1, rho, X, precision="fp32").cpu().numpy()
    B = dense(mesh, k0, k1, rho)
    Xn = X.cpu().numpy()
    for r in range(5):
        err = rel_blocks(Y[r], B @ Xn[r], N)
        print(case, mm, r, err)
        assert max(err.values()) <= TOL["fp32"], err


def test_matvec_multi_rhs_full_size_sampled_rows(P, multi_max):
    """Icosphere L5, k_ext = 10, k_int = 15, rho = 1.5, 4 right-hand sides in
    one multi-vector launch; 24 seed-sampled rows of each block row against
    the oracle's matrix-free rows."""
    import torch
    from oracle.operators import pmchwt_matvec_rows
    mesh = icosphere(5)
    N = mesh.n_vertices
    X = complex_normal((4, 2 * N), seed=0)
    rows = sample_rows(N, 24, seed=1)
    M = P.Mesh.from_inputs(mesh)
    multi_max(4)
    Y = P.pmchwt_matvec(M, 10.0, 15.0, 1.5, torch.from_numpy(X).cuda(),
                        precision="fp32").cpu().numpy()
    for r in (0, 3):
        r1, r2 = pmchwt_matvec_rows(mesh, 10.0, 15.0, 1.5, X[r], rows)
        e1 = np.linalg.norm(Y[r][rows] - r1) / np.linalg.norm(r1)
        e2 = np.linalg.norm(Y[r][N + rows] - r2) / np.linalg.norm(r2)
        print(r, e1, e2)
        assert e1 <= TOL["fp32"] and e2 <= TOL["fp32"]


def test_dense_mfma_gemm_full_size_sampled_rows(P, dense_paths):
    """The batching workload's product: icosphere L5, k_ext = 16, k_int = 24,
    rho = 1.5, the assembled complex64 operator times a 64-column block on
    MFMA; 40 seed-sampled rows of each block row of three columns against the
    oracle's matrix-free rows (<= 1e-5)."""
    import torch
    from oracle.operators import pmchwt_matvec_rows
    dense_paths("dense.gemm_min_rhs", 24)
    mesh = icosphere(5)
    N = mesh.n_vertices
    X = complex_normal((64, 2 * N), seed=2104)
    rows = sample_rows(N, 40, seed=1)
    M = P.Mesh.from_inputs(mesh)
    print("C4 MFMA product, 64 columns", flush=True)
    Y = P.pmchwt_matvec(M, 16.0, 24.0, 1.5, torch.from_numpy(X).cuda(),
                        precision="fp32_dense").cpu().numpy()
    for r in (0, 31, 63):
        r1, r2 = pmchwt_matvec_rows(mesh, 16.0, 24.0, 1.5, X[r], rows)
        e1 = np.linalg.norm(Y[r][rows] - r1) / np.linalg.norm(r1)
        e2 = np.linalg.norm(Y[r][N + rows] - r2) / np.linalg.norm(r2)
        print(r, e1, e2)
        assert e1 <= TOL["fp32"] and e2 <= TOL["fp32"]


@pytest.mark.parametrize("block", [64, 128])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_matvec_workgroup_sizes(P, block, precision):
    """Pair kernel with 64 and 128 test triangles per workgroup (ragged last
    workgroup on the geodesic mesh) against the oracle's dense matrix."""
    old = P.tune_get("farfield.block")
    try:
        P.tune_set("farfield.block", block)
        for case in ("geodesic3_ragged", "two_spheres1"):
            make, k0, k1, rho = CASES[case]
            mesh = make()
            N = mesh.n_vertices
            x = complex_normal(2 * N, seed=0)
            ref = dense(mesh, k0, k1, rho) @ x
            y = gpu_matvec(P, mesh, k0, k1, rho, x, precision)
            err = rel_blocks(y, ref, N)
            print(case, block, precision, err)
            assert max(err.values()) <= TOL[precision], err
    finally:
        P.tune_set("farfield.block", old)


@pytest.fixture
def far_tuning(P):
    old = {k: P.tune_get(k) for k in ("farfield.block", "farfield.symmetric",
                                      "farfield.sym_round_mib")}
    yield lambda k, v: P.tune_set(k, v)
    for k, v in old.items():
        P.tune_set(k, v)


@pytest.mark.parametrize("block", [64, 128, 256])
def test_symmetric_kernel_matches_one_directional(P, far_tuning, block):
    """FP32 kernel that evaluates each separated triangle pair once and adds
    it to the rows of both triangles, against the kernel that evaluates every
    ordered pair (same arithmetic per pair, another order of additions) and
    against the oracle: complex wavenumbers, two objects, ragged last block."""
    far_tuning("farfield.block", block)
    for case in ("C1_ico3", "ico2_lossy", "geodesic3_ragged", "two_spheres1"):
        make, k0, k1, rho = CASES[case]
        mesh = make()
        N = mesh.n_vertices
        print(f"symmetric {case} block {block}", flush=True)
        x = complex_normal(2 * N, seed=3)
        ref = dense(mesh, k0, k1, rho) @ x
        far_tuning("farfield.symmetric", 1)
        ys = gpu_matvec(P, mesh, k0, k1, rho, x, "fp32")
        far_tuning("farfield.symmetric", 0)
        yd = gpu_matvec(P, mesh, k0, k1, rho, x, "fp32")
        d, e = rel_blocks(ys, yd, N), rel_blocks(ys, ref, N)
        print(case, block, d, e)
        assert max(d.values()) <= 2e-6, d
        assert max(e.values()) <= TOL["fp32"], e


@pytest.mark.parametrize("block", [64, 256])
def test_symmetric_kernel_rounds_bitwise(P, far_tuning, block):
    """The symmetric kernel in several launches (a 1 MiB buffer of the
    partial sums of the second triangle's rows: a dozen or more rounds on an
    icosphere of level 4, the last one ragged) gives bitwise the result of
    one launch, and matches the oracle's rows."""
    import torch
    from oracle.operators import pmchwt_matvec_rows
    far_tuning("farfield.block", block)
    far_tuning("farfield.symmetric", 1)
    mesh = icosphere(4)
    N = mesh.n_vertices
    M = P.Mesh.from_inputs(mesh)
    x = complex_normal(2 * N, seed=12)
    xd = torch.from_numpy(x).cuda()
    print(f"symmetric rounds block {block}", flush=True)
    y1 = P.pmchwt_matvec(M, 4.0, 6.0 + 0.5j, 1.5, xd, precision="fp32")
    far_tuning("farfield.sym_round_mib", 1)
    yr = P.pmchwt_matvec(M, 4.0, 6.0 + 0.5j, 1.5, xd, precision="fp32")
    assert torch.equal(y1, yr)
    rows = sample_rows(N, 24, seed=13)
    r1, r2 = pmchwt_matvec_rows(mesh, 4.0, 6.0 + 0.5j, 1.5, x, rows)
    y = yr.cpu().numpy()
    for got, ref in ((y[rows], r1), (y[N + rows], r2)):
        assert np.linalg.norm(got - ref) <= TOL["fp32"] * np.linalg.norm(ref)
    with pytest.raises(P.BemError):
        P.tune_set("farfield.sym_round_mib", 0)


def test_fp32_kernels_large_phases(P, far_tuning):
    """Phases k r / 2 pi above 256 revolutions: both FP32 kernels reduce the
    phase to [0, 1) before v_sin/v_cos.  Against each other (2e-6) and the
    oracle: the FP32 rounding of r and k r / 2 pi leaves a phase error of a
    few t 2^-24 revolutions (t <= 390 here, about 6e-4 rad), hence 2e-3."""
    mesh = icosphere(2)
    k0, k1, rho = 500.0, 700.0, 1.3
    N = mesh.n_vertices
    x = complex_normal(2 * N, seed=5)
    ref = dense(mesh, k0, k1, rho) @ x
    out = {}
    for sym in (1, 0):
        far_tuning("farfield.symmetric", sym)
        out[sym] = gpu_matvec(P, mesh, k0, k1, rho, x, "fp32")
    d, e = rel_blocks(out[1], out[0], N), rel_blocks(out[1], ref, N)
    print(d, e)
    assert max(d.values()) <= 2e-6, d
    assert max(e.values()) <= 2e-3, e
