"""osrc_apply_noalloc (the OSRC apply without device allocation) against
osrc_apply through the C ABI: two calls in a row on one GPU, the second with
a smaller input (fewer vectors on a smaller mesh), each bitwise equal to
osrc_apply on the same input (same kernels, same per-vector order) and within
1e-10 of the oracle; argument errors are rejected on the host before any
launch."""
import numpy as np
import pytest

from bem_inputs import complex_normal, icosphere

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2104_04609_amd as P
    return P


def _case(P, level, n_rhs, k, keps, n_p, seed):
    import torch
    from oracle.osrc import OSRC
    mesh = icosphere(level)
    N = mesh.n_vertices
    M = P.Mesh.from_inputs(mesh)
    X = torch.from_numpy(complex_normal((n_rhs, 2 * N), seed=seed)).cuda()
    ref = P.osrc_apply(M, n_p, np.pi / 3, k, keps, X)          # creates the factors
    out = torch.full_like(X, complex(np.nan, np.nan))
    print(f"osrc_apply_noalloc level {level} n_rhs {n_rhs}", flush=True)
    P.osrc_apply_noalloc(M, n_p, np.pi / 3, k, keps, X, out)
    torch.cuda.synchronize()
    return mesh, M, X, ref, out


def test_noalloc_matches_osrc_apply_twice(P):
    import torch
    from oracle.osrc import OSRC
    cases = [(3, 5, 3.0, 3.4 + 0.9j, 4, 1), (2, 2, 6.0 + 0.3j, 6.5 + 1.1j, 8, 2)]
    for level, n_rhs, k, keps, n_p, seed in cases:
        mesh, M, X, ref, out = _case(P, level, n_rhs, k, keps, n_p, seed)
        assert torch.equal(out, ref), (level, n_rhs)
        N = mesh.n_vertices
        op = OSRC(mesh, k, keps, n_p, np.pi / 3)
        Xn, On = X.cpu().numpy(), out.cpu().numpy()
        for r in range(n_rhs):
            o = op.apply(Xn[r])
            for sl in (slice(0, N), slice(N, 2 * N)):
                assert np.linalg.norm(On[r][sl] - o[sl]) <= 1e-10 * np.linalg.norm(o[sl])


def test_noalloc_rejects_missing_factors_and_oversize(P):
    import torch
    mesh = icosphere(1)
    M = P.Mesh.from_inputs(mesh)
    X = torch.from_numpy(complex_normal((2, 2 * mesh.n_vertices), seed=3)).cuda()
    Y = torch.empty_like(X)
    with pytest.raises(P.BemError) as e:     # no factors for these parameters yet
        P.osrc_apply_noalloc(M, 4, np.pi / 3, 2.0, 2.2 + 0.5j, X, Y)
    assert e.value.code == -1 and "once first" in str(e.value)
    # a mesh whose work vectors exceed the scratch: 16 vectors of level 6
    big = icosphere(6)
    B = P.Mesh.from_inputs(big)
    XB = torch.zeros((16, 2 * big.n_vertices), dtype=torch.complex128, device="cuda")
    P.osrc_apply(B, 4, np.pi / 3, 2.0, 2.2 + 0.5j, XB[:1].contiguous())
    with pytest.raises(P.BemError) as e:
        P.osrc_apply_noalloc(B, 4, np.pi / 3, 2.0, 2.2 + 0.5j, XB, torch.empty_like(XB))
    assert e.value.code == -1 and "exceeds" in str(e.value)
