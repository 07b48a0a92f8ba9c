"""GPU tests of the serving loop (bem_server_*), through the C ABI.

* Each result is the same alone and in a mix of concurrent requests on
  several meshes (bitwise: the kernels reduce in a fixed order and the path
  depends only on the request), and equal to a direct pmchwt_solve.
* Work of several requests is in flight at once (peak_inflight > 1).
* Admission by device-memory budget: a request whose footprint cannot fit is
  completed with BEM_E_NOMEM; the accounted peak stays within the budget;
  resident caches are released when the budget requires it.
"""
import numpy as np
import pytest

from bem_inputs import icosphere, two_spheres, wave_directions

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2104_04609_amd as P
    return P


MESHES = {"ico2": lambda: icosphere(2), "ico3": lambda: icosphere(3),
          "two2": lambda: two_spheres(2, offset=1.5)}

# (mesh, k_ext, k_int, rho, n_waves, precision, path)
REQUESTS = [
    ("ico3", 2.0, 3.0, 1.5, 1, "fp32", 0),
    ("ico2", 3.0, 4.5 + 0.2j, 1.3, 2, "fp64", 0),
    ("two2", 2.0, 3.2, 1.7, 1, "fp32", 1),
    ("ico3", 4.0, 6.0, 1.9, 3, "fp32", 1),
    ("ico2", 1.5, 2.5, 1.2, 1, "fp32", 0),
    ("ico3", 2.5, 4.0, 1.4, 2, "fp64", 0),
]


def _dirs(n, seed):
    return wave_directions(n, seed=seed)


def _run(P, workers, order, budget=0):
    srv = P.Server(hbm_budget=budget, workers=workers)
    ids = {name: srv.add_mesh(m.vertices, m.triangles, m.object_id)
           for name, m in ((n, f()) for n, f in MESHES.items())}
    rids = {}
    for i in order:
        name, k0, k1, rho, nw, prec, path = REQUESTS[i]
        rids[i] = srv.submit(ids[name], k0, k1, rho, _dirs(nw, 10 + i), 1e-8,
                             precision=prec, path=path, maxiter=400)
    out = {i: srv.wait(rid) for i, rid in rids.items()}
    stats = srv.stats()
    srv.close()
    return out, stats


def test_results_alone_equal_in_mix(P):
    import torch
    alone = {}
    for i in range(len(REQUESTS)):
        print("alone", i, REQUESTS[i], flush=True)
        res, _ = _run(P, 1, [i])
        alone[i] = res[i]
    print("mix", flush=True)
    mix, stats = _run(P, 4, list(range(len(REQUESTS)))[::-1])
    print(stats)
    assert stats["completed"] == len(REQUESTS) and stats["rejected"] == 0
    assert stats["peak_inflight"] > 1
    assert stats["peak_bytes"] <= stats["budget"]
    for i in range(len(REQUESTS)):
        sa, ia, ta = alone[i]
        sm, im, tm = mix[i]
        print(i, ta, tm, ia[0])
        assert ta["status"] == 0 and tm["status"] == 0
        assert ta["path"] == tm["path"] == (1 if REQUESTS[i][5] == "fp32" and REQUESTS[i][6] == 1 else 0)
        assert torch.equal(sa, sm), i
        assert all(x["rel_residual"] <= 1e-8 for x in im)
        assert tm["t_submit"] <= tm["t_admit"] <= tm["t_end"]


def test_server_matches_direct_solve(P):
    import torch
    name, k0, k1, rho, nw, prec, path = REQUESTS[3]
    m = MESHES[name]()
    d = _dirs(nw, 13)
    M = P.Mesh.from_inputs(m)
    ref, info, rc = P.pmchwt_solve(M, k0, k1, rho, d, 1e-8, precision=prec, path=path,
                                   maxiter=400)
    srv = P.Server(workers=2)
    mid = srv.add_mesh(m.vertices, m.triangles, m.object_id)
    rid = srv.submit(mid, k0, k1, rho, d, 1e-8, precision=prec, path=path, maxiter=400)
    sol, infos, st = srv.wait(rid)
    srv.close()
    assert rc == 0 and st["status"] == 0
    assert torch.equal(sol, ref)
    assert [x["iterations"] for x in infos] == [x["iterations"] for x in info]


def test_server_per_object_materials_and_formulation(P):
    """A request with a material per object and another formulation equals
    the direct pmchwt_solve_multi bitwise."""
    import torch
    m = MESHES["two2"]()
    k0, ks, rs = 2.0, [3.2, 4.0 + 0.3j], [1.7, 0.9]
    d = _dirs(2, 17)
    M = P.Mesh.from_inputs(m)
    srv = P.Server(workers=2)
    mid = srv.add_mesh(m.vertices, m.triangles, m.object_id)
    for form in ("osrc", "calderon"):
        ref, info, rc = P.pmchwt_solve_multi(M, k0, ks, rs, d, 1e-8, precision="fp32", path=1,
                                             formulation=form)
        rid = srv.submit(mid, k0, ks, rs, d, 1e-8, precision="fp32", path=1, formulation=form)
        sol, infos, st = srv.wait(rid)
        assert rc == 0 and st["status"] == 0
        assert torch.equal(sol, ref), form
        assert [x["iterations"] for x in infos] == [x["iterations"] for x in info]
    with pytest.raises(P.BemError):
        srv.submit(mid, k0, [3.2, 4.0], [1.7, -1.0], d, 1e-8)
    srv.close()


def test_budget_admission_and_rejection(P):
    m3, m5 = icosphere(3), icosphere(5)
    srv = P.Server(hbm_budget=160 << 20, workers=2)
    a = srv.add_mesh(m3.vertices, m3.triangles)
    b = srv.add_mesh(m5.vertices, m5.triangles)
    d = _dirs(1, 3)
    # ico5 on the assembled path: the complex64 operator alone is 3.4 GB
    big = srv.submit(b, 2.0, 3.0, 1.5, d, 1e-6, precision="fp32", path=1)
    small = [srv.submit(a, 2.0 + 0.5 * i, 3.0 + 0.5 * i, 1.5, d, 1e-6, precision="fp32",
                        path=0, maxiter=200) for i in range(4)]
    sol, info, st = srv.wait(big)
    assert st["status"] == -3 and "budget" in st["error"]
    for rid in small:
        sol, info, st = srv.wait(rid)
        assert st["status"] == 0, st
        assert info[0]["rel_residual"] <= 1e-6
    stats = srv.stats()
    print(stats)
    assert stats["rejected"] == 1 and stats["completed"] == 4
    assert stats["peak_bytes"] <= stats["budget"]
    srv.close()


def test_resident_state_released_under_budget(P):
    """A budget that holds one request beside the fresh handles but not the
    cached state of the previous ones: idle handles are trimmed (LRU) and the
    results are unchanged."""
    import torch
    m3 = icosphere(3)
    tw = two_spheres(2, offset=1.5)
    d = _dirs(1, 4)

    def flow(srv):
        a = srv.add_mesh(m3.vertices, m3.triangles)
        b = srv.add_mesh(tw.vertices, tw.triangles, tw.object_id)
        floor = srv.stats()["resident_bytes"]
        out = []
        for mid in (a, b, a):
            r = srv.submit(mid, 2.0, 3.0, 1.5, d, 1e-8, precision="fp64", maxiter=300)
            out.append(srv.wait(r))
        return floor, out

    probe = P.Server(workers=1)
    floor, ref = flow(probe)
    used = probe.stats()["resident_bytes"]
    probe.close()
    fp = max(t["footprint"] for _, _, t in ref)
    assert used > floor + (1 << 20)
    srv = P.Server(hbm_budget=floor + fp + (1 << 20), workers=1)
    _, got = flow(srv)
    stats = srv.stats()
    print(stats, floor, used, fp)
    srv.close()
    assert stats["evictions"] >= 1 and stats["rejected"] == 0
    assert stats["peak_bytes"] <= stats["budget"]
    for (s0, _, t0), (s1, _, t1) in zip(ref, got):
        assert t0["status"] == 0 and t1["status"] == 0
        assert torch.equal(s0, s1)


def test_krylov_growth_accounted(P):
    """A request whose basis outgrows the initial 65 vectors reports the
    growth to the server (krylov_growth_bytes) and equals the direct solve."""
    import torch
    m = icosphere(3)
    d = _dirs(1, 21)
    M = P.Mesh.from_inputs(m)
    # no OSRC (formulation "pmchwt"), k_int = 20 on 1280 triangles, tol 1e-12:
    # the oracle takes 117 iterations
    ref, info, rc = P.pmchwt_solve(M, 12.0, 20.0, 1.5, d, 1e-12, precision="fp64", path=1,
                                   formulation="pmchwt", maxiter=300)
    assert info[0]["iterations"] > 64, info
    srv = P.Server(workers=1)
    mid = srv.add_mesh(m.vertices, m.triangles)
    rid = srv.submit(mid, 12.0, 20.0, 1.5, d, 1e-12, precision="fp64", path=1,
                     formulation="pmchwt", maxiter=300)
    sol, infos, st = srv.wait(rid)
    stats = srv.stats()
    srv.close()
    print(stats, st)
    assert st["status"] == rc
    assert stats["krylov_growth_bytes"] > 0 and stats["reserved_bytes"] == 0
    assert torch.equal(sol, ref)


def test_replicas_share_assembled_operator(P):
    """Requests with the same mesh and wavenumbers running on several
    replicas use one assembled operator (one assembly, counted by the
    library's profiler), and each result equals the direct solve."""
    import torch
    m = icosphere(4)
    M = P.Mesh.from_inputs(m)
    srv = P.Server(workers=3)
    mid = srv.add_mesh(m.vertices, m.triangles)
    ds = [_dirs(2, 30 + i) for i in range(3)]
    P.profile_enable(True)
    try:
        rids = [srv.submit(mid, 4.0, 6.0, 1.5, d, 1e-8, precision="fp32", path=1) for d in ds]
        out = [srv.wait(r) for r in rids]
        torch.cuda.synchronize()
        # the operator is assembled in FP32, or in FP64 and rounded
        # ("solve.residual_dense_gib"): one assembly either way
        n_asm = P.profile_read("dense_assemble")[1] + P.profile_read("dense_assemble_fp64")[1]
    finally:
        P.profile_enable(False)
    stats = srv.stats()
    srv.close()
    print(stats, n_asm)
    assert stats["peak_inflight"] >= 2
    assert n_asm == 1
    for d, (sol, infos, st) in zip(ds, out):
        ref, info, rc = P.pmchwt_solve(M, 4.0, 6.0, 1.5, d, 1e-8, precision="fp32", path=1)
        assert st["status"] == 0 and rc == 0
        assert torch.equal(sol, ref)


def test_invalid_requests(P):
    m = icosphere(1)
    srv = P.Server(workers=1)
    a = srv.add_mesh(m.vertices, m.triangles)
    with pytest.raises(P.BemError):
        srv.submit(a + 7, 2.0, 3.0, 1.5, [[0, 0, 1.0]], 1e-6)
    with pytest.raises(P.BemError):
        srv.submit(a, 2.0, 3.0, -1.0, [[0, 0, 1.0]], 1e-6)
    with pytest.raises(P.BemError):
        srv.wait(12345)
    srv.close()
