#!/usr/bin/env python3
"""Benchmark of the matrix-free permuted PMCHWT matvec and the OSRC-GMRES solve.

Workload: unit sphere, icosphere level 5 (10 242 vertices, 20 480 triangles),
k_ext = 10, k_int = 15, rho = 1.5, plane wave along +z; synthetic seeded
input x (complex standard normal, seed 0) already resident in HBM.

A step is one Galerkin matvec y = B x of the whole operator: source gather,
FP32 pair kernel over all separated triangle pairs, fixed-order reduction to
vertex rows and the FP64 near-field CSR SpMV.  value = T(T-1) triangle-pair
evaluations per second of that step.  The solve comparison (FP64 GMRES vs
FP32 pair kernel + FP64 true-residual refinement, both to 1e-6) and the FP64
matvec are measured in the same run outside the timed steps.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PMCHWT matvec tri-pair evals/s + solve time; FP32+refine vs FP64 @1e-6 res"
K_EXT, K_INT, RHO = 10.0, 15.0, 1.5


def cpu_baseline(mesh, n_test=2048):
    """Oracle (FP64, plain C + OpenMP) matrix-free rows on a seeded sample of
    test triangles against all trial triangles; tri-pair evaluations/s."""
    from bem_inputs import complex_normal, sample_rows
    from oracle import operators as O
    N, T = mesh.n_vertices, mesh.n_triangles
    x = complex_normal(2 * N, seed=0)
    test = sample_rows(T, n_test, seed=3)
    lib = O._load()
    t0 = time.perf_counter()
    O._matvec_tris(mesh, K_EXT, False, test, (x[:N], x[N:], x[:N], x[N:]))
    O._matvec_tris(mesh, K_INT, True, test, (x[:N], x[N:], x[:N], x[N:]))
    dt = time.perf_counter() - t0
    return {"value": n_test * T / dt, "unit": "tri-pair evals/s",
            "cores": int(lib.oracle_num_threads()), "kind": "oracle",
            "sample": f"{n_test} seeded test triangles x all {T} trial triangles, "
                      f"both wavenumbers, 4 operators, FP64 ({dt:.1f} s)"}


def pmc_traffic():
    """HBM bytes per launch of the FP32 pair kernel from the committed PMC
    summary (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel of known size),
    or None when the kernel source has changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "farfield_fp32_ico5_pmc.md")
    try:
        text = open(path).read()
        rec = json.loads(re.search(r"```json\n(.*?)```", text, re.S).group(1))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, AttributeError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    kib = 1024.0
    fetch = rec["fetch_kib"] * kib * rec["copy_bytes"] / (rec["copy_fetch_kib"] * kib)
    write = rec["write_kib"] * kib * rec["copy_bytes"] / (rec["copy_write_kib"] * kib)
    return {"bytes": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
            "source": "profiles/farfield_fp32_ico5_pmc.md"}


def batch_measure(P, M, mesh, mf_step_s):
    """64 plane-wave right-hand sides (normalised Gaussian directions, seed
    2104) at 4 wavenumber pairs k_ext in {4, 8, 12, 16}, k_int = 1.5 k_ext,
    rho = 1.5: assembled complex64 operator x 64-column block on MFMA,
    against the matrix-free FP32 operator on the same block (4 right-hand
    sides per pair-kernel launch).  Then 8 plane waves solved in one lockstep
    group against 8 single-wave solves (FP32 + refinement, assembled path)."""
    import torch
    from bem_inputs import wave_directions
    from paper_2104_04609_amd import roofline as RL
    d = wave_directions(64, seed=2104)
    N = mesh.n_vertices
    out = {"n_rhs": 64, "k_pairs": []}
    for ke in (4.0, 8.0, 12.0, 16.0):
        F = P.pmchwt_rhs(M, ke, d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.profile_enable(True)
        Y = P.pmchwt_matvec(M, ke, 1.5 * ke, 1.5, F, precision="fp32_dense")   # assembles
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        asm_ms, _ = P.profile_read("dense_assemble")
        P.profile_enable(False)
        P.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(3):
            P.pmchwt_matvec(M, ke, 1.5 * ke, 1.5, F, Y, precision="fp32_dense")
        torch.cuda.synchronize()
        gemm_s = (time.perf_counter() - t0) / 3
        kms, kn = P.profile_read("dense_gemm_mfma")
        P.profile_enable(False)
        flops = 8.0 * (2 * N) ** 2 * 64
        # matrix-free FP32 on the same 64-column block
        P.pmchwt_matvec(M, ke, 1.5 * ke, 1.5, F, Y, precision="fp32")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.pmchwt_matvec(M, ke, 1.5 * ke, 1.5, F, Y, precision="fp32")
        torch.cuda.synchronize()
        mf_s = time.perf_counter() - t0
        out["k_pairs"].append({
            "k_ext": ke, "k_int": 1.5 * ke, "assembly_ms": asm_ms,
            "first_call_s": first, "gemm_call_ms": gemm_s * 1e3,
            "mfma_kernel_ms": kms / kn,
            "mfma_tflops": flops / (kms / kn * 1e-3) / 1e12,
            "mfma_frac_of_fp32_matrix_peak": flops / (kms / kn * 1e-3) / 1e12 / RL.PEAK_FP32_TFLOPS,
            "matrix_free_64_rhs_ms": mf_s * 1e3,
            "matrix_free_64_rhs_ms_one_per_launch": 64 * mf_step_s * 1e3})
    # lockstep multi-wave solve against single-wave solves
    d8 = wave_directions(8, seed=2104)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info8, rc8 = P.pmchwt_solve(M, K_EXT, K_INT, RHO, d8, 1e-6, precision="fp32", path=1)
    torch.cuda.synchronize()
    lock_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    for w in range(8):
        P.pmchwt_solve(M, K_EXT, K_INT, RHO, d8[w:w + 1], 1e-6, precision="fp32", path=1)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    out["solve_8_waves"] = {"lockstep_s": lock_s, "one_at_a_time_s": seq_s, "rc": rc8,
                            "speedup": seq_s / lock_s,
                            "max_rel_residual": max(i["rel_residual"] for i in info8),
                            "k_ext": K_EXT, "k_int": K_INT, "path": "assembled (FP32 + refine)"}
    return out


def multi_material_measure(P, RL) -> dict:
    """The paper's multiple-scattering layout (Sec. 3): four spheres, radius
    5 mm, centres (+-15, +-7.5, 0) mm, two of fat and two of bone in water at
    500 kHz (Table 1 media), each sphere an icosphere of level 4 (10 248
    vertices, 20 480 triangles in all).  One FP32 matvec (pair kernel with
    per-object materials) timed over 5 launches, then OSRC-preconditioned
    solves to 1e-6 (FP32 + refinement on the matrix-free and assembled
    paths), and the PMCHWT, Calderon and Mueller formulations on the assembled
    path."""
    import torch
    from bem_inputs import complex_normal, density_ratio, four_spheres, wavenumber
    f, a = 5e5, 5e-3
    mesh = four_spheres(4)
    k0 = wavenumber("water", f, a)
    tissue = ["fat", "bone", "bone", "fat"]
    ks = [wavenumber(t, f, a) for t in tissue]
    rs = [density_ratio(t) for t in tissue]
    M = P.Mesh.from_inputs(mesh)
    N, T = mesh.n_vertices, mesh.n_triangles
    x = torch.from_numpy(complex_normal(2 * N, seed=0)).cuda()
    y = torch.empty_like(x)
    P.pmchwt_matvec_multi(M, k0, ks, rs, x, y, precision="fp32")
    torch.cuda.synchronize()
    P.profile_enable(True)
    for _ in range(5):
        P.pmchwt_matvec_multi(M, k0, ks, rs, x, y, precision="fp32")
    torch.cuda.synchronize()
    kms, kn = P.profile_read("farfield_fp32")
    P.profile_enable(False)
    pairs = RL.far_pairs_per_matvec(mesh.triangles)
    out = {"workload": "four_spheres4 fat/bone 500 kHz", "n_vertices": N, "n_triangles": T,
           "k_ext": [k0.real, k0.imag], "k_int": [[k.real, k.imag] for k in ks], "rho": rs,
           "fp32_kernel_ms": kms / kn,
           "roofline": RL.pair_kernel_roofline(pairs, kms / kn * 1e-3, "fp32",
                                               symmetric=P.tune_get("farfield.symmetric") == 1)}
    d = [[1.0, 0.0, 0.0]]
    for name, path, form in (("osrc_fp32", 0, "osrc"), ("osrc_fp32_dense", 1, "osrc"),
                             ("pmchwt_fp32_dense", 1, "pmchwt"), ("calderon_fp32_dense", 1, "calderon"),
                             ("muller_fp32_dense", 1, "muller")):
        P.pmchwt_solve_multi(M, k0, ks, rs, d, 1e-6, precision="fp32", path=path,
                             formulation=form, maxiter=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, rc = P.pmchwt_solve_multi(M, k0, ks, rs, d, 1e-6, precision="fp32", path=path,
                                           formulation=form)
        torch.cuda.synchronize()
        out[name] = {"seconds": time.perf_counter() - t0, "rc": rc,
                     "iterations": info[0]["iterations"], "rel_residual": info[0]["rel_residual"]}
        print(f"four spheres {name}: {out[name]}", file=sys.stderr, flush=True)
    del M
    return out


def frequency_sweep(P) -> dict:
    """GMRES iterations against frequency (the paper's frequency-dependency
    test, Sec. 3): a sphere of radius 5 mm in water, interior fat or bone
    (Table 1 media), 0.5 - 2.5 MHz, about six elements per wavelength (geodesic
    spheres of 10 n^2 + 2 vertices near the paper's node counts), plane wave
    along +z, tolerance 1e-7 on the preconditioned residual (Sec. 3.1).  Every
    formulation: PMCHWT, Mueller, Calderon, OSRC with the interior and with the
    exterior wavenumber; FP32 assembled operator + FP64 refinement, so the
    count is the total of the inner GMRES iterations.  Then the four-sphere
    layout (two fat, two bone) at 0.5 - 1.5 MHz, wave along +x."""
    import torch
    from bem_inputs import density_ratio, four_spheres, geodesic_sphere, wavenumber
    a = 5e-3
    sizes = {0.5e6: 13, 1.0e6: 27, 1.5e6: 40, 2.0e6: 52, 2.5e6: 65}
    forms = (("pmchwt", "pmchwt", 1), ("muller", "muller", 1), ("calderon", "calderon", 1),
             ("osrc_int", "osrc", 1), ("osrc_ext", "osrc", 0))
    out = []
    for f, n in sizes.items():
        mesh = geodesic_sphere(n)
        M = P.Mesh.from_inputs(mesh)
        k0 = wavenumber("water", f, a)
        for medium in ("fat", "bone"):
            k1, rho = wavenumber(medium, f, a), density_ratio(medium)
            row = {"f_MHz": f / 1e6, "medium": medium, "n_vertices": mesh.n_vertices}
            for name, form, interior in forms:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info, rc = P.pmchwt_solve(M, k0, k1, rho, [[0.0, 0.0, 1.0]], 1e-7,
                                             precision="fp32", path=1, formulation=form,
                                             osrc_interior=interior)
                torch.cuda.synchronize()
                row[name] = {"iterations": info[0]["iterations"],
                             "outer_steps": info[0]["outer_steps"],
                             "seconds": time.perf_counter() - t0, "rc": rc}
            out.append(row)
            print("sweep " + json.dumps(row), file=sys.stderr, flush=True)
        del M
        P.tune_clear()
    # the four-sphere test (two fat, two bone; 6 823 / 26 801 / 59 758 nodes at
    # 0.5 / 1 / 1.5 MHz in the paper; 2 MHz would need a 340 GB assembled operator)
    four = []
    tissue = ["fat", "bone", "bone", "fat"]
    for f, n in {0.5e6: 13, 1.0e6: 26, 1.5e6: 39}.items():
        mesh = four_spheres(geodesic=n)
        M = P.Mesh.from_inputs(mesh)
        k0 = wavenumber("water", f, a)
        ks = [wavenumber(t, f, a) for t in tissue]
        rs = [density_ratio(t) for t in tissue]
        row = {"f_MHz": f / 1e6, "n_vertices": mesh.n_vertices}
        for name, form, interior in forms:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info, rc = P.pmchwt_solve_multi(M, k0, ks, rs, [[1.0, 0.0, 0.0]], 1e-7,
                                               precision="fp32", path=1, formulation=form,
                                               osrc_interior=interior)
            torch.cuda.synchronize()
            row[name] = {"iterations": info[0]["iterations"], "outer_steps": info[0]["outer_steps"],
                         "seconds": time.perf_counter() - t0, "rc": rc}
        four.append(row)
        print("sweep four spheres " + json.dumps(row), file=sys.stderr, flush=True)
        del M
        P.tune_clear()
    return {"frequency_sweep": out, "four_spheres": four}


def sponge_sweep(P) -> dict:
    """The paper's test on a domain with corners and inclusions: a level-2
    Menger sponge of edge 10 mm, bone inside, water outside, plane wave along
    +x, 0.5 / 1 / 1.5 MHz with every voxel face split 4 / 6 / 8 times
    (16 736 / 37 856 / 67 424 vertices; the paper's Gmsh meshes have 13 568 /
    34 975 / 62 291), tolerance 1e-7, every formulation on the FP32 assembled
    operator + FP64 refinement (up to 2 000 iterations).  2 MHz (105 440
    vertices) would need a 356 GB assembled operator."""
    import torch
    from bem_inputs import density_ratio, menger_sponge, wavenumber
    forms = (("pmchwt", "pmchwt", 1), ("muller", "muller", 1), ("calderon", "calderon", 1),
             ("osrc_int", "osrc", 1), ("osrc_ext", "osrc", 0))
    out = []
    for f, k in {0.5e6: 4, 1.0e6: 6, 1.5e6: 8}.items():
        mesh = menger_sponge(2, k, edge=10.0)
        M = P.Mesh.from_inputs(mesh)
        k0, k1, rho = wavenumber("water", f, 1e-3), wavenumber("bone", f, 1e-3), density_ratio("bone")
        row = {"f_MHz": f / 1e6, "n_vertices": mesh.n_vertices}
        for name, form, interior in forms:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info, rc = P.pmchwt_solve(M, k0, k1, rho, [[1.0, 0.0, 0.0]], 1e-7,
                                         precision="fp32", path=1, formulation=form,
                                         osrc_interior=interior, maxiter=2000)
            torch.cuda.synchronize()
            row[name] = {"iterations": info[0]["iterations"], "outer_steps": info[0]["outer_steps"],
                         "seconds": time.perf_counter() - t0, "rc": rc,
                         "rel_residual": info[0]["rel_residual"]}
            print(f"sponge {f / 1e6} MHz {name}: {row[name]}", file=sys.stderr, flush=True)
        out.append(row)
        del M
        P.tune_clear()
    return {"sponge_sweep": out}


def serving_measure(P, n_requests: int, workers: int = 4, seed: int = 5) -> dict:
    """Serving mix: meshes {icosphere L3, L4, L5, ellipsoid (geodesic 45
    scaled by (1, 0.6, 0.4)), two level-4 spheres}, k_ext ~ U[1, 20],
    k_int/k_ext ~ U[1.3, 1.9], rho ~ U[1.2, 2.0], 1-8 plane waves, tol 1e-6,
    FP32 + refinement, auto path (seeded stream, seed 5).  A prefix of the
    stream submitted at once gives the saturated solves/s; the whole stream
    then arrives as a Poisson process at 0.7 x that rate."""
    from bem_inputs import ellipsoid, geodesic_sphere, icosphere, request_stream, two_spheres
    meshes = {"ico3": icosphere(3), "ico4": icosphere(4), "ico5": icosphere(5),
              "ellipsoid45": ellipsoid(geodesic_sphere(45)),
              "two_spheres4": two_spheres(4, offset=1.5)}
    srv = P.Server(workers=workers)
    ids = {k: srv.add_mesh(m.vertices, m.triangles, m.object_id) for k, m in meshes.items()}
    reqs = request_stream(n_requests, seed=seed, rate=1.0)

    def submit(r):
        return srv.submit(ids[r["mesh"]], r["k_ext"], r["k_int"], r["rho"], r["directions"],
                          1e-6, precision="fp32")

    def progress(msg):
        print(f"serving: {msg}", file=sys.stderr, flush=True)

    n_sat = max(8, n_requests // 4)
    t0 = time.perf_counter()
    for i, rid in enumerate([submit(r) for r in reqs[:n_sat]]):
        srv.wait(rid)
        progress(f"saturated phase {i + 1}/{n_sat} done")
    sat = n_sat / (time.perf_counter() - t0)
    print(f"serving: saturated {sat:.2f} solves/s over {n_sat} requests", file=sys.stderr,
          flush=True)
    lam = 0.7 * sat
    t0 = time.perf_counter()
    pending = []
    for i, r in enumerate(reqs):
        dt = r["arrival"] / lam - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        pending.append((r, submit(r)))
        if (i + 1) % 16 == 0:
            progress(f"submitted {i + 1}/{n_requests}")
    results = []
    for i, (r, rid) in enumerate(pending):
        results.append((r, srv.wait(rid)))
        if (i + 1) % 16 == 0:
            progress(f"completed {i + 1}/{n_requests}")
    elapsed = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    lat = np.array([st["t_end"] - st["t_submit"] for _, (_, _, st) in results])
    queue_wait = np.array([st["t_admit"] - st["t_submit"] for _, (_, _, st) in results])
    busy = sum(st["t_end"] - st["t_admit"] for _, (_, _, st) in results)
    bad = [st for _, (_, info, st) in results
           if st["status"] != 0 or max(i["rel_residual"] for i in info) > 1e-6]
    by_mesh = {}
    for r, (_, info, st) in results:
        e = by_mesh.setdefault(r["mesh"], {"n": 0, "latency_s": [], "paths": set()})
        e["n"] += 1
        e["latency_s"].append(st["t_end"] - st["t_submit"])
        e["paths"].add(st["path"])
    return {
        "requests": n_requests, "workers": workers, "seed": seed,
        "saturated_solves_per_s": sat, "saturated_prefix": n_sat,
        "arrival_rate_per_s": lam, "solves_per_s": n_requests / elapsed,
        "waves_per_s": sum(len(r["directions"]) for r in reqs) / elapsed,
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "p50_queue_wait_s": float(np.percentile(queue_wait, 50)),
        "mean_concurrency": busy / elapsed, "peak_inflight": stats["peak_inflight"],
        "peak_bytes": stats["peak_bytes"], "budget": stats["budget"],
        "evictions": stats["evictions"], "rejected": stats["rejected"],
        "failed_or_unconverged": len(bad),
        "per_mesh": {k: {"n": v["n"], "p50_latency_s": float(np.median(v["latency_s"])),
                         "paths": sorted(v["paths"])} for k, v in by_mesh.items()},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-batching", action="store_true")
    ap.add_argument("--serving", type=int, default=32, metavar="N",
                    help="requests of the serving mix to replay (0: skip)")
    ap.add_argument("--frequency-sweep", action="store_true",
                    help="only the iteration-count sweep over frequency (one JSON line)")
    ap.add_argument("--sponge-sweep", action="store_true",
                    help="only the Menger-sponge sweep over frequency (one JSON line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB read + 256 MiB write elementwise kernel 3 times, "
                         "to scale HBM byte counters (FETCH_SIZE, WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus must be 1 "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2104_04609_amd as P
    from paper_2104_04609_amd import roofline as RL
    from bem_inputs import complex_normal, icosphere

    if args.frequency_sweep:
        print(json.dumps(frequency_sweep(P)), flush=True)
        return
    if args.sponge_sweep:
        print(json.dumps(sponge_sweep(P)), flush=True)
        return

    mesh = icosphere(5)
    N, T = mesh.n_vertices, mesh.n_triangles
    M = P.Mesh.from_inputs(mesh)
    x = torch.from_numpy(complex_normal(2 * N, seed=0)).cuda()
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()

    # first call builds the FP64 near-field operator (setup, not timed)
    t0 = time.perf_counter()
    P.pmchwt_matvec(M, K_EXT, K_INT, RHO, x, y, precision="fp32")
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0

    def timed(precision, steps, warmup):
        for _ in range(warmup):
            P.pmchwt_matvec(M, K_EXT, K_INT, RHO, x, y, precision=precision)
        P.profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            P.pmchwt_matvec(M, K_EXT, K_INT, RHO, x, y, precision=precision)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms_k, n_k = P.profile_read(f"farfield_{precision}")
        P.profile_enable(False)
        return dt / steps, ms_k / max(n_k, 1)

    step_s, kern_ms = timed("fp32", args.steps, args.warmup)
    step64_s, kern64_ms = timed("fp64", max(3, args.steps // 4), 1)

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # measured issue rates of FMA and the transcendental instructions
    rates = P.valu_rates()
    pairs = RL.far_pairs_per_matvec(mesh.triangles)
    symmetric = P.tune_get("farfield.symmetric") == 1
    roof = RL.pair_kernel_roofline(pairs, kern_ms * 1e-3, "fp32", rates, symmetric=symmetric)
    traffic = pmc_traffic()
    roof["traffic"] = traffic["bytes"] if traffic else None
    roof["traffic_detail"] = traffic
    roof64 = RL.pair_kernel_roofline(pairs, kern64_ms * 1e-3, "fp64")
    value = T * (T - 1) / step_s

    solve = None
    if not args.no_solve:
        try:
            solve = {}
            # near-field and OSRC factors are built once per handle: warm them so
            # that no timed solve pays for them (untimed, one iteration)
            P.pmchwt_solve(M, K_EXT, K_INT, RHO, [[0, 0, 1]], 1e-6, precision="fp64", path=0,
                           maxiter=1)
            # FP64 GMRES and FP32 + refinement, each matrix-free and on the
            # assembled operator (assembly included in its time)
            for name, prec, path in (("fp64", "fp64", 0), ("fp32", "fp32", 0),
                                     ("fp32_dense", "fp32", 1), ("fp64_dense", "fp64", 1)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sol, info, rc = P.pmchwt_solve(M, K_EXT, K_INT, RHO, [[0, 0, 1]], 1e-6,
                                               precision=prec, path=path)
                torch.cuda.synchronize()
                # "seconds": wall clock around the call, set-up (assembly) included;
                # "solve_seconds": the library's own time of the wave group's solve
                wall = time.perf_counter() - t0
                solve[name] = {**info[0], "seconds": wall, "solve_seconds": info[0]["seconds"],
                               "rc": rc}
            # the autotuner's choice for this shape (matrix-free vs assembled), then a
            # solve on the auto path
            # (fresh handle with warm near field and OSRC, so that assembly, when
            # chosen, is paid inside the timed solve)
            M2 = P.Mesh.from_inputs(mesh)
            P.pmchwt_solve(M2, K_EXT, K_INT, RHO, [[0, 0, 1]], 1e-6, precision="fp64", path=0,
                           maxiter=1)
            tuned = P.autotune(M2, K_EXT, K_INT, RHO, n_rhs=1,
                               expected_matvecs=solve["fp32"]["iterations"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sol, info, rc = P.pmchwt_solve(M2, K_EXT, K_INT, RHO, [[0, 0, 1]], 1e-6,
                                           precision="fp32", path=2)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            solve["fp32_autotuned"] = {**info[0], "seconds": wall,
                                       "solve_seconds": info[0]["seconds"], "rc": rc,
                                       "tune": tuned}
            P.tune_clear()
            del M2
            solve["speedup_fp32_refine_vs_fp64"] = (solve["fp64"]["seconds"] /
                                                    solve["fp32"]["seconds"])
            solve["speedup_fp32_autotuned_vs_fp64"] = (solve["fp64"]["seconds"] /
                                                       solve["fp32_autotuned"]["seconds"])
            solve["speedup_fp32_dense_refine_vs_fp64"] = (solve["fp64"]["seconds"] /
                                                          solve["fp32_dense"]["seconds"])
            # on the assembled operators: FP32 + refinement against FP64 GMRES
            solve["speedup_fp32_dense_vs_fp64_dense"] = (solve["fp64_dense"]["seconds"] /
                                                         solve["fp32_dense"]["seconds"])
            # dense GEMV throughput (operator resident after the solve)
            P.profile_enable(True)
            for _ in range(5):
                P.pmchwt_matvec(M, K_EXT, K_INT, RHO, x, y, precision="fp32_dense")
            torch.cuda.synchronize()
            gms, gn = P.profile_read("dense_gemv")
            P.profile_enable(False)
            gbytes = (2 * N) ** 2 * 8
            solve["dense_gemv"] = {"ms": gms / gn, "GB_per_s": gbytes / (gms / gn * 1e-3) / 1e9,
                                   "matrix_bytes": gbytes}
            P.profile_enable(True)
            for _ in range(5):
                P.pmchwt_matvec(M, K_EXT, K_INT, RHO, x, y, precision="fp64_dense")
            torch.cuda.synchronize()
            gms, gn = P.profile_read("dense_gemv_fp64")
            P.profile_enable(False)
            solve["dense_gemv_fp64"] = {"ms": gms / gn,
                                        "GB_per_s": 2 * gbytes / (gms / gn * 1e-3) / 1e9,
                                        "matrix_bytes": 2 * gbytes}
            # the four formulations compared in the paper (OSRC, PMCHWT, Calderon,
            # Mueller; strong form), FP32 assembled operator + refinement to the
            # same tolerance, each operator assembled and factorised beforehand
            forms = {}
            for form in ("osrc", "pmchwt", "calderon", "muller"):
                P.pmchwt_solve(M, K_EXT, K_INT, RHO, [[0, 0, 1]], 1e-6, precision="fp32", path=1,
                               formulation=form, maxiter=1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info, rc = P.pmchwt_solve(M, K_EXT, K_INT, RHO, [[0, 0, 1]], 1e-6,
                                             precision="fp32", path=1, formulation=form)
                torch.cuda.synchronize()
                forms[form] = {"seconds": time.perf_counter() - t0, "rc": rc,
                               "iterations": info[0]["iterations"],
                               "outer_steps": info[0]["outer_steps"],
                               "rel_residual": info[0]["rel_residual"]}
                print(f"formulation {form}: {forms[form]}", file=sys.stderr, flush=True)
            solve["formulations_fp32_dense"] = forms
            # total field on the 101 x 101 grid of the paper's accuracy test (3 x 3
            # square through the centre, x-y plane) from the last solution
            g = np.linspace(-1.5, 1.5, 101)
            GX, GY = np.meshgrid(g, g)
            pts = torch.from_numpy(np.stack([GX.ravel(), GY.ravel(), np.zeros(GX.size)], 1)).cuda()
            P.pmchwt_field(M, K_EXT, K_INT, RHO, [0, 0, 1.0], sol[0].contiguous(), pts)
            P.profile_enable(True)
            for _ in range(3):
                P.pmchwt_field(M, K_EXT, K_INT, RHO, [0, 0, 1.0], sol[0].contiguous(), pts)
            fms, fn = P.profile_read("field_eval")
            wms, wn = P.profile_read("field_winding")
            P.profile_enable(False)
            fpairs = pts.shape[0] * 6 * T
            solve["field_101x101"] = {"points": int(pts.shape[0]), "kernel_ms": fms / fn,
                                      "winding_ms": wms / wn,
                                      "roofline": RL.field_roofline(fpairs, fms / fn * 1e-3)}
        except P.BemError as e:
            solve = {"error": str(e)}

    multi = None
    if not args.no_solve:
        multi = multi_material_measure(P, RL)

    batching = None
    if not args.no_batching:
        batching = batch_measure(P, M, mesh, step_s)

    serving = serving_measure(P, args.serving) if args.serving > 0 else None

    out = {
        "metric": METRIC, "value": value, "unit": "tri-pair evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_s * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "icosphere L5 unit sphere (10242 vertices, 20480 "
                               "triangles), k_ext=10, k_int=15, rho=1.5; FP32 pair "
                               "kernel + FP64 near field",
                   "n_vertices": N, "n_triangles": T, "k_ext": K_EXT, "k_int": K_INT,
                   "rho": RHO, "parallelism": "single GPU"},
        "roofline": {**roof, "kernel": "farfield_fp32",
                     "kernel_ms": kern_ms, "point_pairs_per_launch": pairs,
                     "flops_per_unit": RL.FLOPS_PER_UPAIR if symmetric else RL.FLOPS_PER_PAIR,
                     "valu_rates": rates},
        "fp64_matvec": {"ms_per_step": step64_s * 1e3,
                        "tri_pair_evals_per_s": T * (T - 1) / step64_s,
                        "kernel_ms": kern64_ms, "roofline_frac": roof64["frac"]},
        "setup_s": setup_s,
        "solve": solve,
        "multi_material": multi,
        "batching": batching,
        "serving": serving,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
