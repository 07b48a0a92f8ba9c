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

Legs reported beside the timed steps (each can be skipped): the OSRC apply
(ms, algorithmic bytes, GB/s), the four-sphere multiple-scattering layout,
batching (assembled complex64 operators x 64 right-hand sides on MFMA), the
smallest workload (icosphere L3, FP64 solve to 1e-8 against the Mie series
and the oracle's own solve), the lossy ellipsoid (40 962 vertices: matvecs,
OSRC, FP64 against FP32 + refinement solves, the compressed operator), the
compressed operator at 1e5 vertices, the 256-request serving stream, and the
oracle baselines on the host cores.

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
            "seconds": dt, "n_test": n_test,
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


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def event_ms(fn, reps):
    """Average milliseconds of fn() over reps calls, HIP events on the current
    stream (the library's calls run on it)."""
    import torch
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def osrc_measure(P, M, k, n_p, theta=np.pi / 3, R=None):
    """OSRC apply (strong form, Sec. 2.6-2.7) at the solver's damped
    wavenumber k_eps = k (1 + 0.4 i (k R)^(-2/3)), R = 0.1 (object radius 1),
    on one and eight vectors: ms per apply, the algorithmic bytes of
    bem_osrc_info and the implied GB/s."""
    import torch
    from bem_inputs import complex_normal
    N = M.n_vertices
    R = R if R is not None else 0.1
    k = complex(k)
    keps = k * (1.0 + 0.4j * (k * R) ** (-2.0 / 3.0))
    info = P.osrc_info(M, n_p, theta, k, keps)
    out = {"k": [complex(k).real, complex(k).imag], "k_eps": [keps.real, keps.imag],
           "pade_terms": n_p, "theta": theta, "info": info}
    for r in (1, 8):
        x = torch.from_numpy(complex_normal(r * 2 * N, seed=11).reshape(r, 2 * N)).cuda()
        y = torch.empty_like(x)
        ms = event_ms(lambda: P.osrc_apply(M, n_p, theta, k, keps, x, y), 20)
        byt = info["bytes_per_apply"] * r
        out[f"vectors_{r}"] = {"ms": ms, "ms_per_vector": ms / r,
                               "algorithmic_GB_per_s": byt / (ms * 1e-3) / 1e9,
                               "frac_of_hbm": byt / (ms * 1e-3) / 1e9 / 8000.0}
    return out


def c1_leg(P, RL, cpu: bool) -> dict:
    """Plain method at the smallest workload: unit sphere as icosphere level 3
    (642 vertices), k_ext = 2, k_int = 3, rho = 1.5, plane wave along +z,
    FP64 GMRES to 1e-8 on the matrix-free path.  With cpu (the oracle legs):
    its far field against the oracle's Mie series (181 polar angles) and the
    oracle's full solve (dense complex128 assembly, sparse LU OSRC, GMRES)
    timed on the host cores."""
    import torch
    from bem_inputs import complex_normal, icosphere
    mesh = icosphere(3)
    N, T = mesh.n_vertices, mesh.n_triangles
    M = P.Mesh.from_inputs(mesh)
    x = torch.from_numpy(complex_normal(2 * N, seed=0)).cuda()
    y = torch.empty_like(x)
    out = {"workload": "icosphere L3 unit sphere (642 vertices), k_ext=2, k_int=3, rho=1.5",
           "n_vertices": N, "n_triangles": T}
    for prec in ("fp32", "fp64"):
        ms = event_ms(lambda: P.pmchwt_matvec(M, 2.0, 3.0, 1.5, x, y, precision=prec), 20)
        out[f"{prec}_matvec"] = {"ms": ms, "tri_pair_evals_per_s": T * (T - 1) / (ms * 1e-3)}
    P.pmchwt_solve(M, 2.0, 3.0, 1.5, [[0, 0, 1]], 1e-8, precision="fp64", path=0, maxiter=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol, info, rc = P.pmchwt_solve(M, 2.0, 3.0, 1.5, [[0, 0, 1]], 1e-8, precision="fp64", path=0)
    torch.cuda.synchronize()
    out["fp64_solve"] = {"seconds": time.perf_counter() - t0, "rc": rc,
                         "iterations": info[0]["iterations"],
                         "rel_residual": info[0]["rel_residual"]}
    if cpu:
        from oracle import mie
        th = np.linspace(0.0, np.pi, 181)
        dirs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
        F = P.far_field(M, 2.0, sol[0].contiguous(), dirs)
        Fm = mie.far_field(2.0, 3.0, 1.5, th)
        out["fp64_solve"]["far_field_rel_error_vs_mie"] = float(np.linalg.norm(F - Fm) /
                                                                np.linalg.norm(Fm))
        from oracle import operators as O
        from oracle.solve import PreconditionedSystem
        t0 = time.perf_counter()
        S = PreconditionedSystem(mesh, 2.0, 3.0, 1.5)
        t1 = time.perf_counter()
        xo, it, hist = S.solve([0.0, 0.0, 1.0], tol=1e-8)
        t2 = time.perf_counter()
        out["oracle_solve"] = {"kind": "oracle", "assembly_and_factor_s": t1 - t0,
                               "gmres_s": t2 - t1, "seconds": t2 - t0, "iterations": it,
                               "cores": int(O._load().oracle_num_threads()),
                               "solution_rel_diff_gpu": float(
                                   np.linalg.norm(sol[0].cpu().numpy() - xo) / np.linalg.norm(xo))}
        out["gpu_speedup_vs_oracle_solve"] = out["oracle_solve"]["seconds"] / out["fp64_solve"]["seconds"]
    del M
    return out


def c2_oracle_extrapolation(mesh, cpu_rows: dict, iterations: int) -> dict:
    """The oracle's full C2 solve, extrapolated (labelled as such): its far
    field rows on a sample of test triangles (the cpu_baseline sample) scaled
    to all triangles stand for the dense assembly (the same integrals), a
    complex128 dense matvec timed at 4096 x 4096 and scaled by (2N / 4096)^2
    (memory bound), and the oracle OSRC apply and mass solves timed at full
    size; GMRES iterations are those of the GPU's FP64 solve of the same
    system (the two agree within 2 at every size the tests run)."""
    from oracle.solve import PreconditionedSystem
    N, T = mesh.n_vertices, mesh.n_triangles
    n_test = cpu_rows["n_test"]
    assembly_s = cpu_rows["seconds"] * T / n_test
    rng = np.random.default_rng(0)
    m = 4096
    A = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    v = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    A @ v
    t0 = time.perf_counter()
    for _ in range(5):
        A @ v
    dense_s = (time.perf_counter() - t0) / 5 * (2 * N / m) ** 2
    del A
    t0 = time.perf_counter()
    S = PreconditionedSystem(mesh, K_EXT, K_INT, RHO, B=np.zeros((1, 1), np.complex128))
    osrc_setup_s = time.perf_counter() - t0
    y = rng.standard_normal(2 * N) + 1j * rng.standard_normal(2 * N)
    S.osrc.apply(S.strong(y))
    t0 = time.perf_counter()
    for _ in range(3):
        S.osrc.apply(S.strong(y))
    osrc_s = (time.perf_counter() - t0) / 3
    total = assembly_s + osrc_setup_s + iterations * (dense_s + osrc_s)
    return {"kind": "oracle", "extrapolated": True, "seconds": total,
            "assembly_s": assembly_s, "osrc_setup_s": osrc_setup_s,
            "dense_matvec_s": dense_s, "osrc_apply_s": osrc_s, "iterations": iterations,
            "method": "assembly = oracle far-field rows of the sampled test triangles x "
                      f"{T}/{n_test}; dense c128 matvec timed at 4096^2 x (2N/4096)^2; OSRC "
                      "apply and mass solves timed at full size; iterations of the GPU FP64 "
                      "solve at tol 1e-6"}


def c3_leg(P, RL, rates, steps: int) -> dict:
    """Precision form: ellipsoid with semi-axes (1, 0.6, 0.4) from an
    icosphere of level 6 (40 962 vertices, 81 920 triangles; max edge about
    lambda_int / 8), k_ext = 20, k_int = 30 + 1.5i (lossy interior), rho = 1.9,
    OSRC with 8 Pade terms.  FP32 and FP64 matrix-free matvecs (tri-pair
    evals/s, kernel roofline of the complex-k_int variant), the OSRC apply,
    FP64 GMRES against FP32 + FP64 true-residual refinement to 1e-6 on the
    matrix-free path, and the compressed operator (H-matrix, ACA 1e-5):
    set-up, memory, ms per product and its error against the FP64 product."""
    import torch
    from bem_inputs import complex_normal, ellipsoid, icosphere
    mesh = ellipsoid(icosphere(6))
    N, T = mesh.n_vertices, mesh.n_triangles
    k0, k1, rho, n_p = 20.0, 30.0 + 1.5j, 1.9, 8
    M = P.Mesh.from_inputs(mesh)
    x = torch.from_numpy(complex_normal(2 * N, seed=0)).cuda()
    y = torch.empty_like(x)
    out = {"workload": "ellipsoid (1, 0.6, 0.4) from icosphere L6 (40962 vertices), "
                       "k_ext=20, k_int=30+1.5i, rho=1.9, 8 Pade terms",
           "n_vertices": N, "n_triangles": T}
    progress("C3 matvecs")
    P.pmchwt_matvec(M, k0, k1, rho, x, y, precision="fp32")   # near field built here
    torch.cuda.synchronize()
    pairs = RL.far_pairs_per_matvec(mesh.triangles)
    symmetric = P.tune_get("farfield.symmetric") == 1
    for prec, reps in (("fp32", steps), ("fp64", 2)):
        P.profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            P.pmchwt_matvec(M, k0, k1, rho, x, y, precision=prec)
        torch.cuda.synchronize()
        step = (time.perf_counter() - t0) / reps
        kms, kn = P.profile_read(f"farfield_{prec}")
        P.profile_enable(False)
        kern = kms / max(kn, 1)
        roof = (RL.pair_kernel_roofline(pairs, kern * 1e-3, "fp32", rates, symmetric=symmetric,
                                        lossy=True) if prec == "fp32"
                else RL.pair_kernel_roofline(pairs, kern * 1e-3, "fp64"))
        out[f"{prec}_matvec"] = {"ms_per_step": step * 1e3, "kernel_ms": kern,
                                 "tri_pair_evals_per_s": T * (T - 1) / step, "roofline": roof}
    y64 = P.pmchwt_matvec(M, k0, k1, rho, x, precision="fp64")
    y32 = P.pmchwt_matvec(M, k0, k1, rho, x, precision="fp32")
    out["fp32_matvec"]["rel_error_vs_fp64"] = float(torch.linalg.norm(y32 - y64) /
                                                    torch.linalg.norm(y64))
    progress("C3 OSRC")
    out["osrc"] = osrc_measure(P, M, k1, n_p)
    progress("C3 compressed operator")
    out["compressed"] = hmat_measure(P, M, k0, k1, rho, x, y64)
    progress("C3 solves")
    P.pmchwt_solve(M, k0, k1, rho, [[0, 0, 1]], 1e-6, precision="fp64", path=0, maxiter=1,
                   pade_terms=n_p)
    solves = {}
    for name, prec, path in (("fp32", "fp32", 0), ("fp64", "fp64", 0),
                             ("fp32_compressed", "fp32", 3)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, rc = P.pmchwt_solve(M, k0, k1, rho, [[0, 0, 1]], 1e-6, precision=prec,
                                     path=path, pade_terms=n_p)
        torch.cuda.synchronize()
        solves[name] = {**info[0], "seconds": time.perf_counter() - t0, "rc": rc}
        progress(f"C3 solve {name}: {solves[name]['seconds']:.2f} s, "
                 f"{solves[name]['iterations']} iterations")
    solves["speedup_fp32_refine_vs_fp64"] = solves["fp64"]["seconds"] / solves["fp32"]["seconds"]
    # the compressed operator was built above (hmat_measure): its set-up added
    solves["fp32_compressed"]["setup_s"] = out["compressed"]["first_call_s"]
    solves["fp32_compressed"]["seconds_with_setup"] = (solves["fp32_compressed"]["seconds"] +
                                                       out["compressed"]["first_call_s"])
    solves["speedup_fp32_compressed_refine_vs_fp64"] = (
        solves["fp64"]["seconds"] / solves["fp32_compressed"]["seconds_with_setup"])
    out["solve"] = solves
    del M
    return out


def hmat_measure(P, M, k0, k1, rho, x, y_ref=None) -> dict:
    """Compressed operator (precision fp32_hmat): first call (tree, ACA, dense
    leaves), device bytes, ms per product (HIP events) and, given an FP64
    product of x, the relative error per block row."""
    import torch
    N = M.n_vertices
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y = P.pmchwt_matvec(M, k0, k1, rho, x, precision="fp32_hmat")
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    st = P.hmat_info(M, k0, k1, rho)
    ms = event_ms(lambda: P.pmchwt_matvec(M, k0, k1, rho, x, y, precision="fp32_hmat"), 5)
    out = {"first_call_s": first, "ms_per_product": ms, "bytes": st["bytes"],
           "dense_complex64_bytes": 32 * N * N, "stats": st}
    if y_ref is not None:
        out["rel_error_vs_fp64"] = [
            float(torch.linalg.norm(y[..., sl] - y_ref[..., sl]) / torch.linalg.norm(y_ref[..., sl]))
            for sl in (slice(0, N), slice(N, 2 * N))]
    return out


def compression_large(P) -> dict:
    """Compressed operator at about 1e5 vertices: geodesic sphere of
    frequency 100 (100 002 vertices, 200 000 triangles), k_ext = 10,
    k_int = 15, rho = 1.5; against one FP32 matrix-free product (the dense
    complex64 operator, 320 GB, does not fit)."""
    import torch
    from bem_inputs import complex_normal, geodesic_sphere
    mesh = geodesic_sphere(100)
    N = mesh.n_vertices
    M = P.Mesh.from_inputs(mesh)
    x = torch.from_numpy(complex_normal(2 * N, seed=0)).cuda()
    progress("1e5-vertex sphere: compressed operator")
    out = {"workload": "geodesic sphere f=100 (100002 vertices, 200000 triangles), "
                       "k_ext=10, k_int=15, rho=1.5", "n_vertices": N,
           "n_triangles": mesh.n_triangles}
    out.update(hmat_measure(P, M, 10.0, 15.0, 1.5, x))
    progress("1e5-vertex sphere: matrix-free FP32 product")
    y = P.pmchwt_matvec(M, 10.0, 15.0, 1.5, x, precision="fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y = P.pmchwt_matvec(M, 10.0, 15.0, 1.5, x, y, precision="fp32")
    torch.cuda.synchronize()
    out["matrix_free_fp32_ms"] = (time.perf_counter() - t0) * 1e3
    yh = P.pmchwt_matvec(M, 10.0, 15.0, 1.5, x, precision="fp32_hmat")
    out["rel_diff_vs_matrix_free_fp32"] = [
        float(torch.linalg.norm(yh[..., sl] - y[..., sl]) / torch.linalg.norm(y[..., sl]))
        for sl in (slice(0, N), slice(N, 2 * N))]
    progress("1e5-vertex sphere: FP32 compressed solve with FP64 residuals")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info, rc = P.pmchwt_solve(M, 10.0, 15.0, 1.5, [[0, 0, 1]], 1e-6, precision="fp32", path=3)
    torch.cuda.synchronize()
    out["solve_fp32_compressed"] = {**info[0], "seconds": time.perf_counter() - t0, "rc": rc,
                                    "note": "OSRC factors and near field built inside the call; "
                                            "compressed operator already built above"}
    del M
    return out


def serving_measure(P, n_requests: int, workers: int = 8, seed: int = 5) -> dict:
    """Serving mix: meshes {icosphere L3, L4, L5, ellipsoid (geodesic 45
    scaled by (1, 0.6, 0.4)), two level-4 spheres}, k_ext ~ U[1, 20],
    k_int/k_ext ~ U[1.3, 1.9], rho ~ U[1.2, 2.0], 1-8 plane waves, tol 1e-6,
    FP32 + refinement, auto path (seeded stream, seed 5), a server of
    `workers` concurrent requests.  Every 4th request of the stream submitted
    at once gives the saturated solves/s; the whole stream then arrives as a
    Poisson process at 0.7 x that rate."""
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

    # saturated throughput: every 4th request of the stream (a sample with
    # the stream's mix) submitted at once
    sample = reqs[::4] if n_requests >= 32 else reqs
    n_sat = len(sample)
    t0 = time.perf_counter()
    for i, rid in enumerate([submit(r) for r in sample]):
        srv.wait(rid)
        if (i + 1) % 8 == 0:
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
        "saturated_solves_per_s": sat, "saturated_sample": n_sat,
        "arrival_rate_per_s": lam, "solves_per_s": n_requests / elapsed,
        "waves_per_s": sum(len(r["directions"]) for r in reqs) / elapsed,
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "p50_queue_wait_s": float(np.percentile(queue_wait, 50)),
        "mean_concurrency": busy / elapsed, "peak_inflight": stats["peak_inflight"],
        "peak_bytes": stats["peak_bytes"], "budget": stats["budget"],
        "evictions": stats["evictions"], "rejected": stats["rejected"],
        "krylov_growth_bytes": stats["krylov_growth_bytes"],
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
    ap.add_argument("--no-c1", action="store_true", help="skip the icosphere L3 leg")
    ap.add_argument("--no-c3", action="store_true", help="skip the lossy-ellipsoid leg")
    ap.add_argument("--no-compression", action="store_true",
                    help="skip the compressed operator at 1e5 vertices")
    ap.add_argument("--no-multi", action="store_true", help="skip the four-sphere leg")
    ap.add_argument("--serving", type=int, default=256, metavar="N",
                    help="requests of the serving mix to replay (0: skip)")
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

    progress("C2 timed matvec steps")
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
        progress("C2 solves")
        try:
            solve = {}
            # near-field and OSRC factors are built once per handle: warm them so
            # that no timed solve pays for them (untimed, one iteration)
            P.pmchwt_solve(M, K_EXT, K_INT, RHO, [[0, 0, 1]], 1e-6, precision="fp64", path=0,
                           maxiter=1)
            # FP64 GMRES and FP32 + refinement, each matrix-free and on the
            # assembled operator (assembly included in its time: each assembled
            # solve on a fresh handle whose near field and OSRC factors are warm)
            for name, prec, path in (("fp64", "fp64", 0), ("fp32", "fp32", 0),
                                     ("fp32_dense", "fp32", 1), ("fp64_dense", "fp64", 1)):
                Ms = M
                if path == 1:
                    Ms = P.Mesh.from_inputs(mesh)
                    P.pmchwt_solve(Ms, K_EXT, K_INT, RHO, [[0, 0, 1]], 1e-6, precision="fp64",
                                   path=0, maxiter=1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sol, info, rc = P.pmchwt_solve(Ms, K_EXT, K_INT, RHO, [[0, 0, 1]], 1e-6,
                                               precision=prec, path=path)
                torch.cuda.synchronize()
                # "seconds": wall clock around the call, set-up (assembly) included;
                # "solve_seconds": the library's own time of the wave group's solve
                wall = time.perf_counter() - t0
                solve[name] = {**info[0], "seconds": wall, "solve_seconds": info[0]["seconds"],
                               "rc": rc}
                if Ms is not M:
                    del Ms
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
            # FP32 refinement with the compressed operator in the inner solves
            # (H-matrix built inside the timed call) and FP64 matrix-free residuals
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info, rc = P.pmchwt_solve(M, K_EXT, K_INT, RHO, [[0, 0, 1]], 1e-6,
                                         precision="fp32", path=3)
            torch.cuda.synchronize()
            solve["fp32_compressed"] = {**info[0], "seconds": time.perf_counter() - t0,
                                        "solve_seconds": info[0]["seconds"], "rc": rc}
            solve["speedup_fp32_compressed_refine_vs_fp64"] = (solve["fp64"]["seconds"] /
                                                               solve["fp32_compressed"]["seconds"])
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

    progress("C2 OSRC apply")
    osrc = osrc_measure(P, M, K_INT, 4)

    multi = None
    if not args.no_solve and not args.no_multi:
        progress("four spheres")
        multi = multi_material_measure(P, RL)

    batching = None
    if not args.no_batching:
        progress("batching")
        batching = batch_measure(P, M, mesh, step_s)
    del M

    c1 = None
    if not args.no_c1:
        progress("C1")
        c1 = c1_leg(P, RL, cpu=not args.no_cpu_baseline)

    c3 = None
    if not args.no_c3:
        progress("C3")
        c3 = c3_leg(P, RL, rates, max(3, args.steps // 4))

    large = None
    if not args.no_compression:
        large = compression_large(P)

    serving = None
    if args.serving > 0:
        progress("serving")
        serving = serving_measure(P, args.serving)

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
        "osrc": osrc,
        "multi_material": multi,
        "batching": batching,
        "c1": c1,
        "c3": c3,
        "compression_1e5": large,
        "serving": serving,
    }
    if not args.no_cpu_baseline:
        progress("oracle baselines")
        cb = cpu_baseline(mesh)
        out["cpu_baseline"] = cb
        if solve and "fp64" in solve:
            ext = c2_oracle_extrapolation(mesh, cb, solve["fp64"]["iterations"])
            ext["gpu_speedup_fp64"] = ext["seconds"] / solve["fp64"]["seconds"]
            ext["gpu_speedup_fp32_refine"] = ext["seconds"] / solve["fp32"]["seconds"]
            out["oracle_c2_solve"] = ext
    print(json.dumps(out))


if __name__ == "__main__":
    main()
