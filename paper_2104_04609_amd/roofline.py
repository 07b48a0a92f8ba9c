"""Algorithmic work model and issue-bound roofline of the matrix-free PMCHWT
pair kernel.

Unit of work: one quadrature point pair (x in tau, y in sigma), both
wavenumbers, all four operators (V, K, K', D in Maue form) fused.  The work
per unit is the itemised count below, frozen before the kernel was tuned:
about 110 flops (FMA = 2) and 5 transcendentals (1/sqrt r^2, sin and cos of
two phases).  The kernel itself now needs fewer flops per pair (it factors
triangle constants out of the point sums); the frozen count stays the unit so
that speed-ups show up as a higher fraction.

Issue-bound model (FP32):  t_pair = F / P32 + sum_t n_t / P_t  with
P32 = 157.3 TFLOP/s (published vector FP32 peak of MI355X) and P_t the issue
rate of each transcendental instruction, measured on the device by
``bem_valu_rates``.  The roofline object reports achieved and peak in
flop-equivalents at the P32 rate, so frac = achieved pairs/s / model pairs/s.
FP64: table-based sin/cos and a refined 1/sqrt counted in flops (55 per
pair), against the 78.6 TFLOP/s FP64 vector peak.  The symmetric FP32
kernel (each separated triangle pair once) uses the unordered point pair
as its unit: 164 flops (the accumulations twice) and the same 5
transcendentals.
"""
from __future__ import annotations

import numpy as np

# itemised per-point-pair count (flops, FMA = 2)
FLOPS_ITEMS = {
    "geometry: y - x, r^2, r, (y - x).n_y, (x - y).n_x": 20,
    "per wavenumber (x2): phase k r / 2pi, G = e^{ikr}/r, F = G (ikr - 1)/r^2": 20,
    "combinations G_V, G_W, G_N (n_x.n_y), F": 16,
    "accumulations: V, K, K', D normal and curl-curl parts": 54,
}
FLOPS_PER_PAIR = sum(FLOPS_ITEMS.values())            # 110
TRANS_PER_PAIR = {"sin_f32": 2, "cos_f32": 2, "rsq_f32": 1}
# FP64: sin and cos of each phase from a 256-entry table of e^{2 pi i n/256}
# and short Taylor series (reduction 5, two series 12, complex product 6
# flops per phase), 1/sqrt from the hardware estimate and two Newton steps (9)
FP64_TRANS_FLOPS_PER_PAIR = 2 * 23 + 9

# VALU instructions per point pair of the tuned FP32 kernel (real wavenumbers,
# one object), counted in its gfx950 assembly: 1890 VALU FP32 instructions per
# 36-pair unrolled trial-triangle iteration, transcendentals excluded.
KERNEL_VALU_PER_PAIR = 52.5

# Symmetric FP32 kernel (each separated triangle pair once, rows of both
# triangles): unit = one unordered point pair.  The geometry, wavenumber and
# combination items serve both directions; the accumulations are done for
# each direction.
FLOPS_ITEMS_SYM = dict(FLOPS_ITEMS)
FLOPS_ITEMS_SYM["accumulations: V, K, K', D normal and curl-curl parts"] = 2 * 54
FLOPS_PER_UPAIR = sum(FLOPS_ITEMS_SYM.values())        # 164
# its instruction stream (real wavenumbers, one object; SQ_INSTS_VALU per
# wave and unordered point pair, 82.4, minus the 5 transcendentals),
# including the per-trial-triangle work and the cross-lane sums of the rows
# of sigma
KERNEL_VALU_PER_UPAIR = 77.4

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
LANE_ISSUE_PER_S = 256 * 4 * 16 * 2.4e9                  # 3.93e13 (wave64 op = 4 cycles)
PEAK_FP32_PLAIN_TFLOPS = 2 * LANE_ISSUE_PER_S / 1e12     # 78.6, plain FP32 FMA
PEAK_FP32_TFLOPS = 157.3                                 # published vector FP32 (packed)
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# quarter-rate assumption, used only when no measured rates are given
QUARTER_RATES = {"fma_f32": LANE_ISSUE_PER_S, "sin_f32": LANE_ISSUE_PER_S / 4,
                 "cos_f32": LANE_ISSUE_PER_S / 4, "rsq_f32": LANE_ISSUE_PER_S / 4,
                 "fma_f64": LANE_ISSUE_PER_S}


def trans_seconds_per_pair(rates: dict) -> float:
    return sum(n / rates[op] for op, n in TRANS_PER_PAIR.items())


def model_pairs_per_s(rates: dict | None = None) -> float:
    """Issue-bound model peak of FP32 point-pair evaluations per second."""
    rates = rates or QUARTER_RATES
    return 1.0 / (FLOPS_PER_PAIR / (PEAK_FP32_TFLOPS * 1e12) + trans_seconds_per_pair(rates))


def flop_eq_per_pair(rates: dict | None = None) -> float:
    """Flop-equivalents per pair at the P32 rate (transcendentals priced by
    their measured issue rate)."""
    rates = rates or QUARTER_RATES
    return FLOPS_PER_PAIR + PEAK_FP32_TFLOPS * 1e12 * trans_seconds_per_pair(rates)


def adjacent_ordered_pairs(triangles: np.ndarray) -> int:
    """Number of ordered triangle pairs sharing >= 1 vertex (incl. tau == sigma)."""
    T = triangles.shape[0]
    nv = int(triangles.max()) + 1
    star = [[] for _ in range(nv)]
    for t, tri in enumerate(triangles):
        for v in tri:
            star[v].append(t)
    count = 0
    for t, tri in enumerate(triangles):
        s = set()
        for v in tri:
            s.update(star[v])
        count += len(s)
    return count


def far_pairs_per_matvec(triangles: np.ndarray) -> int:
    """Point pairs the pair kernel evaluates per matvec (separated pairs x 36)."""
    T = triangles.shape[0]
    return 36 * (T * T - adjacent_ordered_pairs(triangles))


def pair_kernel_roofline(point_pairs: int, seconds_per_launch: float,
                         precision: str = "fp32", rates: dict | None = None,
                         symmetric: bool = False, lossy: bool = False) -> dict:
    """point_pairs: ordered separated point pairs per matvec.  symmetric: the
    FP32 kernel evaluates each unordered pair once (unit = unordered pair).
    lossy: complex interior wavenumber, one more transcendental per pair (the
    decay e^{-Im(k) r} as exp2, priced at the 1/sqrt issue rate: both are
    quarter-rate transcendental instructions) and its multiply (2 flops)."""
    pairs_s = point_pairs / seconds_per_launch
    if precision == "fp32" and symmetric:
        r = rates or QUARTER_RATES
        upairs_s = pairs_s / 2
        tt = trans_seconds_per_pair(r) + (1.0 / r["rsq_f32"] if lossy else 0.0)
        if lossy:
            fe_extra = 2 * 2   # the decay times both accumulated Green's functions
            fe = FLOPS_PER_UPAIR + fe_extra + PEAK_FP32_TFLOPS * 1e12 * tt
            achieved = upairs_s * fe / 1e12
            return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                    "work_unit": "unordered point pair (complex k_int)",
                    "flop_eq_per_unit": fe, "units_per_s": upairs_s,
                    "point_pairs_per_s": pairs_s, "rates_measured": rates is not None}
        fe = FLOPS_PER_UPAIR + PEAK_FP32_TFLOPS * 1e12 * tt
        achieved = upairs_s * fe / 1e12
        t_issue = KERNEL_VALU_PER_UPAIR / r["fma_f32"] + tt
        return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                "work_unit": "unordered point pair", "flop_eq_per_unit": fe,
                "units_per_s": upairs_s, "point_pairs_per_s": pairs_s,
                "model_units_per_s": 1.0 / (FLOPS_PER_UPAIR / (PEAK_FP32_TFLOPS * 1e12) + tt),
                "issue_frac": upairs_s * t_issue, "rates_measured": rates is not None,
                # the same launch priced in the one-directional unit (ordered
                # pairs, 110 flops + 5 transcendentals each): what a kernel
                # evaluating every ordered pair would need to reach
                "frac_ordered_unit": pairs_s / model_pairs_per_s(rates)}
    if precision == "fp32":
        fe = flop_eq_per_pair(rates)
        achieved = pairs_s * fe / 1e12
        out = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
               "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
               "flop_eq_per_pair": fe, "point_pairs_per_s": pairs_s,
               "model_point_pairs_per_s": model_pairs_per_s(rates)}
        r = rates or QUARTER_RATES
        # issue utilisation of the kernel's own instruction stream
        t_issue = KERNEL_VALU_PER_PAIR / r["fma_f32"] + trans_seconds_per_pair(r)
        out["issue_frac"] = pairs_s * t_issue
        out["rates_measured"] = rates is not None
        return out
    fe = FLOPS_PER_PAIR + FP64_TRANS_FLOPS_PER_PAIR
    achieved = pairs_s * fe / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None, "flop_eq_per_pair": fe,
            "point_pairs_per_s": pairs_s}


# Field off the surface (FP64): unit = one (target point, trial quadrature
# point) pair.  y - p, r^2 (8), r and 1/r, phase, decay and G (5), F = G (ikr - 1)
# / r^2 (13), the single- and double-layer accumulations (16): 42 flops; the
# sin/cos of the phase and the square root priced as in the FP64 matvec (23 +
# 9 flops); per triangle (y - p).n (6) and the double-layer product (4) are
# spread over its 6 points.
FIELD_FLOPS_PER_PAIR = 42 + 10 / 6
FIELD_TRANS_FLOPS_PER_PAIR = 23 + 9


def field_roofline(point_pairs: int, seconds_per_launch: float) -> dict:
    pairs_s = point_pairs / seconds_per_launch
    fe = FIELD_FLOPS_PER_PAIR + FIELD_TRANS_FLOPS_PER_PAIR
    achieved = pairs_s * fe / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None, "flop_eq_per_pair": fe,
            "point_pairs_per_s": pairs_s}
