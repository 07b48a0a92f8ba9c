"""Algorithmic work model of the matrix-free PMCHWT pair kernel.

Unit of work: one quadrature point pair (x in tau, y in sigma), both
wavenumbers, all four operators (V, K, K', D in Maue form) fused.  The count
below is the arithmetic the fused kernel performs per point pair for real
wavenumbers and one object, with a fused multiply-add counted as 2 flops.
Transcendentals (1/sqrt r^2, sin and cos of two phases) run at a quarter of
the FMA issue rate on CDNA, so each occupies 4 issue slots = 8 flop-equivalents.
"""
from __future__ import annotations

import numpy as np

# itemised per-point-pair count (flops, FMA = 2)
FLOPS_ITEMS = {
    "difference y - x": 3,
    "r^2 (mul + 2 fma)": 5,
    "r = r^2 / sqrt(r^2)": 1,
    "phases k r / 2pi and reduction, 2 wavenumbers": 6,
    "G_0, G_1 = e^{ikr} / r": 4,
    "F_m r^2 = G_m (i k_m r - 1), 2 wavenumbers": 10,
    "F = (F_0 + F_1) / r^2": 5,
    "G_V, G_W (2 complex axpy)": 8,
    "G_N (k_0^2 G_0 + k_1^2 G_1 / rho) (n_x . n_y)": 14,
    "F (y-x).n_y, F (x-y).n_x": 4,
    "row-1 and row-2 accumulations (4 complex fma pairs)": 32,
    "curl-term weight sum w_x w_y G_W": 4,
}
FLOPS_PER_PAIR = sum(FLOPS_ITEMS.values())            # 96
TRANS_PER_PAIR = 5                                    # rsqrt, 2 sin, 2 cos
TRANS_FLOP_EQ = 8                                     # quarter rate: 4 FMA slots
FLOP_EQ_PER_PAIR = FLOPS_PER_PAIR + TRANS_PER_PAIR * TRANS_FLOP_EQ   # 136

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, FMA = 2 flops
PEAK_FP32_PLAIN_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12   # 78.6 (no packed FP32)
PEAK_FP32_PACKED_TFLOPS = 157.3                            # published, packed
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


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
                         precision: str = "fp32") -> dict:
    achieved = point_pairs * FLOP_EQ_PER_PAIR / seconds_per_launch / 1e12
    peak = PEAK_FP32_PLAIN_TFLOPS if precision == "fp32" else PEAK_FP64_TFLOPS
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": None}
