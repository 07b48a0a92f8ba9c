"""Acoustic media of the paper's benchmarks (Table 1): density rho (kg/m^3),
speed of sound c (m/s) and the power-law attenuation alpha (Np/m/Hz^b at
frequencies in MHz), k = 2 pi f / c + i alpha (f / 1 MHz)^b.  Input data only:
wavenumbers made nondimensional by a length scale (the sphere radius)."""
from __future__ import annotations

import math

MEDIA = {
    "water": (1000.0, 1500.0, 0.015, 2.0),
    "fat": (917.0, 1412.0, 9.334, 1.0),
    "bone": (1912.0, 4080.0, 47.20, 1.0),
}


def wavenumber(medium: str, f_hz: float, length_m: float) -> complex:
    """k of the medium at frequency f, times the length scale."""
    _, c, alpha, b = MEDIA[medium]
    return complex(2 * math.pi * f_hz / c, alpha * (f_hz * 1e-6) ** b) * length_m


def density_ratio(medium: str, exterior: str = "water") -> float:
    return MEDIA[medium][0] / MEDIA[exterior][0]
