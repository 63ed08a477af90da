"""Analytic reference fields for accuracy diagnostics (lattice units).

* Taylor-Green vortex (Sec. 3, eq. tgv_eqs): on a periodic square of side L
  (in cloud units) discretised with streaming distance dx, the velocity decays
  as exp(-2 nu k^2 t) with k = 2 pi / L, nu = (tau - 1/2) / 3 dx^2 / dt, so per
  lattice step the exponent is 2 (tau - 1/2) / 3 (2 pi dx / L)^2.
* Annular channel (Sec. 3, eq. bch_solution): u(r) = -G (r^2 - alpha r +
  beta / r), G = g / (3 nu), in lattice units r/dx.
"""
from __future__ import annotations

import math

import numpy as np


def tgv_decay(tau: float, length: float, dx: float, steps: float) -> float:
    k_lat = 2.0 * math.pi * dx / length
    return math.exp(-2.0 * (tau - 0.5) / 3.0 * k_lat * k_lat * steps)


def tgv_velocity(x, y, length: float, u0: float, tau: float, dx: float, steps: float):
    a = u0 * tgv_decay(tau, length, dx, steps)
    k = 2.0 * math.pi / length
    return a * np.sin(k * x) * np.cos(k * y), -a * np.cos(k * x) * np.sin(k * y)


def annulus_azimuthal(r, r1: float, r2: float, dx: float, g: float, tau: float):
    nu = (tau - 0.5) / 3.0
    rl, r1l, r2l = r / dx, r1 / dx, r2 / dx
    alpha = (r1l * r1l + r1l * r2l + r2l * r2l) / (r1l + r2l)
    beta = (r1l * r1l * r2l * r2l) / (r1l + r2l)
    return -(g / (3.0 * nu)) * (rl * rl - alpha * rl + beta / rl)
