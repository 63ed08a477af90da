"""Closed-form solutions and error measures used to pin the oracle (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Lattice viscosity. The paper prints nu = (tau - 0.5) / c_s^2 (Sec. 2.1);
  its own Taylor-Green settings (tau = 0.8, dx = 1/10, dt = 1e-3 giving
  nu = 1, Sec. 3) require nu = c_s^2 (tau - 1/2) dx^2 / dt, which is the
  standard BGK result and the reading used here.
* Taylor-Green vortex (Sec. 3, eq. tgv_eqs): the velocity decays as
  exp(-2 nu k^2 t) with k = 2 pi / L.
* Annular channel (Sec. 3, eq. bch_solution): u(r) = -G (r^2 - alpha r +
  beta / r), G = g / (3 nu).
* Error norm (Sec. 3, eq. L2norm).
"""
from __future__ import annotations

import math

import numpy as np

CS2 = 1.0 / 3.0


def lattice_viscosity(tau: float) -> float:
    """nu in lattice units (dx = dt = 1)."""
    return CS2 * (tau - 0.5)


def tgv_decay(tau: float, length_lattice: float, steps: float) -> float:
    """Amplitude factor exp(-2 nu k^2 t) after `steps` lattice timesteps on a
    periodic square whose side is `length_lattice` streaming distances."""
    k = 2.0 * math.pi / length_lattice
    return math.exp(-2.0 * lattice_viscosity(tau) * k * k * steps)


def tgv_velocity(x, y, length, u0, decay):
    """u = u0 decay (sin kx cos ky, -cos kx sin ky), k = 2 pi / length."""
    k = 2.0 * math.pi / length
    return (u0 * decay * np.sin(k * x) * np.cos(k * y),
            -u0 * decay * np.cos(k * x) * np.sin(k * y))


def annulus_profile(r, r1, r2, g, nu):
    """Azimuthal velocity of the forced annular channel, eq. bch_solution,
    in whatever consistent units r, g and nu are given."""
    G = g / (3.0 * nu)
    alpha = (r1 * r1 + r1 * r2 + r2 * r2) / (r1 + r2)
    beta = (r1 * r1 * r2 * r2) / (r1 + r2)
    return -G * (r * r - alpha * r + beta / r)


def l2_error(u, u_true) -> float:
    """Normalised discrete L2 norm of eq. L2norm."""
    u = np.asarray(u, dtype=np.float64)
    u_true = np.asarray(u_true, dtype=np.float64)
    return float(np.sqrt(np.sum((u - u_true) ** 2)) / np.sqrt(np.sum(u_true ** 2)))
