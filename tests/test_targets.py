"""The package's analytic fields (the bench's L2 against the analytic flow)
against the oracle's, written independently, and against the closed forms
they must satisfy."""
import math

import numpy as np

from oracle import analytic
from paper_2306_01525_amd import targets


def test_tgv_decay_and_field_match_the_oracle():
    for tau, n_side, steps in ((0.6, 512, 2000), (0.8, 40, 200), (1.3, 100, 37.5)):
        L = 2 * math.pi
        dx = L / n_side
        assert math.isclose(targets.tgv_decay(tau, L, dx, steps),
                            analytic.tgv_decay(tau, n_side, steps), rel_tol=1e-14)
        x, y = np.meshgrid(np.linspace(0, L, 17), np.linspace(0, L, 17))
        ux, uy = targets.tgv_velocity(x, y, L, 0.01, tau, dx, steps)
        ox, oy = analytic.tgv_velocity(x, y, L, 0.01, analytic.tgv_decay(tau, n_side, steps))
        assert np.allclose(ux, ox, rtol=1e-13, atol=0)
        assert np.allclose(uy, oy, rtol=1e-13, atol=0)
    # per step the amplitude falls by exp(-2 nu k^2) in lattice units, nu = (tau - 1/2) / 3
    assert math.isclose(targets.tgv_decay(0.8, 10.0, 1.0, 1.0),
                        math.exp(-2 * 0.1 * (2 * math.pi / 10) ** 2), rel_tol=1e-14)


def test_annulus_profile_matches_the_oracle_and_the_walls():
    r1, r2, dx, g, tau = 1.0, 2.0, 3.6e-3, 1.9e-7, 0.7
    r = np.linspace(r1, r2, 101)
    u = targets.annulus_azimuthal(r, r1, r2, dx, g, tau)
    uo = analytic.annulus_profile(r / dx, r1 / dx, r2 / dx, g, (tau - 0.5) / 3)
    assert np.allclose(u, uo, rtol=1e-12, atol=0)
    scale = np.abs(u).max()
    assert abs(u[0]) < 1e-12 * scale and abs(u[-1]) < 1e-12 * scale   # no slip on both walls
    # r^2 - alpha r + beta / r < 0 between the walls: g > 0 drives u > 0
    assert (u[1:-1] > 0).all()
