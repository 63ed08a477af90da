"""Pin of the oracle's forced, walled path against the analytic annular
channel profile (Sec. 3, eq. bch_solution), plus the closed-form constants."""
import numpy as np

import oracle
from oracle import analytic
from synth import annulus_poisson


def test_profile_constants_and_boundary_values(golden):
    a = golden["annulus_settings"]
    r1, r2 = a["R1"], a["R2"]
    alpha = (r1 * r1 + r1 * r2 + r2 * r2) / (r1 + r2)
    beta = (r1 * r1 * r2 * r2) / (r1 + r2)
    assert abs(alpha - a["alpha"][0] / a["alpha"][1]) < 1e-15
    assert abs(beta - a["beta"][0] / a["beta"][1]) < 1e-15
    assert abs(analytic.annulus_profile(r1, r1, r2, 1.0, 1.0)) < 1e-15
    assert abs(analytic.annulus_profile(r2, r1, r2, 1.0, 1.0)) < 1e-15
    # it solves nu (u'' + u'/r - u/r^2) = -g (finite differences)
    r = np.linspace(1.1, 1.9, 9)
    h = 1e-4
    u = lambda s: analytic.annulus_profile(s, r1, r2, 2.0, 0.5)
    lap = (u(r + h) - 2 * u(r) + u(r - h)) / h ** 2 + (u(r + h) - u(r - h)) / (2 * h) / r \
        - u(r) / r ** 2
    np.testing.assert_allclose(0.5 * lap, -2.0, rtol=1e-5)


def _run_annulus(h, dx, K, m, tau=1.0, g_scale=3.45e-5):
    c = annulus_poisson(1.0, 2.0, h, seed=3)
    nbr, own, W = oracle.build_plan(c, dx, K, m, mode=0)
    g = g_scale * (dx / 0.05) ** 3           # keeps u_max near 0.01 in lattice units
    ax, ay = oracle.azimuthal_force(c.x, c.y, g, c.node_type)
    f = oracle.equilibrium(np.ones(c.n), np.zeros(c.n), np.zeros(c.n))
    prev, steps = None, 0
    nu = analytic.lattice_viscosity(tau)
    while steps < 20000:
        f = oracle.run(f, nbr, own, W, tau, 100, ax, ay, c.node_type, 1.0)
        steps += 100
        _, u, v = oracle.moments(f)
        U = np.hypot(u, v)
        if prev is not None and np.linalg.norm(U - prev) / np.linalg.norm(U) < 1e-10:
            break
        prev = U
    r = np.hypot(c.x, c.y)
    fl = c.node_type == 0
    ut = analytic.annulus_profile(r / dx, 1 / dx, 2 / dx, g, nu)
    uphi = (-c.y * u + c.x * v) / r
    ur = (c.x * u + c.y * v) / r
    return analytic.l2_error(U[fl], np.abs(ut[fl])), analytic.l2_error(uphi[fl], ut[fl]), \
        np.abs(ur[fl]).max() / np.abs(ut).max(), steps


def test_annulus_steady_profile_converges_in_h():
    """dx = 1/20 fixed, the paper's stencil (N_L = 15, P2), equilibrium walls:
    the steady velocity matches the analytic profile and improves when the
    cloud is refined from h = 1/10 to h = 1/20 (Sec. 3, Fig. bch_conv)."""
    e_coarse = _run_annulus(0.1, 0.05, 15, 2)
    e_fine = _run_annulus(0.05, 0.05, 15, 2)
    assert e_fine[3] < 20000 and e_coarse[3] < 20000   # residual reached 1e-10
    assert e_fine[0] < 1e-2 and e_fine[1] < 1e-2
    assert e_fine[0] < e_coarse[0]
    assert e_fine[2] < 1e-2          # flow is azimuthal
