"""Pins of the oracle's lattice Boltzmann arithmetic (CPU).

Each check ties the oracle to something other than itself: the paper's printed
constants, closed-form moment identities of the D2Q9 equilibrium, the
analytic Taylor-Green decay, the second-order convergence of standard LBM, and
the exact reduction of MLBM to standard LBM on a lattice with dx = h.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import analytic
from synth import jittered_lattice, tgv_initial_velocity


def test_d2q9_tables_match_paper(golden):
    ex, ey, w, opp = oracle.tables()
    e = np.array(golden["d2q9_directions"]["e"], dtype=float)
    np.testing.assert_array_equal(ex, e[:, 0])
    np.testing.assert_array_equal(ey, e[:, 1])
    gw = np.array(golden["d2q9_weights"]["numerators"]) / np.array(
        golden["d2q9_weights"]["denominators"])
    np.testing.assert_allclose(w, gw, rtol=0, atol=1e-16)
    # opposite direction: e_k = -e_k'
    np.testing.assert_array_equal(ex[opp], -ex)
    np.testing.assert_array_equal(ey[opp], -ey)


def test_lattice_isotropy():
    ex, ey, w, _ = oracle.tables()
    e = np.stack([ex, ey], 1)
    assert abs(w.sum() - 1) < 1e-15
    np.testing.assert_allclose(w @ e, 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("k,ka,kb->ab", w, e, e), np.eye(2) / 3, atol=1e-16)
    np.testing.assert_allclose(np.einsum("k,ka,kb,kc->abc", w, e, e, e), 0, atol=1e-16)
    d = np.eye(2)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9
    np.testing.assert_allclose(np.einsum("k,ka,kb,kc,kd->abcd", w, e, e, e, e), iso4,
                               atol=1e-16)


@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.0, 0.0), (1.03, 0.02, -0.05),
                                       (0.97, -0.1, 0.07)])
def test_equilibrium_moments(rho, ux, uy):
    """sum feq = rho, sum feq e = rho u, sum feq e e = rho (I/3 + u u)."""
    ex, ey, _, _ = oracle.tables()
    f = oracle.feq(rho, ux, uy)
    e = np.stack([ex, ey], 1)
    u = np.array([ux, uy])
    assert abs(f.sum() - rho) < 1e-15
    np.testing.assert_allclose(f @ e, rho * u, atol=1e-16)
    np.testing.assert_allclose(np.einsum("k,ka,kb->ab", f, e, e),
                               rho * (np.eye(2) / 3 + np.outer(u, u)), atol=1e-15)
    r, vx, vy = oracle.moments(f[None, :])
    assert abs(r[0] - rho) < 1e-15 and abs(vx[0] - ux) < 1e-15 and abs(vy[0] - uy) < 1e-15


def test_collision_conserves_and_force_moments():
    rng = np.random.default_rng(7)
    n = 64
    f = oracle.equilibrium(1 + 0.01 * rng.standard_normal(n), 0.05 * rng.standard_normal(n),
                           0.05 * rng.standard_normal(n))
    f = f + 1e-3 * rng.standard_normal(f.shape)
    ex, ey, _, _ = oracle.tables()
    post = oracle.collide(f, 0.7)
    np.testing.assert_allclose(post.sum(1), f.sum(1), rtol=0, atol=2e-15)
    np.testing.assert_allclose(post @ ex, f @ ex, atol=2e-15)
    np.testing.assert_allclose(post @ ey, f @ ey, atol=2e-15)
    ax = 1e-3 * rng.standard_normal(n)
    ay = 1e-3 * rng.standard_normal(n)
    pf = oracle.collide(f, 0.7, ax, ay)
    F = pf - post
    np.testing.assert_allclose(F.sum(1), 0, atol=1e-16)
    np.testing.assert_allclose(F @ ex, ax, atol=1e-16)
    np.testing.assert_allclose(F @ ey, ay, atol=1e-16)
    # relaxation: the non-equilibrium part shrinks by (1 - 1/tau)
    r, u, v = oracle.moments(f)
    eq = oracle.equilibrium(r, u, v)
    np.testing.assert_allclose(post - eq, (1 - 1 / 0.7) * (f - eq), atol=1e-15)
    # wall nodes are left untouched by collision and force
    nt = np.zeros(n, np.uint8)
    nt[::3] = 1
    pw = oracle.collide(f, 0.7, ax, ay, nt)
    np.testing.assert_array_equal(pw[nt == 1], (post)[nt == 1])


def test_viscosity_reading_matches_paper_settings(golden):
    """nu = c_s^2 (tau - 1/2) dx^2 / dt gives the paper's nu = 1 at tau = 0.8,
    dx = 1/10, dt = 1e-3 (Sec. 3)."""
    s = golden["tgv_settings"]
    nu = analytic.lattice_viscosity(s["tau"]) * s["dx"] ** 2 / s["dt"]
    assert abs(nu - s["nu"]) < 1e-12
    # the printed form (tau - 0.5) / c_s^2 would not
    assert abs((s["tau"] - 0.5) * 3 * s["dx"] ** 2 / s["dt"] - s["nu"]) > 1


def _lbm_tgv(n, u0, tau, steps):
    c = jittered_lattice(n, length=float(n), jitter=0.0)
    ux, uy = tgv_initial_velocity(c.x, c.y, float(n), u0)
    f = oracle.equilibrium(np.ones(c.n), ux, uy)
    f = oracle.lbm_run(f, n, n, tau, steps)
    _, u, v = oracle.moments(f)
    ut, vt = analytic.tgv_velocity(c.x, c.y, float(n), u0,
                                   analytic.tgv_decay(tau, n, steps))
    return analytic.l2_error(u, ut), f


def test_standard_lbm_tgv_second_order():
    """Standard LBM under diffusive scaling converges at second order to the
    analytic Taylor-Green decay (Sec. 3; the paper quotes 2nd order)."""
    errs = []
    for n, u0, steps in [(16, 0.04, 64), (32, 0.02, 256), (64, 0.01, 1024)]:
        e, _ = _lbm_tgv(n, u0, 0.8, steps)
        errs.append(e)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-3
    assert all(1.8 < r < 2.3 for r in rates), (errs, rates)


@pytest.mark.parametrize("mode", [0, 1])
def test_mlbm_on_lattice_equals_standard_lbm(mode):
    """Nodes on the lattice with dx = h: every departure point is a node, the
    shape vector is a unit vector, and MLBM is standard LBM (Sec. 2.1 vs
    Sec. 2.3)."""
    n = 24
    c = jittered_lattice(n, length=float(n), jitter=0.0)
    nbr, own, W = oracle.build_plan(c, 1.0, 12, 2, mode)
    ux, uy = tgv_initial_velocity(c.x, c.y, float(n), 0.03)
    f0 = oracle.equilibrium(np.ones(c.n), ux, uy)
    f_ml = oracle.run(f0, nbr, own, W, 0.8, 200)
    f_lb = oracle.lbm_run(f0, n, n, 0.8, 200)
    err = np.abs(f_ml - f_lb).max() / np.abs(f_lb).max()
    assert err < 1e-13, err


def test_mlbm_tgv_decay_own_stencil_c1():
    """TGV-40, jittered by 0.3 h, K = 12, degree 2, own-node stencils,
    tau = 0.8, u0 = 0.01, 200 steps: velocity follows the analytic decay."""
    c = jittered_lattice(40, seed=1)
    nbr, own, W = oracle.build_plan(c, c.h, 12, 2, mode=1)
    ux, uy = tgv_initial_velocity(c.x, c.y, c.period[0], 0.01)
    f = oracle.run(oracle.equilibrium(np.ones(c.n), ux, uy), nbr, own, W, 0.8, 200)
    rho, u, v = oracle.moments(f)
    ut, vt = analytic.tgv_velocity(c.x, c.y, c.period[0], 0.01,
                                   analytic.tgv_decay(0.8, 40, 200))
    assert analytic.l2_error(u, ut) < 1e-2
    assert analytic.l2_error(v, vt) < 1e-2
    # periodic domain, no force: mass is conserved up to interpolation error
    assert abs(rho.sum() - c.n) / c.n < 1e-6


def test_mlbm_tgv_converges_under_refinement():
    """Paper stencils (closest-node owner), degree 4, K = 30, dx = h,
    diffusive scaling: the L2 error falls as the cloud is refined (Sec. 3)."""
    errs = []
    for n, u0, steps in [(20, 0.02, 100), (40, 0.01, 400)]:
        c = jittered_lattice(n, seed=5, length=float(n))
        nbr, own, W = oracle.build_plan(c, 1.0, 30, 4, mode=0)
        ux, uy = tgv_initial_velocity(c.x, c.y, float(n), u0)
        f = oracle.run(oracle.equilibrium(np.ones(c.n), ux, uy), nbr, own, W, 0.8, steps)
        _, u, _ = oracle.moments(f)
        ut, _ = analytic.tgv_velocity(c.x, c.y, float(n), u0,
                                      analytic.tgv_decay(0.8, n, steps))
        errs.append(analytic.l2_error(u, ut))
    assert errs[1] < 0.5 * errs[0], errs
    assert errs[1] < 5e-3


def test_paper_stencil_small_p2_diverges_reproduces_paper_remark():
    """K = 12, degree 2, closest-node stencils on a 0.3 h jittered cloud
    diverge within 200 steps, as the paper reports divergence for P2 in part
    of its parameter space (Sec. 3). The same cloud with the paper's N_L = 25
    is stable."""
    c = jittered_lattice(40, seed=1)
    ux, uy = tgv_initial_velocity(c.x, c.y, c.period[0], 0.01)
    f0 = oracle.equilibrium(np.ones(c.n), ux, uy)
    nbr, own, W = oracle.build_plan(c, c.h, 12, 2, mode=0)
    _, u, _ = oracle.moments(oracle.run(f0, nbr, own, W, 0.8, 200))
    assert not np.all(np.abs(u) < 0.1)
    nbr, own, W = oracle.build_plan(c, c.h, 25, 2, mode=0)
    _, u, _ = oracle.moments(oracle.run(f0, nbr, own, W, 0.8, 200))
    assert np.all(np.abs(u) < 0.011)
