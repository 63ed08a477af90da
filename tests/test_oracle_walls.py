"""The paper's bounce-back wall rule in the oracle (Sec. 3: boundary nodes on
the wall, each population entering from outside takes the post-streaming
value of the opposite direction at the same node)."""
import math

import numpy as np

import oracle
from oracle import analytic
from synth.clouds import annulus_poisson


def _ex_ey():
    ex, ey, _, _ = oracle.tables()
    return ex, ey


def test_links_are_the_directions_entering_from_outside():
    """A population arriving at a wall node enters from outside exactly when
    its departure point x - e_k dx (dx small) lies outside the fluid: checked
    on the two circles of the annulus at many angles."""
    ex, ey = _ex_ey()
    th = np.linspace(0.0, 2 * np.pi, 97, endpoint=False) + 0.01
    for R, inner in ((1.0, True), (2.0, False)):
        x, y = R * np.cos(th), R * np.sin(th)
        out_n = (-1.0 if inner else 1.0)
        links = oracle.bounce_links(out_n * x / R, out_n * y / R, np.ones(th.size, np.uint8))
        dx = 1e-7
        for k in range(1, 9):
            r = np.hypot(x - ex[k] * dx, y - ey[k] * dx)
            outside = r < R if inner else r > R
            np.testing.assert_array_equal(((links >> (k - 1)) & 1).astype(bool), outside)
    assert (oracle.bounce_links(np.ones(3), np.zeros(3), np.zeros(3, np.uint8)) == 0).all()


def test_reflection_identities():
    """Generic normal: all four opposite pairs are mirrored, so the momentum
    vanishes and rho = f_0 + 2 (sum of the kept populations). Lattice-aligned
    flat wall (fluid above, outward normal (0, -1)): f_2, f_5, f_6 take
    f_4, f_7, f_8; then j_y = 0 and j_x = f_1 - f_3."""
    ex, ey = _ex_ey()
    rng = np.random.default_rng(3)
    f = rng.uniform(0.01, 0.2, size=(2, 9))
    lk = oracle.bounce_links(np.array([math.cos(0.3), 0.0]), np.array([math.sin(0.3), -1.0]),
                             np.ones(2, np.uint8))
    g = oracle.bounce(f, lk)
    kept = [k for k in range(1, 9) if not (lk[0] >> (k - 1)) & 1]
    assert len(kept) == 4
    assert abs(g[0] @ ex) < 1e-15 and abs(g[0] @ ey) < 1e-15
    assert abs(g[0].sum() - (f[0, 0] + 2 * f[0, kept].sum())) < 1e-15
    assert lk[1] == (1 << 1) | (1 << 4) | (1 << 5)        # directions 2, 5, 6
    assert g[1, 2] == f[1, 4] and g[1, 5] == f[1, 7] and g[1, 6] == f[1, 8]
    assert abs(g[1] @ ey) < 1e-15
    assert abs(g[1] @ ex - (f[1, 1] - f[1, 3])) < 1e-15


def test_annulus_bounce_back_steady_profile():
    """tau = 1, the paper's N_L = 15 with P2, dx = 1/40, body force 1e-6: the
    wall nodes come to rest, the steady speed matches eq. bch_solution, and the
    error falls faster than second order from h = 1/10 to h = 1/20."""
    R1, R2, tau, g, dx = 1.0, 2.0, 1.0, 1e-6, 1.0 / 40
    nu = (tau - 0.5) / 3.0
    errs = []
    for h in (0.1, 0.05):
        c = annulus_poisson(R1, R2, h, seed=3)
        r = np.hypot(c.x, c.y)
        s = np.where(r < 0.5 * (R1 + R2), -1.0, 1.0)
        links = oracle.bounce_links(s * c.x / r, s * c.y / r, c.node_type)
        nbr, own, W = oracle.build_plan(c, dx, 15, 2, mode=0)
        ax, ay = oracle.azimuthal_force(c.x, c.y, g, None)
        f = oracle.equilibrium(np.ones(c.n), np.zeros(c.n), np.zeros(c.n))
        f = oracle.run(f, nbr, own, W, tau, 20000, ax, ay, links=links)
        _, u, v = oracle.moments(f)
        U = np.hypot(u, v)
        exact = np.abs(analytic.annulus_profile(r / dx, R1 / dx, R2 / dx, g, nu))
        assert U[c.node_type == 1].max() < 1e-12 * exact.max()
        errs.append(analytic.l2_error(U, exact))
    assert errs[1] < 5e-3
    assert errs[0] / errs[1] > 4.0
