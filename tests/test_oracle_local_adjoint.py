"""The single-node reference of the full-size reversed-step test, checked
on the CPU: its disc search gives the rows of the oracle's transposed
streaming operator over a whole (small) cloud, and its finite-difference
collision Jacobian has the structure BGK fixes (conserved mass and momentum,
relaxation of non-equilibrium parts by 1 - 1/tau)."""
import numpy as np

import oracle
from adjoint_local import collision_jacobian, transposed_row
from synth import jittered_lattice, random_field, tgv_initial_velocity


def test_transposed_rows_match_the_whole_cloud_operator():
    c = jittered_lattice(64, seed=5)
    K, m = 30, 4
    nbr = oracle.knn(c.x, c.y, c.period, K)
    own = oracle.owners(c.x, c.y, c.period, c.h, 0)
    W = oracle.weights(c.x, c.y, c.period, c.h, K, m, nbr, own)
    lam = random_field((c.n, 9), seed=3)
    ref = oracle.stream_transpose(nbr, own, W, lam)
    for q in (0, 63, 64, 1234, 2000, c.n - 1):
        row, mag = transposed_row(c, K, m, lam, q)
        np.testing.assert_allclose(row, ref[q], rtol=0, atol=1e-12 * (1.0 + mag.max()))


def test_collision_jacobian_is_linear_in_direction():
    """C is affine in f along any direction that keeps rho and u (a
    non-equilibrium part): there the Jacobian is (1 - 1/tau) I."""
    tau = 0.6
    ux, uy = tgv_initial_velocity(np.array([0.3]), np.array([1.1]), 2 * np.pi, 0.05)
    f = oracle.equilibrium(np.ones(1), ux, uy)[0]
    J = collision_jacobian(f, tau)
    ex, ey, _, _ = oracle.tables()
    # a direction with zero mass and momentum: d = e_1 + e_3 - e_2 - e_4
    d = np.zeros(9)
    d[[1, 3]] = 1.0
    d[[2, 4]] = -1.0
    assert abs(d.sum()) == 0 and abs(d @ ex) == 0 and abs(d @ ey) == 0
    np.testing.assert_allclose(J @ d, (1.0 - 1.0 / tau) * d, atol=1e-8)
    # mass and momentum are conserved by the collision: their rows of J^T
    np.testing.assert_allclose(np.ones(9) @ J, np.ones(9), atol=1e-8)
    np.testing.assert_allclose(ex @ J, ex, atol=1e-8)
    np.testing.assert_allclose(ey @ J, ey, atol=1e-8)
