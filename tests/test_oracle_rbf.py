"""Pins of the oracle's RBF interpolation and local solves (CPU).

* LU with partial pivoting against systems with a known solution.
* The interpolant built from the collocation equations (coefficients gamma,
  pi of eq. rbf_interp_set_augmented) evaluated directly at p equals the
  shape-vector form w_L(p) . f_L (eq. shape_vector).
* Exact reproduction of every monomial in the augmentation set, partition of
  unity, unit vector at a stencil node, invariance to shift/scale/rotation.
* Interpolation-only convergence on the paper's smooth test function
  (Sec. 4, Fig. interp_test): slopes between 2 and 5.
"""
import math

import numpy as np
import pytest

import oracle
from synth import jittered_lattice


def _stencil(seed, K):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-1, 1, (4 * K, 2)) * 0.03
    pts[0] = 0.0
    d = np.hypot(pts[:, 0], pts[:, 1])
    order = np.argsort(d)[:K]
    return pts[order, 0].copy(), pts[order, 1].copy()


def test_paper_poly_set_sizes(golden):
    ps = golden["poly_sets"]
    assert oracle.poly_count(2) == ps["size_P2"]
    assert oracle.poly_count(4) == ps["size_P4"]
    assert oracle.poly_count(3) == 10


def test_lu_solves_known_systems():
    rng = np.random.default_rng(3)
    for nn in (5, 18, 45):
        A = rng.standard_normal((nn, nn))
        x = rng.standard_normal(nn)
        b = A @ x
        np.testing.assert_allclose(oracle.lu_solve(A, b), x, rtol=0, atol=1e-10 * np.abs(x).max())
    # a matrix that needs pivoting (zero leading entry) with an integer solution
    A = np.array([[0.0, 2, 1], [1, 1, 1], [2, 1, 0]])
    x = np.array([1.0, -2.0, 3.0])
    np.testing.assert_allclose(oracle.lu_solve(A, A @ x), x, atol=1e-14)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.lu_solve(np.ones((4, 4)), np.ones(4))


@pytest.mark.parametrize("K,m", [(12, 2), (20, 3), (30, 4), (25, 2)])
def test_shape_vector_equals_coefficient_interpolant(K, m):
    rx, ry = _stencil(K, K)
    px, py = 0.011, -0.007
    w = oracle.shape_vector(rx, ry, px, py, m)
    Phi, phi = oracle.local_system(rx, ry, px, py, m)
    rng = np.random.default_rng(K)
    fL = rng.standard_normal(K)
    # coefficients of eq. rbf_interp_set_augmented, then F(p) = coef . phi(p)
    coef = oracle.lu_solve(Phi, np.concatenate([fL, np.zeros(Phi.shape[0] - K)]))
    assert abs(coef @ phi - w @ fL) < 1e-10 * np.abs(fL).max()
    # the collocation matrix is symmetric (which is what makes the transposition
    # in eq. shape_vector legitimate)
    np.testing.assert_allclose(Phi, Phi.T, atol=0)


@pytest.mark.parametrize("K,m", [(12, 2), (20, 3), (30, 4)])
def test_monomial_reproduction_and_unity(K, m, golden):
    rx, ry = _stencil(100 + K, K)
    px, py = -0.004, 0.009
    w = oracle.shape_vector(rx, ry, px, py, m)
    exps = golden["poly_sets"]["exponents_P4"][: oracle.poly_count(m)]
    for a, b in exps:
        exact = px ** a * py ** b
        got = w @ (rx ** a * ry ** b)
        assert abs(got - exact) < 1e-10 * max(1.0, 0.03 ** (a + b)), (a, b, got, exact)
    assert abs(w.sum() - 1) < 1e-12


@pytest.mark.parametrize("K,m", [(12, 2), (30, 4)])
def test_unit_vector_at_stencil_node(K, m):
    rx, ry = _stencil(200 + K, K)
    for j in (0, 3, K - 1):
        w = oracle.shape_vector(rx, ry, rx[j], ry[j], m)
        e = np.zeros(K)
        e[j] = 1
        np.testing.assert_allclose(w, e, atol=1e-10)


def test_shape_vector_invariances():
    """r^3 with complete polynomials: invariant to shift, scale and rotation."""
    K, m = 20, 3
    rx, ry = _stencil(77, K)
    px, py = 0.006, 0.004
    w0 = oracle.shape_vector(rx, ry, px, py, m)
    th = 0.7
    c, s = math.cos(th), math.sin(th)
    w_rot = oracle.shape_vector(c * rx - s * ry, s * rx + c * ry, c * px - s * py,
                                s * px + c * py, m)
    w_scale = oracle.shape_vector(37 * rx, 37 * ry, 37 * px, 37 * py, m)
    # shift: move the centre to stencil member 3 (local coordinates relative to it)
    w_shift = oracle.shape_vector(rx - rx[3], ry - ry[3], px - rx[3], py - ry[3], m)
    for w in (w_rot, w_scale, w_shift):
        np.testing.assert_allclose(w, w0, atol=1e-10)


def test_interpolation_only_convergence():
    """f = 0.01 sin 2 pi x cos 2 pi y on the unit periodic square, dx = 1/10,
    departure points x - e_k dx, the paper's stencils (closest-node owner):
    the L2 error falls with a slope between 2 and 5 (Sec. 4, Fig. interp_test)."""
    ex, ey, _, _ = oracle.tables()
    for m, K in ((2, 25), (4, 25)):
        errs, hs = [], []
        for n in (20, 40, 80):
            c = jittered_lattice(n, length=1.0, seed=11 + n)
            nbr, own, W = oracle.build_plan(c, 0.1, K, m, mode=0)
            F = 0.01 * np.sin(2 * np.pi * c.x) * np.cos(2 * np.pi * c.y)
            num = den = 0.0
            for k in range(1, 9):
                val = np.einsum("ij,ij->i", W[:, k, :], F[nbr[own[:, k]]])
                px, py = c.x - ex[k] * 0.1, c.y - ey[k] * 0.1
                tr = 0.01 * np.sin(2 * np.pi * px) * np.cos(2 * np.pi * py)
                num += np.sum((val - tr) ** 2)
                den += np.sum(tr ** 2)
            errs.append(math.sqrt(num / den))
            hs.append(1.0 / n)
        slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
        assert 2.0 <= slope <= 5.5, (m, errs, slope)


def test_d0_weights_are_identity():
    """The population at rest departs from the node itself: its shape vector is
    the unit vector on the stencil centre."""
    c = jittered_lattice(16, seed=2, length=1.0)
    nbr, own, W = oracle.build_plan(c, 1 / 16, 12, 2, mode=0)
    np.testing.assert_array_equal(own[:, 0], np.arange(c.n))
    e = np.zeros(12)
    e[0] = 1
    np.testing.assert_allclose(W[:, 0, :], np.broadcast_to(e, (c.n, 12)), atol=1e-10)
