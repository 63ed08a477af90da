"""Pins of the oracle's discrete adjoint: dot-product identity of the
transposed streaming, complex-step derivatives of the same forward code, and
central finite differences (CPU, FP64)."""
import numpy as np
import pytest

import oracle
from synth import jittered_lattice, random_field, tgv_initial_velocity


@pytest.fixture(scope="module")
def small_setup():
    c = jittered_lattice(10, seed=21, length=10.0)
    nbr, own, W = oracle.build_plan(c, 1.0, 20, 3, mode=0)
    u0x, u0y = tgv_initial_velocity(c.x, c.y, 10.0, 0.02)
    tx, ty = tgv_initial_velocity(c.x, c.y, 10.0, 0.015)
    return c, nbr, own, W, u0x, u0y, tx, ty


def test_stream_transpose_dot_product(small_setup):
    c, nbr, own, W, *_ = small_setup
    v = random_field((c.n, 9), 1)
    lam = random_field((c.n, 9), 2)
    lhs = np.sum(oracle.stream(nbr, own, W, v) * lam)
    rhs = np.sum(v * oracle.stream_transpose(nbr, own, W, lam))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_adjoint_matches_complex_step(small_setup):
    c, nbr, own, W, u0x, u0y, tx, ty = small_setup
    tau, steps = 0.7, 12
    J, gx, gy, gt = oracle.adjoint(nbr, own, W, tau, steps, 1.0, u0x, u0y, tx, ty)
    eps = 1e-30
    for seed in (3, 4, 5):
        vx = random_field(c.n, seed)
        vy = random_field(c.n, seed + 10)
        jr, ji = oracle.loss_cs(nbr, own, W, tau, steps, 1.0, u0x, u0y, tx, ty,
                                u0x_im=eps * vx, u0y_im=eps * vy)
        assert abs(jr - J) < 1e-14 * abs(J)
        dd = ji / eps
        assert abs(dd - (gx @ vx + gy @ vy)) < 1e-10 * abs(dd), (dd, gx @ vx + gy @ vy)
    _, ji = oracle.loss_cs(nbr, own, W, tau, steps, 1.0, u0x, u0y, tx, ty, tau_im=eps)
    assert abs(ji / eps - gt) < 1e-10 * abs(gt)


def test_complex_step_matches_central_differences(small_setup):
    c, nbr, own, W, u0x, u0y, tx, ty = small_setup
    tau, steps = 0.7, 12
    _, ji = oracle.loss_cs(nbr, own, W, tau, steps, 1.0, u0x, u0y, tx, ty, tau_im=1e-30)
    h = 1e-6
    jp, _ = oracle.loss_cs(nbr, own, W, tau + h, steps, 1.0, u0x, u0y, tx, ty)
    jm, _ = oracle.loss_cs(nbr, own, W, tau - h, steps, 1.0, u0x, u0y, tx, ty)
    fd = (jp - jm) / (2 * h)
    assert abs(fd - ji / 1e-30) < 1e-6 * abs(fd)
