"""The adjoint workload at full size: Taylor-Green at 262,144 nodes (K = 30,
degree 4, paper stencils, tau 0.6), 500 steps checkpointed every 50, gradient
of J = 1/2 sum |u(T) - u*|^2 with respect to the initial velocity field and
tau, through the checkpointed rollout. The target u* is the analytic decay of
a vortex 10 % weaker than the initial one, so the misfit is not a near
cancellation of the two fields.

FP64: the adjoint gradient against central differences of the FP64 forward
along a smooth direction of u0 and in tau, and against the FP64 oracle's
complex-step derivatives on the same cloud. FP32 (the benchmarked path):
against the FP64 gradient, within the FP32 rounding bound carried through the
misfit, and the rollout that stores every state against the checkpointed one."""
import math

import numpy as np
import pytest

import oracle
from gpu_common import rel_l2, say, tol_fp32
from synth import jittered_lattice, tgv_initial_velocity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_SIDE, K, M_DEG, TAU, U0, STEPS, SEG = 512, 30, 4, 0.6, 0.01, 500, 50


def _plan(c, precision):
    from paper_2306_01525_amd import Params, Plan
    p = Params(dx=c.h, K=K, degree=M_DEG, tau=TAU, stencil_mode=0, precision=precision,
               with_adjoint=1)
    return Plan.build(c.x, c.y, c.period, p)


def _loss(plan, u0x, u0y, tx, ty):
    from paper_2306_01525_amd.autograd import Rollout
    ro = Rollout(plan, STEPS, SEG)
    ro.forward(u0x, u0y)
    return float(ro.loss(tx, ty).item())


def _grad(plan, u0x, u0y, tx, ty, store_all=False):
    from paper_2306_01525_amd.autograd import Rollout
    ro = Rollout(plan, STEPS, SEG, store_all)
    ro.forward(u0x, u0y)
    J = float(ro.loss(tx, ty).item())
    gx, gy, gt = ro.backward()
    return J, gx.cpu().numpy(), gy.cpu().numpy(), float(gt.item())


def test_fullsize_gradient_fd_and_fp32():
    from paper_2306_01525_amd import targets
    c = jittered_lattice(N_SIDE, seed=2)
    L = c.period[0]
    u0x, u0y = tgv_initial_velocity(c.x, c.y, L, U0)
    tx, ty = targets.tgv_velocity(c.x, c.y, L, 0.9 * U0, TAU, c.h, STEPS)
    tx_t = torch.tensor(tx, device="cuda")
    ty_t = torch.tensor(ty, device="cuda")

    say("FP64 rollout + adjoint, n =", c.n)
    p64 = _plan(c, 1)
    J64, gx64, gy64, gt64 = _grad(p64, u0x, u0y, tx_t, ty_t)
    # smooth direction (slowly decaying modes carry the signal to time T)
    k = 2 * math.pi / L
    dx = np.cos(k * c.x) * np.sin(2 * k * c.y)
    dy = np.sin(3 * k * c.x + 0.4)
    D = float(gx64 @ dx + gy64 @ dy)
    eps = 1e-6
    Jp = _loss(p64, u0x + eps * dx, u0y + eps * dy, tx_t, ty_t)
    Jm = _loss(p64, u0x - eps * dx, u0y - eps * dy, tx_t, ty_t)
    fd = (Jp - Jm) / (2 * eps)
    et = 1e-6
    p64.set_tau(TAU + et)
    Jtp = _loss(p64, u0x, u0y, tx_t, ty_t)
    p64.set_tau(TAU - et)
    Jtm = _loss(p64, u0x, u0y, tx_t, ty_t)
    p64.close()
    fdt = (Jtp - Jtm) / (2 * et)
    say("J %.6e; direction: adjoint %.9e vs FD %.9e; tau: adjoint %.9e vs FD %.9e"
        % (J64, D, fd, gt64, fdt))
    # central differences: O(eps^2) truncation, rounding of J ~ 1e-16 J / eps
    assert abs(D - fd) <= 1e-6 * abs(D) + 1e-9 * J64
    assert abs(gt64 - fdt) <= 1e-6 * abs(gt64) + 1e-9 * J64

    # the FP64 oracle on the same cloud: its loss and its complex-step
    # derivatives J(u0 + i h d) and J(tau + i h) (exact to rounding, no
    # cancellation) along the same direction and in tau
    say("oracle: build and complex-step rollouts on the whole cloud")
    nbr, own, W = oracle.build_plan(c, c.h, K, M_DEG, 0, search="tree")
    hcs = 1e-30
    Jo, Jd = oracle.loss_cs(nbr, own, W, TAU, STEPS, 1.0, u0x, u0y, tx, ty,
                            u0x_im=hcs * dx, u0y_im=hcs * dy)
    _, Jt = oracle.loss_cs(nbr, own, W, TAU, STEPS, 1.0, u0x, u0y, tx, ty, tau_im=hcs)
    del nbr, own, W
    Dcs, Tcs = Jd / hcs, Jt / hcs
    say("oracle: J %.12e vs GPU %.12e; direction %.12e vs GPU %.12e; tau %.12e vs GPU %.12e"
        % (Jo, J64, Dcs, D, Tcs, gt64))
    # the gradient carries rounding relative to its own size; the direction
    # is nearly orthogonal to it, so the directional derivative is compared
    # on the scale |grad| |d| (measured 7.7e-13 relative in J, 1.7e-12 in tau)
    scale = math.sqrt(float(gx64 @ gx64 + gy64 @ gy64) * float(dx @ dx + dy @ dy))
    say("oracle: |D - D_cs| / (|grad| |d|) %.2e" % (abs(D - Dcs) / scale))
    assert abs(J64 - Jo) <= 4e-12 * Jo
    assert abs(D - Dcs) <= 1e-10 * scale
    assert abs(gt64 - Tcs) <= 1e-11 * abs(Tcs)

    say("FP32 rollout + adjoint")
    p32 = _plan(c, 0)
    J32, gx32, gy32, gt32 = _grad(p32, u0x, u0y, tx_t, ty_t)
    # every state stored by the forward (501 states, 4.7 GB) instead of the
    # checkpoints: the same reversed steps on the same recorded states
    Js, gxs, gys, gts = _grad(p32, u0x, u0y, tx_t, ty_t, store_all=True)
    p32.close()
    ds = max(np.abs(gxs - gx32).max(), np.abs(gys - gy32).max()) / np.abs(
        np.concatenate([gx32, gy32])).max()
    say("FP32 stored vs checkpointed: J diff %.2e, grad u0 max diff %.2e, dtau diff %.2e"
        % (abs(Js - J32), ds, abs(gts - gt32)))
    assert abs(Js - J32) <= 1e-14 * J32
    assert ds <= 1e-6 and abs(gts - gt32) <= 1e-6 * abs(gt32)
    # the FP32 state is within tol_fp32(T) of the FP64 one relative to |u|; the
    # misfit e = u(T) - u* is 10x smaller than u, and the reverse sweep adds
    # its own rounding of the same order
    ratio = math.sqrt((tx @ tx + ty @ ty) / 0.81) / math.sqrt(2.0 * J64)
    bound = 2.0 * tol_fp32(STEPS) * (ratio + 1.0)
    eg = rel_l2(np.concatenate([gx32, gy32]), np.concatenate([gx64, gy64]))
    et32 = abs(gt32 - gt64) / abs(gt64)
    say("FP32: J %.6e vs %.6e, grad u0 rel %.2e, dtau rel %.2e (bound %.2e)"
        % (J32, J64, eg, et32, bound))
    assert abs(J32 - J64) <= bound * J64
    assert eg < bound
    assert et32 < bound
