"""Differentiable MLBM rollout: checkpointed forward, hand-written adjoint.

Loss: J = 1/2 sum_i |u_i(f^T) - u*_i|^2 after T steps from f^0 = feq(rho0, u0).
Gradients with respect to the initial velocity u0 and the relaxation time tau.

Forward keeps the pre-collision state f at the start of every segment of C
steps. Backward walks the segments in reverse: it recomputes the segment from
its checkpoint while recording every pre-collision state (mlbm_step_record),
then applies C reversed steps (mlbm_step_adjoint). Memory: (T/C + 1) + C states
instead of T. With store_all the forward records all T + 1 states instead
(T + 1 states of 36 bytes a node in FP32: 4.7 GB for 500 steps of 262,144
nodes) and the backward runs the reversed steps alone, without recomputing.
Every numeric operation runs in the HIP library.
"""
from __future__ import annotations

import torch

from .mlbm import Plan


class Rollout:
    """One checkpointed rollout on a plan. The relaxation time in force when
    forward() runs is recorded, and backward() recomputes and differentiates
    at that value whatever the plan holds by then (the plan's value is put
    back afterwards), so several rollouts on one plan may be differentiated in
    any order. With store_all every pre-collision state of the forward is
    kept (the segment length is then unused) and nothing is recomputed."""

    def __init__(self, plan: Plan, steps: int, segment: int = 50, store_all: bool = False):
        if steps < 1 or segment < 1:
            raise ValueError("steps and segment must be positive")
        self.plan = plan
        self.tau = None
        self.T = int(steps)
        self.C = int(segment)
        self.nseg = (self.T + self.C - 1) // self.C
        self.store = bool(store_all)
        self.rec = None
        self.ckpt = None
        self.J = None

    def _seg_len(self, c):
        return min(self.C, self.T - c * self.C)

    def forward(self, u0x, u0y, stream=None):
        """Run T steps; returns f^T (pre-collision) and keeps checkpoints."""
        plan = self.plan
        self.u0 = (u0x, u0y)
        self.tau = float(plan.params.tau)
        if self.store:
            # f^0 .. f^T; f^n is the pre-collision state the reversed step n uses
            rec = torch.empty((self.T + 1, 9, plan.n), dtype=plan.state_dtype,
                              device=plan.device)
            plan.init_f(u0x, u0y, f=rec[0], stream=stream)
            g = plan.collide(rec[0], stream=stream)
            plan.step_record(g, plan.new_state(), self.T, rec[1:], stream=stream)
            self.rec = rec
            self.ckpt = [rec[self.T]]
            return rec[self.T]
        ck = [plan.init_f(u0x, u0y, stream=stream)]
        g = plan.collide(ck[0], stream=stream)
        other = plan.new_state()
        for c in range(self.nseg):
            L = self._seg_len(c)
            if L > 1:
                res = plan.step(g, other, L - 1, stream=stream)
                if res is other:
                    g, other = other, g
            f_end = plan.new_state()
            res = plan.step_record(g, other, 1, f_end, stream=stream)
            g, other = other, g
            ck.append(f_end)
        self.ckpt = ck
        return ck[-1]

    def loss(self, ux_t, uy_t, stream=None):
        self.target = (ux_t, uy_t)
        lam, J = self.plan.loss_seed(self.ckpt[-1], ux_t, uy_t, stream=stream)
        self.lam_T = lam
        self.J = J
        return J

    def backward(self, stream=None):
        """Returns (dJ/du0x, dJ/du0y, dJ/dtau) as device tensors."""
        plan = self.plan
        held = float(plan.params.tau)
        if held != self.tau:
            plan.set_tau(self.tau)
        try:
            return self._backward(stream)
        finally:
            if held != self.tau:
                plan.set_tau(held)

    def _backward(self, stream):
        plan = self.plan
        lam = self.lam_T
        lam_other = plan.new_state()
        dtau = torch.zeros(1, dtype=torch.float64, device=plan.device)
        if self.store:
            for t in reversed(range(self.T)):
                plan.step_adjoint(self.rec[t], lam, lam_other, dtau, stream=stream)
                lam, lam_other = lam_other, lam
            gx, gy = plan.init_adjoint(self.u0[0], self.u0[1], lam, stream=stream)
            return gx, gy, dtau
        rec = torch.empty((self.C, 9, plan.n), dtype=plan.state_dtype, device=plan.device)
        g = plan.new_state()
        other = plan.new_state()
        for c in reversed(range(self.nseg)):
            L = self._seg_len(c)
            rec[0].copy_(self.ckpt[c])
            if L > 1:
                plan.collide(self.ckpt[c], g, stream=stream)
                plan.step_record(g, other, L - 1, rec[1:L], stream=stream)
            for t in reversed(range(L)):
                plan.step_adjoint(rec[t], lam, lam_other, dtau, stream=stream)
                lam, lam_other = lam_other, lam
        gx, gy = plan.init_adjoint(self.u0[0], self.u0[1], lam, stream=stream)
        return gx, gy, dtau


class MLBMRollout(torch.autograd.Function):
    """J = MLBMRollout.apply(u0x, u0y, tau, plan, steps, ux_t, uy_t, segment, store_all).

    u0x, u0y: float64 CUDA tensors [n] (user order); tau: 0-d float64 tensor.
    Returns J (0-d float64). Backward gives dJ/du0x, dJ/du0y, dJ/dtau."""

    @staticmethod
    def forward(ctx, u0x, u0y, tau, plan, steps, ux_t, uy_t, segment=50, store_all=False):
        plan.set_tau(float(tau))
        ro = Rollout(plan, steps, segment, store_all)
        ro.forward(u0x.detach(), u0y.detach())
        J = ro.loss(ux_t, uy_t)
        ctx.ro = ro
        return J.reshape(())

    @staticmethod
    def backward(ctx, gJ):
        gx, gy, gt = ctx.ro.backward()
        ctx.ro = None
        return gJ * gx, gJ * gy, (gJ * gt).reshape(()), None, None, None, None, None, None


def rollout_loss(plan, u0x, u0y, tau, steps, ux_t, uy_t, segment=50, store_all=False):
    return MLBMRollout.apply(u0x, u0y, tau, plan, steps, ux_t, uy_t, segment, store_all)
