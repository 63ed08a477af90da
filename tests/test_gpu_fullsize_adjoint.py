"""The reversed step at full size (262,144 nodes, K = 30, degree 4, paper
stencil rule, FP32, the launch the benchmark times): sampled nodes against the
oracle computed one node at a time, lam^n(q) = C'(f^n(q))^T (S^T lam^{n+1})(q)
with the transposed row and the BGK Jacobian of adjoint_local."""
import numpy as np
import pytest

import oracle
from adjoint_local import collision_jacobian, transposed_row
from gpu_common import say
from synth import jittered_lattice, random_field, tgv_initial_velocity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_SIDE, K, M_DEG, TAU, U0 = 512, 30, 4, 0.6, 0.01


def test_fullsize_reversed_step_sampled():
    from paper_2306_01525_amd import MLBM_FP32_DEV, Params, Plan
    c = jittered_lattice(N_SIDE, seed=2)
    ux, uy = tgv_initial_velocity(c.x, c.y, c.period[0], U0)
    n = c.n
    lam_u = random_field((n, 9), seed=77)                  # lam^{n+1}, user order
    say("building the FP32 plan with adjoint tables at full size, n =", n)
    p = Params(dx=c.h, K=K, degree=M_DEG, tau=TAU, stencil_mode=0, precision=MLBM_FP32_DEV,
               with_adjoint=1)
    plan = Plan.build(c.x, c.y, c.period, p)
    perm = plan.export("perm")                              # internal -> user
    assert np.array_equal(np.sort(perm), np.arange(n))
    fn = plan.init_f(ux, uy)                                # f^n = feq(1, u0)
    lam_i = torch.tensor(lam_u[perm].T.astype(np.float32).copy(), device=fn.device)
    lam_o = plan.new_state()
    dtau = torch.zeros(1, dtype=torch.float64, device=fn.device)
    plan.step_adjoint(fn, lam_i, lam_o, dtau)
    torch.cuda.synchronize()
    got_i = lam_o.cpu().numpy().astype(np.float64)          # [9][n] internal
    got = np.empty((n, 9))
    got[perm] = got_i.T
    plan.close()
    # f^n is an equilibrium, so the tau partials vanish
    assert abs(float(dtau.item())) < 1e-6

    rng = np.random.default_rng(321)
    sample = np.concatenate([rng.choice(n, 40, replace=False), [0, n - 1, N_SIDE - 1]])
    worst = 0.0
    for q in sample:
        row, mag = transposed_row(c, K, M_DEG, lam_u, int(q))
        f = oracle.equilibrium(np.ones(1), ux[q:q + 1], uy[q:q + 1])[0]
        J = collision_jacobian(f, TAU)
        want = J.T @ row
        # FP32 sums of about K terms and FP32 weights: bound by the magnitude
        bound = 1e-5 * (np.abs(J).T @ mag) + 1e-6
        err = np.abs(got[q] - want)
        worst = max(worst, float((err / bound).max()))
        assert (err <= bound).all(), (q, got[q], want, bound)
    say("sampled %d nodes: worst |lam_gpu - lam_oracle| / bound = %.3f" % (sample.size, worst))
