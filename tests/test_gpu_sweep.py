"""A seeded sweep over the parameter space: random stencil sizes, degrees,
stencil rules, relaxation times, jitter amplitudes (including none, with exact
ties) and cloud sizes, each built and stepped on the GPU in both precisions
and compared with the oracle after 1 and 5 steps."""
import numpy as np
import pytest

from gpu_common import TOL_FP64, oracle_run, rel_l2, say, tgv_case, tol_fp32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _draw(count=16, seed=2024):
    r = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < count:
        m = int(r.integers(2, 5))
        M = (m + 1) * (m + 2) // 2
        K = int(r.integers(M + 6, min(48, 64 - M) + 1))
        n_side = int(r.integers(max(8, int(np.ceil(np.sqrt(K))) + 2), 46))
        jitter = float(r.choice([0.0, 0.1, 0.3, 0.4]))
        out.append(dict(n_side=n_side, K=K, m=m, mode=int(r.integers(0, 2)),
                        tau=float(r.uniform(0.55, 1.2)), jitter=jitter,
                        seed=int(r.integers(1, 10_000))))
    return out


CASES = _draw()


@pytest.mark.parametrize("case", CASES, ids=["n%d-K%d-m%d-mode%d-j%.1f" % (
    c["n_side"], c["K"], c["m"], c["mode"], c["jitter"]) for c in CASES])
def test_sweep_matches_oracle(case):
    from paper_2306_01525_amd import Params, Plan
    c, ux, uy = tgv_case(case["n_side"], case["K"], case["m"], case["mode"], seed=case["seed"],
                         jitter=case["jitter"])
    K, m, mode, tau = case["K"], case["m"], case["mode"], case["tau"]
    _, ref = oracle_run(c, c.h, K, m, mode, tau, ux, uy, [1, 5])
    for prec, tol in ((1, lambda s: TOL_FP64), (0, tol_fp32)):
        p = Params(dx=c.h, K=K, degree=m, tau=tau, stencil_mode=mode, precision=prec)
        plan = Plan.build(c.x, c.y, c.period, p)
        g, other, done = plan.init(ux, uy), plan.new_state(), 0
        for s in (1, 5):
            res = plan.step(g, other, s - done)
            if res is other:
                g, other = other, g
            done = s
            _, u, v = (a.cpu().numpy() for a in plan.moments(g))
            e = rel_l2(np.stack([u, v]), np.stack(ref[s][1:]))
            say("%s %s step %d: rel L2 %.2e (tol %.1e)"
                % (case, "fp64" if prec else "fp32", s, e, tol(s)))
            assert e < tol(s)
        assert plan.device_error() == 0
        plan.close()
