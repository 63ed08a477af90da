"""The paper's convergence studies on the GPU: interpolation alone (Sec. 4,
Fig. interp_test) and the Taylor-Green error map against the standard LBM
(Sec. 3, Figs. h_dx_explained and tgv_conv_P), on a reduced grid. One point
of the map and the interpolation operator are checked against the oracle;
the rest against what the paper reports."""
import math

import numpy as np
import pytest

import oracle
from gpu_common import rel_l2, say
from synth import jittered_lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_interpolation_operator_matches_oracle():
    from paper_2306_01525_amd import Params, Plan
    ex, ey, _, _ = oracle.tables()
    for mode in (0, 1):
        c = jittered_lattice(40, length=1.0, seed=51)
        nbr, own, W = oracle.build_plan(c, 0.1, 25, 4, mode=mode)
        f = 0.01 * np.sin(2 * np.pi * c.x) * np.cos(2 * np.pi * c.y)
        want = np.stack([np.einsum("ij,ij->i", W[:, k, :], f[nbr[own[:, k]]]) for k in range(1, 9)])
        p = Params(dx=0.1, K=25, degree=4, tau=0.8, stencil_mode=mode, precision=1)
        plan = Plan.build(c.x, c.y, c.period, p)
        got = plan.interpolate(f).cpu().numpy()
        plan.close()
        err = float(np.abs(got - want).max())
        say("mode %d: max |GPU - oracle| of the interpolated field %.2e" % (mode, err))
        assert err < 1e-13


def test_interpolation_convergence_slopes():
    """Slopes of the interpolation error between 2 and 5 (Sec. 4); P4 above P2."""
    from paper_2306_01525_amd.studies import interpolation_convergence
    rec, slopes = interpolation_convergence(n_sides=(20, 40, 80, 160))
    say("interpolation L2:", ["P%d h=1/%d %.2e" % (r["degree"], r["n_side"], r["l2"]) for r in rec])
    say("slopes:", slopes)
    assert 2.0 <= slopes[2] <= 5.5
    assert 2.0 <= slopes[4] <= 5.5
    assert slopes[4] > slopes[2] + 1.0


def test_tgv_error_map_point_matches_oracle():
    """dx_ML = 1/10, h = 1/20, P4, paper stencils: the 29 steps to t_end on the
    GPU (FP64) against the oracle on the same cloud and initial state."""
    from paper_2306_01525_amd import studies
    from paper_2306_01525_amd import Params, Plan
    dx, h, m, K = 0.1, 0.05, 4, 25
    c = jittered_lattice(20, length=1.0, seed=5 + 20)
    steps = studies._steps(dx)
    ux, uy = studies._tgv_lattice_units(c.x, c.y, dx)
    plan = Plan.build(c.x, c.y, c.period, Params(dx=dx, K=K, degree=m, tau=studies.TAU,
                                                 stencil_mode=0, precision=1))
    g = plan.step(plan.init(ux, uy), plan.new_state(), steps)
    _, u_g, v_g = (a.cpu().numpy() for a in plan.moments(g))
    plan.close()
    nbr, own, W = oracle.build_plan(c, dx, K, m, mode=0)
    f = oracle.run(oracle.equilibrium(np.ones(c.n), ux, uy), nbr, own, W, studies.TAU, steps)
    _, u_o, v_o = oracle.moments(f)
    d = rel_l2(np.stack([u_g, v_g]), np.stack([u_o, v_o]))
    say("error-map point after %d steps: GPU vs oracle %.2e" % (steps, d))
    assert d < 1e-11


def test_tgv_error_map_reproduces_the_papers_observations():
    """Reduced map (dx_ML = 1/10, 1/40; h = 1/10 .. 1/80) plus one dx_ML =
    1/160 column, P2 and P4, and the standard LBM:
    * the LBM converges at second order;
    * refined in h, the MLBM error stops at the LBM error of dx = dx_ML;
    * P4 is more accurate than P2 on coarse clouds;
    * with dx_ML = 1/160 and P4 the MLBM is more accurate than the LBM on the
      same number of nodes (h = 1/40 and 1/80)."""
    from paper_2306_01525_amd.studies import lbm_errors, tgv_error_map
    lbm = {round(1 / r["dx"]): r["l2_u"] for r in lbm_errors(dxs=(1 / 10, 1 / 20, 1 / 40, 1 / 80))}
    say("LBM L2:", lbm)
    orders = [math.log2(lbm[a] / lbm[2 * a]) for a in (10, 20, 40)]
    assert all(1.85 < o < 2.15 for o in orders), orders
    res = tgv_error_map(dx_ml=(1 / 10, 1 / 40), hs=(1 / 10, 1 / 20, 1 / 40, 1 / 80))
    e = {(round(1 / r["dx_ml"]), round(1 / r["h"]), r["degree"]): r["l2_u"] for r in res}
    say("MLBM L2:", {k: "%.2e" % v for k, v in sorted(e.items())})
    for dxi in (10, 40):
        for m in (2, 4):
            assert abs(e[(dxi, 80, m)] / lbm[dxi] - 1.0) < 0.05
    assert e[(40, 20, 4)] < e[(40, 20, 2)]
    assert e[(40, 10, 2)] > e[(40, 20, 2)] > e[(40, 40, 2)]
    fine = tgv_error_map(dx_ml=(1 / 160,), hs=(1 / 40, 1 / 80), degrees=(4,))
    for r in fine:
        n = round(1 / r["h"])
        say("dx_ML 1/160, h 1/%d, P4: MLBM %.2e vs LBM on %d^2 nodes %.2e"
            % (n, r["l2_u"], n, lbm[n]))
        assert r["l2_u"] < 0.5 * lbm[n]
