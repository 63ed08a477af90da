"""GPU time stepping against the oracle: on imported oracle weights (isolates
the step kernel) and end to end (GPU build + GPU steps)."""
import numpy as np
import pytest

import oracle
from gpu_common import (EPS32, TOL_FP64, annulus_case, first_step_bounds,
                        first_step_rounding_bounds, oracle_run, rel_l2, say, tgv_case,
                        tol_fp32, weight_bounds)
from synth import tgv_initial_velocity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _params(dx, K, m, mode, precision, tau, **kw):
    from paper_2306_01525_amd import Params
    return Params(dx=dx, K=K, degree=m, tau=tau, stencil_mode=mode, precision=precision, **kw)


def _gpu_run(plan, ux, uy, steps_list, rho=None):
    g = plan.init(ux, uy, rho=rho)
    other = plan.new_state()
    out = {}
    done = 0
    for s in sorted(steps_list):
        res = plan.step(g, other, s - done)
        if res is other:
            g, other = other, g
        done = s
        rho_g, ux_g, uy_g = plan.moments(g)
        out[s] = (rho_g.cpu().numpy(), ux_g.cpu().numpy(), uy_g.cpu().numpy())
    return out


def _compare(ref, got, tol, label, node_factor=3.0):
    for s in sorted(ref):
        r_o, u_o, v_o = ref[s]
        r_g, u_g, v_g = got[s]
        eu = rel_l2(np.stack([u_g, v_g]), np.stack([u_o, v_o]))
        en = float(np.hypot(u_g - u_o, v_g - v_o).max() / np.hypot(u_o, v_o).max())
        er = float(np.abs(r_g - r_o).max())
        say("  %s step %d: rel L2 velocity %.3e, max node %.3e, max |drho| %.3e (tol %.1e)"
            % (label, s, eu, en, er, tol(s)))
        assert eu < tol(s), (label, s, eu)
        assert en < node_factor * tol(s), (label, s, en)
        assert er < tol(s), (label, s, er)


STEP_CASES = [
    ("c1-own", 40, 12, 2, 1, 0.8),
    ("paper-K25-m2", 40, 25, 2, 0, 0.8),
    ("paper-K30-m4-tau0.6", 33, 30, 4, 0, 0.6),
    ("own-K20-m3", 29, 20, 3, 1, 0.7),
]


@pytest.mark.parametrize("label,nside,K,m,mode,tau", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_step_on_imported_weights(label, nside, K, m, mode, tau):
    """Oracle stencils and weights imported into the GPU plan: the step kernel
    alone is compared with the oracle after 1, 10 and 200 steps."""
    from paper_2306_01525_amd import Plan
    c, ux, uy = tgv_case(nside, K, m, mode)
    steps = [1, 10, 200]
    (nbr, own, W), ref = oracle_run(c, c.h, K, m, mode, tau, ux, uy, steps)
    for prec, tol in ((1, lambda s: TOL_FP64), (0, tol_fp32)):
        say("case", label, "precision", prec, "n", c.n)
        plan = Plan.from_arrays(c.x, c.y, nbr, own, W, _params(c.h, K, m, mode, prec, tau))
        got = _gpu_run(plan, ux, uy, steps)
        _compare(ref, got, tol, "%s/%s" % (label, "fp64" if prec else "fp32"))
        plan.close()


E2E_CASES = [
    ("c1-own", 40, 12, 2, 1, 0.8, 200),
    ("paper-K30-m4", 48, 30, 4, 0, 0.6, 100),
    ("ragged-rect-paper-K20-m3", None, 20, 3, 0, 0.7, 50),
    # the smallest cloud the boundary accepts, n = K: every stencil is the
    # whole cloud, one partial tile
    ("n-equals-K-paper", 4, 16, 2, 0, 0.8, 20),
    ("n-equals-K-own", 4, 16, 2, 1, 0.8, 20),
]


@pytest.mark.parametrize("label,nside,K,m,mode,tau,steps", E2E_CASES, ids=[c[0] for c in E2E_CASES])
def test_end_to_end_matches_oracle(label, nside, K, m, mode, tau, steps):
    from paper_2306_01525_amd import Plan
    if nside is None:
        c, ux, uy = tgv_case(31, K, m, mode, ny=23, length_y=2 * np.pi * 23 / 31)
        ux, uy = tgv_initial_velocity(c.x, c.y, c.period[0], 0.01)
    else:
        c, ux, uy = tgv_case(nside, K, m, mode)
    _, ref = oracle_run(c, c.h, K, m, mode, tau, ux, uy, [1, steps])
    for prec, tol in ((1, lambda s: TOL_FP64), (0, tol_fp32)):
        say("case", label, "precision", prec, "n", c.n)
        plan = Plan.build(c.x, c.y, c.period, _params(c.h, K, m, mode, prec, tau))
        got = _gpu_run(plan, ux, uy, [1, steps])
        _compare(ref, got, tol, "%s/%s" % (label, "fp64" if prec else "fp32"))
        plan.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_open_cloud_without_walls_matches_oracle(mode):
    """A jittered square that is neither periodic nor walled: departure points
    beyond its edge are extrapolated with the owner's stencil (the paper is
    silent), on both sides alike; both precisions. Without walls the edge
    amplifies any difference: the oracle alone grows a 1e-14 perturbation by
    1.5 per step here (it decays by 0.9 per step on the same cloud made
    periodic), and GPU against oracle in FP64 goes from 6.6e-14 after one step
    to 1.1e-11 after ten, so the run is compared over three steps."""
    from dataclasses import replace
    from paper_2306_01525_amd import Plan
    c, ux, uy = tgv_case(30, 20, 3, mode, seed=23)
    c = replace(c, period=(0.0, 0.0))
    K, m, tau = 20, 3, 0.8
    _, ref = oracle_run(c, c.h, K, m, mode, tau, ux, uy, [1, 3])
    for prec, tol in ((1, lambda s: TOL_FP64), (0, tol_fp32)):
        plan = Plan.build(c.x, c.y, c.period, _params(c.h, K, m, mode, prec, tau))
        got = _gpu_run(plan, ux, uy, [1, 3])
        _compare(ref, got, tol, "open/%d/%s" % (mode, "fp64" if prec else "fp32"))
        assert plan.device_error() == 0
        plan.close()


def test_annulus_walls_and_force_match_oracle():
    """Open cloud, equilibrium walls, azimuthal body force (Sec. 3)."""
    from paper_2306_01525_amd import Plan
    c = annulus_case(0.1)
    dx, K, m, tau, g = 0.1, 15, 2, 1.0, 1e-4
    zeros = np.zeros(c.n)
    _, ref = oracle_run(c, dx, K, m, 0, tau, zeros, zeros, [1, 20, 300], force=g)
    for prec, tol in ((1, lambda s: TOL_FP64), (0, tol_fp32)):
        say("case annulus precision", prec, "n", c.n)
        p = _params(dx, K, m, 0, prec, tau, force_kind=1, force_mag=g, wall_kind=1, rho_wall=1.0)
        plan = Plan.build(c.x, c.y, c.period, p, node_type=c.node_type)
        got = _gpu_run(plan, zeros, zeros, [1, 20, 300])
        _compare(ref, got, tol, "annulus/%s" % ("fp64" if prec else "fp32"))
        plan.close()


def test_graph_replay_equals_eager():
    from paper_2306_01525_amd import Plan
    c, ux, uy = tgv_case(24, 20, 3, 0)
    plan = Plan.build(c.x, c.y, c.period, _params(c.h, 20, 3, 0, 0, 0.8))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g0 = plan.init(ux, uy, stream=s)
        a = g0.clone()
        b = plan.new_state()
        ea = g0.clone()
        eb = plan.new_state()
        plan.graph_create(a, b, 10, s)
        for rep in range(3):
            plan.graph_launch(s)                   # 10 steps: result back in a
            res = plan.step(ea, eb, 10, stream=s)  # eager reference
            assert res is ea
            s.synchronize()
            say("graph replay", rep)
            assert torch.equal(a, ea)
    plan.close()


def test_fp32_mass_conservation():
    """Periodic, no force: the corrected FP32 weights keep the partition of
    unity, so total mass drifts only by rounding."""
    from paper_2306_01525_amd import Plan
    c, ux, uy = tgv_case(64, 30, 4, 0)
    plan = Plan.build(c.x, c.y, c.period, _params(c.h, 30, 4, 0, 0, 0.6))
    got = _gpu_run(plan, ux, uy, [500])
    drift = abs(got[500][0].sum() - c.n) / c.n
    say("fp32 mass drift after 500 steps", drift)
    assert drift < 1e-6


def test_tiles_cover_the_workload_and_fallback_path_matches():
    """Compact clouds use LDS gather tables on every tile; a streaming
    distance of 4 h spreads the owners of a tile beyond the table caps, so
    those tiles gather from global memory; both paths match the oracle."""
    from paper_2306_01525_amd import Plan
    c, ux, uy = tgv_case(48, 20, 3, 0)
    plan = Plan.build(c.x, c.y, c.period, _params(c.h, 20, 3, 0, 0, 0.8))
    say("tiles: lds bytes", plan.info.step_lds_bytes, "fallback", plan.info.fallback_tiles)
    assert plan.info.step_lds_bytes > 0 and plan.info.fallback_tiles == 0
    plan.close()
    dx = 4 * c.h
    _, ref = oracle_run(c, dx, 20, 3, 0, 0.8, ux, uy, [1, 30])
    plan = Plan.build(c.x, c.y, c.period, _params(dx, 20, 3, 0, 0, 0.8))
    say("dx = 4h: lds bytes", plan.info.step_lds_bytes, "fallback", plan.info.fallback_tiles)
    assert plan.info.fallback_tiles > 0
    got = _gpu_run(plan, ux, uy, [1, 30])
    _compare(ref, got, tol_fp32, "dx4h/fp32")
    plan.close()


def test_step_variants_are_bitwise_identical_and_autotune_picks_one():
    from paper_2306_01525_amd import Plan
    ca = annulus_case(0.05)
    walled = Plan.build(ca.x, ca.y, ca.period,
                        _params(0.05, 20, 3, 0, 0, 0.7, force_kind=1, force_mag=1e-5,
                                wall_kind=1, rho_wall=1.0), node_type=ca.node_type)
    za = np.zeros(ca.n)
    c, ux, uy = tgv_case(40, 30, 4, 0)
    plan = Plan.build(c.x, c.y, c.period, _params(c.h, 30, 4, 0, 0, 0.6))
    for pl, vx, vy in ((walled, za, za), (plan, ux, uy)):
        ref = rec_ref = None
        for v in range(10):   # 0-5 one lane per node, 6-9 two
            pl.set_variant(v)
            g = pl.init(vx, vy)
            g = pl.step(g, pl.new_state(), 25)
            # the recording step (pre-collision populations kept for the
            # adjoint) takes the same variant
            rec = torch.empty((3, 9, pl.n), dtype=g.dtype, device=g.device)
            g = pl.step_record(g, pl.new_state(), 3, rec)
            if ref is None:
                ref, rec_ref = g.clone(), rec.clone()
            else:
                assert torch.equal(g, ref), v
                assert torch.equal(rec, rec_ref), v
    walled.close()
    a, b = plan.new_state(), plan.new_state()
    ms = plan.autotune(plan.init(ux, uy, g=a), b, 5)
    say("variant ms/step", ["%.4f" % m for m in ms], "chosen", plan.info.variant)
    assert len(ms) == 10 and all(m > 0 for m in ms)
    assert ms[plan.info.variant] == min(ms)
    plan.close()



EXTREME_CASES = [
    # (label, K, degree, mode, steps compared, FP64 tolerance): the largest
    # stencil (K + M = 63 and 54 unknowns, the widest local solve and kNN paths,
    # 16 index words per stencil) and the smallest (K = M = 6: the polynomial
    # block alone fixes the weights). Six-point quadratic interpolation is
    # poorly conditioned on near-regular points (condition numbers up to ~2e7,
    # weights up to ~2e3): the two solvers' weights there agree only to the
    # conditioning bound, and the run diverges within a few tens of steps in
    # the oracle and on the GPU alike, so that case is compared after the first
    # step only, node by node, against the bound the weights imply (None).
    ("K48-m4-paper", 48, 4, 0, [1, 40], lambda s: TOL_FP64),
    ("K48-m2-own", 48, 2, 1, [1, 40], lambda s: TOL_FP64),
    ("K6-m2-own", 6, 2, 1, [1], None),
]


@pytest.mark.parametrize("label,K,m,mode,steps,tol64", EXTREME_CASES,
                         ids=[c[0] for c in EXTREME_CASES])
def test_extreme_stencil_sizes_match_oracle(label, K, m, mode, steps, tol64):
    from paper_2306_01525_amd import Plan
    c, ux, uy = tgv_case(30, K, m, mode, seed=17)
    tau = 0.8
    say("case", label, "n", c.n)
    (nbr, own, W), ref = oracle_run(c, c.h, K, m, mode, tau, ux, uy, steps)
    wb = weight_bounds(c, nbr, own, W, K, m)
    for prec in (1, 0):
        plan = Plan.build(c.x, c.y, c.period, _params(c.h, K, m, mode, prec, tau))
        if prec == 1:
            np.testing.assert_array_equal(plan.export("nbr"), nbr)
            dW = np.abs(plan.export("W")[:, 1:, :] - W[:, 1:, :]).max(axis=2)
            say("  max |W_gpu - W_oracle| = %.2e, largest fraction of its bound %.2e"
                % (dW.max(), (dW / wb[:, 1:]).max()))
            assert (dW <= wb[:, 1:]).all()
        got = _gpu_run(plan, ux, uy, steps)
        if tol64 is None:
            # one step from equilibrium: per-node bound from the weight bounds
            # plus the rounding of the step in the state's precision
            f0 = oracle.equilibrium(np.ones(c.n), ux, uy)
            b = first_step_bounds(nbr, own, wb, f0) + first_step_rounding_bounds(
                nbr, own, W, f0, 2.0 ** -53 if prec else EPS32)
            r_o, u_o, v_o = ref[1]
            r_g, u_g, v_g = got[1]
            worst = max(float((np.abs(a - o) / b).max())
                        for a, o in ((r_g, r_o), (r_g * u_g, r_o * u_o), (r_g * v_g, r_o * v_o)))
            say("  %s step 1: largest |moment difference| / bound %.2e"
                % ("fp64" if prec else "fp32", worst))
            assert worst <= 1.0
        else:
            tol = tol64 if prec == 1 else (lambda s: max(tol_fp32(s), tol64(s)))
            _compare(ref, got, tol, "%s/%s" % (label, "fp64" if prec else "fp32"))
        plan.close()
