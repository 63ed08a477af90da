"""Several clouds in one plan: one launch per step over all tiles of all
clouds, and the whole workload (build + init + steps) as one HIP graph."""
import numpy as np
import pytest

from gpu_common import dense_strip, oracle_run, rel_l2, say, tgv_case, tol_fp32
from synth import annulus_poisson, jittered_lattice, tgv_initial_velocity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SPECS = [  # (n_side, K, degree, tau, seed): uneven sizes, ragged tiles
    (23, 12, 2, 0.55, 1), (40, 30, 4, 0.9, 2), (17, 20, 3, 0.7, 3), (33, 12, 2, 1.0, 4),
    (51, 20, 3, 0.62, 5),
]


def _clouds(mode=0):
    from paper_2306_01525_amd import Params
    clouds, params, u = [], [], []
    for n_side, K, m, tau, seed in SPECS:
        c = jittered_lattice(n_side, seed=seed)
        ux, uy = tgv_initial_velocity(c.x, c.y, c.period[0], 0.01)
        clouds.append((c.x, c.y, c.period, None))
        params.append(Params(dx=c.h, K=K, degree=m, tau=tau, stencil_mode=mode if K >= 20 else 1))
        u.append((ux, uy))
    return clouds, params, u


def test_batched_plan_equals_single_plans_and_oracle():
    from paper_2306_01525_amd import Params, Plan
    clouds, params, u = _clouds()
    # batched step needs a common stencil rule: use own-node stencils for all
    for p in params:
        p.stencil_mode = 1
    ux = np.concatenate([a for a, _ in u])
    uy = np.concatenate([b for _, b in u])
    bp = Plan.build_batch(clouds, params)
    say("batched plan: clouds", len(bp.sizes), "nodes", bp.n)
    g = bp.init(ux, uy)
    g = bp.step(g, bp.new_state(), 20)
    rho_b, ux_b, uy_b = (a.cpu().numpy() for a in bp.moments(g))
    for c, ((x, y, period, _), p) in enumerate(zip(clouds, params)):
        sp = Plan.build(x, y, period, p)
        gs = sp.init(*u[c])
        gs = sp.step(gs, sp.new_state(), 20)
        assert torch.equal(gs, bp.cloud_view(g, c)), c
        sp.close()
    # and against the oracle, cloud by cloud
    for c, (n_side, K, m, tau, seed) in enumerate(SPECS):
        cl, ux0, uy0 = tgv_case(n_side, K, m, 1, seed=seed)
        _, ref = oracle_run(cl, cl.h, K, m, 1, tau, ux0, uy0, [20])
        sl = slice(bp.offsets[c], bp.offsets[c] + bp.sizes[c])
        e = rel_l2(np.stack([ux_b[sl], uy_b[sl]]), np.stack(ref[20][1:]))
        say("  cloud %d (n %d, K %d): rel L2 vs oracle %.2e" % (c, bp.sizes[c], K, e))
        assert e < tol_fp32(20)
    bp.close()


def test_batch_with_fewer_tiles_than_xcds_and_clouds_out_of_k_order():
    """Four tiles over eight XCD ranges (some ranges empty), clouds passed with
    K falling (the launch lays their tiles out by K): every cloud still steps
    bitwise like its single-cloud plan."""
    from paper_2306_01525_amd import Params, Plan
    specs = [(12, 30, 4, 0.8, 21), (10, 20, 3, 0.7, 22), (17, 12, 2, 0.9, 23)]  # 144, 100, 289 nodes
    clouds, params, u = [], [], []
    for n_side, K, m, tau, seed in specs:
        c = jittered_lattice(n_side, seed=seed)
        clouds.append((c.x, c.y, c.period, None))
        params.append(Params(dx=c.h, K=K, degree=m, tau=tau, stencil_mode=1))
        u.append(tgv_initial_velocity(c.x, c.y, c.period[0], 0.01))
    ux = np.concatenate([a for a, _ in u])
    uy = np.concatenate([b for _, b in u])
    bp = Plan.build_batch(clouds, params)
    g = bp.step(bp.init(ux, uy), bp.new_state(), 7)
    for c, ((x, y, period, _), p) in enumerate(zip(clouds, params)):
        sp = Plan.build(x, y, period, p)
        gs = sp.step(sp.init(*u[c]), sp.new_state(), 7)
        assert torch.equal(gs, bp.cloud_view(g, c)), c
        sp.close()
    assert bp.device_error() == 0
    bp.close()


def test_mixed_batch_falls_back_to_per_cloud_launches():
    """An annulus with walls and force next to a periodic cloud: no common
    batched kernel, each cloud is stepped by its own launch."""
    from paper_2306_01525_amd import Params, Plan
    a = annulus_poisson(1.0, 2.0, 0.1, seed=3)
    t = jittered_lattice(30, seed=6)
    pa = Params(dx=0.1, K=15, degree=2, tau=1.0, force_kind=1, force_mag=1e-4, wall_kind=1)
    pt = Params(dx=t.h, K=20, degree=3, tau=0.8)
    clouds = [(a.x, a.y, a.period, a.node_type), (t.x, t.y, t.period, None)]
    tux, tuy = tgv_initial_velocity(t.x, t.y, t.period[0], 0.01)
    ux = np.concatenate([np.zeros(a.n), tux])
    uy = np.concatenate([np.zeros(a.n), tuy])
    bp = Plan.build_batch(clouds, [pa, pt])
    g = bp.step(bp.init(ux, uy), bp.new_state(), 15)
    for c, (cl, p, u0) in enumerate([(clouds[0], pa, (np.zeros(a.n), np.zeros(a.n))),
                                     (clouds[1], pt, (tux, tuy))]):
        sp = Plan.build(cl[0], cl[1], cl[2], p, node_type=cl[3])
        gs = sp.step(sp.init(*u0), sp.new_state(), 15)
        assert torch.equal(gs, bp.cloud_view(g, c)), c
        sp.close()
    bp.close()


def test_build_graph_replays_equal_eager():
    """Build + init + steps captured once and replayed three times, with eager
    work and synchronisation in between; every replay equals an eager run."""
    from paper_2306_01525_amd import Plan
    clouds, params, u = _clouds()
    for p in params:
        p.stencil_mode = 1
    ux = np.concatenate([a for a, _ in u])
    uy = np.concatenate([b for _, b in u])
    eager = Plan.build_batch(clouds, params)
    ge = eager.step(eager.init(ux, uy), eager.new_state(), 12)
    s = torch.cuda.Stream()
    plan, g_a, g_b, res = Plan.build_graph(clouds, params, ux, uy, 12, s)
    for rep in range(3):
        plan.graph_launch(s)
        s.synchronize()
        say("graph replay", rep, "device error", plan.device_error())
        assert torch.equal(res, ge), rep
        assert plan.device_error() == 0
        ge2 = eager.step(eager.init(ux, uy), eager.new_state(), 12)   # eager work between
        torch.cuda.synchronize()
        assert torch.equal(ge2, ge)
    plan.close()
    eager.close()


def test_set_tau_reaches_every_cloud_of_a_batched_plan():
    """The batched step reads each cloud's relaxation time from the device
    descriptor table: after set_tau every cloud steps exactly like a
    single-cloud plan built at the new value, and the graph created before
    the change is dropped."""
    from paper_2306_01525_amd import Plan
    clouds, params, u = _clouds()
    for p in params:
        p.stencil_mode = 1
    ux = np.concatenate([a for a, _ in u])
    uy = np.concatenate([b for _, b in u])
    bp = Plan.build_batch(clouds, params)
    g = bp.step(bp.init(ux, uy), bp.new_state(), 3)
    new_tau = 0.77
    bp.set_tau(new_tau)
    g = bp.step(bp.init(ux, uy), bp.new_state(), 10)
    for c, (x, y, period, _) in enumerate(clouds):
        p = params[c]
        assert p.tau == new_tau
        sp = Plan.build(x, y, period, p)
        gs = sp.step(sp.init(*u[c]), sp.new_state(), 10)
        assert torch.equal(gs, bp.cloud_view(g, c)), c
        sp.close()
    bp.close()


@pytest.mark.parametrize("variant", [0, 6])
def test_captured_plan_sends_tiles_beyond_its_lds_to_the_global_path(variant):
    """A plan built inside a graph capture sizes the FP32 step's LDS before
    its tables exist (40 KiB up to K = 30). On a cloud whose largest tile needs
    more, those tiles gather from global memory and the captured plan still
    steps bitwise like the eager plan, which stages every tile. (The strip's
    nodes are far closer than the streaming distance, which is not a stable
    setting (the run would pass the speed limit within 15 steps): three steps
    compare the arithmetic of the two paths.)"""
    from paper_2306_01525_amd import Params, Plan
    x, y, period, h = dense_strip()
    p = Params(dx=h, K=30, degree=4, tau=0.8, stencil_mode=0)
    ux, uy = tgv_initial_velocity(x, y, period[0], 0.01)
    eager = Plan.build(x, y, period, p)
    need = int(eager.info.step_lds_bytes)
    say("largest tile needs %d bytes of LDS; fallback tiles %d" % (need, int(eager.info.fallback_tiles)))
    assert need > 40 * 1024 and int(eager.info.fallback_tiles) == 0
    eager.set_variant(variant)
    ge = eager.step(eager.init(ux, uy), eager.new_state(), 3)
    s = torch.cuda.Stream()
    plan, g_a, g_b, res = Plan.build_graph([(x, y, period, None)], [p], ux, uy, 3, s, variant)
    plan.graph_launch(s)
    s.synchronize()
    say("device error words: captured %d, eager %d" % (plan.device_error(), eager.device_error()))
    assert plan.device_error() == eager.device_error() == 0
    assert torch.equal(res.reshape(-1), ge.reshape(-1))
    plan.close()
    eager.close()


def _batch_draw(count=4, seed=99):
    r = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        mode = int(r.integers(0, 2))
        clouds = []
        for _ in range(int(r.integers(2, 8))):
            m = int(r.integers(2, 5))
            K = {2: 20, 3: 25, 4: 30}[m] if mode == 0 else int(r.integers(12, 41))
            clouds.append(dict(n_side=int(r.integers(8, 70)), K=max(K, (m + 1) * (m + 2) // 2 + 2),
                               m=m, tau=float(r.uniform(0.55, 1.0)), seed=int(r.integers(1, 9999))))
        out.append(dict(mode=mode, clouds=clouds))
    return out


@pytest.mark.parametrize("batch", _batch_draw(), ids=lambda b: "mode%d-%dclouds" % (
    b["mode"], len(b["clouds"])))
def test_random_batches_equal_single_plans(batch):
    """Seeded random batches (2-7 clouds of 64 to 4,761 nodes, their own K,
    degree and tau, one stencil rule): every cloud of the batched plan steps
    bitwise like its own single-cloud plan."""
    from paper_2306_01525_amd import Params, Plan
    clouds, params, u = [], [], []
    for s in batch["clouds"]:
        c = jittered_lattice(s["n_side"], seed=s["seed"])
        clouds.append((c.x, c.y, c.period, None))
        params.append(Params(dx=c.h, K=min(s["K"], c.n), degree=s["m"], tau=s["tau"],
                             stencil_mode=batch["mode"]))
        u.append(tgv_initial_velocity(c.x, c.y, c.period[0], 0.01))
    ux = np.concatenate([a for a, _ in u])
    uy = np.concatenate([b for _, b in u])
    bp = Plan.build_batch(clouds, params)
    g = bp.step(bp.init(ux, uy), bp.new_state(), 9)
    for c, ((x, y, period, _), p) in enumerate(zip(clouds, params)):
        sp = Plan.build(x, y, period, p)
        gs = sp.step(sp.init(*u[c]), sp.new_state(), 9)
        assert torch.equal(gs, bp.cloud_view(g, c)), c
        sp.close()
    assert bp.device_error() == 0
    bp.close()
