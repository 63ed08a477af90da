"""Clouds at the size limits. A cloud of 12.25M nodes (3,500 x 3,500 jittered
lattice, K = 30, degree 4, paper stencils), where the FP64 shape vectors hold
8 K n = 2.9e9 values, past 2^31: the first step at sampled nodes, half of
them among the last internal (Hilbert) positions, against the oracle formed
node by node. And the adjoint at the largest cloud its tables allow."""
import numpy as np
import pytest

import oracle
from gpu_common import say, tol_fp32_node
from synth import jittered_lattice, tgv_initial_velocity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_SIDE, K, M_DEG, TAU, U0, WIN = 3500, 30, 4, 0.6, 0.01, 8


def _window(c, i):
    """User indices (ascending) of the lattice cells within WIN of node i's
    cell, which holds every node closer than (WIN - 0.6) h to it."""
    ix, iy = i % N_SIDE, i // N_SIDE
    d = np.arange(-WIN, WIN + 1)
    jx, jy = np.meshgrid((ix + d) % N_SIDE, (iy + d) % N_SIDE)
    return np.unique((jy * N_SIDE + jx).ravel())


def _knn(c, i):
    """The oracle's K nearest of node i over its window; exact because the
    K-th distance stays inside the window's sure radius (asserted)."""
    idx = _window(c, i)
    loc = oracle.knn_one(c.x[idx], c.y[idx], c.period, K, int(np.searchsorted(idx, i)))
    st = idx[loc]
    L = c.period[0]
    dx = (c.x[st[-1]] - c.x[i] + L / 2) % L - L / 2
    dy = (c.y[st[-1]] - c.y[i] + L / 2) % L - L / 2
    assert np.hypot(dx, dy) < (WIN - 0.6) * c.h
    return st


def _nearest(c, i, px, py):
    idx = _window(c, i)
    s = idx[oracle.nearest(c.x[idx], c.y[idx], c.period, px, py)]
    L = c.period[0]
    d = np.hypot((c.x[s] - px + L / 2) % L - L / 2, (c.y[s] - py + L / 2) % L - L / 2)
    assert d < (WIN - 2.0) * c.h
    return int(s)


def test_large_cloud_first_step_at_sampled_nodes():
    from paper_2306_01525_amd import Params, Plan
    c = jittered_lattice(N_SIDE, seed=6)
    ux, uy = tgv_initial_velocity(c.x, c.y, c.period[0], U0)
    res = {}
    for prec in (1, 0):
        p = Params(dx=c.h, K=K, degree=M_DEG, tau=TAU, stencil_mode=0, precision=prec)
        say("building precision %d plan, n = %d" % (prec, c.n))
        plan = Plan.build(c.x, c.y, c.period, p)
        if prec == 1:
            perm = plan.export("perm")       # internal position -> user index
        g1 = plan.step(plan.init(ux, uy), plan.new_state(), 1)
        res[prec] = tuple(a.cpu().numpy() for a in plan.moments(g1))
        assert plan.device_error() == 0
        plan.close()
        del g1
        torch.cuda.empty_cache()
    rng = np.random.default_rng(7)
    tail = perm[c.n - c.n // 100:]
    sample = np.concatenate([rng.choice(tail, 16, replace=False), perm[-1:],
                             rng.choice(c.n, 16, replace=False)])
    ex, ey, _, _ = oracle.tables()
    L = c.period[0]
    emax64 = emax32 = 0.0
    for i in sample:
        f = np.empty(9)
        for k in range(9):
            px, py = c.x[i] - ex[k] * c.h, c.y[i] - ey[k] * c.h
            s = _nearest(c, i, px, py) if k else int(i)
            st = _knn(c, s)
            rx = (c.x[st] - c.x[s] + L / 2) % L - L / 2
            ry = (c.y[st] - c.y[s] + L / 2) % L - L / 2
            qx = (px - c.x[s] + L / 2) % L - L / 2
            qy = (py - c.y[s] + L / 2) % L - L / 2
            w = oracle.shape_vector(rx, ry, qx, qy, M_DEG)
            post = oracle.collide(oracle.equilibrium(np.ones(K), ux[st], uy[st]), TAU)
            f[k] = w @ post[:, k]
        r, u, v = oracle.moments(f[None, :])
        for prec in (1, 0):
            rg, ug, vg = (a[i] for a in res[prec])
            e = max(abs(r[0] - rg), abs(u[0] - ug) / U0, abs(v[0] - vg) / U0)
            if prec:
                emax64 = max(emax64, e)
            else:
                emax32 = max(emax32, e)
    say("%d sampled nodes (17 among the last 1 %% of positions): largest difference after one "
        "step FP64 %.2e, FP32 %.2e" % (sample.size, emax64, emax32))
    # as at 262,144 nodes: K TOL_W |f| for FP64 (measured 7e-14); the FP32
    # per-node bound after one step (measured 1.9e-7)
    assert emax64 < 1e-10
    assert emax32 < tol_fp32_node(1)


def test_adjoint_at_the_table_limit_satisfies_the_dot_product_identity():
    """2,991^2 = 8,946,081 nodes at K = 30: the transposed operator holds
    8 K n = 2,147,059,440 entries, just below the 2^31 - 1 the row pointers
    allow. For the one-step map F(f) = S(C(f)) and seeded random directions,
    <lam, J df> (central difference of the GPU forward, FP64) equals
    <J^T lam, df> (one reversed step)."""
    from paper_2306_01525_amd import Params, Plan
    n_side = 2991
    c = jittered_lattice(n_side, seed=8)
    assert 2 ** 31 - 1_000_000 < 8 * K * c.n <= 2 ** 31 - 1
    ux, uy = tgv_initial_velocity(c.x, c.y, c.period[0], U0)
    p = Params(dx=c.h, K=K, degree=M_DEG, tau=TAU, stencil_mode=0, precision=1, with_adjoint=1)
    say("building FP64 plan with the adjoint tables, n = %d" % c.n)
    plan = Plan.build(c.x, c.y, c.period, p)
    f0 = plan.init_f(ux, uy)
    gen = torch.Generator(device="cuda").manual_seed(11)
    df = torch.randn(f0.shape, generator=gen, device="cuda", dtype=torch.float64)
    lam = torch.randn(f0.shape, generator=gen, device="cuda", dtype=torch.float64)
    eps = 1e-7

    def F(f):
        rec = plan.new_state()
        plan.step_record(plan.collide(f), plan.new_state(), 1, rec)
        return rec

    jdf = (F(f0 + eps * df) - F(f0 - eps * df)) / (2 * eps)
    lam_n = plan.new_state()
    dtau = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.step_adjoint(f0, lam, lam_n, dtau)
    a = float(torch.dot(lam.reshape(-1), jdf.reshape(-1)))
    b = float(torch.dot(lam_n.reshape(-1), df.reshape(-1)))
    say("<lam, J df> %.12e, <J^T lam, df> %.12e, relative difference %.2e" % (a, b, abs(a - b) / abs(b)))
    assert plan.device_error() == 0
    # measured 1.8e-11: the central difference's truncation is O(eps^2) and its
    # rounding about 1e-16 |F| / eps per entry, averaged over 80M entries
    assert abs(a - b) <= 1e-10 * abs(b)
    plan.close()
