"""GPU weight build (stencils, owners, shape vectors) against the oracle."""
import numpy as np
import pytest

import oracle
from gpu_common import TOL_W, annulus_case, dense_strip, say, tgv_case, weight_bounds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _build(c, dx, K, m, mode, precision=0):
    from paper_2306_01525_amd import Params, Plan
    p = Params(dx=dx, K=K, degree=m, tau=0.8, stencil_mode=mode, precision=precision)
    return Plan.build(c.x, c.y, c.period, p, node_type=c.node_type)


CASES = [
    # (label, cloud factory, dx factor, K, m, mode)
    ("tgv40-K12-m2-own", lambda: tgv_case(40, 12, 2, 1)[0], 1.0, 12, 2, 1),
    ("tgv40-K25-m2-paper", lambda: tgv_case(40, 25, 2, 0)[0], 1.0, 25, 2, 0),
    ("tgv37x41-K30-m4-paper", lambda: tgv_case(37, 30, 4, 0, ny=41, length_y=7.0)[0], 1.0, 30, 4, 0),
    ("tgv23-K20-m3-own", lambda: tgv_case(23, 20, 3, 1, seed=7)[0], 0.7, 20, 3, 1),
    ("annulus-h0.1-K15-m2-paper", lambda: annulus_case(0.1), None, 15, 2, 0),
    ("tgv30-K47-m4-own", lambda: tgv_case(30, 47, 4, 1, seed=3)[0], 1.0, 47, 4, 1),
    ("tgv32-K40-m3-paper", lambda: tgv_case(32, 40, 3, 0, seed=5)[0], 1.0, 40, 3, 0),
    ("lattice16-K12-m2-paper", lambda: tgv_case(16, 12, 2, 0, jitter=0.0, length=16.0)[0], 1.0, 12, 2, 0),
]


@pytest.mark.parametrize("label,make,dxf,K,m,mode", CASES, ids=[c[0] for c in CASES])
def test_build_matches_oracle(label, make, dxf, K, m, mode):
    c = make()
    dx = 0.1 if dxf is None else dxf * c.h
    say("case", label, "n", c.n)
    plan = _build(c, dx, K, m, mode)
    nbr_g = plan.export("nbr")
    own_g = plan.export("owner")
    W_g = plan.export("W")
    perm = plan.export("perm")
    assert sorted(perm.tolist()) == list(range(c.n))
    nbr_o = oracle.knn(c.x, c.y, c.period, K)
    own_o = oracle.owners(c.x, c.y, c.period, dx, mode)
    np.testing.assert_array_equal(nbr_g, nbr_o)
    np.testing.assert_array_equal(own_g, own_o)
    W_o = oracle.weights(c.x, c.y, c.period, dx, K, m, nbr_o, own_o)
    err = np.abs(W_g[:, 1:, :] - W_o[:, 1:, :]).max()
    say("  max |W_gpu - W_oracle| =", err)
    assert err < TOL_W
    # k = 0 is the identity on both sides
    np.testing.assert_allclose(W_o[:, 0, 0], 1.0, atol=1e-10)
    plan.close()


# K and degree whose K + M unknowns (33 to 48) take the 48-unknown matrix-core
# solver: every remainder of K + M modulo 4 (the last panel of four pivot
# columns only partly used) and both ends of the range.
MFMA_RANGE = [(18, 4, 0), (24, 3, 1), (30, 2, 0), (24, 4, 1), (32, 3, 0), (32, 4, 1),
              (33, 4, 0), (38, 3, 1)]


@pytest.mark.parametrize("K,m,mode", MFMA_RANGE,
                         ids=["K%d-m%d-n%d" % (K, m, K + (m + 1) * (m + 2) // 2)
                              for K, m, _ in MFMA_RANGE])
def test_48_unknown_solver_over_its_range(K, m, mode):
    c, _, _ = tgv_case(20, K, m, mode, seed=11)
    plan = _build(c, c.h, K, m, mode)
    nbr_o = oracle.knn(c.x, c.y, c.period, K)
    own_o = oracle.owners(c.x, c.y, c.period, c.h, mode)
    np.testing.assert_array_equal(plan.export("nbr"), nbr_o)
    np.testing.assert_array_equal(plan.export("owner"), own_o)
    W_o = oracle.weights(c.x, c.y, c.period, c.h, K, m, nbr_o, own_o)
    err = np.abs(plan.export("W")[:, 1:, :] - W_o[:, 1:, :]).max()
    say("K %d degree %d (%d unknowns), mode %d: max |W_gpu - W_oracle| = %.2e"
        % (K, m, K + oracle.poly_count(m), mode, err))
    assert err < TOL_W
    assert plan.device_error() == 0
    plan.close()


def test_build_with_crowded_owners_matches_oracle():
    """Weights on the dense-strip cloud, where nodes beside the strip own
    more than 16 departure points: the 48-unknown matrix-core solver solves
    them in groups of 16 (K 30, degree 4, paper rule)."""
    from paper_2306_01525_amd import Params, Plan
    x, y, period, h = dense_strip()
    K, m = 30, 4
    p = Params(dx=h, K=K, degree=m, tau=0.8, stencil_mode=0)
    plan = Plan.build(x, y, period, p)
    nbr_o = oracle.knn(x, y, period, K)
    own_o = oracle.owners(x, y, period, h, 0)
    counts = np.bincount(own_o[:, 1:].ravel(), minlength=x.shape[0])
    say("largest number of departure points of one owner:", counts.max())
    assert counts.max() > 16
    np.testing.assert_array_equal(plan.export("nbr"), nbr_o)
    np.testing.assert_array_equal(plan.export("owner"), own_o)
    W_o = oracle.weights(x, y, period, h, K, m, nbr_o, own_o)
    d = np.abs(plan.export("W") - W_o).max(axis=2)[:, 1:]            # [n][8]
    # the stencils at the strip's edges are lopsided and their systems far
    # worse conditioned than on the lattices: each (node, direction) is held
    # to the backward-error bound of its owner's system
    from types import SimpleNamespace
    c = SimpleNamespace(x=x, y=y, period=period, n=x.shape[0])
    b = weight_bounds(c, nbr_o, own_o, W_o, K, m)[:, 1:]
    worst = np.unravel_index(np.argmax(d / b), d.shape)
    say("max |W_gpu - W_oracle| = %.2e; worst against its bound: %.2e of %.2e (owner of %d points)"
        % (d.max(), d[worst], b[worst], counts[own_o[worst[0], worst[1] + 1]]))
    assert (d <= np.maximum(b, TOL_W)).all()
    assert plan.device_error() == 0
    plan.close()


def test_build_rejects_bad_parameters():
    from paper_2306_01525_amd import MLBMError, Params, Plan
    c, _, _ = tgv_case(10, 12, 2, 0)
    for kw in (dict(K=5, degree=2), dict(K=12, degree=1), dict(K=8, degree=3),
               dict(K=12, degree=2, tau=0.5)):
        p = Params(dx=c.h, tau=kw.pop("tau", 0.8), **kw)
        with pytest.raises(MLBMError):
            Plan.build(c.x, c.y, c.period, p)


@pytest.mark.parametrize("K,m", [(12, 2), (30, 4), (48, 4)])
def test_singular_stencil_is_reported(K, m):
    """Nodes on a straight line make every local system singular (the
    monomials of degree >= 2 are not unisolvent), for each solver shape: two
    systems per wavefront (24 unknowns) and one (48 and 64)."""
    from paper_2306_01525_amd import MLBMError, Params, Plan
    n = 61
    x = np.linspace(0.0, 1.0, n)
    y = 2.0 * x + 0.5
    p = Params(dx=0.01, K=K, degree=m, tau=0.8, stencil_mode=1)
    with pytest.raises(MLBMError) as ei:
        Plan.build(x, y, (0.0, 0.0), p)
    assert ei.value.status == -2


@pytest.mark.parametrize("mode", [0, 1])
def test_duplicate_node_is_reported_singular(mode):
    """Two nodes at the same place: every stencil that holds both has two
    equal rows (and columns) in its local system, which is singular; the
    build reports it (the lower-index twin owns the departure points near it
    in the paper's rule, and every node owns its own in the other)."""
    from paper_2306_01525_amd import MLBMError, Params, Plan
    c, _, _ = tgv_case(20, 20, 3, mode, seed=13)
    x, y = c.x.copy(), c.y.copy()
    x[150], y[150] = x[77], y[77]
    with pytest.raises(MLBMError) as ei:
        Plan.build(x, y, c.period, Params(dx=c.h, K=20, degree=3, tau=0.8, stencil_mode=mode))
    assert ei.value.status == -2


@pytest.mark.parametrize("mode", [0, 1])
def test_tile_tables_are_consistent(mode):
    """Gather tables of the FP32 step, checked on the CPU before any step
    uses them: halo lists sorted, unique and in range; local owners and
    local stencils map back to the global owners and stencils."""
    c, _, _ = tgv_case(64, 30, 4, mode, seed=9)
    plan = _build(c, c.h, 30, 4, mode)
    perm = plan.export("perm")
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(c.n)
    nbr_u = plan.export("nbr")            # user order, user indices
    own_u = plan.export("owner")
    # internal order, internal indices
    nbr_i = iperm[nbr_u[perm]]
    own_i = iperm[own_u[perm]]
    td = plan.export("tdesc")
    hl = plan.export("hlist")
    words = plan.export("nbrL")
    # three 10-bit halo positions per word -> [ntiles][ocap][K]
    nl = np.stack([(words >> (10 * s_)) & 1023 for s_ in range(3)], axis=-1)
    nl = nl.reshape(words.shape[0], words.shape[1], -1)[:, :, :30]
    ol = plan.export("ownerL") if mode == 0 else None
    T = int(plan.info.tile_nodes)
    say("mode", mode, "tiles", td.shape[0], "max nh", td[:, 1].max(), "max no", td[:, 0].max())
    assert (td[:, 1] > 0).all()
    for t in range(td.shape[0]):
        no, nh = td[t]
        base, cnt = t * T, min(T, c.n - t * T)
        H = hl[t, :nh]
        assert (H >= 0).all() and (H < c.n).all()
        assert (np.diff(H) > 0).all()
        if mode == 0:
            O = np.unique(own_i[base:base + cnt, 1:])
        else:
            O = np.arange(base, base + cnt)
        assert O.size == no
        np.testing.assert_array_equal(H[nl[t, :no, :]], nbr_i[O])
        if mode == 0:
            np.testing.assert_array_equal(O[ol[:, base:base + cnt].T], own_i[base:base + cnt, 1:])
    plan.close()


def _uncompact(units, hd, lw, n, fill):
    """Row heads compacted per group of 64 nodes ([units][8]: group g from
    unit 64 g lw, slot e a block of the group's nodes with hd > e in node
    order, entries 0-3 of the block's units before entries 4-7) back to
    [8][lw][n], with `fill` where a node has no unit."""
    n64 = (n + 63) // 64 * 64
    G = n64 // 64
    H = np.zeros(n64, dtype=np.int64)
    H[:n] = hd
    act = np.arange(lw)[:, None, None] < H.reshape(G, 64)[None]   # [lw][G][64]
    cnt = act.sum(axis=2)
    start = np.cumsum(cnt, axis=0) - cnt                          # units of earlier slots
    u0 = (np.arange(G) * 64 * lw)[None, :] + start                 # [lw][G] first unit
    rank = np.cumsum(act, axis=2) - 1
    e, g, l_ = np.nonzero(act)
    flat = units.reshape(-1)
    k = np.arange(8)[:, None]
    at = 8 * u0[e, g][None] + 4 * ((k // 4) * cnt[e, g][None] + rank[e, g, l_][None]) + k % 4
    out = np.full((8, lw, n64), fill, dtype=units.dtype)
    out[:, e, g * 64 + l_] = flat[at]
    return out[:, :, :n]


@pytest.mark.parametrize("mode,precision,K,m", [(0, 0, 30, 4), (1, 1, 30, 4), (1, 0, 48, 4),
                                                (0, 0, 12, 2)])
def test_adjoint_tables_are_consistent(mode, precision, K, m):
    """Transposed stencil operator and the gather tables of the adjoint step,
    checked on the CPU before any adjoint step uses them: row lengths and row
    heads match the transpose of the forward stencils (rows sorted by arriving
    node), inverse halo lists are sorted, unique and in range, and the local
    columns map back to the row heads. The fill stages 128-node tiles up to
    K = 30 in FP32 and 64-node tiles for FP64 or larger K."""
    from paper_2306_01525_amd import Params, Plan
    c, _, _ = tgv_case(61, K, m, mode, seed=9)   # 3,721 nodes: a partial last group of 64
    p = Params(dx=c.h, K=K, degree=m, tau=0.8, stencil_mode=mode, precision=precision,
               with_adjoint=1)
    plan = Plan.build(c.x, c.y, c.period, p)
    n = c.n
    perm = plan.export("perm")
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(n)
    nbr_i = iperm[plan.export("nbr")[perm]]
    own_i = iperm[plan.export("owner")[perm]]
    ptr = plan.export("tr_ptr")
    lw = K + 4
    hd = np.minimum(np.diff(ptr).reshape(8, n), lw).max(axis=0)
    ecol = _uncompact(plan.export("ell_col"), hd, lw, n, -1)            # [8][slot][n]
    td = plan.export("tdescT")
    il = plan.export("ilist")
    words = _uncompact(plan.export("elocal"), (hd + 2) // 3, (lw + 2) // 3, n, 0)
    # every slot of a node's head is there, padded with its own index
    pad = (np.arange(lw)[None, :, None] >= np.diff(ptr).reshape(8, 1, n)) \
        & (np.arange(lw)[None, :, None] < hd[None, None, :])
    assert (ecol[pad] == np.broadcast_to(np.arange(n), ecol.shape)[pad]).all()
    el = np.stack([(words >> (10 * s_)) & 1023 for s_ in range(3)], axis=2)
    el = el.reshape(8, -1, n)[:, :lw, :]              # [8][lw][n] (slot-major)
    assert (el[:, :, :][np.arange(lw)[None, :, None] >= np.diff(ptr).reshape(8, 1, n)] == 0).all()
    assert ptr[0] == 0 and ptr[-1] == 8 * K * n and (np.diff(ptr) >= 0).all()
    lens = np.diff(ptr).reshape(8, n)
    arrive = np.repeat(np.arange(n), K)
    for k in range(1, 9):
        S = nbr_i[own_i[:, k]] if mode == 0 else nbr_i
        src = S.ravel()
        np.testing.assert_array_equal(lens[k - 1], np.bincount(src, minlength=n))
        order = np.lexsort((arrive, src))
        rows_src, rows_arr = src[order], arrive[order]
        start = np.concatenate([[0], np.cumsum(lens[k - 1])[:-1]])
        slot = np.arange(src.size) - start[rows_src]
        head = slot < lw
        np.testing.assert_array_equal(ecol[k - 1][slot[head], rows_src[head]], rows_arr[head])
    T = int(plan.info.tile_nodes)
    say("mode", mode, "precision", precision, "tiles", td.size, "max |I_t|", td.max(),
        "global tiles", int((td == 0).sum()))
    assert (td > 0).all()
    assert td.max() <= 1024
    for t in range(td.size):
        ni = td[t]
        I = il[t, :ni]
        assert (I >= 0).all() and (I < n).all() and (np.diff(I) > 0).all()
        ms = np.arange(t * T, min(n, (t + 1) * T))
        for k in range(8):
            hl = np.minimum(lens[k, ms], lw)
            mask = np.arange(lw)[:, None] < hl[None, :]
            np.testing.assert_array_equal(I[el[k][:, ms][mask]], ecol[k][:, ms][mask])
    plan.close()


def test_fp32_weights_only_plan_steps_like_the_full_plan():
    """A plan built with fp32_weights_only holds no FP64 shape vectors: its
    buffer is smaller by 64 K bytes per node; its steps (one cloud, a batch,
    the static-workspace build) and its gradient are bitwise those of the full
    plan; the calls that need the FP64 vectors refuse."""
    from paper_2306_01525_amd import MLBMError, Params, Plan
    from paper_2306_01525_amd.autograd import rollout_loss
    from synth import jittered_lattice, tgv_initial_velocity
    c, ux, uy = tgv_case(48, 30, 4, 0, seed=4)
    ux, uy = tgv_initial_velocity(c.x, c.y, c.period[0], 0.01)

    def prm(lean, K=30, m=4, **kw):
        return Params(dx=c.h, K=K, degree=m, tau=0.8, stencil_mode=0,
                      fp32_weights_only=int(lean), **kw)

    full = Plan.build(c.x, c.y, c.period, prm(False))
    lean = Plan.build(c.x, c.y, c.period, prm(True))
    stat = Plan.build(c.x, c.y, c.period, prm(True), static_workspace=True)
    saved = full._buf.numel() - lean._buf.numel()
    say("plan bytes per node: full %.0f, fp32_weights_only %.0f"
        % (full._buf.numel() / c.n, lean._buf.numel() / c.n))
    assert saved >= 64 * 30 * c.n
    g_full = full.step(full.init(ux, uy), full.new_state(), 20)
    for q in (lean, stat):
        assert torch.equal(q.step(q.init(ux, uy), q.new_state(), 20), g_full)
        assert q.device_error() == 0
    for call in (lambda: lean.export("W"), lambda: lean.interpolate(np.zeros(c.n))):
        with pytest.raises(MLBMError) as ei:
            call()
        assert ei.value.status == -5
    for q in (full, lean, stat):
        q.close()
    # built, initialised and stepped inside one captured graph, replayed twice
    s = torch.cuda.Stream()
    gp, _, _, res = Plan.build_graph([(c.x, c.y, c.period, None)], [prm(True)], ux, uy, 20, s)
    for _ in range(2):
        gp.graph_launch(s)
        s.synchronize()
        assert torch.equal(res.reshape(-1), g_full.reshape(-1))
    assert gp.device_error() == 0
    gp.close()

    # a batch of two clouds
    c2 = jittered_lattice(30, seed=8)
    u2x, u2y = tgv_initial_velocity(c2.x, c2.y, c2.period[0], 0.01)
    clouds = [(c.x, c.y, c.period, None), (c2.x, c2.y, c2.period, None)]
    bx, by = np.concatenate([ux, u2x]), np.concatenate([uy, u2y])
    states = []
    for lean_flag in (False, True):
        b = Plan.build_batch(clouds, [prm(lean_flag), prm(lean_flag, K=20, m=3)])
        states.append(b.step(b.init(bx, by), b.new_state(), 10))
        b.close()
    assert torch.equal(states[0], states[1])

    # the gradient of a short checkpointed rollout
    tx, ty = (torch.tensor(a, device="cuda") for a in (ux, uy))
    grads = []
    for lean_flag in (False, True):
        q = Plan.build(c.x, c.y, c.period, prm(lean_flag, with_adjoint=1))
        u0x = torch.tensor(ux, device="cuda", requires_grad=True)
        u0y = torch.tensor(uy, device="cuda", requires_grad=True)
        tau = torch.tensor(0.8, dtype=torch.float64, device="cuda", requires_grad=True)
        J = rollout_loss(q, u0x, u0y, tau, 6, 0.5 * tx, 0.5 * ty, 3)
        J.backward()
        grads.append((J.detach(), u0x.grad, u0y.grad, tau.grad))
        q.close()
    for a, b in zip(*grads):
        assert torch.equal(a, b)
