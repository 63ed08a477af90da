"""Sticky device error words (mlbm_device_error): conditions forced from the
host are reported with their codes and nodes. A NaN population and a fast
initial node are data; a halo index overwritten in the plan buffer is clamped
by the kernels to node 0 before any load, so none of these can fault."""
import numpy as np
import pytest

from gpu_common import say, tgv_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _plan(precision, with_adjoint=0):
    from paper_2306_01525_amd import Params, Plan
    c, ux, uy = tgv_case(20, 20, 3, 0)
    p = Params(dx=c.h, K=20, degree=3, tau=0.8, stencil_mode=0, precision=precision,
               with_adjoint=with_adjoint)
    return c, ux, uy, Plan.build(c.x, c.y, c.period, p)


@pytest.mark.parametrize("precision", [0, 1])
def test_nonfinite_population_is_flagged_by_the_next_step(precision):
    from paper_2306_01525_amd import MLBM_DEVERR_NONFINITE
    c, ux, uy, plan = _plan(precision)
    g = plan.step(plan.init(ux, uy), plan.new_state(), 3)
    assert plan.device_error() == 0
    assert plan.device_error_nodes() == (-1, -1)
    perm = plan.export("perm")
    p = 57                      # internal position; its rest population streams to itself only
    g[0, p] = float("nan")
    plan.step(g, plan.new_state(), 1)
    err = plan.device_error()
    _, node = plan.device_error_nodes()
    say("precision %d: error bits %d, node %d (user index of position %d: %d)"
        % (precision, err, node, p, perm[p]))
    assert err == MLBM_DEVERR_NONFINITE
    assert node == perm[p]
    plan.clear_device_error()
    assert plan.device_error() == 0
    assert plan.device_error_nodes() == (-1, -1)
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_speed_above_the_limit_is_flagged_by_the_diagnostics(precision):
    """A node started at |u| = 0.45 (Mach 0.78): the moments, the L2 sums and
    the residual pass each report it."""
    from paper_2306_01525_amd import MLBM_DEVERR_SPEED
    c, ux, uy, plan = _plan(precision)
    ux = ux.copy()
    ux[13] = 0.45
    g = plan.init(ux, uy)
    assert plan.device_error() == 0      # the initial state is not checked
    for name, call in (("moments", lambda: plan.moments(g)),
                       ("l2", lambda: plan.l2_sums(g, torch.zeros(c.n, dtype=torch.float64,
                                                                  device="cuda"),
                                                   torch.zeros(c.n, dtype=torch.float64,
                                                               device="cuda"))),
                       ("residual", lambda: plan.residual(
                           g, torch.zeros(c.n, dtype=torch.float64, device="cuda")))):
        call()
        err = plan.device_error()
        _, node = plan.device_error_nodes()
        say("precision %d, %s: error bits %d, node %d" % (precision, name, err, node))
        assert err == MLBM_DEVERR_SPEED and node == 13
        plan.clear_device_error()
        assert plan.device_error() == 0
    plan.close()


def _corrupt_first_list(plan, table, entry, value):
    """Overwrite entry `entry` of tile 0's list `table` ('hlist' or 'ilist')
    inside the plan buffer with `value`. The list's place in the buffer is
    found from its exported contents: the unique 256-byte aligned offset where
    every tile's used entries appear."""
    used = plan.export("tdesc")[:, 1] if table == "hlist" else plan.export("tdescT")
    lists = plan.export(table)
    hcap = lists.shape[1]
    buf = plan._buf.cpu().numpy().copy()
    words = buf[: buf.size // 4 * 4].view(np.int32)
    first = lists[0, : used[0]]
    hits = []
    for off in range(0, words.size - lists.size + 1, 64):
        if words[off] != first[0] or not np.array_equal(words[off: off + used[0]], first):
            continue
        if all(np.array_equal(words[off + t * hcap: off + t * hcap + used[t]], lists[t, : used[t]])
               for t in range(lists.shape[0])):
            hits.append(off)
    assert len(hits) == 1, hits
    assert entry < used[0]
    words[hits[0] + entry] = value
    plan._buf.copy_(torch.from_numpy(buf).to(plan._buf.device))
    torch.cuda.synchronize()
    assert plan.export(table)[0, entry] == value


@pytest.mark.parametrize("precision", [0, 1])
def test_out_of_range_halo_index_is_clamped_and_flagged(precision):
    from paper_2306_01525_amd import MLBM_DEVERR_INDEX
    c, ux, uy, plan = _plan(precision)
    assert (plan.export("tdesc")[:, 1] > 0).all()     # every tile stages its halo
    g = plan.init(ux, uy)
    plan.step(g, plan.new_state(), 1)
    assert plan.device_error() == 0
    _corrupt_first_list(plan, "hlist", 5, c.n + 7)
    plan.step(g, plan.new_state(), 1)
    err = plan.device_error()
    say("precision %d: error bits after the corrupted halo %d" % (precision, err))
    assert err & MLBM_DEVERR_INDEX
    plan.close()


def test_out_of_range_inverse_halo_index_is_clamped_and_flagged():
    from paper_2306_01525_amd import MLBM_DEVERR_INDEX
    c, ux, uy, plan = _plan(1, with_adjoint=1)
    assert (plan.export("tdescT") > 0).all()
    f = plan.init_f(ux, uy)
    lam = torch.ones_like(f)
    dtau = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.step_adjoint(f, lam, torch.empty_like(f), dtau)
    assert plan.device_error() == 0
    _corrupt_first_list(plan, "ilist", 3, -5)
    plan.step_adjoint(f, lam, torch.empty_like(f), dtau)
    err = plan.device_error()
    say("error bits after the corrupted inverse halo %d" % err)
    assert err & MLBM_DEVERR_INDEX
    plan.close()
