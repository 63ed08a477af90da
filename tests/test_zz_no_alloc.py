"""mlbm_build_weights_static, the build for callers that cannot allocate:
its plans equal those of mlbm_build_weights with a caller workspace, on two
calls in a row (the second on a smaller cloud, over what the first left in
the library's fixed workspace), and a build that needs more than the fixed
workspace is refused before any device work."""
import ctypes

import numpy as np
import pytest

from gpu_common import say, tgv_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ITEMS = ("perm", "nbr", "owner", "W", "tdesc", "hlist", "nbrL", "ownerL", "caps")


def _compare(c, ux, uy, p):
    from paper_2306_01525_amd import Plan
    ref = Plan.build(c.x, c.y, c.period, p)
    got = Plan.build(c.x, c.y, c.period, p, static_workspace=True)
    for item in ITEMS + (("tdescT", "ilist", "tr_ptr") if p.with_adjoint else ()):
        a, b = ref.export(item), got.export(item)
        if item in ("hlist", "nbrL", "ilist"):   # the used part of each tile's list
            td = ref.export("tdescT") if item == "ilist" else ref.export("tdesc")
            for t in range(td.shape[0]):
                u = td[t] if item == "ilist" else (td[t, 1] if item == "hlist" else td[t, 0])
                np.testing.assert_array_equal(a[t, :u], b[t, :u], err_msg=item)
        else:
            np.testing.assert_array_equal(a, b, err_msg=item)
    ga = ref.step(ref.init(ux, uy), ref.new_state(), 7)
    gb = got.step(got.init(ux, uy), got.new_state(), 7)
    assert torch.equal(ga, gb)
    if p.with_adjoint:   # the transposed operator, through one reversed step
        f = ref.init_f(ux, uy)
        lam = torch.linspace(-1.0, 1.0, f.numel(), device="cuda").reshape(f.shape).to(f.dtype)
        out = []
        for plan in (ref, got):
            dtau = torch.zeros(1, dtype=torch.float64, device="cuda")
            lam_n = torch.empty_like(f)
            plan.step_adjoint(f, lam, lam_n, dtau)
            out.append((lam_n, dtau))
        assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    assert got.device_error() == 0
    say("n %d K %d adjoint %d: static-workspace plan equal to the caller-workspace plan"
        % (c.n, p.K, p.with_adjoint))
    ref.close()
    got.close()


def test_static_workspace_build_equals_caller_workspace_build_twice():
    from paper_2306_01525_amd import Params
    c1, ux1, uy1 = tgv_case(96, 30, 4, 0, seed=11)
    c2, ux2, uy2 = tgv_case(37, 20, 3, 0, seed=12)
    for c, ux, uy, K, m, adj in ((c1, ux1, uy1, 30, 4, 1), (c2, ux2, uy2, 20, 3, 0)):
        p = Params(dx=c.h, K=K, degree=m, tau=0.7, stencil_mode=0, precision=0,
                   with_adjoint=adj)
        _compare(c, ux, uy, p)


def test_static_workspace_refuses_a_build_beyond_its_size():
    from paper_2306_01525_amd import Params, _lib
    from paper_2306_01525_amd._lib import MLBM_EUNSUPPORTED
    n = 1_200_000
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    p = Params(dx=0.01, K=30, degree=4, tau=0.7, stencil_mode=0, precision=0).to_c()
    cl = _lib.Cloud(n, x.data_ptr(), x.data_ptr(), None, 1.0, 1.0, None, None)
    L = _lib.load()
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.mlbm_weights_query(ctypes.byref(cl), ctypes.byref(p), 1, ctypes.byref(pb),
                                ctypes.byref(wb)) == 0
    h = ctypes.c_void_p()
    st = L.mlbm_build_weights_static(ctypes.byref(cl), ctypes.byref(p), 1, None, pb.value,
                                     ctypes.byref(h), None)
    msg = L.mlbm_last_error().decode()
    say("refused:", msg)
    assert st == MLBM_EUNSUPPORTED and "static workspace" in msg and not h.value
