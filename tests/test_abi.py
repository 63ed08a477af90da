"""The C-ABI library loads and exports every entry point that include/mlbm.h
declares; host-side argument checks work without a GPU (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mlbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mlbm_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2306_01525_amd import _lib
    L = _lib.load()
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding knows every declared entry point
    assert set(names) <= set(_lib.SIGNATURES), set(names) - set(_lib.SIGNATURES)


def _query(n=100, **kw):
    from paper_2306_01525_amd import _lib
    L = _lib.load()
    p = dict(dx=0.1, K=12, degree=2, stencil_mode=0, precision=0, tau=0.8, rho0=1.0,
             force_kind=0, force_mag=0.0, wall_kind=0, rho_wall=1.0, with_adjoint=0)
    p.update(kw)
    cp = _lib.Params(**p)
    cl = _lib.Cloud(n, None, None, None, 1.0, 1.0, None, None)
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    st = L.mlbm_weights_query(ctypes.byref(cl), ctypes.byref(cp), 1, ctypes.byref(pb),
                              ctypes.byref(wb))
    return st, pb.value, wb.value


def test_query_sizes_grow_with_problem():
    st, pb, wb = _query()
    assert st == 0 and pb > 0 and wb > 0
    st2, pb2, _ = _query(n=1000)
    assert st2 == 0 and pb2 > pb
    st3, pb3, _ = _query(precision=1)
    assert st3 == 0
    st4, pb4, _ = _query(with_adjoint=1)
    assert st4 == 0 and pb4 > pb


@pytest.mark.parametrize("kw,code", [
    (dict(degree=1), -1), (dict(degree=5), -1), (dict(K=5), -1), (dict(K=8, degree=3), -1),
    (dict(tau=0.5), -1), (dict(dx=0.0), -1), (dict(dx=0.6), -1), (dict(precision=7), -1),
    (dict(stencil_mode=3), -1), (dict(K=49), -1), (dict(n=10), -1),
    (dict(with_adjoint=1, force_kind=1), -5),
    (dict(with_adjoint=1, K=48, degree=4, n=5_600_000), -5), (dict(K=6, n=268_435_456), -5),
    (dict(fp32_weights_only=1, precision=1), -1), (dict(fp32_weights_only=2), -1),
])
def test_query_rejects_invalid(kw, code):
    st, _, _ = _query(**kw)
    assert st == code
    from paper_2306_01525_amd import _lib
    assert len(_lib.load().mlbm_last_error()) > 0


def test_fp32_weights_only_moves_the_fp64_shape_vectors_to_the_workspace():
    """The FP64 shape vectors (8 directions x K doubles per node) leave the
    plan for the workspace; imported plans keep them and refuse the flag."""
    import ctypes
    from paper_2306_01525_amd import _lib
    n, K = 1000, 12
    st0, pb0, wb0 = _query(n=n, K=K)
    st1, pb1, wb1 = _query(n=n, K=K, fp32_weights_only=1)
    assert st0 == st1 == 0
    assert pb0 - pb1 >= 8 * K * n * 8 and wb1 - wb0 >= 8 * K * n * 8
    p = _lib.Params(dx=0.1, K=K, degree=2, stencil_mode=0, precision=0, tau=0.8, rho0=1.0,
                    fp32_weights_only=1)
    size = ctypes.c_size_t()
    assert _lib.load().mlbm_import_query(n, ctypes.byref(p), ctypes.byref(size)) == -5


PLAN_CALLS = {   # entry point -> its arguments after the plan (pointers null)
    "mlbm_plan_get_info": [None],
    "mlbm_plan_export": [0, 0, None, 0],
    "mlbm_plan_set_tau": [0.8],
    "mlbm_plan_set_variant": [1],
    "mlbm_init": [None, None, None, None, None],
    "mlbm_init_f": [None, None, None, None, None],
    "mlbm_collide": [None, None, None],
    "mlbm_step": [None, None, 1, None, None],
    "mlbm_step_record": [None, None, 1, None, None, None],
    "mlbm_moments": [None, None, None, None, None],
    "mlbm_l2_sums": [None, None, None, None, None],
    "mlbm_interpolate": [None, None, None],
    "mlbm_residual": [None, None, None, None],
    "mlbm_loss_seed": [None, None, None, None, None, None],
    "mlbm_step_adjoint": [None, None, None, None, None],
    "mlbm_init_adjoint": [None, None, None, None, None, None],
    "mlbm_autotune": [None, None, 1, None, None, None],
    "mlbm_graph_create": [None, None, 1, None],
    "mlbm_graph_launch": [None],
    "mlbm_device_error_nodes": [None, None],
    "mlbm_device_error_clear": [None],
}


@pytest.mark.parametrize("name", sorted(PLAN_CALLS))
def test_plan_calls_reject_a_null_plan(name):
    """Every entry point that takes a plan returns MLBM_EINVAL for a null one
    (checked before any device work), with a message."""
    from paper_2306_01525_amd import _lib
    L = _lib.load()
    assert getattr(L, name)(None, *PLAN_CALLS[name]) == -1
    assert len(L.mlbm_last_error()) > 0


def test_null_plan_device_error_and_destroy():
    from paper_2306_01525_amd import _lib
    L = _lib.load()
    assert L.mlbm_device_error(None) == 0
    assert L.mlbm_plan_destroy(None) == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2306_01525_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        _lib.load()
