"""ctypes view of include/mlbm.h. Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libmlbm.so")

MLBM_OK = 0
MLBM_EINVAL = -1
MLBM_ESINGULAR = -2
MLBM_EHIP = -3
MLBM_ESMALLBUF = -4
MLBM_EUNSUPPORTED = -5

MLBM_FP32_DEV = 0
MLBM_FP64 = 1
# sticky device error bits (mlbm_device_error)
MLBM_DEVERR_SINGULAR = 1
MLBM_DEVERR_INDEX = 2
MLBM_DEVERR_NONFINITE = 4
MLBM_DEVERR_SPEED = 8
MLBM_STENCIL_PAPER = 0
MLBM_STENCIL_OWN = 1

_c_i32 = ctypes.c_int32
_c_i64 = ctypes.c_int64
_c_d = ctypes.c_double
_c_p = ctypes.c_void_p
_c_sz = ctypes.c_size_t


class Cloud(ctypes.Structure):
    _fields_ = [("n", _c_i32), ("x", _c_p), ("y", _c_p), ("node_type", _c_p),
                ("period_x", _c_d), ("period_y", _c_d), ("normal_x", _c_p), ("normal_y", _c_p)]


class Params(ctypes.Structure):
    _fields_ = [("dx", _c_d), ("K", _c_i32), ("degree", _c_i32), ("stencil_mode", _c_i32),
                ("precision", _c_i32), ("tau", _c_d), ("rho0", _c_d), ("force_kind", _c_i32),
                ("force_mag", _c_d), ("wall_kind", _c_i32), ("rho_wall", _c_d),
                ("with_adjoint", _c_i32), ("fp32_weights_only", _c_i32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_clouds", _c_i32), ("n_total", _c_i64), ("K", _c_i32), ("degree", _c_i32),
                ("stencil_mode", _c_i32), ("precision", _c_i32), ("state_bytes", _c_sz),
                ("tile_nodes", _c_i64), ("step_lds_bytes", _c_i32), ("fallback_tiles", _c_i32),
                ("variant", _c_i32)]


_P = ctypes.POINTER
# name -> (restype, argtypes); every symbol declared in include/mlbm.h
SIGNATURES = {
    "mlbm_weights_query": (_c_i32, [_P(Cloud), _P(Params), _c_i32, _P(_c_sz), _P(_c_sz)]),
    "mlbm_build_weights": (_c_i32, [_P(Cloud), _P(Params), _c_i32, _c_p, _c_sz, _c_p, _c_sz,
                                    _P(_c_p), _c_p]),
    "mlbm_import_query": (_c_i32, [_c_i32, _P(Params), _P(_c_sz)]),
    "mlbm_import_weights": (_c_i32, [_c_i32, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _P(Params),
                                     _c_p, _c_sz, _P(_c_p), _c_p]),
    "mlbm_plan_get_info": (_c_i32, [_c_p, _P(PlanInfo)]),
    "mlbm_plan_export": (_c_i32, [_c_p, _c_i32, _c_i32, _c_p, _c_sz]),
    "mlbm_plan_destroy": (_c_i32, [_c_p]),
    "mlbm_plan_set_tau": (_c_i32, [_c_p, _c_d]),
    "mlbm_init": (_c_i32, [_c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "mlbm_init_f": (_c_i32, [_c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "mlbm_collide": (_c_i32, [_c_p, _c_p, _c_p, _c_p]),
    "mlbm_step": (_c_i32, [_c_p, _c_p, _c_p, _c_i32, _P(_c_i32), _c_p]),
    "mlbm_step_record": (_c_i32, [_c_p, _c_p, _c_p, _c_i32, _c_p, _P(_c_i32), _c_p]),
    "mlbm_moments": (_c_i32, [_c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "mlbm_l2_sums": (_c_i32, [_c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "mlbm_residual": (_c_i32, [_c_p, _c_p, _c_p, _c_p, _c_p]),
    "mlbm_interpolate": (_c_i32, [_c_p, _c_p, _c_p, _c_p]),
    "mlbm_lbm_init": (_c_i32, [_c_i32, _c_i32, _c_i32, _c_d, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "mlbm_lbm_step": (_c_i32, [_c_i32, _c_i32, _c_i32, _c_d, _c_d, _c_p, _c_p, _c_i32, _c_p,
                               _c_p]),
    "mlbm_lbm_moments": (_c_i32, [_c_i32, _c_i32, _c_i32, _c_d, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "mlbm_loss_seed": (_c_i32, [_c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "mlbm_step_adjoint": (_c_i32, [_c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "mlbm_init_adjoint": (_c_i32, [_c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "mlbm_autotune": (_c_i32, [_c_p, _c_p, _c_p, _c_i32, _c_p, _P(_c_i32), _c_p]),
    "mlbm_plan_set_variant": (_c_i32, [_c_p, _c_i32]),
    "mlbm_build_graph": (_c_i32, [_P(Cloud), _P(Params), _c_i32, _c_p, _c_sz, _c_p, _c_sz,
                                  _c_p, _c_p, _c_p, _c_p, _c_p, _c_i32, _c_i32, _P(_c_p), _c_p]),
    "mlbm_graph_create": (_c_i32, [_c_p, _c_p, _c_p, _c_i32, _c_p]),
    "mlbm_graph_launch": (_c_i32, [_c_p, _c_p]),
    "mlbm_last_error": (ctypes.c_char_p, []),
    "mlbm_device_error": (_c_i32, [_c_p]),
    "mlbm_build_weights_static": (_c_i32, [_P(Cloud), _P(Params), _c_i32, _c_p, _c_sz, _P(_c_p),
                                           _c_p]),
    "mlbm_device_error_nodes": (_c_i32, [_c_p, _P(_c_i32), _P(_c_i32)]),
    "mlbm_device_error_clear": (_c_i32, [_c_p, _c_p]),
}

_lib = None


class MLBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("mlbm status %d: %s" % (status, msg))
        self.status = status


def load():
    """Load the built HIP library; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("the MLBM HIP library is not built (%s missing); run "
                              "paper_2306_01525_amd.build.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != MLBM_OK:
        raise MLBMError(status, load().mlbm_last_error().decode(errors="replace"))
