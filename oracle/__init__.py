"""Plain FP64 CPU oracle of the Meshless Lattice Boltzmann Method.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers. The GPU library never imports,
links or executes anything in this package, and this package imports nothing
from the GPU library.

The arithmetic lives in ``mlbm_oracle.c`` (built with gcc into
``_build/libmlbm_oracle.so``); this module only marshals numpy arrays.
Layouts are node-major: nbr [n][K], owner [n][9], W [n][9][K], f [n][9].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import analytic  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mlbm_oracle.c")
_INC = os.path.join(_HERE, "lbm_core.inc")
_LIB = os.path.join(_HERE, "_build", "libmlbm_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FMA contraction)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if not force and os.path.exists(_LIB) and \
            os.path.getmtime(_LIB) >= max(os.path.getmtime(_SRC), os.path.getmtime(_INC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=gnu11", "-fopenmp",
           "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double

_SIGS = {
    "orc_tables": (None, [_P, _P, _P, _P]),
    "orc_threads": (_I, []),
    "orc_set_threads": (None, [_I]),
    "orc_knn_one": (None, [_I, _P, _P, _D, _D, _I, _I, _P]),
    "orc_knn": (None, [_I, _P, _P, _D, _D, _I, _P]),
    "orc_nearest": (_I, [_I, _P, _P, _D, _D, _D, _D]),
    "orc_owners": (None, [_I, _P, _P, _D, _D, _D, _I, _P]),
    "orc_knn_cand": (_I, [_I, _P, _P, _D, _D, _I, _I, _P, _P]),
    "orc_owners_cand": (_I, [_I, _P, _P, _D, _D, _D, _I, _P, _P]),
    "orc_poly_count": (_I, [_I]),
    "orc_local_system": (_I, [_I, _I, _P, _P, _D, _D, _P, _P]),
    "orc_lu_solve": (_I, [_I, _P, _P, _P]),
    "orc_shape_vector": (_I, [_I, _I, _P, _P, _D, _D, _P]),
    "orc_weights": (_I, [_I, _P, _P, _D, _D, _D, _I, _I, _P, _P, _P]),
    "orc_feq": (None, [_D, _D, _D, _P]),
    "orc_equilibrium": (None, [_I, _P, _P, _P, _P]),
    "orc_moments": (None, [_I, _P, _P, _P, _P]),
    "orc_collide": (None, [_I, _P, _D, _P, _P, _P, _P]),
    "orc_stream": (None, [_I, _I, _P, _P, _P, _P, _P]),
    "orc_walls": (None, [_I, _P, _D, _P]),
    "orc_azimuthal_force": (None, [_I, _P, _P, _D, _P, _P, _P]),
    "orc_run": (None, [_I, _I, _P, _P, _P, _D, _P, _P, _P, _D, _I, _P]),
    "orc_run_links": (None, [_I, _I, _P, _P, _P, _D, _P, _P, _P, _I, _P]),
    "orc_bounce": (None, [_I, _P, _P]),
    "orc_lbm_run": (None, [_I, _I, _D, _I, _P]),
    "orc_loss_cs": (None, [_I, _I, _P, _P, _P, _D, _D, _I, _D, _P, _P, _P, _P, _P, _P,
                           _P, _P]),
    "orc_adjoint": (None, [_I, _I, _P, _P, _P, _D, _I, _D, _P, _P, _P, _P, _P, _P, _P,
                           _P]),
    "orc_stream_transpose": (None, [_I, _I, _P, _P, _P, _P, _P]),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# --------------------------------------------------------------------------
# D2Q9 tables
# --------------------------------------------------------------------------

def tables():
    ex, ey, w = np.zeros(9), np.zeros(9), np.zeros(9)
    opp = np.zeros(9, dtype=np.int32)
    lib().orc_tables(_p(ex), _p(ey), _p(w), _p(opp))
    return ex, ey, w, opp


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def knn(x, y, period, K):
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    nbr = np.empty((n, K), dtype=np.int32)
    lib().orc_knn(n, _p(x), _p(y), float(period[0]), float(period[1]), K, _p(nbr))
    return nbr


def knn_one(x, y, period, K, c):
    x, y = _f64(x), _f64(y)
    out = np.empty(K, dtype=np.int32)
    lib().orc_knn_one(x.shape[0], _p(x), _p(y), float(period[0]), float(period[1]), K,
                      int(c), _p(out))
    return out


def nearest(x, y, period, px, py):
    x, y = _f64(x), _f64(y)
    return int(lib().orc_nearest(x.shape[0], _p(x), _p(y), float(period[0]),
                                 float(period[1]), float(px), float(py)))


def owners(x, y, period, dx, mode):
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    own = np.empty((n, 9), dtype=np.int32)
    lib().orc_owners(n, _p(x), _p(y), float(period[0]), float(period[1]), float(dx),
                     int(mode), _p(own))
    return own


# Candidate lists for large clouds: scipy's k-d tree reports the C nearest
# nodes of every query point; the C functions take the exact answer from them
# (or fall back to brute force where the list cannot be shown to hold it).
KNN_EXTRA = 8        # candidates beyond K per stencil query
OWNER_CAND = 4       # candidates per departure point

last_fallbacks = {"knn": 0, "owners": 0}


def _tree(x, y, period):
    from scipy.spatial import cKDTree
    pts = np.stack([x, y], axis=1)
    periodic = period[0] > 0 and period[1] > 0
    return cKDTree(pts, boxsize=(period[0], period[1]) if periodic else None), periodic


def _wrap_query(px, py, period, periodic):
    if periodic:
        px = np.mod(px, period[0])
        py = np.mod(py, period[1])
        px[px >= period[0]] = 0.0
        py[py >= period[1]] = 0.0
    return np.stack([px, py], axis=1)


def knn_tree(x, y, period, K):
    """Same result as knn(), from k-d tree candidate lists."""
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    C = min(n, K + KNN_EXTRA)
    tree, periodic = _tree(x, y, period)
    _, cand = tree.query(_wrap_query(x.copy(), y.copy(), period, periodic), k=C,
                         workers=threads())
    cand = _i32(np.asarray(cand).reshape(n, C))
    nbr = np.empty((n, K), dtype=np.int32)
    last_fallbacks["knn"] = int(lib().orc_knn_cand(n, _p(x), _p(y), float(period[0]),
                                                   float(period[1]), K, C, _p(cand), _p(nbr)))
    return nbr


def owners_tree(x, y, period, dx, mode):
    """Same result as owners(), from k-d tree candidate lists (mode 0)."""
    if mode != 0:
        return owners(x, y, period, dx, mode)
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    ex, ey, _, _ = tables()
    px = (x[:, None] - ex[None, 1:] * dx).ravel()
    py = (y[:, None] - ey[None, 1:] * dx).ravel()
    C = min(n, OWNER_CAND)
    tree, periodic = _tree(x, y, period)
    _, cand = tree.query(_wrap_query(px, py, period, periodic), k=C, workers=threads())
    cand = _i32(np.asarray(cand).reshape(n * 8, C))
    own = np.empty((n, 9), dtype=np.int32)
    last_fallbacks["owners"] = int(lib().orc_owners_cand(
        n, _p(x), _p(y), float(period[0]), float(period[1]), float(dx), C, _p(cand), _p(own)))
    return own


# --------------------------------------------------------------------------
# RBF interpolation
# --------------------------------------------------------------------------

def poly_count(m):
    return int(lib().orc_poly_count(int(m)))


def local_system(rx, ry, px, py, m):
    rx, ry = _f64(rx), _f64(ry)
    K = rx.shape[0]
    nn = K + poly_count(m)
    Phi = np.empty((nn, nn))
    phi = np.empty(nn)
    lib().orc_local_system(K, int(m), _p(rx), _p(ry), float(px), float(py), _p(Phi),
                           _p(phi))
    return Phi, phi


def lu_solve(A, b):
    A = _f64(A).copy()
    b = _f64(b)
    x = np.empty_like(b)
    st = lib().orc_lu_solve(A.shape[0], _p(A), _p(b), _p(x))
    if st:
        raise np.linalg.LinAlgError("oracle LU: singular")
    return x


def shape_vector(rx, ry, px, py, m):
    rx, ry = _f64(rx), _f64(ry)
    w = np.empty(rx.shape[0])
    st = lib().orc_shape_vector(rx.shape[0], int(m), _p(rx), _p(ry), float(px),
                                float(py), _p(w))
    if st:
        raise np.linalg.LinAlgError("oracle shape vector: singular local system")
    return w


def weights(x, y, period, dx, K, m, nbr, own):
    x, y = _f64(x), _f64(y)
    nbr, own = _i32(nbr), _i32(own)
    n = x.shape[0]
    W = np.empty((n, 9, K))
    st = lib().orc_weights(n, _p(x), _p(y), float(period[0]), float(period[1]),
                           float(dx), K, int(m), _p(nbr), _p(own), _p(W))
    if st:
        raise np.linalg.LinAlgError("oracle weights: singular at node %d" % (-st - 1))
    return W


# --------------------------------------------------------------------------
# lattice Boltzmann
# --------------------------------------------------------------------------

def feq(rho, ux, uy):
    out = np.empty(9)
    lib().orc_feq(float(rho), float(ux), float(uy), _p(out))
    return out


def equilibrium(rho, ux, uy):
    rho, ux, uy = _f64(rho), _f64(ux), _f64(uy)
    f = np.empty((rho.shape[0], 9))
    lib().orc_equilibrium(rho.shape[0], _p(rho), _p(ux), _p(uy), _p(f))
    return f


def moments(f):
    f = _f64(f)
    n = f.shape[0]
    rho, ux, uy = np.empty(n), np.empty(n), np.empty(n)
    lib().orc_moments(n, _p(f), _p(rho), _p(ux), _p(uy))
    return rho, ux, uy


def collide(f, tau, ax=None, ay=None, node_type=None):
    f = _f64(f)
    out = np.empty_like(f)
    ax = None if ax is None else _f64(ax)
    ay = None if ay is None else _f64(ay)
    nt = None if node_type is None else np.ascontiguousarray(node_type, dtype=np.uint8)
    lib().orc_collide(f.shape[0], _p(f), float(tau), _p(ax), _p(ay), _p(nt), _p(out))
    return out


def stream(nbr, own, W, fpost):
    nbr, own, W, fpost = _i32(nbr), _i32(own), _f64(W), _f64(fpost)
    out = np.empty_like(fpost)
    lib().orc_stream(fpost.shape[0], nbr.shape[1], _p(nbr), _p(own), _p(W), _p(fpost),
                     _p(out))
    return out


def stream_transpose(nbr, own, W, lam):
    nbr, own, W, lam = _i32(nbr), _i32(own), _f64(W), _f64(lam)
    out = np.empty_like(lam)
    lib().orc_stream_transpose(lam.shape[0], nbr.shape[1], _p(nbr), _p(own), _p(W),
                               _p(lam), _p(out))
    return out


def walls(f, node_type, rho_w):
    f = _f64(f).copy()
    nt = np.ascontiguousarray(node_type, dtype=np.uint8)
    lib().orc_walls(f.shape[0], _p(nt), float(rho_w), _p(f))
    return f


def azimuthal_force(x, y, g, node_type=None):
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    ax, ay = np.empty(n), np.empty(n)
    nt = None if node_type is None else np.ascontiguousarray(node_type, dtype=np.uint8)
    lib().orc_azimuthal_force(n, _p(x), _p(y), float(g), _p(nt), _p(ax), _p(ay))
    return ax, ay


def bounce_links(nx, ny, node_type):
    """Populations that enter the fluid from outside at wall nodes: bit k-1 of
    the result is set where node_type != 0 and e_k . n < 0, n = the outward
    normal of the fluid domain (Sec. 3, bounce-back walls)."""
    ex, ey, _, _ = tables()
    nx, ny = _f64(nx), _f64(ny)
    nt = np.asarray(node_type)
    bits = (ex[None, 1:] * nx[:, None] + ey[None, 1:] * ny[:, None] < 0.0) & (nt[:, None] != 0)
    return (bits.astype(np.int64) << np.arange(8)).sum(axis=1).astype(np.uint8)


def bounce(f, links):
    f = _f64(f).copy()
    lk = np.ascontiguousarray(links, dtype=np.uint8)
    lib().orc_bounce(f.shape[0], _p(lk), _p(f))
    return f


def run(f, nbr, own, W, tau, steps, ax=None, ay=None, node_type=None, rho_w=1.0, links=None):
    """Advance f ([n][9], copied) by `steps` MLBM timesteps. With `links`
    (from bounce_links) the walls are the bounce-back rule and the force acts
    at every node; otherwise wall nodes (node_type) hold feq(rho_w, 0)."""
    f = _f64(f).copy()
    nbr, own, W = _i32(nbr), _i32(own), _f64(W)
    ax = None if ax is None else _f64(ax)
    ay = None if ay is None else _f64(ay)
    if links is not None:
        lk = np.ascontiguousarray(links, dtype=np.uint8)
        lib().orc_run_links(f.shape[0], nbr.shape[1], _p(nbr), _p(own), _p(W), float(tau),
                            _p(ax), _p(ay), _p(lk), int(steps), _p(f))
        return f
    nt = None if node_type is None else np.ascontiguousarray(node_type, dtype=np.uint8)
    lib().orc_run(f.shape[0], nbr.shape[1], _p(nbr), _p(own), _p(W), float(tau), _p(ax),
                  _p(ay), _p(nt), float(rho_w), int(steps), _p(f))
    return f


def lbm_run(f, nx, ny, tau, steps):
    """Standard LBM on a periodic nx x ny lattice (node iy*nx + ix)."""
    f = _f64(f).copy()
    lib().orc_lbm_run(int(nx), int(ny), float(tau), int(steps), _p(f))
    return f


def loss_cs(nbr, own, W, tau, steps, rho0, u0x, u0y, tx, ty, tau_im=0.0, u0x_im=None,
            u0y_im=None):
    nbr, own, W = _i32(nbr), _i32(own), _f64(W)
    n = nbr.shape[0]
    z = np.zeros(n)
    u0x, u0y, tx, ty = _f64(u0x), _f64(u0y), _f64(tx), _f64(ty)
    u0x_im = z if u0x_im is None else _f64(u0x_im)
    u0y_im = z if u0y_im is None else _f64(u0y_im)
    jr, ji = ctypes.c_double(), ctypes.c_double()
    lib().orc_loss_cs(n, nbr.shape[1], _p(nbr), _p(own), _p(W), float(tau), float(tau_im),
                      int(steps), float(rho0), _p(u0x), _p(u0x_im), _p(u0y), _p(u0y_im),
                      _p(tx), _p(ty), ctypes.byref(jr), ctypes.byref(ji))
    return jr.value, ji.value


def adjoint(nbr, own, W, tau, steps, rho0, u0x, u0y, tx, ty):
    """Returns (J, dJ/du0x, dJ/du0y, dJ/dtau)."""
    nbr, own, W = _i32(nbr), _i32(own), _f64(W)
    n = nbr.shape[0]
    u0x, u0y, tx, ty = _f64(u0x), _f64(u0y), _f64(tx), _f64(ty)
    gx, gy = np.empty(n), np.empty(n)
    J, gt = ctypes.c_double(), ctypes.c_double()
    lib().orc_adjoint(n, nbr.shape[1], _p(nbr), _p(own), _p(W), float(tau), int(steps),
                      float(rho0), _p(u0x), _p(u0y), _p(tx), _p(ty), ctypes.byref(J),
                      _p(gx), _p(gy), ctypes.byref(gt))
    return J.value, gx, gy, gt.value


# --------------------------------------------------------------------------
# whole-setup helpers
# --------------------------------------------------------------------------

def build_plan(cloud, dx, K, m, mode=0, search="brute"):
    """Stencils, owners and shape vectors of a cloud (Appendix A, init loop).
    search: "brute" scans every node per query; "tree" takes the same answers
    from k-d tree candidate lists (for clouds of 10^5 nodes and more)."""
    if search == "tree":
        nbr = knn_tree(cloud.x, cloud.y, cloud.period, K)
        own = owners_tree(cloud.x, cloud.y, cloud.period, dx, mode)
    else:
        nbr = knn(cloud.x, cloud.y, cloud.period, K)
        own = owners(cloud.x, cloud.y, cloud.period, dx, mode)
    W = weights(cloud.x, cloud.y, cloud.period, dx, K, m, nbr, own)
    return nbr, own, W
