"""Thin Python binding of the MLBM C-ABI on top of PyTorch device memory.

Every computation runs in the HIP library; this module only allocates torch
buffers of the queried sizes, passes their addresses and the current stream,
and converts status codes into exceptions.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import MLBM_FP32_DEV, MLBM_FP64, MLBM_STENCIL_OWN, MLBM_STENCIL_PAPER  # noqa: F401
from ._lib import MLBMError, check


def _ptr(t):
    """Address of a tensor. The caller must hold a reference to `t` until the
    enqueued work has consumed it (a temporary freed here would be handed to
    the next allocation on the same stream)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _addr(t):
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _order(stream, *tensors):
    """Inputs staged on torch's current stream are consumed on `stream`: make
    `stream` wait for their copies and keep their memory until it is done."""
    if stream is None:
        return
    cur = torch.cuda.current_stream()
    if stream != cur:
        stream.wait_stream(cur)
        for t in tensors:
            if t is not None:
                t.record_stream(stream)


def _f64(t, device):
    if t is None:
        return None
    t = torch.as_tensor(t, dtype=torch.float64, device=device)
    return t.contiguous()


@dataclass
class Params:
    dx: float
    K: int
    degree: int
    tau: float
    stencil_mode: int = MLBM_STENCIL_PAPER
    precision: int = MLBM_FP32_DEV
    rho0: float = 1.0
    force_kind: int = 0
    force_mag: float = 0.0
    wall_kind: int = 0
    rho_wall: float = 1.0
    with_adjoint: int = 0
    fp32_weights_only: int = 0

    def to_c(self) -> _lib.Params:
        return _lib.Params(self.dx, self.K, self.degree, self.stencil_mode, self.precision,
                           self.tau, self.rho0, self.force_kind, self.force_mag,
                           self.wall_kind, self.rho_wall, self.with_adjoint,
                           self.fp32_weights_only)


class Plan:
    """A built MLBM plan: stencils, owners and shape vectors of one cloud."""

    def __init__(self, handle, plan_buf, params, n: int, device, sizes=None, keep=()):
        self._h = handle
        self._buf = plan_buf          # keeps the caller-owned plan memory alive
        self._keep = keep             # inputs a captured graph still reads
        self.params = params[0] if isinstance(params, (list, tuple)) else params
        self.params_list = list(params) if isinstance(params, (list, tuple)) else [params]
        self.n = n
        self.sizes = list(sizes) if sizes is not None else [n]
        self.offsets = [sum(self.sizes[:i]) for i in range(len(self.sizes))]
        self.device = device
        info = _lib.PlanInfo()
        check(_lib.load().mlbm_plan_get_info(self._h, ctypes.byref(info)))
        self.info = info
        self.state_dtype = torch.float64 if self.params.precision == MLBM_FP64 else torch.float32

    # ---- construction ----------------------------------------------------
    @classmethod
    def build(cls, x, y, period, params: Params, node_type=None, device="cuda",
              stream=None, normals=None, static_workspace=False):
        """normals: (nx, ny), the outward normal of the fluid domain at wall
        nodes (user order); needed by bounce-back walls (wall_kind 2).
        static_workspace: build through mlbm_build_weights_static (the
        library's own fixed workspace; no temporary device buffer)."""
        L = _lib.load()
        x = _f64(x, device)
        y = _f64(y, device)
        nt = None
        if node_type is not None:
            nt = torch.as_tensor(node_type, dtype=torch.uint8, device=device).contiguous()
        nx = ny = None
        if normals is not None:
            nx, ny = _f64(normals[0], device), _f64(normals[1], device)
        n = int(x.shape[0])
        _order(stream, x, y, nt, nx, ny)
        cloud = _lib.Cloud(n, x.data_ptr(), y.data_ptr(), nt.data_ptr() if nt is not None else None,
                           float(period[0]), float(period[1]), _addr(nx), _addr(ny))
        cp = params.to_c()
        pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        check(L.mlbm_weights_query(ctypes.byref(cloud), ctypes.byref(cp), 1, ctypes.byref(pb),
                                   ctypes.byref(wb)))
        plan_buf = torch.empty(pb.value, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        if static_workspace:
            check(L.mlbm_build_weights_static(ctypes.byref(cloud), ctypes.byref(cp), 1,
                                              _ptr(plan_buf), pb.value, ctypes.byref(h),
                                              _stream(stream)))
        else:
            ws = torch.empty(wb.value, dtype=torch.uint8, device=device)
            check(L.mlbm_build_weights(ctypes.byref(cloud), ctypes.byref(cp), 1, _ptr(plan_buf),
                                       pb.value, _ptr(ws), wb.value, ctypes.byref(h),
                                       _stream(stream)))
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        return cls(h, plan_buf, params, n, device)

    @staticmethod
    def _clouds(clouds, device):
        """clouds: list of (x, y, period, node_type or None[, (nx, ny) normals])."""
        keep, cs = [], []
        for cl in clouds:
            x, y, period, nt = cl[:4]
            xt, yt = _f64(x, device), _f64(y, device)
            ntt = None if nt is None else torch.as_tensor(nt, dtype=torch.uint8,
                                                          device=device).contiguous()
            nx = ny = None
            if len(cl) > 4 and cl[4] is not None:
                nx, ny = _f64(cl[4][0], device), _f64(cl[4][1], device)
            keep += [xt, yt, ntt, nx, ny]
            cs.append(_lib.Cloud(int(xt.shape[0]), xt.data_ptr(), yt.data_ptr(),
                                 ntt.data_ptr() if ntt is not None else None,
                                 float(period[0]), float(period[1]), _addr(nx), _addr(ny)))
        return (_lib.Cloud * len(cs))(*cs), keep

    @classmethod
    def build_batch(cls, clouds, params_list, device="cuda", stream=None):
        """One plan over several clouds; per-node arrays are concatenated in
        cloud order and the state is a flat tensor of [9][n_c] blocks."""
        L = _lib.load()
        carr, keep = cls._clouds(clouds, device)
        parr = (_lib.Params * len(params_list))(*[p.to_c() for p in params_list])
        _order(stream, *keep)
        pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        check(L.mlbm_weights_query(carr, parr, len(params_list), ctypes.byref(pb), ctypes.byref(wb)))
        plan_buf = torch.empty(pb.value, dtype=torch.uint8, device=device)
        ws = torch.empty(wb.value, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(L.mlbm_build_weights(carr, parr, len(params_list), _ptr(plan_buf), pb.value,
                                   _ptr(ws), wb.value, ctypes.byref(h), _stream(stream)))
        (torch.cuda.current_stream() if stream is None else stream).synchronize()
        sizes = [c.n for c in carr]
        return cls(h, plan_buf, list(params_list), sum(sizes), device, sizes)

    @classmethod
    def build_graph(cls, clouds, params_list, ux, uy, n_steps, stream, variant=0, rho=None,
                    device="cuda"):
        """Capture build + initial state + n_steps steps of all clouds into
        one HIP graph (nothing runs yet). Returns (plan, g_a, g_b, result):
        plan.graph_launch(stream) runs it; `result` holds the final state."""
        L = _lib.load()
        carr, keep = cls._clouds(clouds, device)
        parr = (_lib.Params * len(params_list))(*[p.to_c() for p in params_list])
        rho, ux, uy = (_f64(a, device) for a in (rho, ux, uy))
        keep += [rho, ux, uy]
        torch.cuda.current_stream().synchronize()
        pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        check(L.mlbm_weights_query(carr, parr, len(params_list), ctypes.byref(pb), ctypes.byref(wb)))
        plan_buf = torch.empty(pb.value, dtype=torch.uint8, device=device)
        ws = torch.empty(wb.value, dtype=torch.uint8, device=device)
        sizes = [c.n for c in carr]
        dt = torch.float64 if params_list[0].precision == MLBM_FP64 else torch.float32
        g_a = torch.empty(9 * sum(sizes), dtype=dt, device=device)
        g_b = torch.empty_like(g_a)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        check(L.mlbm_build_graph(carr, parr, len(params_list), _ptr(plan_buf), pb.value, _ptr(ws),
                                 wb.value, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(g_a), _ptr(g_b),
                                 int(n_steps), int(variant), ctypes.byref(h), _stream(stream)))
        plan = cls(h, plan_buf, list(params_list), sum(sizes), device, sizes,
                   keep=tuple(keep) + (ws,))
        return plan, g_a, g_b, (g_b if n_steps % 2 else g_a)

    def cloud_view(self, t, c):
        """[9][n_c] view of cloud c inside a state tensor, or the [n_c] slice of
        a per-node tensor."""
        o, n = self.offsets[c], self.sizes[c]
        if t.dim() == 1 and t.shape[0] == 9 * self.n:
            return t[9 * o: 9 * (o + n)].view(9, n)
        if t.dim() == 2 and len(self.sizes) == 1:
            return t
        return t[o: o + n]

    @classmethod
    def from_arrays(cls, x, y, nbr, owner, W, params: Params, node_type=None, device="cuda"):
        """Plan from host arrays (test hook): nbr [n][K], owner [n][9] (user
        indices), W [n][9][K] FP64; no reordering."""
        import numpy as np
        L = _lib.load()
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        owner = np.ascontiguousarray(owner, dtype=np.int32)
        W = np.ascontiguousarray(W, dtype=np.float64)
        n = x.shape[0]
        nt = None if node_type is None else np.ascontiguousarray(node_type, dtype=np.uint8)
        cp = params.to_c()
        pb = ctypes.c_size_t()
        check(L.mlbm_import_query(n, ctypes.byref(cp), ctypes.byref(pb)))
        plan_buf = torch.empty(pb.value, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        a = lambda arr: None if arr is None else arr.ctypes.data_as(ctypes.c_void_p)
        check(L.mlbm_import_weights(n, a(x), a(y), a(nt), a(nbr), a(owner), a(W),
                                    ctypes.byref(cp), _ptr(plan_buf), pb.value,
                                    ctypes.byref(h), _stream()))
        return cls(h, plan_buf, params, n, device)

    def close(self):
        if self._h:
            _lib.load().mlbm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state ---------------------------------------------------------------
    def new_state(self):
        if len(self.sizes) > 1:
            return torch.empty(9 * self.n, dtype=self.state_dtype, device=self.device)
        return torch.empty((9, self.n), dtype=self.state_dtype, device=self.device)

    def init(self, ux=None, uy=None, rho=None, g=None, stream=None):
        g = self.new_state() if g is None else g
        rho, ux, uy = (_f64(a, self.device) for a in (rho, ux, uy))
        _order(stream, rho, ux, uy)
        check(_lib.load().mlbm_init(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(g),
                                    _stream(stream)))
        return g

    def init_f(self, ux=None, uy=None, rho=None, f=None, stream=None):
        f = self.new_state() if f is None else f
        rho, ux, uy = (_f64(a, self.device) for a in (rho, ux, uy))
        _order(stream, rho, ux, uy)
        check(_lib.load().mlbm_init_f(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(f),
                                      _stream(stream)))
        return f

    def collide(self, f, g=None, stream=None):
        g = self.new_state() if g is None else g
        check(_lib.load().mlbm_collide(self._h, _ptr(f), _ptr(g), _stream(stream)))
        return g

    def step(self, g_a, g_b, n_steps: int, stream=None):
        """Advance n_steps; returns the buffer that holds the result."""
        rb = ctypes.c_int32()
        check(_lib.load().mlbm_step(self._h, _ptr(g_a), _ptr(g_b), int(n_steps),
                                    ctypes.byref(rb), _stream(stream)))
        return g_b if rb.value else g_a

    def step_record(self, g_a, g_b, n_steps: int, f_rec, stream=None):
        rb = ctypes.c_int32()
        check(_lib.load().mlbm_step_record(self._h, _ptr(g_a), _ptr(g_b), int(n_steps),
                                           _ptr(f_rec), ctypes.byref(rb), _stream(stream)))
        return g_b if rb.value else g_a

    def moments(self, g, stream=None):
        rho = torch.empty(self.n, dtype=torch.float64, device=self.device)
        ux = torch.empty_like(rho)
        uy = torch.empty_like(rho)
        check(_lib.load().mlbm_moments(self._h, _ptr(g), _ptr(rho), _ptr(ux), _ptr(uy),
                                       _stream(stream)))
        return rho, ux, uy

    def l2_sums(self, g, ux_t, uy_t, stream=None):
        out = torch.empty(4, dtype=torch.float64, device=self.device)
        ux_t, uy_t = _f64(ux_t, self.device), _f64(uy_t, self.device)
        _order(stream, ux_t, uy_t)
        check(_lib.load().mlbm_l2_sums(self._h, _ptr(g), _ptr(ux_t), _ptr(uy_t), _ptr(out),
                                       _stream(stream)))
        return out

    def interpolate(self, field, stream=None):
        """The streaming operator applied to a scalar field (user order):
        returns FP64 [8][n], row k-1 = the field interpolated at x_i - e_k dx."""
        field = _f64(field, self.device)
        out = torch.empty((8, self.n), dtype=torch.float64, device=self.device)
        _order(stream, field, out)
        check(_lib.load().mlbm_interpolate(self._h, _ptr(field), _ptr(out), _stream(stream)))
        return out

    def residual(self, g, speed, stream=None):
        """Relative change of the speed field since the check that filled
        `speed` (device FP64 [n], overwritten with the current speed)."""
        out = torch.empty(4, dtype=torch.float64, device=self.device)
        _order(stream, out)
        check(_lib.load().mlbm_residual(self._h, _ptr(g), _ptr(speed), _ptr(out), _stream(stream)))
        if stream is not None:
            torch.cuda.current_stream().wait_stream(stream)
        s = out.cpu().tolist()
        return (s[0] / s[1]) ** 0.5 if s[1] > 0 else float("inf")

    def run_to_steady(self, g, tol=1e-8, check_every=100, max_steps=500_000, plateau=10,
                      stream=None):
        """Step until the residual between checks `check_every` steps apart
        falls below `tol`, stops decreasing for `plateau` checks in a row
        (FP32 can level off above tol; plateau=None never stops on this), or
        `max_steps` is reached. Returns (state, steps, residual, reason) with
        reason 'tol', 'plateau' or 'max_steps'."""
        other = self.new_state()
        speed = torch.zeros(self.n, dtype=torch.float64, device=self.device)
        _order(stream, speed)
        self.residual(g, speed, stream)
        steps, best, stall, r = 0, float("inf"), 0, float("inf")
        while steps < max_steps:
            res = self.step(g, other, check_every, stream=stream)
            if res is other:
                g, other = other, g
            steps += check_every
            r = self.residual(g, speed, stream)
            if r < tol:
                return g, steps, r, "tol"
            if r < best:
                best, stall = r, 0
            else:
                stall += 1
                if plateau is not None and stall >= plateau:
                    return g, steps, r, "plateau"
        return g, steps, r, "max_steps"

    def l2(self, g, ux_t, uy_t):
        """(L2 of the u-component, L2 of the velocity vector), eq. L2norm."""
        s = self.l2_sums(g, ux_t, uy_t).cpu().tolist()
        return (s[2] / s[3]) ** 0.5, (s[0] / s[1]) ** 0.5

    # ---- adjoint ---------------------------------------------------------------
    def loss_seed(self, f_T, ux_t, uy_t, stream=None):
        lam = self.new_state()
        J = torch.empty(1, dtype=torch.float64, device=self.device)
        ux_t, uy_t = _f64(ux_t, self.device), _f64(uy_t, self.device)
        _order(stream, ux_t, uy_t)
        check(_lib.load().mlbm_loss_seed(self._h, _ptr(f_T), _ptr(ux_t), _ptr(uy_t), _ptr(lam),
                                         _ptr(J), _stream(stream)))
        return lam, J

    def step_adjoint(self, f_n, lam_next, lam_n, dtau, stream=None):
        check(_lib.load().mlbm_step_adjoint(self._h, _ptr(f_n), _ptr(lam_next), _ptr(lam_n),
                                            _ptr(dtau), _stream(stream)))
        return lam_n

    def init_adjoint(self, u0x, u0y, lam0, stream=None):
        gx = torch.empty(self.n, dtype=torch.float64, device=self.device)
        gy = torch.empty_like(gx)
        u0x, u0y = _f64(u0x, self.device), _f64(u0y, self.device)
        _order(stream, u0x, u0y)
        check(_lib.load().mlbm_init_adjoint(self._h, _ptr(u0x), _ptr(u0y), _ptr(lam0),
                                            _ptr(gx), _ptr(gy), _stream(stream)))
        return gx, gy

    # ---- tuning ----------------------------------------------------------------
    def autotune(self, g_a, g_b, n_steps: int = 20, stream=None):
        """Time every FP32 step variant on this cloud and keep the fastest;
        returns the milliseconds per step of each variant. Advances g_a/g_b."""
        ms = (ctypes.c_float * 16)()
        nv = ctypes.c_int32()
        check(_lib.load().mlbm_autotune(self._h, _ptr(g_a), _ptr(g_b), int(n_steps), ms,
                                        ctypes.byref(nv), _stream(stream)))
        self._refresh_info()
        return [ms[i] for i in range(nv.value)]

    def set_variant(self, v: int):
        check(_lib.load().mlbm_plan_set_variant(self._h, int(v)))
        self._refresh_info()

    def _refresh_info(self):
        info = _lib.PlanInfo()
        check(_lib.load().mlbm_plan_get_info(self._h, ctypes.byref(info)))
        self.info = info

    # ---- graphs ----------------------------------------------------------------
    def graph_create(self, g_a, g_b, n_steps: int, stream):
        check(_lib.load().mlbm_graph_create(self._h, _ptr(g_a), _ptr(g_b), int(n_steps),
                                            _stream(stream)))

    def graph_launch(self, stream):
        check(_lib.load().mlbm_graph_launch(self._h, _stream(stream)))

    # ---- inspection --------------------------------------------------------------
    def export(self, what: str):
        """Internal arrays: 'perm'; in user order 'nbr' [n][K], 'owner' [n][9],
        'W' [n][9][K] (FP64); tile tables of the FP32 step in internal order
        'tdesc' [ntiles][2], 'hlist' [ntiles][hcap], 'nbrL' [ntiles][ocap][ceil(K/3)]
        (three 10-bit halo positions per word),
        'ownerL' [8][n], 'caps' (ocap, hcap); adjoint tables (with_adjoint) 'tdescT'
        [ntiles], 'ilist' [ntiles][hcap], 'tr_ptr' [8n+1], and the row heads compacted
        per group of 64 nodes (see mlbm_plan_export): 'ell_col' [(K+4) n64][8],
        'elocal' [ceil((K+4)/3) n64][8], n64 = n rounded up to a multiple of 64."""
        import numpy as np
        K = self.params.K
        nt = (self.n + int(self.info.tile_nodes) - 1) // int(self.info.tile_nodes)
        codes = {"perm": 0, "nbr": 1, "owner": 2, "W": 3, "tdesc": 4, "hlist": 5, "nbrL": 6,
                 "ownerL": 7, "caps": 8, "tdescT": 9, "ilist": 10, "elocal": 11, "tr_ptr": 12,
                 "ell_col": 13}
        code = codes[what]
        lw = K + 4
        n64 = (self.n + 63) // 64 * 64
        if code in (5, 10):
            shape, dt = (nt, int(self.export("caps")[1])), np.int32
        elif code == 6:
            shape, dt = (nt, int(self.export("caps")[0]), (K + 2) // 3), np.uint32
        else:
            shape, dt = {0: ((self.n,), np.int32), 1: ((self.n, K), np.int32),
                         2: ((self.n, 9), np.int32), 3: ((self.n, 9, K), np.float64),
                         4: ((nt, 2), np.int32), 7: ((8, self.n), np.uint16),
                         8: ((2,), np.int32), 9: ((nt,), np.int32),
                         11: (((lw + 2) // 3 * n64, 8), np.uint32),
                         12: ((8 * self.n + 1,), np.int32),
                         13: ((lw * n64, 8), np.int32)}[code]
        out = np.empty(shape, dtype=dt)
        check(_lib.load().mlbm_plan_export(self._h, 0, code, out.ctypes.data_as(ctypes.c_void_p),
                                           out.nbytes))
        return out

    def set_tau(self, tau: float):
        """Same relaxation time for every cloud of the plan."""
        check(_lib.load().mlbm_plan_set_tau(self._h, float(tau)))
        for p in self.params_list:
            p.tau = float(tau)

    def device_error(self) -> int:
        """Sticky device error bits (MLBM_DEVERR_*), 0 when none."""
        return int(_lib.load().mlbm_device_error(self._h))

    def device_error_nodes(self):
        """(first singular node, first diverged node), user indices, -1 = none."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(_lib.load().mlbm_device_error_nodes(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def clear_device_error(self, stream=None):
        check(_lib.load().mlbm_device_error_clear(self._h, _stream(stream)))
