"""Standard lattice Boltzmann on a periodic lattice (eq. LBM_streaming): the
reference method the paper compares MLBM against. Every step runs in the HIP
library; this module only allocates torch buffers and passes addresses."""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import MLBM_FP32_DEV, MLBM_FP64, check
from .mlbm import _f64, _ptr, _stream


class Lattice:
    """nx x ny periodic D2Q9 lattice, node (ix, iy) at index iy * nx + ix."""

    def __init__(self, nx: int, ny: int, tau: float, precision: int = MLBM_FP32_DEV,
                 rho0: float = 1.0, device="cuda"):
        self.nx, self.ny, self.n = int(nx), int(ny), int(nx) * int(ny)
        self.tau, self.precision, self.rho0 = float(tau), int(precision), float(rho0)
        self.device = device
        self.state_dtype = torch.float64 if precision == MLBM_FP64 else torch.float32
        _lib.load()

    def new_state(self):
        return torch.empty(9 * self.n, dtype=self.state_dtype, device=self.device)

    def init(self, ux, uy, rho=None, g=None, stream=None):
        g = self.new_state() if g is None else g
        ux, uy, rho = (_f64(a, self.device) for a in (ux, uy, rho))
        check(_lib.load().mlbm_lbm_init(self.nx, self.ny, self.precision, self.rho0, _ptr(rho),
                                        _ptr(ux), _ptr(uy), _ptr(g), _stream(stream)))
        return g

    def step(self, g_a, g_b, n_steps: int, stream=None):
        rb = ctypes.c_int32()
        check(_lib.load().mlbm_lbm_step(self.nx, self.ny, self.precision, self.tau, self.rho0,
                                        _ptr(g_a), _ptr(g_b), int(n_steps), ctypes.byref(rb),
                                        _stream(stream)))
        return g_b if rb.value else g_a

    def moments(self, g, stream=None):
        rho = torch.empty(self.n, dtype=torch.float64, device=self.device)
        ux, uy = torch.empty_like(rho), torch.empty_like(rho)
        check(_lib.load().mlbm_lbm_moments(self.nx, self.ny, self.precision, self.rho0, _ptr(g),
                                           _ptr(rho), _ptr(ux), _ptr(uy), _stream(stream)))
        return rho, ux, uy
