"""The export layout of the compacted adjoint heads (items 11 and 13 of
mlbm_plan_export), checked on the CPU: units written one by one with the
formula of the header (group g from unit 64 g lw; slot e a block of c units
for the group's nodes with hd > e, in node order; entry k-1 of unit r of a
block starting at unit u0 at element 8 u0 + 4 ((k-1)/4 c + r) + (k-1)%4)
are read back by the decoder the GPU tests use."""
import numpy as np

from test_gpu_build import _uncompact


def test_uncompact_inverts_the_documented_layout():
    rng = np.random.default_rng(1)
    n, lw = 150, 7                      # a partial last group of 64
    hd = rng.integers(0, lw + 1, n)
    hd[64:128] = 0                      # a group with no units at all
    n64 = (n + 63) // 64 * 64
    src = rng.integers(0, 1000, (8, lw, n))
    units = np.full((n64 * lw, 8), -5)
    flat = units.reshape(-1)
    for g in range(n64 // 64):
        off = 0
        for e in range(lw):
            lanes = [l for l in range(64) if g * 64 + l < n and hd[g * 64 + l] > e]
            c, u0 = len(lanes), g * 64 * lw + off
            for r, l in enumerate(lanes):
                for k in range(8):
                    flat[8 * u0 + 4 * ((k // 4) * c + r) + k % 4] = src[k, e, g * 64 + l]
            off += c
    out = _uncompact(units, hd, lw, n, -1)
    mask = np.broadcast_to(np.arange(lw)[None, :, None] < hd[None, None, :], out.shape)
    assert (out[mask] == src[mask]).all()
    assert (out[~mask] == -1).all()
