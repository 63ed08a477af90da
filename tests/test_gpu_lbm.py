"""Standard lattice Boltzmann on the GPU (eq. LBM_streaming) against the
oracle's index-shift LBM, and the regular-lattice special case of the MLBM
(unit-vector shape vectors) against it on the GPU."""
import numpy as np
import pytest

import oracle
from gpu_common import TOL_FP64, rel_l2, say, tol_fp32
from synth import tgv_initial_velocity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _tgv_lattice(nx, ny, u0=0.01):
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny))
    x, y = ix.ravel().astype(float), iy.ravel().astype(float)
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    ux = u0 * np.sin(kx * x) * np.cos(ky * y)
    uy = -u0 * (kx / ky) * np.cos(kx * x) * np.sin(ky * y)
    return x, y, ux, uy


@pytest.mark.parametrize("nx,ny", [(40, 32), (37, 29), (1, 5)])
def test_lbm_matches_oracle(nx, ny):
    """Non-square and odd lattices (x/y mix-ups and wrap errors show), and a
    one-column lattice where every x shift wraps onto itself."""
    from paper_2306_01525_amd._lib import MLBM_FP32_DEV, MLBM_FP64
    from paper_2306_01525_amd.lbm import Lattice
    x, y, ux, uy = _tgv_lattice(nx, ny)
    rng = np.random.default_rng(nx * 100 + ny)
    rho = 1.0 + 1e-3 * rng.standard_normal(nx * ny)
    tau, steps = 0.8, 150
    f = oracle.equilibrium(rho, ux, uy)
    f = oracle.lbm_run(f, nx, ny, tau, steps)
    r_o, u_o, v_o = oracle.moments(f)
    for prec, tol in ((MLBM_FP64, TOL_FP64), (MLBM_FP32_DEV, tol_fp32(steps))):
        lat = Lattice(nx, ny, tau, prec)
        g = lat.init(ux, uy, rho=rho)
        g = lat.step(g, lat.new_state(), steps)
        r_g, u_g, v_g = (a.cpu().numpy() for a in lat.moments(g))
        # relative to the initial field: on the one-column lattice the flow
        # decays by e^-47 in 150 steps, and only rounding-level noise is left
        e = float(np.linalg.norm(np.stack([u_g - u_o, v_g - v_o])) /
                  np.linalg.norm(np.stack([ux, uy])))
        er = float(np.abs(r_g - r_o).max())
        say("lattice %dx%d precision %d: rel L2 velocity %.2e, max |drho| %.2e" % (nx, ny, prec, e, er))
        assert e < tol and er < tol


def test_lbm_rejects_bad_arguments():
    from paper_2306_01525_amd import MLBMError
    from paper_2306_01525_amd.lbm import Lattice
    lat = Lattice(8, 8, 0.8)
    g = lat.new_state()
    with pytest.raises(MLBMError):
        lat.step(g, g, 1)
    with pytest.raises(MLBMError):
        Lattice(8, 8, 0.5).step(g, lat.new_state(), 1)
    with pytest.raises(MLBMError):
        Lattice(0, 8, 0.8).init(np.zeros(0), np.zeros(0))


@pytest.mark.parametrize("mode", [0, 1])
def test_mlbm_on_regular_lattice_equals_lbm(mode):
    """No jitter and dx = h: every departure point is a node, its shape vector
    is a unit vector, and the MLBM step is the index-shift step. With the
    paper's rule the departure node is its own owner and the unit vector is
    exact; with own-node stencils it comes out of the local solve, exact up to
    that solve's rounding (about 1e-14 per step)."""
    from paper_2306_01525_amd import Params, Plan
    from paper_2306_01525_amd._lib import MLBM_FP64
    from paper_2306_01525_amd.lbm import Lattice
    n_side, tau, steps = 32, 0.7, 200
    x, y, ux, uy = _tgv_lattice(n_side, n_side)
    p = Params(dx=1.0, K=12, degree=2, tau=tau, stencil_mode=mode, precision=MLBM_FP64)
    plan = Plan.build(x, y, (float(n_side), float(n_side)), p)
    gm = plan.step(plan.init(ux, uy), plan.new_state(), steps)
    _, um, vm = (a.cpu().numpy() for a in plan.moments(gm))
    plan.close()
    lat = Lattice(n_side, n_side, tau, MLBM_FP64)
    gl = lat.step(lat.init(ux, uy), lat.new_state(), steps)
    _, ul, vl = (a.cpu().numpy() for a in lat.moments(gl))
    e = rel_l2(np.stack([um, vm]), np.stack([ul, vl]))
    say("mode %d: MLBM on the lattice vs LBM after %d steps: %.2e" % (mode, steps, e))
    assert e < TOL_FP64
