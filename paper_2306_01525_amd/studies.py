"""The paper's convergence studies, run on the GPU.

* `tgv_error_map`: the Taylor-Green study of Sec. 3 (Fig. h_dx_explained and
  Fig. tgv_conv_P): the L2 error of the u-component at t_end over a grid of
  streaming distances dx_ML and node spacings h, for P2 and P4 augmentation.
* `lbm_errors`: the standard LBM on the same flow at dx = h (the black curve
  of Fig. tgv_conv_P).
* `interpolation_convergence`: interpolation alone (Sec. 4, Fig.
  interp_test), one build and one application of the streaming operator per
  cloud.
* `annulus_convergence`: the annular channel of Sec. 3 (Fig. bch_conv) with
  the paper's bounce-back walls and settings, run to the steady state.
* `annulus_workload_steady`: the ~490,000-node annular workload (equilibrium
  walls, tau = 0.7, K = 20, degree 3) from rest to the steady state.

Flow and scaling follow Sec. 3: the unit periodic square, u = U0 cos 2 pi x
sin 2 pi y, v = -U0 sin 2 pi x cos 2 pi y decaying as exp(-2 nu k^2 t) with
k = 2 pi, U0 = 1, nu = 1, tau = 0.8, dt = 1e-3 at dx = 1/10 and dt
proportional to dx^2 (diffusive scaling), t_end = ln 10 / (2 nu k^2), and the
number of steps is round(t_end / dt). The paper's Poisson-disk clouds are
replaced by lattices of side 1/h jittered by U[-0.3 h, 0.3 h] (seeded).

Run as `python -m paper_2306_01525_amd.studies` for the full maps (JSON on
stdout).
"""
from __future__ import annotations

import json
import math

import numpy as np

TWO_PI = 2.0 * math.pi
NU, U0, TAU = 1.0, 1.0, 0.8
T_END = math.log(10.0) / (2.0 * NU * TWO_PI ** 2)


def _dt(dx: float) -> float:
    """Diffusive scaling from dt = 1e-3 at dx = 1/10."""
    return 1e-3 * (dx / 0.1) ** 2


def _tgv_lattice_units(x, y, dx: float):
    """Initial velocity in lattice units (U0 dt / dx)."""
    s = U0 * _dt(dx) / dx
    return (s * np.cos(TWO_PI * x) * np.sin(TWO_PI * y),
            -s * np.sin(TWO_PI * x) * np.cos(TWO_PI * y))


def _steps(dx: float) -> int:
    return int(round(T_END / _dt(dx)))


def _decay(steps: int, dx: float) -> float:
    return math.exp(-2.0 * NU * TWO_PI ** 2 * steps * _dt(dx))


def tgv_error_map(dx_ml=(1 / 10, 1 / 40, 1 / 160),
                  hs=(1 / 10, 1 / 20, 1 / 40, 1 / 80, 1 / 160, 1 / 320),
                  degrees=(2, 4), K: int = 25, precision: int = 1, seed: int = 5,
                  stencil_mode: int = 0, device="cuda"):
    """One record per (dx_ML, h, degree): nodes, steps and the L2 error of the
    u-component at t_end (NaN when the run diverged)."""
    from .mlbm import Params, Plan
    from synth import jittered_lattice
    out = []
    for h in hs:
        n_side = int(round(1.0 / h))
        c = jittered_lattice(n_side, length=1.0, seed=seed + n_side)
        for dx in dx_ml:
            steps = _steps(dx)
            ux, uy = _tgv_lattice_units(c.x, c.y, dx)
            a = _decay(steps, dx)
            for m in degrees:
                p = Params(dx=dx, K=K, degree=m, tau=TAU, stencil_mode=stencil_mode,
                           precision=precision)
                plan = Plan.build(c.x, c.y, c.period, p, device=device)
                g = plan.step(plan.init(ux, uy), plan.new_state(), steps)
                l2 = plan.l2(g, a * ux, a * uy)[0]
                plan.close()
                out.append({"dx_ml": dx, "h": h, "degree": m, "nodes": c.n, "steps": steps,
                            "l2_u": l2 if math.isfinite(l2) else float("nan")})
    return out


def lbm_errors(dxs=(1 / 10, 1 / 20, 1 / 40, 1 / 80, 1 / 160), precision: int = 1,
               device="cuda"):
    """The standard LBM on the regular lattice of spacing dx, same flow."""
    from .lbm import Lattice
    out = []
    for dx in dxs:
        n = int(round(1.0 / dx))
        ix, iy = np.meshgrid(np.arange(n), np.arange(n))
        x, y = ix.ravel() * dx, iy.ravel() * dx
        steps = _steps(dx)
        ux, uy = _tgv_lattice_units(x, y, dx)
        lat = Lattice(n, n, TAU, precision, device=device)
        g = lat.step(lat.init(ux, uy), lat.new_state(), steps)
        _, u, _ = lat.moments(g)
        u = u.cpu().numpy()
        t = _decay(steps, dx) * ux
        out.append({"dx": dx, "nodes": n * n, "steps": steps,
                    "l2_u": float(np.linalg.norm(u - t) / np.linalg.norm(t))})
    return out


def interpolation_convergence(n_sides=(20, 40, 80, 160), degrees=(2, 4), K: int = 25,
                              dx: float = 0.1, seed: int = 11, stencil_mode: int = 0,
                              device="cuda"):
    """f = 0.01 sin 2 pi x cos 2 pi y on the unit periodic square, interpolated
    at every departure point x_i - e_k dx (k = 1..8); L2 error over all of them
    per cloud, and the least-squares slope of log L2 against log h."""
    from .mlbm import Params, Plan
    from synth import jittered_lattice
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
    records, slopes = [], {}
    for m in degrees:
        hs, errs = [], []
        for n in n_sides:
            c = jittered_lattice(n, length=1.0, seed=seed + n)
            p = Params(dx=dx, K=K, degree=m, tau=TAU, stencil_mode=stencil_mode, precision=1)
            plan = Plan.build(c.x, c.y, c.period, p, device=device)
            f = 0.01 * np.sin(TWO_PI * c.x) * np.cos(TWO_PI * c.y)
            got = plan.interpolate(f).cpu().numpy()
            plan.close()
            px = c.x[None, :] - ex[1:, None] * dx
            py = c.y[None, :] - ey[1:, None] * dx
            exact = 0.01 * np.sin(TWO_PI * px) * np.cos(TWO_PI * py)
            e = float(np.linalg.norm(got - exact) / np.linalg.norm(exact))
            records.append({"degree": m, "n_side": n, "h": 1.0 / n, "l2": e})
            hs.append(1.0 / n)
            errs.append(e)
        slopes[m] = float(np.polyfit(np.log(hs), np.log(errs), 1)[0])
    return records, slopes


def annulus_speed(r, dx: float, g: float, tau: float, r1: float = 1.0, r2: float = 2.0):
    """|u_phi| of eq. bch_solution in lattice units (r in cloud units)."""
    nu = (tau - 0.5) / 3.0
    rl, a, b = r / dx, r1 / dx, r2 / dx
    alpha = (a * a + a * b + b * b) / (a + b)
    beta = (a * a * b * b) / (a + b)
    return np.abs((g / (3.0 * nu)) * (rl * rl - alpha * rl + beta / rl))


def annulus_convergence(hs=(1 / 10, 1 / 20, 1 / 40, 1 / 55, 1 / 80, 1 / 110), dx: float = 1 / 160,
                        K: int = 15, degree: int = 2, tau: float = 1.0, g: float = 1e-6,
                        tol: float = 1e-10, max_steps: int = 500_000, precision: int = 1,
                        seed: int = 3, device="cuda"):
    """The annular channel of Sec. 3 with the paper's settings: R1 = 1, R2 = 2,
    azimuthal acceleration g (lattice units) at every node, bounce-back walls
    on boundary nodes placed on the circles, dx_ML = 1/160, tau = 1, N_L = 15
    with P2, from rest until the residual between checks 100 steps apart
    falls below `tol` (or a plateau, or max_steps). One record per h: nodes,
    steps, why the run stopped, the L2 error of the speed against eq.
    bch_solution and the largest speed at a wall node."""
    from .mlbm import Params, Plan
    from synth.clouds import annulus_poisson
    out = []
    for h in hs:
        c = annulus_poisson(1.0, 2.0, h, seed=seed)
        r = np.hypot(c.x, c.y)
        sgn = np.where(r < 1.5, -1.0, 1.0)          # outward normal of the fluid domain
        p = Params(dx=dx, K=K, degree=degree, tau=tau, stencil_mode=0, precision=precision,
                   force_kind=1, force_mag=g, wall_kind=2)
        plan = Plan.build(c.x, c.y, c.period, p, node_type=c.node_type, device=device,
                          normals=(sgn * c.x / r, sgn * c.y / r))
        zeros = np.zeros(c.n)
        # the start from rest rings with sound waves that make the residual
        # wander for a while: FP64 runs stop on the threshold or the limit only
        gs, steps, res, why = plan.run_to_steady(plan.init(zeros, zeros), tol=tol,
                                                 check_every=100, max_steps=max_steps,
                                                 plateau=None if precision == 1 else 50)
        _, u, v = (a.cpu().numpy() for a in plan.moments(gs))
        plan.close()
        U = np.hypot(u, v)
        exact = annulus_speed(r, dx, g, tau)
        out.append({"h": h, "nodes": c.n, "steps": steps, "residual": res, "stop": why,
                    "l2_speed": float(np.linalg.norm(U - exact) / np.linalg.norm(exact)),
                    "wall_speed_max": float(U[c.node_type == 1].max() / exact.max())})
    return out


def annulus_workload_steady(precision: int = 0, n_target: int = 500_000, tau: float = 0.7,
                            g: float | None = None, K: int = 20, degree: int = 3,
                            tol: float = 1e-8, max_steps: int = 500_000, plateau: int = 10,
                            check_every: int = 100, fixed_steps: int | None = None,
                            seed: int = 3, device="cuda"):
    """The annular-channel workload at full size run from rest to the steady
    state (Sec. 3, with the workload's walls and threshold): about 490,000
    Poisson-disk nodes between r = 1 and r = 2 (h chosen for n_target), dx =
    h, K = 20 with degree 3, the paper's stencil rule, tau = 0.7, equilibrium
    wall nodes, azimuthal acceleration g in lattice units (default: the
    paper's g = 1e-6 at dx_ML = 1/160 under diffusive scaling to h). Stops
    when the residual between checks `check_every` steps apart falls below
    `tol`, after `plateau` checks without a new minimum, or at max_steps; with
    fixed_steps, runs exactly that many steps instead. Returns the stop
    record, the L2 errors of the azimuthal velocity and of the speed against
    eq. bch_solution, the largest radial over the largest azimuthal speed, the
    wall speed, and the velocity field (user order) for comparisons."""
    import time as _time
    import torch
    from .mlbm import Params, Plan
    from .targets import annulus_azimuthal
    from synth.clouds import annulus_force, annulus_h_for_count, annulus_poisson
    c = annulus_poisson(1.0, 2.0, annulus_h_for_count(1.0, 2.0, n_target), seed=seed)
    g = annulus_force(c.h) if g is None else g
    p = Params(dx=c.h, K=K, degree=degree, tau=tau, stencil_mode=0, precision=precision,
               force_kind=1, force_mag=g, wall_kind=1, rho_wall=1.0)
    plan = Plan.build(c.x, c.y, c.period, p, node_type=c.node_type, device=device)
    zeros = np.zeros(c.n)
    torch.cuda.synchronize()
    t0 = _time.perf_counter()
    if fixed_steps is None:
        gs, steps, res, why = plan.run_to_steady(plan.init(zeros, zeros), tol=tol,
                                                 check_every=check_every, max_steps=max_steps,
                                                 plateau=plateau)
    else:
        gs = plan.step(plan.init(zeros, zeros), plan.new_state(), fixed_steps)
        steps, res, why = fixed_steps, float("nan"), "fixed"
    torch.cuda.synchronize()
    wall_s = _time.perf_counter() - t0
    _, u, v = (a.cpu().numpy() for a in plan.moments(gs))
    err = plan.device_error()
    plan.close()
    r = np.hypot(c.x, c.y)
    ut = (-u * c.y + v * c.x) / r
    ur = (u * c.x + v * c.y) / r
    exact = annulus_azimuthal(r, 1.0, 2.0, c.h, g, tau)
    fluid = c.node_type == 0
    return {"precision": precision, "nodes": c.n, "h": c.h, "g": g,
            "u_max_analytic": float(np.abs(exact).max()), "steps": steps, "stop": why,
            "residual": res, "seconds": wall_s, "device_error": err,
            "l2_u_phi": float(np.linalg.norm(ut - exact) / np.linalg.norm(exact)),
            "l2_speed": float(np.linalg.norm(np.hypot(u, v) - np.abs(exact)) /
                              np.linalg.norm(exact)),
            "max_radial_over_azimuthal": float(np.abs(ur[fluid]).max() / np.abs(exact).max()),
            "wall_speed_max": float(np.hypot(u, v)[~fluid].max()),
            "u": u, "v": v}


def main():
    res = {"tgv_error_map": tgv_error_map(), "lbm": lbm_errors(),
           "annulus": annulus_convergence()}
    rec, slopes = interpolation_convergence()
    res["interpolation"] = {"records": rec, "slopes": {str(k): v for k, v in slopes.items()}}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
