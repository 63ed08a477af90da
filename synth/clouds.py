"""Seeded point clouds shaped like the paper's workloads.

* Taylor-Green clouds: a square periodic domain discretised by a regular
  lattice whose nodes are displaced independently in x and y by a uniform
  random offset (a stand-in for the relaxed Poisson-disk clouds of the paper's
  Taylor-Green study, Sec. 3, whose node files are not available).
* Annular channel: boundary nodes equally spaced on both walls plus an interior
  Poisson-disk sample with minimum spacing h (the paper's annulus, Sec. 3,
  is discretised this way with boundary nodes placed exactly on the walls).
* Batched: a list of Taylor-Green cloud specifications of uneven size.

Every draw uses numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class Cloud:
    x: np.ndarray                  # float64 [n]
    y: np.ndarray                  # float64 [n]
    node_type: np.ndarray | None   # uint8 [n]: 0 fluid, 1 wall; None = all fluid
    period: tuple[float, float]    # (Lx, Ly) > 0 periodic; (0, 0) open
    h: float                       # nominal node spacing

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _wrap(v: np.ndarray, length: float) -> np.ndarray:
    v = np.mod(v, length)
    v[v >= length] -= length
    v[v < 0.0] = 0.0
    return v


def jittered_lattice(n_side: int, length: float = TWO_PI, jitter: float = 0.3,
                     seed: int = 0, ny: int | None = None,
                     length_y: float | None = None) -> Cloud:
    """n_side x ny lattice on [0,Lx) x [0,Ly), node (ix, iy) at (ix*h, iy*h),
    each coordinate displaced by U[-jitter*h, +jitter*h] and wrapped.
    User order is row-major with x fastest."""
    ny = n_side if ny is None else ny
    length_y = length if length_y is None else length_y
    hx = length / n_side
    hy = length_y / ny
    ix, iy = np.meshgrid(np.arange(n_side, dtype=np.float64),
                         np.arange(ny, dtype=np.float64), indexing="xy")
    x = (ix * hx).ravel()
    y = (iy * hy).ravel()
    if jitter:
        rng = _rng(seed)
        x = x + rng.uniform(-jitter * hx, jitter * hx, x.shape[0])
        y = y + rng.uniform(-jitter * hy, jitter * hy, y.shape[0])
    x = _wrap(x, length)
    y = _wrap(y, length_y)
    return Cloud(np.ascontiguousarray(x), np.ascontiguousarray(y), None,
                 (float(length), float(length_y)), float(min(hx, hy)))


def annulus_poisson(r_in: float, r_out: float, h: float, seed: int = 0,
                    rounds: int = 24) -> Cloud:
    """Annulus r_in <= r <= r_out. Wall nodes: round(2*pi*r/h) equally spaced
    nodes on each circle (node_type 1). Interior: Poisson-disk sample with
    minimum spacing h, drawn by phased parallel dart throwing on a background
    grid of cell size h/sqrt(2) (at most one point per cell; cells processed in
    3x3 phases so that concurrent candidates cannot conflict)."""
    rng = _rng(seed)
    pts_x: list[np.ndarray] = []
    pts_y: list[np.ndarray] = []
    for r in (r_in, r_out):
        nb = int(round(TWO_PI * r / h))
        phi = (np.arange(nb) + 0.5) * (TWO_PI / nb)
        pts_x.append(r * np.cos(phi))
        pts_y.append(r * np.sin(phi))
    bx = np.concatenate(pts_x)
    by = np.concatenate(pts_y)

    cell = h / math.sqrt(2.0)
    lo = -r_out - 2 * cell
    g = int(math.ceil((2 * r_out + 4 * cell) / cell)) + 1
    cap = bx.shape[0] + int(1.2 * math.pi * (r_out ** 2 - r_in ** 2) / (cell * cell))
    # point store with a far-away sentinel at index `cap`; the background grid
    # (flattened, g x g) holds a point index per cell or the sentinel
    px = np.full(cap + 1, 1e18)
    py = np.full(cap + 1, 1e18)
    grid = np.full(g * g, cap, dtype=np.int64)
    count = 0

    def insert(xs, ys):
        nonlocal count
        cx = ((xs - lo) / cell).astype(np.int64)
        cy = ((ys - lo) / cell).astype(np.int64)
        k = xs.shape[0]
        px[count:count + k] = xs
        py[count:count + k] = ys
        # wall nodes may share a cell: the grid keeps the last, and interior
        # candidates are checked against the wall nodes separately below
        grid[cx * g + cy] = np.arange(count, count + k)
        count += k

    insert(bx, by)

    ci = np.arange(g)
    cxx, cyy = np.meshgrid(ci, ci, indexing="ij")
    ccx = lo + (cxx + 0.5) * cell
    ccy = lo + (cyy + 0.5) * cell
    rc = np.hypot(ccx, ccy)
    in_band = (rc > r_in - cell) & (rc < r_out + cell)
    offs = [a * g + b for a in range(-2, 3) for b in range(-2, 3)]
    wall_sorted = np.argsort(np.arctan2(by, bx))
    wall_ang = np.arctan2(by, bx)[wall_sorted]

    inner = np.zeros_like(in_band)
    inner[2:-2, 2:-2] = True
    phase_cells = [np.nonzero(in_band & inner & (cxx % 3 == phx) & (cyy % 3 == phy))
                   for phx in range(3) for phy in range(3)]
    for _ in range(rounds):
        for ph in range(9):
            kx, ky = phase_cells[ph]
            lin = kx * g + ky
            empty = grid[lin] == cap
            kx, ky, lin = kx[empty], ky[empty], lin[empty]
            phase_cells[ph] = (kx, ky)
            if kx.size == 0:
                continue
            cand_x = lo + (kx + rng.random(kx.size)) * cell
            cand_y = lo + (ky + rng.random(ky.size)) * cell
            rr = np.hypot(cand_x, cand_y)
            ok = (rr >= r_in) & (rr <= r_out)
            for o in offs:
                nb_idx = grid[lin + o]
                d2 = (px[nb_idx] - cand_x) ** 2 + (py[nb_idx] - cand_y) ** 2
                ok &= d2 >= h * h
            near_wall = ok & ((rr < r_in + h) | (rr > r_out - h))
            if near_wall.any():
                idx = np.nonzero(near_wall)[0]
                ang = np.arctan2(cand_y[idx], cand_x[idx])
                pos = np.searchsorted(wall_ang, ang)
                nw = wall_sorted.shape[0]
                bad = np.zeros(idx.size, dtype=bool)
                for off in range(-4, 5):
                    w = wall_sorted[(pos + off) % nw]
                    d2 = (bx[w] - cand_x[idx]) ** 2 + (by[w] - cand_y[idx]) ** 2
                    bad |= d2 < h * h
                ok[idx[bad]] = False
            if ok.any():
                insert(cand_x[ok], cand_y[ok])
    x = px[:count].copy()
    y = py[:count].copy()
    node_type = np.zeros(count, dtype=np.uint8)
    node_type[:bx.shape[0]] = 1
    return Cloud(x, y, node_type, (0.0, 0.0), float(h))


def annulus_h_for_count(r_in: float, r_out: float, n_target: int) -> float:
    """Spacing that gives about n_target nodes for a dart-throwing sample
    (covering density about 0.68 / h^2)."""
    area = math.pi * (r_out ** 2 - r_in ** 2)
    return math.sqrt(0.68 * area / n_target)


def annulus_force(h: float, dx_paper: float = 1.0 / 160.0, g_paper: float = 1e-6) -> float:
    """Azimuthal acceleration (lattice units) of an annulus stepped with
    streaming distance h: the paper's g = 1e-6 at dx_ML = 1/160 carried to h
    under diffusive scaling (tau fixed, so dt goes as dx^2 and a lattice
    acceleration as dx^3). The flow is then the paper's physical flow: the
    same Reynolds number, a Mach number smaller by h / dx_paper."""
    return g_paper * (h / dx_paper) ** 3


def batched_tgv_specs(n_clouds: int = 64, n_min: float = 1e4, n_max: float = 2e5,
                      seed: int = 4) -> list[dict]:
    """Specifications of uneven Taylor-Green clouds: N_c log-uniform in
    [n_min, n_max], n_side = round(sqrt(N_c)), tau in [0.55, 1.0], degree in
    {2, 3, 4} with stencil size {20, 25, 30} (the smallest sizes that kept
    every cloud of the set stable at tau near 0.55: 12 diverges there)."""
    rng = _rng(seed)
    specs = []
    kk = {2: 20, 3: 25, 4: 30}
    for c in range(n_clouds):
        nc = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        n_side = int(round(math.sqrt(nc)))
        tau = float(rng.uniform(0.55, 1.0))
        m = int(rng.integers(2, 5))
        specs.append(dict(n_side=n_side, tau=tau, degree=m, K=kk[m],
                          seed=1000 + c))
    return specs


def tgv_initial_velocity(x: np.ndarray, y: np.ndarray, length: float,
                         u0: float) -> tuple[np.ndarray, np.ndarray]:
    """Taylor-Green vortex at t = 0 on a periodic square of side `length`:
    u = u0 (sin kx cos ky, -cos kx sin ky), k = 2 pi / length."""
    k = TWO_PI / length
    return (u0 * np.sin(k * x) * np.cos(k * y),
            -u0 * np.cos(k * x) * np.sin(k * y))


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded standard-normal field (test vectors, adjoint seeds)."""
    return scale * _rng(seed).standard_normal(shape)
