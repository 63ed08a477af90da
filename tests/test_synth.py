"""The seeded input generators (the workloads' input recipe): the properties
each one promises, and that a seed fixes its output."""
import math

import numpy as np
from scipy.spatial import cKDTree

from synth.clouds import (annulus_force, annulus_h_for_count, annulus_poisson,
                          batched_tgv_specs, jittered_lattice, tgv_initial_velocity)


def test_jittered_lattice_stays_within_its_jitter_and_box():
    n, L = 40, 2 * math.pi
    c = jittered_lattice(n, seed=1)
    h = L / n
    assert c.n == n * n and c.period == (L, L) and c.h == h
    assert (c.x >= 0).all() and (c.x < L).all() and (c.y >= 0).all() and (c.y < L).all()
    ix, iy = np.arange(c.n) % n, np.arange(c.n) // n          # row-major, x fastest
    dx = (c.x - ix * h + L / 2) % L - L / 2
    dy = (c.y - iy * h + L / 2) % L - L / 2
    assert np.abs(dx).max() <= 0.3 * h and np.abs(dy).max() <= 0.3 * h
    assert np.abs(dx).max() > 0.25 * h                        # the jitter is really used
    c2 = jittered_lattice(n, seed=1)
    assert np.array_equal(c.x, c2.x) and np.array_equal(c.y, c2.y)
    assert not np.array_equal(c.x, jittered_lattice(n, seed=2).x)


def test_annulus_is_a_poisson_disk_sample_with_walls_on_both_circles():
    r1, r2, h = 1.0, 2.0, 0.05
    c = annulus_poisson(r1, r2, h, seed=3)
    r = np.hypot(c.x, c.y)
    wall = c.node_type == 1
    assert c.period == (0.0, 0.0)
    assert (r >= r1 - 1e-12).all() and (r <= r2 + 1e-12).all()
    # walls: round(2 pi r / h) nodes equally spaced on each circle
    for rad in (r1, r2):
        on = wall & (np.abs(r - rad) < 1e-12)
        assert on.sum() == round(2 * math.pi * rad / h)
        ang = np.sort(np.arctan2(c.y[on], c.x[on]))
        gaps = np.diff(np.concatenate([ang, [ang[0] + 2 * math.pi]]))
        assert np.allclose(gaps, 2 * math.pi / on.sum())
    assert wall.sum() == round(2 * math.pi * r1 / h) + round(2 * math.pi * r2 / h)
    # interior nodes keep at least h from every other node
    d, _ = cKDTree(np.column_stack([c.x, c.y])).query(
        np.column_stack([c.x[~wall], c.y[~wall]]), k=2)
    assert d[:, 1].min() >= h * (1 - 1e-12)
    # and cover the band at about 0.68 / h^2
    density = (~wall).sum() * h * h / (math.pi * (r2 ** 2 - r1 ** 2))
    assert 0.6 < density < 0.75
    c2 = annulus_poisson(r1, r2, h, seed=3)
    assert np.array_equal(c.x, c2.x)


def test_annulus_spacing_for_a_node_count():
    h = annulus_h_for_count(1.0, 2.0, 20_000)
    n = annulus_poisson(1.0, 2.0, h, seed=3).n
    assert 0.9 * 20_000 < n < 1.1 * 20_000


def test_annulus_force_under_diffusive_scaling():
    assert annulus_force(1.0 / 160.0) == 1e-6
    assert annulus_force(1.0 / 320.0) == 1e-6 / 8


def test_batched_specs_cover_the_stated_ranges():
    specs = batched_tgv_specs(64, seed=4)
    assert len(specs) == 64
    n = np.array([s["n_side"] ** 2 for s in specs])
    assert n.min() >= 0.95e4 and n.max() <= 2.05e5
    assert {s["degree"] for s in specs} == {2, 3, 4}
    assert all(s["K"] == {2: 20, 3: 25, 4: 30}[s["degree"]] for s in specs)
    assert all(0.55 <= s["tau"] <= 1.0 for s in specs)
    assert len({s["seed"] for s in specs}) == 64
    assert n.sum() == 3_831_809                          # the workload's node count
    assert batched_tgv_specs(64, seed=4) == specs


def test_tgv_initial_velocity_is_the_divergence_free_vortex():
    L, u0 = 2 * math.pi, 0.01
    x, y = np.meshgrid(np.linspace(0, L, 33), np.linspace(0, L, 33))
    ux, uy = tgv_initial_velocity(x, y, L, u0)
    assert np.allclose(ux, u0 * np.sin(x) * np.cos(y))
    assert np.allclose(uy, -u0 * np.cos(x) * np.sin(y))
    e = 1e-6     # du/dx + dv/dy = 0 by central differences
    up, um = tgv_initial_velocity(x + e, y, L, u0), tgv_initial_velocity(x - e, y, L, u0)
    vp, vm = tgv_initial_velocity(x, y + e, L, u0), tgv_initial_velocity(x, y - e, L, u0)
    div = (up[0] - um[0]) / (2 * e) + (vp[1] - vm[1]) / (2 * e)
    assert np.abs(div).max() < 1e-9
