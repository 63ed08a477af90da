"""Pins of the oracle's stencil and owner searches against brute force written
independently in numpy (CPU)."""
import numpy as np
import pytest

import oracle
from synth import annulus_poisson, jittered_lattice


def _np_min_image(d, L):
    if L <= 0:
        return d
    return d - L * np.round(d / L)


def _np_knn(x, y, period, K, c):
    dx = _np_min_image(x - x[c], period[0])
    dy = _np_min_image(y - y[c], period[1])
    d2 = dx * dx + dy * dy
    idx = np.arange(x.shape[0])
    others = idx != c
    order = np.lexsort((idx[others], d2[others]))
    return np.concatenate([[c], idx[others][order][: K - 1]])


@pytest.mark.parametrize("kind", ["periodic", "annulus"])
def test_knn_matches_bruteforce(kind):
    if kind == "periodic":
        c = jittered_lattice(13, length=1.0, seed=9, ny=11, length_y=0.8)
    else:
        c = annulus_poisson(1.0, 2.0, 0.2, seed=2)
    K = 20
    nbr = oracle.knn(c.x, c.y, c.period, K)
    for i in range(c.n):
        ref = _np_knn(c.x, c.y, c.period, K, i)
        # equal sets and equal ordering by distance (ties are measure-zero here)
        np.testing.assert_array_equal(nbr[i], ref)
        np.testing.assert_array_equal(oracle.knn_one(c.x, c.y, c.period, K, i), ref)


def test_knn_ties_break_by_index_on_lattice():
    c = jittered_lattice(8, length=8.0, jitter=0.0)
    nbr = oracle.knn(c.x, c.y, c.period, 9)
    i = 3 * 8 + 3
    # the four axis neighbours at distance 1, ascending index, then the four diagonals
    assert set(nbr[i, 1:5]) == {i - 8, i - 1, i + 1, i + 8}
    assert set(nbr[i, 5:9]) == {i - 9, i - 7, i + 7, i + 9}
    # with room for one diagonal only, the lowest index wins the exact tie
    nbr6 = oracle.knn(c.x, c.y, c.period, 6)
    assert nbr6[i, 5] == i - 9
    np.testing.assert_array_equal(nbr6[i, 1:5], [i - 8, i - 1, i + 1, i + 8])


def test_owners_match_bruteforce():
    c = jittered_lattice(12, length=1.0, seed=4)
    ex, ey, _, _ = oracle.tables()
    dx = 1 / 12
    own = oracle.owners(c.x, c.y, c.period, dx, 0)
    for i in range(c.n):
        for k in range(9):
            px, py = c.x[i] - ex[k] * dx, c.y[i] - ey[k] * dx
            d = _np_min_image(c.x - px, 1.0) ** 2 + _np_min_image(c.y - py, 1.0) ** 2
            assert own[i, k] == int(np.argmin(d))
    own1 = oracle.owners(c.x, c.y, c.period, dx, 1)
    np.testing.assert_array_equal(own1, np.repeat(np.arange(c.n)[:, None], 9, 1))


def test_periodic_wrap_is_minimum_image():
    """A node near x = 0 and one near x = L are neighbours across the seam."""
    x = np.array([0.01, 0.99, 0.5, 0.3])
    y = np.array([0.5, 0.5, 0.5, 0.5])
    nbr = oracle.knn(x, y, (1.0, 1.0), 2)
    assert nbr[0, 1] == 1 and nbr[1, 1] == 0
    nbr_open = oracle.knn(x, y, (0.0, 0.0), 2)
    assert nbr_open[0, 1] == 3


@pytest.mark.parametrize("kind", ["periodic", "annulus", "lattice"])
def test_tree_candidates_give_the_bruteforce_answers(kind, monkeypatch):
    """The k-d tree candidate path used for full-size clouds returns exactly
    the brute-force stencils and owners, including exact lattice ties; with no
    spare candidates the ties at the cut cannot be settled from the list and
    the fallback to brute force must still give the same answers."""
    if kind == "periodic":
        c = jittered_lattice(21, length=1.0, seed=5, ny=17, length_y=0.81)
    elif kind == "annulus":
        c = annulus_poisson(1.0, 2.0, 0.12, seed=4)
    else:
        c = jittered_lattice(10, length=10.0, jitter=0.0)
    for extra in (8, 0):
        monkeypatch.setattr(oracle, "KNN_EXTRA", extra)
        monkeypatch.setattr(oracle, "OWNER_CAND", 4 if extra else 1)
        for K in (6, 13, 20):
            np.testing.assert_array_equal(oracle.knn_tree(c.x, c.y, c.period, K),
                                          oracle.knn(c.x, c.y, c.period, K))
            if extra == 0:
                assert oracle.last_fallbacks["knn"] > 0
        dx = 0.9 * c.h
        np.testing.assert_array_equal(oracle.owners_tree(c.x, c.y, c.period, dx, 0),
                                      oracle.owners(c.x, c.y, c.period, dx, 0))
        if extra == 0:
            assert oracle.last_fallbacks["owners"] == 8 * c.n
    if kind == "lattice":
        # on the lattice every departure point sits on a node: the list of one
        # candidate holds the owner but cannot prove it, the others can
        monkeypatch.setattr(oracle, "OWNER_CAND", 4)
        np.testing.assert_array_equal(oracle.owners_tree(c.x, c.y, c.period, c.h, 0),
                                      oracle.owners(c.x, c.y, c.period, c.h, 0))
        assert oracle.last_fallbacks["owners"] == 0
