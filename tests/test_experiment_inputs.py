"""Paper-shaped inputs (Sec. 9): regular-polygon point picking and the leaf
lattices the experiments fill (CPU only).

Point picking is pinned to closed forms of the uniform distribution on a
regular n-gon: zero mean offset, mean squared distance from the centre
R^2 (1 + 2 cos^2(pi/n)) / 6, every point inside the polygon, equal mass in
the n central triangles and in the two halves of each.  The leaf lattices
are pinned to the oracle's CellIndex / cell centres: every full-tree leaf is
a distinct valid cell whose centre the oracle reproduces, and every picked
point lands in its own cell."""
import math

import numpy as np
import pytest

from paper_1204_3105_amd import experiments as ex
from paper_1204_3105_amd import inputs


@pytest.mark.parametrize("n", [3, 4, 6, 7])
def test_polygon_points_moments(n):
    g = inputs.rng(n)
    R, rot, c = 0.7, 0.4, (0.3, -1.2)
    x, y = inputs.polygon_points(g, [c[0]], [c[1]], n, R, rot, 400000)
    dx, dy = x - c[0], y - c[1]
    assert abs(dx.mean()) < 4e-3 and abs(dy.mean()) < 4e-3
    m2 = R * R * (1 + 2 * math.cos(math.pi / n) ** 2) / 6
    assert abs((dx * dx + dy * dy).mean() / m2 - 1) < 5e-3
    # inside: for every edge normal at rot + pi/n + 2 pi k/n, offset . normal <= apothem
    ap = R * math.cos(math.pi / n)
    th = rot + math.pi / n + 2 * math.pi * np.arange(n) / n
    proj = np.outer(dx, np.cos(th)) + np.outer(dy, np.sin(th))
    assert proj.max() <= ap * (1 + 1e-12)
    # mass per central triangle and per half-triangle (chi-square at ~5 sigma)
    ang = np.mod(np.arctan2(dy, dx) - rot, 2 * math.pi)
    tri = np.minimum((ang / (2 * math.pi / n)).astype(int), n - 1)
    half = (np.mod(ang, 2 * math.pi / n) > math.pi / n).astype(int)
    cnt = np.bincount(2 * tri + half, minlength=2 * n)
    e = len(x) / (2 * n)
    chi2 = ((cnt - e) ** 2 / e).sum()
    assert chi2 < 2 * n + 5 * math.sqrt(4 * n), (cnt, chi2)


def test_polygon_points_counts_and_order():
    g = inputs.rng(5)
    x, y = inputs.polygon_points(g, [0.0, 10.0, 20.0], [0.0, 0.0, 0.0], [3, 4, 6], [1.0, 1.0, 1.0],
                                 [0.0, 0.0, 0.0], [5, 0, 7])
    assert len(x) == 12
    assert np.all(np.abs(x[:5]) <= 1) and np.all(np.abs(x[5:] - 20) <= 1)


@pytest.mark.parametrize("tiling,L", [("quad", 3), ("sept", 2), ("sept", 3), ("tri", 3)])
def test_leaf_lattice_matches_oracle_cells(orc, tiling, L):
    cells = ex.leaf_cells(tiling, L)
    base = {"quad": 4, "sept": 7, "tri": 4}[tiling]
    assert len(cells["cx"]) == base ** L
    g = orc.geom(tiling, L, *cells["geometry"])
    keys = orc.cell_index(g, cells["cx"], cells["cy"], L)
    assert np.all(keys >= 0) and len(np.unique(keys)) == len(keys)
    cx, cy = orc.cell_center(g, keys, L)
    assert np.allclose(cx, cells["cx"], atol=1e-12) and np.allclose(cy, cells["cy"], atol=1e-12)
    # picked points land in their own cell
    w = ex.cell_workload(tiling, L, len(keys), 9, seed=3)
    own = np.repeat(keys[w["cells"]], 9)
    for x, y in ((w["xs"], w["ys"]), (w["xt"], w["yt"])):
        got = orc.cell_index(g, x, y, L)
        assert np.array_equal(got, own)


def test_s_opt_and_nearest_cells():
    # p (c N/M)^(1/2) at p = 12, N = M: 24.87, 32.50, 24.61
    assert [ex.s_opt(t, 12) for t in ex.TILINGS] == [25, 32, 25]
    assert ex.s_opt("quad", 1, ratio=0.0) == 1
    cells = ex.leaf_cells("quad", 2)
    sel = ex.nearest_cells(cells, 4)
    assert sorted(zip(cells["cx"][sel], cells["cy"][sel])) == [(0.375, 0.375), (0.375, 0.625),
                                                               (0.625, 0.375), (0.625, 0.625)]
