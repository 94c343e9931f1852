"""The planner's septree constants, derived again from the oracle's cells.

Septree cells above the leaf level are GBT-prefix aggregates of leaf
hexagons (Sec. 5: a level-l address is the first l digits of a leaf's), not
the level-invariant hexagons of the separation argument (Sec. 7), so two
constants the planner uses are measured on the aggregates:

- the separation ratio q = max(r/R, 1/(1 + rho/r)) behind the order rule
  p = ceil(ln eps / ln q) - 1 (Sec. 8 error bounds), with r the aggregate's
  circumradius about its CellCenter, R the distance from that centre to the
  nearest point outside its closed neighbourhood, and rho = d - 2r for the
  nearest NeighborsE4 centre at distance d;
- the inscribed radius of the level-L root aggregate about the root centre,
  as a multiple c_L of sqrt(7)^L leaf spacings, which places the root over
  the points' bounding disk.

Both are computed here by brute force over the oracle's leaf centres
(CellCenter of every leaf key of the cells involved, at several leaf depths
below a level-2 cell) and compared with the values in the library's source:
the septree entry of the q table in plan.hip and kSeptInscribed in
fmm_tables.h.  The library's order rule is then checked against the measured
q over a dense range of eps.
"""
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1204_3105_amd", "csrc")
ANG = np.arange(6) * math.pi / 3   # hexagon vertex angles (circumradius = leaf size)


def source_q_table():
    src = open(os.path.join(CSRC, "plan.hip")).read()
    body = re.search(r"static const double kQ\[3\]\s*=\s*\{(.*?)\};", src, re.S).group(1)
    body = re.sub(r"//[^\n]*", "", body)
    return [float(v) for v in body.replace("\n", " ").split(",") if v.strip()]


def source_inscribed_table():
    src = open(os.path.join(CSRC, "fmm_tables.h")).read()
    body = re.search(r"kSeptInscribed\[\d+\]\s*=\s*\{(.*?)\};", src, re.S).group(1)
    return [float(v) for v in body.replace("\n", " ").split(",") if v.strip()]


def aggregate_radius(orc, g, key, level):
    """Largest distance from CellCenter(key, level) to a vertex of one of the
    cell's leaf hexagons (leaf keys key * 7^k + j)."""
    k = g.L - level
    cx0, cy0 = orc.cell_center(g, [key], level)
    n = 7 ** k
    best = 0.0
    for a in range(0, n, 1 << 22):
        keys = np.arange(key * n + a, key * n + min(n, a + (1 << 22)), dtype=np.int64)
        lx, ly = orc.cell_center(g, keys, g.L)
        d2 = (lx - cx0[0]) ** 2 + (ly - cy0[0]) ** 2
        far = d2 >= max(0.0, math.sqrt(d2.max()) - 2.0 * g.size) ** 2   # only these can hold the farthest vertex
        vx = lx[far][:, None] + g.size * np.cos(ANG)[None, :] - cx0[0]
        vy = ly[far][:, None] + g.size * np.sin(ANG)[None, :] - cy0[0]
        best = max(best, float(np.sqrt(vx * vx + vy * vy).max()))
    return best


def hexagon_distance(px, py, size):
    """Distance from the origin to the hexagons of circumradius `size`
    centred at (px, py) (vertices at 0, 60, ..., 300 degrees)."""
    best = np.full(px.shape, np.inf)
    for v in range(6):
        ax, ay = px + size * math.cos(ANG[v]), py + size * math.sin(ANG[v])
        bx, by = px + size * math.cos(ANG[(v + 1) % 6]), py + size * math.sin(ANG[(v + 1) % 6])
        ex, ey = bx - ax, by - ay
        t = np.clip((-ax * ex - ay * ey) / (ex * ex + ey * ey), 0.0, 1.0)
        best = np.minimum(best, np.hypot(ax + t * ex, ay + t * ey))
    return best


def separation(orc, k, with_R=True):
    """(r/R, rho/r, q) of the level-2 cell 0 of a septree k levels deeper
    (r/R only if with_R).  Cell 0's closed neighbourhood is the level-1 cell
    0; its NeighborsE4 are the 42 other level-2 cells, which surround it."""
    lvl = 2
    g = orc.geom("sept", lvl + k, 0.0, 0.0, 1.0)
    closed = [0] + orc.neighbors(g, 0, lvl)
    e4 = orc.e4(g, 0, lvl)
    assert len(closed) == 7 and len(e4) == 42 and not set(closed) & set(e4)
    cx0, cy0 = orc.cell_center(g, [0], lvl)
    r = aggregate_radius(orc, g, 0, lvl)
    ex, ey = orc.cell_center(g, np.array(e4), lvl)
    d = float(np.min(np.hypot(ex - cx0[0], ey - cy0[0])))
    # R: nearest leaf hexagon of the surrounding cells (all leaves of the
    # E4 cells; those within reach of the closed neighbourhood decide it)
    if not with_R:
        return None, (d - 2 * r) / r, r / (d - r)
    n = 7 ** k
    R = math.inf
    for c in e4:
        keys = np.arange(c * n, (c + 1) * n, dtype=np.int64)
        lx, ly = orc.cell_center(g, keys, g.L)
        px, py = lx - cx0[0], ly - cy0[0]
        near = np.hypot(px, py) < 2.5 * r + 2.0 * g.size
        if near.any():
            R = min(R, float(hexagon_distance(px[near], py[near], g.size).min()))
    return r / R, (d - 2 * r) / r, r / (d - r)


@pytest.fixture(scope="module")
def measured(orc):
    """k = 0..6 levels above the leaves with r/R; 7 and 8 without (their
    r/R would cost a brute force over tens of millions of leaves)."""
    m = {k: separation(orc, k) for k in range(0, 7)}
    m.update({k: separation(orc, k, with_R=False) for k in (7, 8)})
    return m


def test_septree_ratios_leaf_levels_are_the_hexagon_values(measured):
    # one and two levels above the leaves the aggregates keep the hexagon
    # values of the cost table: r/R = 1/2, rho/r = 1
    for k in (0, 1):
        r_R, rho_r, q = measured[k]
        assert abs(r_R - 0.5) < 1e-12 and abs(rho_r - 1.0) < 1e-12 and abs(q - 0.5) < 1e-12


def test_septree_ratios_coarse_levels(measured):
    # the aggregates grow ragged above that: rho/r falls to 0.912 (k = 2..4)
    # and 0.907 (k = 5..7); r/R stays below 1/(1 + rho/r), so rho/r sets q
    for k in (2, 3, 4):
        assert abs(measured[k][1] - 0.91217603) < 1e-7
    for k in (5, 6, 7):
        assert abs(measured[k][1] - 0.90704645) < 1e-7
    # eight levels above, the aggregate's farthest vertex moves out again
    assert abs(measured[8][1] - 0.90681919) < 1e-7
    for k in range(7):
        r_R, rho_r, q = measured[k]
        assert r_R <= q + 1e-12
        assert 0.5 - 1e-12 <= r_R < 0.5230


def test_planner_q_is_the_supremum(measured):
    """The planner's septree q is at least every measured q (eight levels
    above the leaves included), and above it by less than 1e-9."""
    q_sup = max(v[2] for v in measured.values())
    q_src = source_q_table()[1]
    assert q_src >= q_sup - 1e-15, (q_src, q_sup)
    assert q_src - q_sup < 1e-9, (q_src, q_sup)


def test_order_rule_uses_measured_q(measured):
    from paper_1204_3105_amd import fmm
    q_sup = max(v[2] for v in measured.values())
    for eps in np.logspace(-1.0, -14.0, 400):
        want = max(1, math.ceil(math.log(eps) / math.log(q_sup)) - 1)
        assert fmm.order_for_eps("sept", float(eps)) == want, eps


def inscribed(orc, L):
    """Radius of the largest disk about the root centre (leaf 0) inside the
    union of the 7^L leaf hexagons of the level-L root, by brute force: the
    lattice hexagons next to the union that are not in it, and the nearest of
    them.  In leaf spacings (sqrt(3) x circumradius) over sqrt(7)^L."""
    g = orc.geom("sept", L, 0.0, 0.0, 1.0)
    cx, cy = orc.cell_center(g, np.arange(7 ** L, dtype=np.int64), L)
    # lattice directions: the six level-1 cells around cell 0 of a depth-1 tree
    nx, ny = orc.cell_center(orc.geom("sept", 1, 0.0, 0.0, 1.0), np.arange(1, 7), 1)
    basis = np.linalg.inv(np.array([[nx[0], nx[1]], [ny[0], ny[1]]]))

    def code(x, y):
        ab = np.rint(basis @ np.vstack([x, y])).astype(np.int64)
        return ab[0] * 1000003 + ab[1]

    inside = code(cx, cy)
    best = math.inf
    for j in range(6):
        ox, oy = cx + nx[j], cy + ny[j]
        out = ~np.isin(code(ox, oy), inside)
        if out.any():
            best = min(best, float(hexagon_distance(ox[out], oy[out], 1.0).min()))
    return best / (math.sqrt(7) ** L * math.sqrt(3))


def test_root_inscribed_table(orc):
    tab = source_inscribed_table()
    assert len(tab) >= 8
    for L in range(0, 8):
        c = inscribed(orc, L)
        assert abs(c - tab[L]) < 1e-12, (L, c, tab[L])
