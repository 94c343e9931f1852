"""Pins for the oracle's cell addressing (paper Secs. 4-7), CPU only.

Every check here compares the oracle with something other than itself: the
paper's worked examples (tests/golden/paper_examples.json), an independent
Eisenstein-integer model of GBT arithmetic, brute-force nearest-centre
(Voronoi) assignment, geometric vertex sharing computed from polygon
vertices, and the separation ratios of the paper's cost table.
"""
import json
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")

GOLD = os.path.join(os.path.dirname(__file__), "golden")
EX = json.load(open(os.path.join(GOLD, "paper_examples.json")))


def b7(s):
    return int(str(s), 7)


def b4(s):
    return int(str(s), 4)


# ------------------------------------------------------------------ GBT model
# Eisenstein integers a + b w with w = exp(i pi/3), w^2 = w - 1.  Digit k in
# 1..6 is w^(k-1); the base is beta = 1 + 2w (|beta|^2 = 7).
def e_mul(x, y):
    a, b = x
    c, d = y
    return (a * c - b * d, a * d + b * c + b * d)


def e_add(x, y):
    return (x[0] + y[0], x[1] + y[1])


W = (0, 1)
DIGIT = [(0, 0), (1, 0)]
for _ in range(5):
    DIGIT.append(e_mul(DIGIT[-1], W))
BETA = (1, 2)


def gbt_value(key):
    """Eisenstein value of a base-7 GBT index given as an integer."""
    val, pw = (0, 0), (1, 0)
    while key > 0:
        val = e_add(val, e_mul(DIGIT[key % 7], pw))
        pw = e_mul(pw, BETA)
        key //= 7
    return val


def test_gbt_model_matches_paper_table():
    """The printed unit-addition table is vector addition of w^(k-1)."""
    rows = [l.split() for l in open(os.path.join(GOLD, "gbt_unit_table.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    for r in rows:
        a = int(r[0])
        for b in range(1, 7):
            printed = b7(r[b])
            assert gbt_value(printed) == e_add(DIGIT[a], DIGIT[b]), (a, b, r[b])


def test_gbt_add_units_against_table_and_model(orc):
    rows = [l.split() for l in open(os.path.join(GOLD, "gbt_unit_table.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        a = int(r[0])
        for b in range(1, 7):
            assert orc.gbt_add(a, b) == b7(r[b])
            assert orc.gbt_add(b, a) == b7(r[b])
        assert orc.gbt_add(a, 0) == a


def test_gbt_add_random_multidigit(orc):
    rng = np.random.default_rng(7)
    for _ in range(3000):
        a = int(rng.integers(0, 7 ** 6))
        b = int(rng.integers(0, 7 ** 6))
        s = orc.gbt_add(a, b)
        assert s >= 0
        assert gbt_value(s) == e_add(gbt_value(a), gbt_value(b))


def test_paper_gbt_examples(orc):
    for a, b, c in EX["gbt_sum"]["cases"]:
        assert orc.gbt_add(b7(a), b7(b)) == b7(c)
    for a, b, c, d in EX["gbt_zero_extension"]["cases"] + EX["gbt_zero_extension_higher"]["cases"]:
        assert orc.gbt_add(orc.gbt_add(b7(a), b7(b)), b7(c)) == b7(d)


def test_paper_septree_neighbors(orc):
    for case in EX["sept_neighbors"]["cases"]:
        g = orc.geom("sept", 3, 0.0, 0.0, 1.0)
        got = orc.neighbors(g, b7(case["cell"]), case["level"])
        assert got == sorted(b7(v) for v in case["neighbors"])


def test_septree_base_is_rotation_and_scale():
    """beta has |beta| = sqrt 7 and arg beta = arctan(sqrt(3)/2) (Sec. 5, App. D)."""
    ex = EX["gbt_rotation"]
    w = complex(0.5, math.sqrt(3) / 2)
    beta = 1 + 2 * w
    assert abs(abs(beta) - ex["scale"]) < 1e-14
    assert abs(math.degrees(math.atan2(beta.imag, beta.real)) - ex["theta_deg"]) < 1e-12
    assert abs(math.atan(math.sqrt(3) / 2) - math.atan2(beta.imag, beta.real)) < 1e-15


def test_paper_septree_center_decomposition(orc):
    L = 4
    g = orc.geom("sept", L, 0.25, -0.5, 0.01)
    for key in ("sept_center_decomposition", "sept_center_32"):
        for case in EX[key]["cases"]:
            lvl = len(case["cell"])
            cx, cy = orc.cell_center(g, b7(case["cell"]), lvl)
            sx = sy = 0.0
            for part in case["parts"]:
                px, py = orc.cell_center(g, b7(part), lvl)
                sx += px[0] - g.ox
                sy += py[0] - g.oy
            assert abs(cx[0] - g.ox - sx) < 1e-15 and abs(cy[0] - g.oy - sy) < 1e-15


def test_septree_polar_center_formula(orc):
    """eq. (septreecenter), evaluated in floating point, agrees with the
    exact lattice centres."""
    L = 4
    r = 0.01
    g = orc.geom("sept", L, 0.1, 0.2, r)
    worst = 0.0
    for lvl in range(1, L + 1):
        for key in range(7 ** lvl):
            cx, cy = orc.cell_center(g, key, lvl)
            px, py = orc.sept_center_polar(g, key, lvl)
            worst = max(worst, abs(cx[0] - px), abs(cy[0] - py))
    assert worst < 1e-12 * r * 7 ** (L / 2) * 10


def test_septree_center_is_gbt_value(orc):
    """Leaf centre = Eisenstein value of the key on the lattice with unit
    digit 1 at 30 degrees and spacing r sqrt(3)."""
    L = 3
    r = 0.02
    g = orc.geom("sept", L, 0.0, 0.0, r)
    rot = complex(math.cos(math.pi / 6), math.sin(math.pi / 6)) * r * math.sqrt(3)
    w = complex(0.5, math.sqrt(3) / 2)
    for key in range(7 ** L):
        a, b = gbt_value(key)
        z = (a + b * w) * rot
        cx, cy = orc.cell_center(g, key, L)
        assert abs(z - complex(cx[0], cy[0])) < 1e-14


def test_paper_tq_examples(orc):
    for case in EX["tq_adjacent"]["cases"]:
        d = {"L": 0, "R": 1, "V": 2}[case["direction"]]
        assert orc.tq_adjacent(b4(case["cell"]), case["level"], d) == b4(case["result"])
    for case in EX["tq_orientation"]["cases"]:
        cell = case["cell"]
        got = [orc.tq_is_up(b4(cell[:i]), i) for i in range(1, len(cell) + 1)]
        assert got == case["orientations"]
    # Table D: at level 1 a direction has a neighbour iff the entry is starred.
    for t, row in enumerate(EX["tq_table_D"]["rows"]):
        for d, ent in enumerate(row):
            res = orc.tq_adjacent(t, 1, d)
            if ent.endswith("*"):
                assert res == int(ent[0])
            else:
                assert res is None
    # Deeper, the neighbour across an edge (found from the lattice) has the
    # table's destination type as its last digit, and a starred entry means
    # the neighbour is a sibling (same parent); the way back crosses the same
    # edge, which is the other cell's right edge for a left step and so on.
    D = [[int(e[0]) for e in row] for row in EX["tq_table_D"]["rows"]]
    star = [[e.endswith("*") for e in row] for row in EX["tq_table_D"]["rows"]]
    for lvl in range(2, 6):
        for key in range(4 ** lvl):
            t = key & 3
            for d in range(3):
                res = orc.tq_adjacent(key, lvl, d)
                if star[t][d]:
                    assert res is not None and res >> 2 == key >> 2, (lvl, key, d)
                else:
                    assert res is None or res >> 2 != key >> 2, (lvl, key, d)
                if res is not None:
                    assert res & 3 == D[t][d], (lvl, key, d)
                    assert orc.tq_adjacent(res, lvl, (1, 0, 2)[d]) == key


def test_tq_isup_is_zero_parity(orc):
    for lvl in range(1, 6):
        for key in range(4 ** lvl):
            digits = [(key >> (2 * (lvl - i))) & 3 for i in range(1, lvl + 1)]
            expect = 1 if digits.count(0) % 2 == 0 else -1
            assert orc.tq_is_up(key, lvl) == expect


# ------------------------------------------------------------ Voronoi pins
def all_centers(orc, g, lvl):
    n = (7 if g.tiling == 1 else 4) ** lvl
    keys = np.arange(n, dtype=np.int64)
    cx, cy = orc.cell_center(g, keys, lvl)
    return keys, cx, cy


def nearest(keys, cx, cy, x, y):
    d2 = (cx[None, :] - x[:, None]) ** 2 + (cy[None, :] - y[:, None]) ** 2
    return keys[np.argmin(d2, axis=1)], np.sort(d2, axis=1)


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_cell_index_is_nearest_centre(orc, tiling):
    rng = np.random.default_rng(11)
    if tiling == "quad":
        g = orc.geom("quad", 5, -0.3, 0.2, 1.7)
        x = g.ox + g.size * rng.random(4000)
        y = g.oy + g.size * rng.random(4000)
        levels = range(0, 6)
    elif tiling == "sept":
        g = orc.geom("sept", 4, 0.3, -0.1, 0.05)
        # Inside the root aggregate's inscribed disk (radius > 0.43 sqrt(7)^L r sqrt(3)).
        rad = 0.43 * 7 ** 2 * 0.05 * math.sqrt(3) * np.sqrt(rng.random(4000))
        ang = 2 * np.pi * rng.random(4000)
        x, y = g.ox + rad * np.cos(ang), g.oy + rad * np.sin(ang)
        levels = [4]
    else:
        g = orc.geom("tri", 5, 0.1, 0.4, 0.03)
        rho0 = 2 ** 4 * 0.03
        rad = rho0 * np.sqrt(rng.random(4000))
        ang = 2 * np.pi * rng.random(4000)
        x, y = g.ox + rad * np.cos(ang), g.oy + rad * np.sin(ang)
        levels = range(0, 6)
    for lvl in levels:
        keys, cx, cy = all_centers(orc, g, lvl)
        got = orc.cell_index(g, x, y, lvl)
        want, d2 = nearest(keys, cx, cy, x, y)
        # Skip points within rounding of a Voronoi boundary.
        if d2.shape[1] > 1:
            clear = (d2[:, 1] - d2[:, 0]) > 1e-12 * (d2[:, 1] + 1e-30)
        else:
            clear = np.ones(len(x), dtype=bool)
        assert clear.mean() > 0.99
        assert np.array_equal(got[clear], want[clear]), (tiling, lvl)


def test_septree_out_of_root_is_rejected(orc):
    g = orc.geom("sept", 2, 0.0, 0.0, 0.1)
    assert orc.cell_index(g, np.array([5.0]), np.array([5.0]), 2)[0] == -1


@pytest.mark.parametrize("tiling,L", [("quad", 4), ("sept", 4), ("tri", 5)])
def test_cell_index_of_centre_round_trip(orc, tiling, L):
    g = orc.geom(tiling, L, 0.2, 0.3, 0.05 if tiling != "quad" else 1.0)
    for lvl in range(1, L + 1):
        keys, cx, cy = all_centers(orc, g, lvl)
        if tiling == "sept":
            # Only the leaf level has Voronoi cells; coarse cells are aggregates.
            if lvl != L:
                continue
        got = orc.cell_index(g, cx, cy, lvl)
        assert np.array_equal(got, keys)


# ------------------------------------------------------ geometric neighbours
def quad_geo_neighbors(orc, g, key, lvl):
    ix, iy = orc.center_units(g, key, lvl)
    n = 2 ** lvl
    out = set()
    for k in range(4 ** lvl):
        jx, jy = orc.center_units(g, k, lvl)
        if k != key and max(abs(jx - ix), abs(jy - iy)) == 1:
            out.add(k)
    return out


def tq_vertices(orc, g, key, lvl):
    """Triangle vertices in integer units (U, V): x = U sqrt(3)/2 r, y = V r/2."""
    U, V = orc.center_units(g, key, lvl)
    R = 2 ** (g.L - lvl)
    up = orc.tq_is_up(key, lvl)
    return {(U, V + 2 * up * R), (U - R, V - up * R), (U + R, V - up * R)}


def tq_geo_neighbors_all(orc, g, lvl):
    verts = {k: tq_vertices(orc, g, k, lvl) for k in range(4 ** lvl)}
    by_vertex = {}
    for k, vs in verts.items():
        for v in vs:
            by_vertex.setdefault(v, set()).add(k)
    out = {}
    for k, vs in verts.items():
        s = set()
        for v in vs:
            s |= by_vertex[v]
        s.discard(k)
        out[k] = s
    return out


def sept_leaf_geo_neighbors(orc, g, key):
    b, c = orc.center_units(g, key, g.L)
    out = set()
    for k in range(7 ** g.L):
        bb, cc = orc.center_units(g, k, g.L)
        db, dc = bb - b, cc - c
        # squared distance in units of r^2, times 4: 9 db^2 + 3 (2 dc + db)^2
        if 9 * db * db + 3 * (2 * dc + db) ** 2 == 12:
            out.add(k)
    return out


def test_quad_neighbors_geometric(orc):
    g = orc.geom("quad", 3, 0.0, 0.0, 1.0)
    for lvl in (1, 2, 3):
        for key in range(4 ** lvl):
            assert set(orc.neighbors(g, key, lvl)) == quad_geo_neighbors(orc, g, key, lvl)


def test_tq_neighbors_geometric(orc):
    g = orc.geom("tri", 5, 0.0, 0.0, 1.0)
    for lvl in (1, 2, 3, 4, 5):
        geo = tq_geo_neighbors_all(orc, g, lvl)
        for key in range(4 ** lvl):
            assert set(orc.neighbors(g, key, lvl)) == geo[key], (lvl, key)


def test_sept_leaf_neighbors_geometric(orc):
    g = orc.geom("sept", 3, 0.0, 0.0, 1.0)
    for key in range(7 ** 3):
        assert set(orc.neighbors(g, key, 3)) == sept_leaf_geo_neighbors(orc, g, key)


def test_sept_aggregate_neighbors_touch(orc):
    """A coarse septree cell's Neighbors are exactly the aggregates that hold
    a leaf adjacent to one of its leaves (restricted to the root)."""
    L = 4
    g = orc.geom("sept", L, 0.0, 0.0, 1.0)
    leaf_nb = {k: set(orc.neighbors(g, k, L)) for k in range(7 ** L)}
    for lvl in (1, 2, 3):
        div = 7 ** (L - lvl)
        for key in range(7 ** lvl):
            touch = set()
            for leaf in range(key * div, (key + 1) * div):
                touch |= {m // div for m in leaf_nb[leaf]}
            touch.discard(key)
            assert set(orc.neighbors(g, key, lvl)) == touch, (lvl, key)


def closed(orc, g, key, lvl):
    return set(orc.neighbors(g, key, lvl)) | {key}


@pytest.mark.parametrize("tiling,L,P4", [("quad", 4, 27), ("sept", 4, 42), ("tri", 5, 39)])
def test_e4_definition_and_interior_count(orc, tiling, L, P4):
    g = orc.geom(tiling, L, 0.0, 0.0, 1.0)
    base = 7 if tiling == "sept" else 4
    counts = []
    for lvl in range(1, L + 1):
        for key in range(base ** lvl):
            par = key // base
            pn = closed(orc, g, par, lvl - 1) if lvl > 1 else {0}
            want = {c * base + d for c in pn for d in range(base)} - closed(orc, g, key, lvl)
            got = orc.e4(g, key, lvl)
            assert set(got) == want and len(got) == len(want)
            full_parent = len(closed(orc, g, par, lvl - 1)) == {"quad": 9, "sept": 7, "tri": 13}[tiling]
            full_self = len(closed(orc, g, key, lvl)) == {"quad": 9, "sept": 7, "tri": 13}[tiling]
            if lvl > 1 and full_parent and full_self:
                counts.append(len(got))
    assert counts and set(counts) == {P4}


def test_cost_table_p2(orc):
    tab = EX["cost_table"]
    for tiling, L in (("quad", 3), ("sept", 3), ("tri", 4)):
        g = orc.geom(tiling, L, 0.0, 0.0, 1.0)
        base = 7 if tiling == "sept" else 4
        sizes = [len(orc.neighbors(g, k, L)) + 1 for k in range(base ** L)]
        assert max(sizes) == tab[tiling]["P2"]


# ------------------------------------------------------- separation ratios
def point_poly_dist(px, py, poly):
    """Distance from a point to a convex polygon (vertices in CCW or CW order)."""
    n = len(poly)
    inside = True
    sgn = None
    best = math.inf
    for i in range(n):
        ax, ay = poly[i]
        bx, by = poly[(i + 1) % n]
        cross = (bx - ax) * (py - ay) - (by - ay) * (px - ax)
        s = cross > 0
        if sgn is None:
            sgn = s
        elif s != sgn and abs(cross) > 1e-15:
            inside = False
        ex, ey = bx - ax, by - ay
        t = max(0.0, min(1.0, ((px - ax) * ex + (py - ay) * ey) / (ex * ex + ey * ey)))
        best = min(best, math.hypot(ax + t * ex - px, ay + t * ey - py))
    return 0.0 if inside else best


def cell_polygon(orc, g, key, lvl):
    cx, cy = orc.cell_center(g, key, lvl)
    cx, cy = cx[0], cy[0]
    if g.tiling == 0:
        h = g.size / 2 ** lvl / 2
        return [(cx - h, cy - h), (cx + h, cy - h), (cx + h, cy + h), (cx - h, cy + h)]
    if g.tiling == 2:
        R = g.size * 2 ** (g.L - lvl)
        up = orc.tq_is_up(key, lvl)
        return [(cx, cy + up * R), (cx - R * math.sqrt(3) / 2, cy - up * R / 2),
                (cx + R * math.sqrt(3) / 2, cy - up * R / 2)]
    r = g.size
    return [(cx + r * math.cos(k * math.pi / 3), cy + r * math.sin(k * math.pi / 3)) for k in range(6)]


@pytest.mark.parametrize("tiling,L,levels", [("quad", 5, (3, 4, 5)), ("tri", 6, (3, 4, 5, 6)),
                                             ("sept", 3, (3,))])
def test_separation_ratios_match_cost_table(orc, tiling, L, levels):
    """r/R and rho/r of interior cells equal the paper's table values, where
    r = cell circumradius, R = distance from the centre to the nearest cell
    outside the closed neighbourhood, rho = min E4 centre distance - 2r."""
    tab = EX["cost_table"][tiling]
    g = orc.geom(tiling, L, 0.0, 0.0, 1.0)
    base = 7 if tiling == "sept" else 4
    n_full = {"quad": 9, "sept": 7, "tri": 13}[tiling]
    for lvl in levels:
        if tiling == "quad":
            r = g.size / 2 ** lvl * math.sqrt(2) / 2
        else:
            r = g.size * (2 ** (g.L - lvl) if tiling == "tri" else 1.0)
        keys = np.arange(base ** lvl)
        cx_all, cy_all = orc.cell_center(g, keys, lvl)
        ratios_R, ratios_rho = [], []
        rng = np.random.default_rng(lvl)
        for key in rng.permutation(keys):
            key = int(key)
            cl = closed(orc, g, key, lvl)
            if len(cl) != n_full or any(len(closed(orc, g, m, lvl)) != n_full for m in cl):
                continue
            cx, cy = cx_all[key], cy_all[key]
            d = np.hypot(cx_all - cx, cy_all - cy)
            near = [int(m) for m in keys[d < 6 * r] if int(m) not in cl]
            R = min(point_poly_dist(cx, cy, cell_polygon(orc, g, m, lvl)) for m in near)
            ratios_R.append(r / R)
            if lvl > 1 and len(closed(orc, g, key // base, lvl - 1)) == n_full:
                e4 = orc.e4(g, key, lvl)
                dmin = np.min(d[np.array(e4)])
                ratios_rho.append((dmin - 2 * r) / r)
            if len(ratios_R) >= 25 and len(ratios_rho) >= 10:
                break
        assert ratios_R and ratios_rho, (tiling, lvl)
        assert abs(max(ratios_R) - tab["r_over_R"]) < 1e-9, (tiling, lvl, max(ratios_R))
        assert abs(min(ratios_R) - tab["r_over_R"]) < 1e-9, (tiling, lvl, min(ratios_R))
        assert abs(min(ratios_rho) - tab["rho_over_r"]) < 1e-9, (tiling, lvl, min(ratios_rho))
