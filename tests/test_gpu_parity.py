"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Keys, the sorted permutation, the per-level cells and ranges, and the
interaction lists must match bit for bit; potentials must match to relative
L2 <= 1e-12 on the FP64 path (the oracle and the GPU use the same geometry,
exported by the plan, and the same p).
"""
import sys

import numpy as np
import pytest

from paper_1204_3105_amd import inputs

pytestmark = pytest.mark.gpu

TILES = ["quad", "sept", "tri"]
TID = {"quad": 0, "sept": 1, "tri": 2}
BASE = {"quad": 4, "sept": 7, "tri": 4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    from paper_1204_3105_amd import fmm
    fmm.lib()
    return fmm


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def geom_of(orc, plan, tiling):
    inf = plan.info()
    return orc.geom(tiling, inf["lmax"], *inf["geometry"]), inf


def level_keys(keys, tiling, L, l):
    if tiling == "sept":
        return keys // 7 ** (L - l)
    return keys >> (2 * (L - l))


def check_tree(F, orc, plan, w, tiling, list_sample=None):
    """Keys, permutations, cells, occupancy and ranges of every level
    bit-exact against the oracle; E4 lists of the target cells of every
    level >= 1 and near lists of the leaves against the oracle's, for all
    target cells or, with list_sample, a seeded sample of that many per level."""
    g, inf = geom_of(orc, plan, tiling)
    L = inf["lmax"]
    ex = plan.export_points()
    ks = orc.cell_index(g, w.xs, w.ys, L)
    kt = orc.cell_index(g, w.xt, w.yt, L)
    assert (ks >= 0).all() and (kt >= 0).all()
    assert np.array_equal(ex["src_keys"], ks), "source keys differ"
    assert np.array_equal(ex["tgt_keys"], kt), "target keys differ"
    assert np.array_equal(ex["src_perm"], np.argsort(ks, kind="stable"))
    assert np.array_equal(ex["tgt_perm"], np.argsort(kt, kind="stable"))
    sks = np.sort(ks)
    tks = np.sort(kt)
    w4 = inf["e4_width"]
    for l in range(L + 1):
        lv = plan.export_level(l)
        ls = level_keys(sks, tiling, L, l)
        lt = level_keys(tks, tiling, L, l)
        us, ut = np.unique(ls), np.unique(lt)
        cells = np.union1d(us, ut)
        assert np.array_equal(lv["keys"], cells), ("cells", l)
        occ = np.isin(cells, us).astype(int) + 2 * np.isin(cells, ut).astype(int)
        assert np.array_equal(lv["occupancy"], occ), ("occupancy", l)
        sb = np.searchsorted(ls, cells, "left")
        se = np.searchsorted(ls, cells, "right")
        tb = np.searchsorted(lt, cells, "left")
        te = np.searchsorted(lt, cells, "right")
        src_range = np.where((occ & 1)[:, None] > 0, np.stack([sb, se], 1), 0)
        tgt_range = np.where((occ & 2)[:, None] > 0, np.stack([tb, te], 1), 0)
        assert np.array_equal(lv["src_range"], src_range), ("src ranges", l)
        assert np.array_equal(lv["tgt_range"], tgt_range), ("tgt ranges", l)
        # E4 lists of target cells, restricted to source-occupied cells.
        pick = np.flatnonzero((occ & 2) > 0)
        if list_sample is not None and len(pick) > list_sample:
            pick = np.sort(np.random.default_rng(l).choice(pick, list_sample, replace=False))
        if l >= 1:
            tc = cells[pick]
            out, cnt = orc.e4_many(g, tc, l)
            rows = lv["e4"][pick]
            for i in range(len(tc)):
                want = np.sort(out[i, : cnt[i]][np.isin(out[i, : cnt[i]], us)])
                got = rows[i][rows[i] >= 0]
                assert np.array_equal(got, want), ("e4", l, tc[i])
        if l == L:
            tc = cells[pick]
            out, cnt = orc.neighbors_many(g, tc, l)
            rows = lv["near"][pick]
            for i in range(len(tc)):
                nb = np.concatenate([out[i, : cnt[i]], [tc[i]]])
                want = np.sort(nb[np.isin(nb, us)])
                got = rows[i][rows[i] >= 0]
                assert np.array_equal(got, want), ("near", tc[i])
    return g, inf


@pytest.mark.parametrize("tiling", TILES)
@pytest.mark.parametrize("n,seed", [(3000, 1), (20011, 2)])
def test_tree_and_fp64_potential_same_points(F, orc, tiling, n, seed):
    say("case", tiling, n, seed)
    w = inputs.uniform_square(n, seed=seed)
    with F.Plan(tiling, w.xs, w.ys, eps=1e-10, precision="fp64", leaf_size=32) as plan:
        g, inf = check_tree(F, orc, plan, w, tiling)
        phi = plan.eval(w.u)
        ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt, w.yt)
        assert rel(phi, ref) <= 1e-12, rel(phi, ref)


@pytest.mark.parametrize("tiling", TILES)
def test_fp64_separate_clustered(F, orc, tiling):
    say("clustered", tiling)
    w = inputs.gaussian_mixture(6000, 5000, seed=3)
    with F.Plan(tiling, w.xs, w.ys, w.xt, w.yt, eps=1e-6, precision="fp64", leaf_size=40) as plan:
        g, inf = check_tree(F, orc, plan, w, tiling)
        phi = plan.eval(w.u)
        ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt, w.yt)
        assert rel(phi, ref) <= 1e-12
        d1 = orc.direct_principal(w.xs, w.ys, w.u, w.xt, w.yt)
        assert rel(phi.real, d1.real) <= 1e-6


@pytest.mark.parametrize("tiling", TILES)
def test_fp64_matches_direct_sum_at_eps(F, orc, tiling):
    """N = M = 4096 uniform (the points of the quadtree p = 20 case), eps-derived p: rel L2 vs the
    principal direct sum (Re) and the branch-aware direct sum (complex)."""
    say("direct", tiling)
    w = inputs.uniform_square(4096, seed=1)
    with F.Plan(tiling, w.xs, w.ys, eps=1e-10, precision="fp64", leaf_size=32) as plan:
        g, inf = geom_of(orc, plan, tiling)
        phi = plan.eval(w.u)
    d1 = orc.direct_principal(w.xs, w.ys, w.u, w.xt, w.yt)
    d2 = orc.direct_branch_aware(g, w.xs, w.ys, w.u, w.xt, w.yt)
    assert rel(phi.real, d1.real) <= 1e-10
    assert rel(phi, d2) <= 1e-10


def test_quad_4096_p20(F, orc):
    """Quadtree FP64, N = M = 4096 uniform, p = 20, mean <= 32 per leaf."""
    w = inputs.uniform_square(4096, seed=1)
    with F.Plan("quad", w.xs, w.ys, eps=1e-6, p=20, precision="fp64", leaf_size=32) as plan:
        g, inf = geom_of(orc, plan, "quad")
        assert inf["p"] == 20 and inf["lmax"] == 4
        phi = plan.eval(w.u)
    ref = orc.fmm(g, 20, w.xs, w.ys, w.u, w.xt, w.yt)
    assert rel(phi, ref) <= 1e-12
    d1 = orc.direct_principal(w.xs, w.ys, w.u, w.xt, w.yt)
    assert rel(phi.real, d1.real) <= 1e-6


@pytest.mark.parametrize("tiling", TILES)
def test_edge_cases(F, orc, tiling):
    say("edges", tiling)
    rng = np.random.default_rng(5)
    # empty sources: Phi = 0
    xt, yt = rng.random(100), rng.random(100)
    with F.Plan(tiling, np.zeros(0), np.zeros(0), xt, yt, eps=1e-6, precision="fp64") as p:
        assert np.all(p.eval(np.zeros(0)) == 0)
    # empty targets
    xs, ys, u = rng.random(50), rng.random(50), rng.uniform(-1, 1, 50)
    with F.Plan(tiling, xs, ys, np.zeros(0), np.zeros(0), eps=1e-6, precision="fp64") as p:
        assert p.eval(u).shape == (0,)
    # a single point (source = target): no self interaction
    with F.Plan(tiling, xs[:1], ys[:1], eps=1e-6, precision="fp64") as p:
        assert np.all(p.eval(u[:1]) == 0)
    # two points, exact log
    with F.Plan(tiling, xs[:2], ys[:2], eps=1e-6, precision="fp64") as p:
        phi = p.eval(u[:2])
        want0 = u[1] * np.log(complex(xs[0] - xs[1], ys[0] - ys[1]))
        assert abs(phi[0].real - want0.real) < 1e-14
    # duplicate points: coincident pairs skipped in both codes
    xd = np.concatenate([xs, xs[:10]])
    yd = np.concatenate([ys, ys[:10]])
    ud = np.concatenate([u, u[:10]])
    with F.Plan(tiling, xd, yd, eps=1e-10, precision="fp64", leaf_size=8) as p:
        g, inf = geom_of(orc, p, tiling)
        phi = p.eval(ud)
    ref = orc.fmm(g, inf["p"], xd, yd, ud, xd, yd)
    assert rel(phi, ref) <= 1e-12


def test_invalid_inputs(F):
    w = inputs.uniform_square(100, seed=1)
    with pytest.raises(F.FMMError):
        F.Plan("quad", w.xs, w.ys, eps=0.0)
    bad = w.xs.copy()
    bad[3] = np.nan
    with pytest.raises(F.FMMError):
        F.Plan("quad", bad, w.ys, eps=1e-6)
    with pytest.raises(F.FMMError):
        F.Plan("quad", w.xs, w.ys, eps=1e-6, geometry=(0.5, 0.5, 0.1), lmax=2)


@pytest.mark.parametrize("tiling", TILES)
def test_fp64_symmetric_uneven_leaves(F, orc, tiling):
    """FP64, targets = sources, clustered with leaf 160 and 400 repeated
    points: the symmetric near field takes neighbour pairs whose lower leaf
    has at most two chunks of 64 targets once for both sides and the rest
    one-sided; coincident points are skipped.  Same bar as every FP64
    potential."""
    g = inputs.rng(43)
    xs, ys = inputs.gaussian_mixture_points(g, 12000, 6, 0.03)
    xs = np.concatenate([xs, xs[:400]])
    ys = np.concatenate([ys, ys[:400]])
    u = g.uniform(-1.0, 1.0, len(xs))
    with F.Plan(tiling, xs, ys, p=12, precision="fp64", leaf_size=160) as plan:
        inf = plan.info()
        phi = plan.eval(u)
        lv = plan.export_level(inf["lmax"])
    big = int(np.sum(np.diff(lv["src_range"], axis=1) > 128))
    g2 = orc.geom(tiling, inf["lmax"], *inf["geometry"])
    ref = orc.fmm(g2, inf["p"], xs, ys, u, xs, ys)
    e = rel(phi, ref)
    say("fp64 symmetric %s L=%d leaves>128: %d, rel_l2=%.3e" % (tiling, inf["lmax"], big, e))
    assert big > 0
    assert e <= 1e-12


def test_fp64_symmetric_every_tile_shape(F, orc):
    """FP64, targets = sources, quadtree at explicit depths chosen so that the
    leaves take every shape of the symmetric near field: blocks of four rows
    (items of up to 48 targets, 2..12 blocks), blocks of eight rows (49..96
    targets, 7..12 blocks) and chunks of 64 (larger leaves).  Same bar as
    every FP64 potential."""
    seen = set()
    for n, L, seed in ((12000, 5, 61), (12000, 4, 62), (20000, 4, 63)):
        w = inputs.uniform_square(n, seed=seed)
        with F.Plan("quad", w.xs, w.ys, eps=1e-10, precision="fp64", lmax=L) as plan:
            inf = plan.info()
            phi = plan.eval(w.u)
            lv = plan.export_level(L)
        sizes = np.diff(lv["tgt_range"], axis=1).ravel()
        for m in sizes[sizes > 0]:
            items = [m] if m <= 96 else [64] * (m // 64) + ([m % 64] if m % 64 else [])
            for c in items:
                seen.add((4, max(2, (c + 3) // 4)) if c <= 48 else (8, (c + 7) // 8))
        g = orc.geom("quad", L, *inf["geometry"])
        ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt, w.yt)
        e = rel(phi, ref)
        say("tile shapes: n=%d L=%d leaves %d..%d, rel_l2=%.3e" % (n, L, sizes[sizes > 0].min(), sizes.max(), e))
        assert e <= 1e-12
    need = {(4, b) for b in range(2, 13)} | {(8, b) for b in range(7, 13)}
    assert need <= seen, sorted(need - seen)
