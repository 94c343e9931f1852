"""GPU parity of the mixed-precision form (BF16x3 MFMA M2L, FP32 compensated
P2P, FP64 monopole/log terms, P2M, M2M, L2L, L2P) against the FP64 oracle
on the same tree and p.  The bar is the requested eps = 1e-6 in relative L2
(the error is printed for every case)."""
import sys

import numpy as np
import pytest

from paper_1204_3105_amd import inputs

pytestmark = pytest.mark.gpu
EPS = 1e-6


@pytest.fixture(scope="module")
def F():
    from paper_1204_3105_amd import fmm
    fmm.lib()
    return fmm


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run(F, orc, tiling, w, **kw):
    with F.Plan(tiling, w.xs, w.ys, None if w.same else w.xt, None if w.same else w.yt,
                eps=EPS, precision="mixed", **kw) as plan:
        inf = plan.info()
        assert inf["precision"] == "mixed"
        phi = plan.eval(w.u)
    g = orc.geom(tiling, inf["lmax"], *inf["geometry"])
    ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt, w.yt)
    return phi, ref, inf


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
@pytest.mark.parametrize("n,seed,leaf", [(4096, 1, 32), (30011, 2, 64)])
def test_mixed_uniform(F, orc, tiling, n, seed, leaf):
    w = inputs.uniform_square(n, seed=seed)
    phi, ref, inf = run(F, orc, tiling, w, leaf_size=leaf)
    e = rel(phi, ref)
    print("mixed %s n=%d p=%d L=%d rel_l2=%.3e" % (tiling, n, inf["p"], inf["lmax"], e), flush=True)
    assert e <= EPS


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_mixed_clustered_separate(F, orc, tiling):
    w = inputs.gaussian_mixture(12000, 9000, seed=3)
    phi, ref, inf = run(F, orc, tiling, w, leaf_size=64)
    e = rel(phi, ref)
    print("mixed clustered %s rel_l2=%.3e" % (tiling, e), flush=True)
    assert e <= EPS


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_mixed_against_direct_sum(F, orc, tiling):
    w = inputs.uniform_square(4096, seed=1)
    phi, ref, inf = run(F, orc, tiling, w, leaf_size=32)
    d1 = orc.direct_principal(w.xs, w.ys, w.u, w.xt, w.yt)
    e = rel(phi.real, d1.real)
    print("mixed %s vs direct rel_l2(Re)=%.3e" % (tiling, e), flush=True)
    assert e <= EPS


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_mixed_unit_disk_high_order(F, orc, tiling):
    """Mixed arithmetic at a higher order (eps = 1e-8 asks for p up to 36):
    the error floor of the split products stays below 1e-6."""
    w = inputs.unit_disk(20000, seed=4)
    with F.Plan(tiling, w.xs, w.ys, eps=1e-8, precision="mixed") as plan:
        inf = plan.info()
        phi = plan.eval(w.u)
    g = orc.geom(tiling, inf["lmax"], *inf["geometry"])
    ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt, w.yt)
    e = rel(phi, ref)
    print("mixed disk %s p=%d rel_l2=%.3e" % (tiling, inf["p"], e), flush=True)
    assert e <= 1e-6


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_mixed_symmetric_uneven_leaves(F, orc, tiling):
    """Targets = sources, clustered, with 400 repeated points: leaves range
    from a few to several hundred points, so the symmetric near field takes
    the pairs whose lower leaf has at most two chunks of 64 targets for both
    sides and the others one-sided from both leaves; coincident points are
    skipped.  The leaf neighbour lists it relies on are symmetric."""
    g = inputs.rng(41)
    xs, ys = inputs.gaussian_mixture_points(g, 14000, 6, 0.03)
    xs = np.concatenate([xs, xs[:400]])
    ys = np.concatenate([ys, ys[:400]])
    u = g.uniform(-1.0, 1.0, len(xs))
    with F.Plan(tiling, xs, ys, eps=EPS, precision="mixed", leaf_size=160) as plan:
        inf = plan.info()
        phi = plan.eval(u)
        lv = plan.export_level(inf["lmax"])
    sizes = np.diff(lv["src_range"], axis=1).ravel()
    big = int(np.sum(sizes > 128))
    nb = {int(k): set(int(c) for c in row if c >= 0) for k, row in zip(lv["keys"], lv["near"])}
    for a, row in nb.items():
        for b in row:
            assert a in nb[b], ("near lists not symmetric", a, b)
    g2 = orc.geom(tiling, inf["lmax"], *inf["geometry"])
    ref = orc.fmm(g2, inf["p"], xs, ys, u, xs, ys)
    e = rel(phi, ref)
    print("mixed symmetric %s L=%d leaves>128: %d of %d, rel_l2=%.3e" %
          (tiling, inf["lmax"], big, len(sizes), e), flush=True)
    assert big > 0
    assert e <= EPS


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_near_stream_option_same_result(F, prec):
    """The near field on the plan's own stream (after the far field) gives
    bitwise the potential of the default side-stream schedule."""
    w = inputs.uniform_square(30011, seed=5)
    out = {}
    for ns in ("side", "own"):
        with F.Plan("tri", w.xs, w.ys, eps=1e-6, precision=prec, near_stream=ns) as plan:
            out[ns] = plan.eval(w.u)
    print("near_stream own vs side (%s): equal %s" % (prec, np.array_equal(out["own"], out["side"])), flush=True)
    assert np.array_equal(out["own"], out["side"])
