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
def test_mixed_request_below_floor_takes_fp64(F, orc, tiling):
    """A mixed request at eps = 1e-8, below the mixed arithmetic's floor
    (about 2e-8 in relative L2), is resolved to the FP64 form, which meets
    the FP64 bar against the oracle; at eps = 1e-6 it stays mixed."""
    w = inputs.unit_disk(20000, seed=4)
    with F.Plan(tiling, w.xs, w.ys, eps=1e-8, precision="mixed") as plan:
        inf = plan.info()
        phi = plan.eval(w.u)
    assert inf["precision"] == "fp64"
    g = orc.geom(tiling, inf["lmax"], *inf["geometry"])
    ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt, w.yt)
    e = rel(phi, ref)
    print("mixed request at eps 1e-8, disk %s p=%d rel_l2=%.3e" % (tiling, inf["p"], e), flush=True)
    assert e <= 1e-12
    with F.Plan(tiling, w.xs, w.ys, eps=1e-6, precision="mixed") as plan:
        assert plan.info()["precision"] == "mixed"
