"""The cost-model depth rule (depth="cost", FMM_DEPTH_COST) on clustered
inputs: the chosen level is deeper than the mean-occupancy level where
clusters make leaves crowded, and the plan at that level is still the paper's
uniform-depth tree, so keys, lists and potentials keep the oracle's bars
(trees bit-exact; FP64 rel L2 <= 1e-12, mixed <= eps on sampled targets)."""
import sys

import numpy as np
import pytest

from paper_1204_3105_amd import inputs
from test_gpu_parity import check_tree

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    from paper_1204_3105_amd import fmm
    fmm.lib()
    return fmm


def clustered_same(n, seed):
    g = inputs.rng(seed)
    xs, ys = inputs.gaussian_mixture_points(g, n, 8, 0.02)
    u = g.uniform(-1.0, 1.0, n)
    return inputs.Workload(xs, ys, u, xs, ys, True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_cost_depth_clustered_same_points(F, orc, tiling):
    w = clustered_same(200003, 41)
    say("depth rule: clustered 200003 same points, %s" % tiling)
    with F.Plan(tiling, w.xs, w.ys, eps=1e-6, precision="fp64") as pm:
        L0 = pm.info()["lmax"]
    plan = F.Plan(tiling, w.xs, w.ys, eps=1e-6, precision="fp64", depth="cost")
    inf = plan.info()
    say("  mean rule L=%d, cost rule L=%d" % (L0, inf["lmax"]))
    assert L0 <= inf["lmax"] <= L0 + 3
    if tiling == "quad":
        assert inf["lmax"] > L0
    check_tree(F, orc, plan, w, tiling)
    phi = plan.eval(w.u)
    plan.close()
    idx = inputs.subsample(w.n_tgt, 256, 42)
    g = orc.geom(tiling, inf["lmax"], *inf["geometry"])
    ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
    e = rel(phi[idx], ref)
    say("  tree bit-exact; FP64 rel L2 vs oracle %.3e" % e)
    assert e <= 1e-12


@pytest.mark.parametrize("tiling", ["sept", "tri"])
def test_cost_depth_clustered_sources_uniform_targets(F, orc, tiling):
    import torch
    w = inputs.gaussian_mixture(1 << 20, 1 << 20, seed=43)
    say("depth rule: 1M Gaussian-mixture sources -> 1M uniform targets, %s, mixed eps 1e-6" % tiling)
    dev = torch.device("cuda:0")
    src = torch.tensor(w.xs + 1j * w.ys, dtype=torch.complex128, device=dev)
    tgt = torch.tensor(w.xt + 1j * w.yt, dtype=torch.complex128, device=dev)
    u = torch.tensor(w.u, dtype=torch.float64, device=dev)
    plan = F.Plan(tiling, src=src, tgt=tgt, eps=1e-6, precision="mixed", depth="cost")
    phi = plan.eval(u).cpu().numpy()
    inf = plan.info()
    plan.close()
    idx = inputs.subsample(w.n_tgt, 128, 44)
    g = orc.geom(tiling, inf["lmax"], *inf["geometry"])
    ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
    e = rel(phi[idx], ref)
    say("  L=%d p=%d mixed rel L2 vs oracle %.3e" % (inf["lmax"], inf["p"], e))
    assert e <= 1e-6


def test_cost_depth_uniform_and_small(F, orc):
    say("depth rule: uniform 30011 and tiny inputs")
    w = inputs.uniform_square(30011, seed=45)
    with F.Plan("quad", w.xs, w.ys, eps=1e-10, precision="fp64", depth="cost") as plan:
        phi = plan.eval(w.u)
        inf = plan.info()
    g = orc.geom("quad", inf["lmax"], *inf["geometry"])
    idx = inputs.subsample(w.n_tgt, 256, 46)
    ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
    assert rel(phi[idx], ref) <= 1e-12
    for n in (1, 2, 7):
        v = inputs.uniform_square(n, seed=47)
        with F.Plan("sept", v.xs, v.ys, eps=1e-6, depth="cost") as plan:
            out = plan.eval(v.u)
        assert np.all(np.isfinite(out))
