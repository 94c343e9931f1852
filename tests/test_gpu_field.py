"""The field output Phi'(y) = sum_i u_i / (y - x_i) (fmm_eval_field) against
the oracle's FMM field on the same exported geometry and p.

Bars: FP64 plans rel L2 <= 1e-12 against the oracle's FMM field (the same
arithmetic as the potential's bar); mixed plans rel L2 <= eps against it
(the field's near part in compensated FP32, the far part through the
BF16x3 M2L, as the potential); both within their eps of the direct field.
For a plan whose targets are its sources eval takes the symmetric near field
and eval_field the one-sided one; their potentials agree to 1e-13 (FP64) and
eps / 10 (mixed) in relative L2.
"""
import sys

import numpy as np
import pytest

from paper_1204_3105_amd import inputs

pytestmark = pytest.mark.gpu
TILES = ["quad", "sept", "tri"]


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


@pytest.mark.parametrize("tiling", TILES)
@pytest.mark.parametrize("prec,eps", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_field_same_points(F, orc, tiling, prec, eps):
    w = inputs.uniform_square(20011, seed=31)
    say("field %s %s eps %g N=M=20011 (host pointers)" % (tiling, prec, eps))
    with F.Plan(tiling, w.xs, w.ys, eps=eps, precision=prec, leaf_size=64) as plan:
        phi, fld = plan.eval_field(w.u)
        phi2 = plan.eval(w.u)
        inf = plan.info()
    # eval takes the symmetric near field here (targets = sources),
    # eval_field the one-sided one: the two potentials agree to the rounding
    # of the near sums (FP64, or FP32 in the mixed form)
    e_pp = rel(phi, phi2)
    say("  %s phi(eval_field) vs phi(eval) %.3e" % (prec, e_pp))
    assert e_pp <= (1e-13 if prec == "fp64" else eps / 10)
    g = orc.geom(tiling, inf["lmax"], *inf["geometry"])
    rphi, rfld = orc.fmm_field(g, inf["p"], w.xs, w.ys, w.u, w.xt, w.yt)
    d = orc.direct_field(w.xs, w.ys, w.u, w.xt, w.yt)
    e_or, e_dir, e_phi = rel(fld, rfld), rel(fld, d), rel(phi, rphi)
    say("  p=%d L=%d field vs oracle %.3e, vs direct %.3e; phi vs oracle %.3e"
        % (inf["p"], inf["lmax"], e_or, e_dir, e_phi))
    assert e_or <= (1e-12 if prec == "fp64" else eps)
    assert e_dir <= eps


@pytest.mark.parametrize("tiling", ["sept", "tri"])
def test_field_separate_clustered(F, orc, tiling):
    w = inputs.gaussian_mixture(12007, 5003, seed=32)
    say("field %s clustered 12007 -> 5003, fp64 p=16 and mixed eps 1e-6" % tiling)
    for prec, kw in (("fp64", dict(p=16, eps=1e-6)), ("mixed", dict(eps=1e-6))):
        with F.Plan(tiling, w.xs, w.ys, w.xt, w.yt, precision=prec, leaf_size=32, **kw) as plan:
            _, fld = plan.eval_field(w.u)
            inf = plan.info()
        g = orc.geom(tiling, inf["lmax"], *inf["geometry"])
        _, rfld = orc.fmm_field(g, inf["p"], w.xs, w.ys, w.u, w.xt, w.yt)
        e = rel(fld, rfld)
        say("  %s p=%d field vs oracle %.3e" % (prec, inf["p"], e))
        assert e <= (1e-12 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("tiling", TILES)
def test_field_full_size_device(F, orc, tiling):
    """2^20 uniform points on torch's stream (the benchmark's launch shape),
    mixed and FP64 at eps 1e-6; 256 sampled targets against the oracle's FMM
    field over all sources."""
    import torch
    w = inputs.uniform_square(1 << 20, seed=2)
    say("field %s 2^20 device eps 1e-6" % tiling)
    dev = torch.device("cuda:0")
    src = torch.tensor(w.xs + 1j * w.ys, dtype=torch.complex128, device=dev)
    u = torch.tensor(w.u, dtype=torch.float64, device=dev)
    idx = inputs.subsample(w.n_tgt, 256, 33)
    ref = None
    for prec in ("fp64", "mixed"):
        plan = F.Plan(tiling, src=src, tgt=src, eps=1e-6, precision=prec, leaf_size=64)
        phi, fld = plan.eval_field(u)
        phi_only = plan.eval(u)
        inf = plan.info()
        plan.close()
        # symmetric near field in eval (targets = sources)
        d = float(torch.linalg.norm(phi - phi_only) / torch.linalg.norm(phi_only))
        say("  %s phi(eval_field) vs phi(eval) %.3e" % (prec, d))
        assert d <= (1e-13 if prec == "fp64" else 1e-7)
        fld = fld.cpu().numpy()
        if ref is None:
            g = orc.geom(tiling, inf["lmax"], *inf["geometry"])
            _, ref = orc.fmm_field(g, inf["p"], w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
        e = rel(fld[idx], ref)
        say("  %s p=%d L=%d sampled field vs oracle %.3e" % (prec, inf["p"], inf["lmax"], e))
        assert e <= (1e-12 if prec == "fp64" else 1e-6)


def test_field_edge_cases(F):
    say("field edge cases: no sources, one source")
    with F.Plan("quad", np.zeros(0), np.zeros(0), np.array([0.1, 0.7]), np.array([0.2, 0.3]),
                eps=1e-6) as plan:
        phi, fld = plan.eval_field(np.zeros(0))
        assert np.all(phi == 0) and np.all(fld == 0)
    xs, ys = np.array([0.25]), np.array([0.5])
    xt, yt = np.array([0.25, 0.75, 0.5]), np.array([0.5, 0.5, 0.9])
    with F.Plan("tri", xs, ys, xt, yt, eps=1e-10, precision="fp64") as plan:
        _, fld = plan.eval_field(np.array([2.0]))
    want = 2.0 / ((xt - xs[0]) + 1j * (yt - ys[0]))
    want[0] = 0
    assert np.max(np.abs(fld - want)) < 1e-12
