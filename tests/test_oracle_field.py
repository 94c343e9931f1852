"""Pins for the oracle's field output Phi'(y) = sum_i u_i / (y - x_i), the
derivative in y of eq. 2 (CPU only).

Re Phi is harmonic away from the sources, so the derivative of the analytic
Phi at y is c_1 = (2 / (K rho)) sum_k Re Phi(y + rho e^(i theta_k)) e^(-i theta_k)
over K equally spaced points of a source-free circle (the trapezoid rule on a
circle converges geometrically, here to rounding).  This uses only the
logarithm sums, so it checks the field formula (sign, conjugation,
coincident-pair rule) of the direct field and, on circles inside one target
leaf, the derivative of the local expansion in the oracle's FMM field.
"""
import numpy as np
import pytest

from paper_1204_3105_amd import inputs
from test_oracle_fmm import quad_geom, sept_geom, tri_geom

K = 48


def circle_derivative(values_re, rho):
    th = 2 * np.pi * np.arange(K) / K
    return (2.0 / (K * rho)) * (values_re.reshape(-1, K) * np.exp(-1j * th)).sum(axis=1)


def circle_points(xt, yt, rho):
    th = 2 * np.pi * np.arange(K) / K
    cx = (xt[:, None] + rho[:, None] * np.cos(th)).ravel()
    cy = (yt[:, None] + rho[:, None] * np.sin(th)).ravel()
    return cx, cy


def nearest_source(xs, ys, xt, yt):
    d = np.hypot(xt[:, None] - xs[None, :], yt[:, None] - ys[None, :])
    return d.min(axis=1)


def test_direct_field_is_derivative_of_potential(orc):
    w = inputs.uniform_square(600, seed=21, m=200, targets_same=False)
    rho = 0.3 * nearest_source(w.xs, w.ys, w.xt, w.yt)
    cx, cy = circle_points(w.xt, w.yt, rho)
    pot = orc.direct_principal(w.xs, w.ys, w.u, cx, cy).real
    want = circle_derivative(pot, rho)
    got = orc.direct_field(w.xs, w.ys, w.u, w.xt, w.yt)
    scale = np.sum(np.abs(w.u) / np.hypot(w.xt[:, None] - w.xs, w.yt[:, None] - w.ys), axis=1)
    assert np.max(np.abs(got - want) / scale) < 1e-11


def test_direct_field_special_cases(orc):
    # two equal sources symmetric about the target: the field vanishes
    f = orc.direct_field(np.array([0.2, 0.6]), np.array([0.5, 0.5]), np.array([0.7, 0.7]),
                         np.array([0.4]), np.array([0.5]))
    assert abs(f[0]) < 1e-15
    # one source: u / (y - x); a coincident pair is skipped
    f = orc.direct_field(np.array([0.0, 1.0]), np.array([0.0, 1.0]), np.array([2.0, 5.0]),
                         np.array([0.0]), np.array([1.0]))
    assert f[0] == 2.0 / (0 + 1j) + 5.0 / (-1 + 0j)
    f = orc.direct_field(np.array([0.3]), np.array([0.3]), np.array([1.0]), np.array([0.3]), np.array([0.3]))
    assert f[0] == 0


def test_fmm_field_potential_matches_fmm(orc):
    w = inputs.uniform_square(1500, seed=22)
    g = quad_geom(orc, w.xs, w.ys, 3)
    phi, fld = orc.fmm_field(g, 12, w.xs, w.ys, w.u, w.xt, w.yt)
    assert np.array_equal(phi, orc.fmm(g, 12, w.xs, w.ys, w.u, w.xt, w.yt))


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_fmm_field_is_derivative_of_fmm_potential(orc, tiling):
    """On circles inside the target's leaf and clear of every source, the
    FMM potential is the leaf's local expansion plus exact near terms, an
    analytic function; its circle derivative must equal the FMM field to
    rounding, at any p (p = 6 here, far from converged)."""
    w = inputs.uniform_square(1200, seed=23, m=400, targets_same=False)
    if tiling == "quad":
        g = quad_geom(orc, np.r_[w.xs, w.xt], np.r_[w.ys, w.yt], 3)
    elif tiling == "sept":
        g = sept_geom(orc, 0.5, 0.5, 0.05, 4)
    else:
        g = tri_geom(orc, 0.5, 0.5, 0.75, 4)
    L = g.L
    rho = 0.25 * nearest_source(w.xs, w.ys, w.xt, w.yt)
    ex, ey = circle_points(w.xt, w.yt, 1.02 * rho)
    own = orc.cell_index(g, w.xt, w.yt, L)
    inside = (own >= 0) & np.all(orc.cell_index(g, ex, ey, L).reshape(-1, K) == own[:, None], axis=1)
    assert inside.sum() > 100
    xt, yt, rho = w.xt[inside], w.yt[inside], rho[inside]
    cx, cy = circle_points(xt, yt, rho)
    p = 6
    pot = orc.fmm(g, p, w.xs, w.ys, w.u, cx, cy).real
    want = circle_derivative(pot, rho)
    _, got = orc.fmm_field(g, p, w.xs, w.ys, w.u, xt, yt)
    scale = np.sum(np.abs(w.u)) / rho
    assert np.max(np.abs(got - want) / scale) < 1e-11


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_fmm_field_converges_to_direct_field(orc, tiling):
    w = inputs.uniform_square(1500, seed=24)
    if tiling == "quad":
        g = quad_geom(orc, w.xs, w.ys, 3)
    elif tiling == "sept":
        g = sept_geom(orc, 0.5, 0.5, 0.05, 4)
    else:
        g = tri_geom(orc, 0.5, 0.5, 0.75, 4)
    d = orc.direct_field(w.xs, w.ys, w.u, w.xt, w.yt)
    errs = []
    for p in (6, 12, 18, 40):
        _, fld = orc.fmm_field(g, p, w.xs, w.ys, w.u, w.xt, w.yt)
        errs.append(np.linalg.norm(fld - d) / np.linalg.norm(d))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-11
