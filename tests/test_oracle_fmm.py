"""Pins for the oracle's expansions, translations and full sweep, CPU only.

The oracle FMM is checked against: closed forms (a single source is
u Log(y - x)), exactness of the multipole and local shifts (Greengard-Rokhlin
Lemmas 2.3 and 2.5 are exact rearrangements), the monopole invariant
a_0 = sum u_i, brute-force direct sums (principal for Re, branch-aware for
the full complex value), the truncation bound of the paper's Sec. 8 and the
geometric decay of the error in p.
"""
import math

import numpy as np
import pytest

from paper_1204_3105_amd import inputs


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def quad_geom(orc, xs, ys, L):
    x0, y0 = min(xs.min(), 0.0), min(ys.min(), 0.0)
    w = max(xs.max() - x0, ys.max() - y0) * (1 + 2.0 ** -20)
    return orc.geom("quad", L, x0, y0, w)


def sept_geom(orc, cx, cy, r, L):
    return orc.geom("sept", L, cx, cy, r)


def tri_geom(orc, cx, cy, rho, L):
    return orc.geom("tri", L, cx, cy, 2.0 * rho / 2 ** L)


# ------------------------------------------------------------------ operators
def test_p2m_single_source_closed_form(orc):
    """One source: the multipole expansion reproduces u Log(z - x) outside
    the disk, with error below (r/R)^(p+1)/(1 - r/R) (|w|^(p+1) tail)."""
    p = 20
    c = 0.3 + 0.2j
    x, u = c + 0.1 * np.exp(0.7j), 0.8
    a = orc.p2m(p, c, [x.real], [x.imag], [u])
    assert a[0] == pytest.approx(u)
    zs = c + 0.4 * np.exp(1j * np.linspace(0, 2 * np.pi, 17)[:-1])
    got = orc.mpole_eval(p, a, c, zs.real, zs.imag)
    want = u * np.log(zs - x)
    q = 0.1 / 0.4
    bound = abs(u) * q ** (p + 1) / ((p + 1) * (1 - q))
    assert np.max(np.abs(got.real - want.real)) <= bound * 1.01
    # Imaginary parts agree up to a multiple of 2 pi u (branch of the log).
    k = (got.imag - want.imag) / (2 * np.pi * u)
    assert np.max(np.abs(got - want - 2j * np.pi * u * np.round(k))) <= bound * 1.01


def test_m2m_is_exact(orc):
    """Shifting a child's multipole to the parent equals forming the
    parent's multipole directly from the same sources (Lemma 2.3)."""
    p = 25
    rng = np.random.default_rng(3)
    cc = 0.25 + 0.25j
    cp = 0.5 + 0.5j
    x = cc + 0.2 * (rng.random(30) - 0.5) + 0.2j * (rng.random(30) - 0.5)
    u = rng.uniform(-1, 1, 30)
    a_child = orc.p2m(p, cc, x.real, x.imag, u)
    a_parent = orc.p2m(p, cp, x.real, x.imag, u)
    shifted = orc.m2m(p, a_child, cc - cp)
    scale = 0.5 ** np.arange(p + 1)
    assert np.max(np.abs(shifted - a_parent) / scale) < 1e-13
    # A planted error in the shift (wrong sign of z0) is detected.
    wrong = orc.m2m(p, a_child, cp - cc)
    assert np.max(np.abs(wrong - a_parent) / scale) > 1e-3


def test_l2l_is_exact(orc):
    """The local shift re-expands the same polynomial (Lemma 2.5)."""
    p = 18
    rng = np.random.default_rng(5)
    b = rng.standard_normal(p + 1) + 1j * rng.standard_normal(p + 1)
    cp, cc = 0.1 + 0.2j, 0.15 + 0.17j
    bc = orc.l2l(p, b, cc - cp)
    z = cc + 0.05 * (rng.random(20) - 0.5) + 0.05j * (rng.random(20) - 0.5)
    v1 = orc.l2p(p, b, cp, z.real, z.imag)
    v2 = orc.l2p(p, bc, cc, z.real, z.imag)
    assert np.max(np.abs(v1 - v2)) < 1e-13 * np.max(np.abs(v1))


def test_m2l_matches_far_sum(orc):
    """The local expansion from M2L agrees with the direct sum of the
    sources within the (1/(1+rho/r))^(p+1) bound."""
    p = 10
    rng = np.random.default_rng(9)
    cs, ct = 0.0 + 0.0j, 2.0 + 0.5j
    r = 0.5
    n = 40
    x = cs + r * np.sqrt(rng.random(n)) * np.exp(2j * np.pi * rng.random(n))
    u = rng.uniform(-1, 1, n)
    a = orc.p2m(p, cs, x.real, x.imag, u)
    b = orc.m2l(p, a, cs, ct)
    y = ct + r * np.sqrt(rng.random(25)) * np.exp(2j * np.pi * rng.random(25))
    got = orc.l2p(p, b, ct, y.real, y.imag)
    # Branch of M2L: Log(c_T - c_S) + Log((y - x)/(c_T - c_S)).
    dc = ct - cs
    want = np.array([np.sum(u * (np.log(dc) + np.log((yy - x) / dc))) for yy in y])
    d = abs(ct - cs)
    q = r / (d - r)
    bound = np.sum(np.abs(u)) * (q ** (p + 1) / (1 - q)) * 4
    err = np.max(np.abs(got - want))
    assert err <= bound + 1e-13
    assert err > 1e-12          # truncation, not rounding, is being measured
    # p = 30 drives the truncation error below 1e-12.
    a30 = orc.p2m(30, cs, x.real, x.imag, u)
    got30 = orc.l2p(30, orc.m2l(30, a30, cs, ct), ct, y.real, y.imag)
    assert np.max(np.abs(got30 - want)) < 1e-12


def test_m2l_log_branch_on_negative_axis(orc):
    """Horizontally aligned cells with the source to the right: the log
    term takes +pi (canonical +0 imaginary part)."""
    p = 4
    a = np.zeros(p + 1, dtype=complex)
    a[0] = 1.0
    b = orc.m2l(p, a, 2.0 + 0.5j, 0.0 + 0.5j)
    assert b[0].imag == pytest.approx(math.pi)


# -------------------------------------------------------------- upward pass
@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_monopole_invariant(orc, tiling):
    w = inputs.uniform_square(3000, seed=21)
    if tiling == "quad":
        g = quad_geom(orc, w.xs, w.ys, 4)
    elif tiling == "sept":
        g = sept_geom(orc, 0.5, 0.5, 0.035, 4)
    else:
        g = tri_geom(orc, 0.5, 0.5, 0.75, 5)
    p = 10
    for lvl in range(1, g.L + 1):
        keys, coef = orc.upward_level(g, p, w.xs, w.ys, w.u, lvl)
        lk = orc.cell_index(g, w.xs, w.ys, lvl)
        for k, a in zip(keys, coef):
            assert abs(a[0] - w.u[lk == k].sum()) < 1e-12
            assert a[0].imag == 0.0


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_upward_pass_equals_direct_p2m(orc, tiling):
    """After M2M, each coarse multipole equals P2M of its sources formed
    directly at the coarse centre (the shift is exact)."""
    w = inputs.uniform_square(1500, seed=22)
    if tiling == "quad":
        g = quad_geom(orc, w.xs, w.ys, 4)
    elif tiling == "sept":
        g = sept_geom(orc, 0.5, 0.5, 0.035, 4)
    else:
        g = tri_geom(orc, 0.5, 0.5, 0.75, 5)
    p = 16
    lvl = 2
    keys, coef = orc.upward_level(g, p, w.xs, w.ys, w.u, lvl)
    lk = orc.cell_index(g, w.xs, w.ys, lvl)
    cx, cy = orc.cell_center(g, keys, lvl)
    for k, a, x0, y0 in zip(keys, coef, cx, cy):
        m = lk == k
        direct = orc.p2m(p, complex(x0, y0), w.xs[m], w.ys[m], w.u[m])
        rad = np.max(np.abs((w.xs[m] + 1j * w.ys[m]) - complex(x0, y0)))
        scale = np.maximum(rad, 1e-300) ** np.arange(p + 1) * max(1.0, np.abs(direct[0]))
        assert np.max(np.abs(direct - a) / scale) < 1e-11


# -------------------------------------------------------------- full sweep
def uniform_4096(orc, n=4096, seed=1):
    w = inputs.uniform_square(n, seed=seed)
    return w, quad_geom(orc, w.xs, w.ys, 4)


def test_fmm_quad_4096_against_direct(orc):
    """Quadtree, N = M = 4096 uniform, p = 20, mean 16 per leaf: relative
    L2 error of Re vs the principal direct sum and of the complex value vs
    the branch-aware direct sum."""
    w, g = uniform_4096(orc)
    phi = orc.fmm(g, 20, w.xs, w.ys, w.u, w.xt, w.yt)
    d1 = orc.direct_principal(w.xs, w.ys, w.u, w.xt, w.yt)
    d2 = orc.direct_branch_aware(g, w.xs, w.ys, w.u, w.xt, w.yt)
    assert rel(phi.real, d1.real) < 1e-8
    assert rel(phi, d2) < 1e-8
    assert np.array_equal(d1.real, d2.real) or rel(d1.real, d2.real) < 1e-14
    # Im differs from the principal sum by multiples of 2 pi u_i only.
    assert np.max(np.abs(phi.imag - d1.imag)) > 1.0


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_fmm_converges_to_branch_aware_sum(orc, tiling):
    w = inputs.uniform_square(2000, seed=4)
    if tiling == "quad":
        g = quad_geom(orc, w.xs, w.ys, 3)
    elif tiling == "sept":
        g = sept_geom(orc, 0.5, 0.5, 0.04, 4)
    else:
        g = tri_geom(orc, 0.5, 0.5, 0.75, 4)
    d1 = orc.direct_principal(w.xs, w.ys, w.u, w.xt, w.yt)
    d2 = orc.direct_branch_aware(g, w.xs, w.ys, w.u, w.xt, w.yt)
    phi = orc.fmm(g, 45, w.xs, w.ys, w.u, w.xt, w.yt)
    assert rel(phi.real, d1.real) < 1e-12
    assert rel(phi, d2) < 1e-12


@pytest.mark.parametrize("tiling,q", [("quad", 0.5469), ("sept", 0.5244), ("tri", 0.6076)])
def test_error_decays_geometrically_in_p(orc, tiling, q):
    """Sec. 9: the error falls exponentially in p, at a rate no slower than
    the separation ratio q of the tiling."""
    w = inputs.uniform_square(1200, seed=8)
    if tiling == "quad":
        g = quad_geom(orc, w.xs, w.ys, 3)
    elif tiling == "sept":
        g = sept_geom(orc, 0.5, 0.5, 0.05, 4)
    else:
        g = tri_geom(orc, 0.5, 0.5, 0.75, 4)
    d2 = orc.direct_branch_aware(g, w.xs, w.ys, w.u, w.xt, w.yt)
    errs = []
    for p in (4, 8, 12, 16, 20):
        phi = orc.fmm(g, p, w.xs, w.ys, w.u, w.xt, w.yt)
        errs.append(np.max(np.abs(phi - d2)))
    errs = np.array(errs)
    assert np.all(np.diff(np.log(errs)) < 0)
    rate = (errs[-1] / errs[0]) ** (1.0 / 16)
    assert rate < q * 1.02


@pytest.mark.parametrize("tiling", ["quad", "tri"])
def test_error_within_truncation_bound(orc, tiling):
    """Per target, |Phi - D2| is below the sum over far cells of the M2L
    bound sum|u| / rho * (1/(1+rho/r))^(p+1) of Sec. 8 with the tiling's
    table value of rho/r (bound read in units of the cell radius)."""
    w = inputs.uniform_square(1500, seed=12)
    rho_r = {"quad": 2 * (math.sqrt(2) - 1), "tri": math.sqrt(7) - 2}[tiling]
    if tiling == "quad":
        g = quad_geom(orc, w.xs, w.ys, 3)
    else:
        g = tri_geom(orc, 0.5, 0.5, 0.75, 4)
    p = 8
    d2 = orc.direct_branch_aware(g, w.xs, w.ys, w.u, w.xt, w.yt)
    phi = orc.fmm(g, p, w.xs, w.ys, w.u, w.xt, w.yt)
    q = 1.0 / (1.0 + rho_r)
    bound = np.sum(np.abs(w.u)) * q ** (p + 1) / (1 - q) * g.L
    assert np.max(np.abs(phi - d2)) < bound


def test_single_source_closed_form(orc):
    rng = np.random.default_rng(2)
    xs, ys, u = np.array([0.31]), np.array([0.77]), np.array([0.6])
    xt, yt = rng.random(500), rng.random(500)
    g = orc.geom("quad", 4, 0.0, 0.0, 1.0)
    phi = orc.fmm(g, 40, xs, ys, u, xt, yt)
    want = u[0] * np.log((xt - xs[0]) + 1j * (yt - ys[0]))
    assert np.max(np.abs(phi.real - want.real)) < 1e-13
    k = (phi.imag - want.imag) / (2 * np.pi * u[0])
    assert np.max(np.abs(k - np.round(k))) < 1e-12


def test_no_far_field_reduces_to_direct(orc):
    """With L = 1 no cell pair is well separated: the FMM is the direct sum."""
    w = inputs.uniform_square(600, seed=3)
    g = quad_geom(orc, w.xs, w.ys, 1)
    phi = orc.fmm(g, 10, w.xs, w.ys, w.u, w.xt, w.yt)
    d1 = orc.direct_principal(w.xs, w.ys, w.u, w.xt, w.yt)
    assert np.max(np.abs(phi - d1)) < 1e-12


def test_separate_targets_and_sample_invariance(orc):
    """With fixed geometry, the FMM value of a target does not depend on
    which other targets are evaluated (used to sample large workloads)."""
    w = inputs.uniform_square(3000, seed=6, m=2000, targets_same=False)
    g = quad_geom(orc, np.concatenate([w.xs, w.xt]), np.concatenate([w.ys, w.yt]), 4)
    full = orc.fmm(g, 12, w.xs, w.ys, w.u, w.xt, w.yt)
    idx = inputs.subsample(len(w.xt), 100, seed=1)
    part = orc.fmm(g, 12, w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
    assert np.array_equal(part, full[idx])
    d1 = orc.direct_principal(w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
    assert rel(part.real, d1.real) < 1e-5


def test_coincident_pairs_are_skipped(orc):
    xs = np.array([0.2, 0.2, 0.7])
    ys = np.array([0.3, 0.3, 0.1])
    u = np.array([1.0, 2.0, -0.5])
    d1 = orc.direct_principal(xs, ys, u, xs[:1], ys[:1])
    want = u[2] * np.log(complex(0.2 - 0.7, 0.3 - 0.1))
    assert abs(d1[0] - want) < 1e-15


def test_direct_on_a_lattice_takes_plus_pi_on_the_cut(orc):
    """D1 on a 9 x 7 lattice, targets = sources: many differences are exactly
    negative real (equal y, +0 imaginary part), where the principal Log has
    Im = +pi; coincident pairs are skipped.  Brute force with numpy's complex
    log on the same differences."""
    gx, gy = np.meshgrid(np.arange(9) / 9.0, np.arange(7) / 7.0)
    x, y = gx.ravel(), gy.ravel()
    u = np.random.default_rng(31).uniform(-1.0, 1.0, x.size)
    got = orc.direct_principal(x, y, u, x, y)
    want = np.zeros(x.size, dtype=complex)
    for j in range(x.size):
        for i in range(x.size):
            if i != j:
                want[j] += u[i] * np.log(complex(x[j] - x[i], y[j] - y[i]))
    assert np.max(np.abs(got - want)) <= 1e-13 * np.sum(np.abs(u)) * 10
    # a pair on the cut: the left neighbour seen from its right neighbour's
    # source has Im exactly pi
    assert np.log(complex(x[0] - x[1], y[0] - y[1])).imag == np.pi


@pytest.mark.parametrize("tiling", ["quad", "sept", "tri"])
def test_fmm_on_a_lattice_converges_to_branch_aware_sum(orc, tiling):
    """A 40 x 40 regular lattice, targets = sources: pairs exactly on the
    branch cut (equal y), pairs with dx = 0, points on cell edges.  At p = 45
    the FMM equals the branch-aware direct sum to rounding, and Re the
    principal one."""
    k = 40
    gx, gy = np.meshgrid(np.arange(k) / k, np.arange(k) / k)
    x, y = gx.ravel().copy(), gy.ravel().copy()
    u = np.random.default_rng(32).uniform(-1.0, 1.0, x.size)
    if tiling == "quad":
        g = quad_geom(orc, x, y, 3)
    elif tiling == "sept":
        g = sept_geom(orc, 0.5, 0.5, 0.04, 4)
    else:
        g = tri_geom(orc, 0.5, 0.5, 0.75, 4)
    d1 = orc.direct_principal(x, y, u, x, y)
    d2 = orc.direct_branch_aware(g, x, y, u, x, y)
    phi = orc.fmm(g, 45, x, y, u, x, y)
    assert rel(phi.real, d1.real) < 1e-12
    assert rel(phi, d2) < 1e-12
