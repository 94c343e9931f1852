"""Seeded synthetic workloads for the 2D log-kernel FMM.

This module draws random inputs only; it holds none of the method's
arithmetic.  The test suite and the benchmark feed the same arrays to the GPU
library and to the CPU oracle.  All draws use numpy's PCG64 generator; the
draw order is source x, source y, strengths, then targets.

The paper's experiments use synthetic uniform points (Sec. 9); the shapes
below (unit square, Gaussian clusters, unit disk, a Poisson request stream)
are the workload families the benchmark is quoted on.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MEBI = 1 << 20


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclass
class Workload:
    xs: np.ndarray
    ys: np.ndarray
    u: np.ndarray
    xt: np.ndarray
    yt: np.ndarray
    same: bool = False            # targets are the source array itself
    meta: dict = field(default_factory=dict)

    @property
    def n_src(self) -> int:
        return len(self.xs)

    @property
    def n_tgt(self) -> int:
        return len(self.xt)


def uniform_square(n: int, seed: int, m: int | None = None, targets_same: bool = True) -> Workload:
    """n sources uniform in [0,1]^2 with strengths U[-1,1]; targets are the
    sources (targets_same) or m separate uniform draws."""
    g = rng(seed)
    xs = g.random(n)
    ys = g.random(n)
    u = g.uniform(-1.0, 1.0, n)
    if targets_same:
        return Workload(xs, ys, u, xs, ys, True, {"kind": "uniform_square", "seed": seed})
    m = n if m is None else m
    xt = g.random(m)
    yt = g.random(m)
    return Workload(xs, ys, u, xt, yt, False, {"kind": "uniform_square", "seed": seed})


def gaussian_mixture_points(g: np.random.Generator, n: int, k: int, sigma: float):
    centres = g.random((k, 2))
    label = g.integers(0, k, n)
    pts = centres[label] + sigma * g.standard_normal((n, 2))
    return pts[:, 0].copy(), pts[:, 1].copy()


def gaussian_mixture(n_src: int, n_tgt: int, seed: int, k: int = 8, sigma: float = 0.02) -> Workload:
    """Sources from k isotropic Gaussians (centres U[0,1]^2, equal weights),
    strengths N(0,1); targets uniform in [0,1]^2, a separate draw."""
    g = rng(seed)
    xs, ys = gaussian_mixture_points(g, n_src, k, sigma)
    u = g.standard_normal(n_src)
    xt = g.random(n_tgt)
    yt = g.random(n_tgt)
    return Workload(xs, ys, u, xt, yt, False,
                    {"kind": "gaussian_mixture", "seed": seed, "k": k, "sigma": sigma})


def unit_disk(n: int, seed: int) -> Workload:
    """n points uniform in the unit disk (radius sqrt(U), angle 2 pi U),
    strengths U[-1,1], targets = sources."""
    g = rng(seed)
    rad = np.sqrt(g.random(n))
    ang = 2.0 * np.pi * g.random(n)
    xs = rad * np.cos(ang)
    ys = rad * np.sin(ang)
    u = g.uniform(-1.0, 1.0, n)
    return Workload(xs, ys, u, xs, ys, True, {"kind": "unit_disk", "seed": seed})


@dataclass
class Request:
    t_arrival: float
    tiling: str
    eps: float
    work: Workload


def serving_stream(n_requests: int, seed: int, rate: float, n_lo: float = 1e3, n_hi: float = 2e6,
                   max_n: int | None = None) -> list:
    """Poisson stream of solve requests: N = round(10^U(log10 n_lo, log10 n_hi)),
    sources uniform in [0,1]^2 or a 4-Gaussian mixture (sigma 0.03) with a
    50/50 seeded choice, tiling uniform over the three, eps in {1e-4, 1e-8},
    strengths U[-1,1], targets = sources.  Arrival gaps ~ Exp(rate)."""
    g = rng(seed)
    t = 0.0
    out = []
    tilings = ("quad", "sept", "tri")
    for _ in range(n_requests):
        t += g.exponential(1.0 / rate)
        n = int(round(10.0 ** g.uniform(np.log10(n_lo), np.log10(n_hi))))
        if max_n is not None:
            n = min(n, max_n)
        tiling = tilings[int(g.integers(0, 3))]
        eps = (1e-4, 1e-8)[int(g.integers(0, 2))]
        clustered = bool(g.integers(0, 2))
        if clustered:
            xs, ys = gaussian_mixture_points(g, n, 4, 0.03)
        else:
            xs = g.random(n)
            ys = g.random(n)
        u = g.uniform(-1.0, 1.0, n)
        w = Workload(xs, ys, u, xs, ys, True,
                     {"kind": "gaussian4" if clustered else "uniform_square"})
        out.append(Request(t, tiling, eps, w))
    return out


def polygon_points(g: np.random.Generator, cx, cy, n_sides, radius, rotation, counts):
    """Uniform points in regular polygons by the point picking of Sec. 9.

    Cell c is the regular n_sides[c]-gon with centre (cx[c], cy[c]),
    circumradius radius[c] and its first vertex at angle rotation[c]; it gets
    counts[c] points.  The polygon is cut into n isosceles triangles (centre
    and one edge); each triangle's two halves (split along its altitude) fit
    together into an s/2 x a rectangle (s the edge, a the apothem).  A point
    (x, y) uniform in the rectangle, folded back onto the half-triangle it
    lies in, is uniform in the triangle, and a third uniform z picks the
    triangle.  Draw order: x, y, z for all points of all cells.  Returns the
    (x, y) arrays, cell after cell."""
    cx, cy = np.asarray(cx, dtype=np.float64), np.asarray(cy, dtype=np.float64)
    n_sides = np.broadcast_to(np.asarray(n_sides, dtype=np.int64), cx.shape)
    radius = np.broadcast_to(np.asarray(radius, dtype=np.float64), cx.shape)
    rotation = np.broadcast_to(np.asarray(rotation, dtype=np.float64), cx.shape)
    counts = np.broadcast_to(np.asarray(counts, dtype=np.int64), cx.shape)
    cell = np.repeat(np.arange(len(cx)), counts)
    total = len(cell)
    x, y, z = g.random(total), g.random(total), g.random(total)
    n = n_sides[cell]
    half = np.pi / n
    s2 = radius[cell] * np.sin(half)          # half the edge
    a = radius[cell] * np.cos(half)           # apothem
    px, py = x * s2, y * a                    # uniform in the rectangle [0, s/2] x [0, a]
    # Local frame of the triangle: centre at 0, its edge's midpoint at (0, a).
    # Above the diagonal from (0, 0) to (s/2, a): the right half as it is;
    # below it: reflected onto the left half.
    below = py * s2 < px * a
    lx = np.where(below, px - s2, px)
    ly = np.where(below, a - py, py)
    k = np.minimum((z * n).astype(np.int64), n - 1)
    th = rotation[cell] + half + 2.0 * np.pi * k / n   # direction of triangle k's apothem
    ct, st = np.cos(th), np.sin(th)
    return cx[cell] + ly * ct + lx * st, cy[cell] + ly * st - lx * ct


def subsample(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct sorted indices out of n (k >= n gives all)."""
    if k >= n:
        return np.arange(n)
    return np.sort(rng(seed).choice(n, size=k, replace=False))
