"""The experiments of Sec. 9 re-run on the GPU.

Inputs are the paper's: S_opt uniform sources and S_opt separate uniform
targets in every occupied leaf cell (Table of FMM properties: S_opt =
p (c N/M)^(1/2) with c = 116/27, 308/42, 164/39 for quadtree, septree and
triangle-quadtree), drawn by regular-polygon point picking
(inputs.polygon_points); N is varied by the number of occupied leaf cells
(the cells nearest the root's centre).  Strengths are U[-1, 1].

Sweeps:
  n   runtime and max |Re(Phi_FMM - Phi_direct)| against N = M at p = 12,
      for two leaf levels per tiling, with the GPU direct sum timed beside
      it (the FMM/direct crossover);
  p   the same against p at N = M = 5120.
The FMM runs with the tree geometry given explicitly (leaf level and cell
lattice fixed, as in the paper), in FP64; the reference is the FP64 GPU
direct sum.  Times are wall-clock medians of plan + evaluate (and of the
direct sum) with device-resident inputs.

    python -m paper_1204_3105_amd.experiments --sweep n
    python -m paper_1204_3105_amd.experiments --sweep p
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import fmm, inputs

TILINGS = ("quad", "sept", "tri")
# S_opt coefficient c in p (c N / M)^(1/2), Table of FMM properties.
SOPT_COEF = {"quad": 116.0 / 27.0, "sept": 308.0 / 42.0, "tri": 164.0 / 39.0}
# Two leaf levels per tiling for the N sweep (4^L, 7^L, 4^L leaves).
N_SWEEP_LEVELS = {"quad": (5, 7), "sept": (3, 5), "tri": (5, 7)}


def s_opt(tiling: str, p: int, ratio: float = 1.0) -> int:
    """Optimal points per cell (N/M = ratio), rounded to the nearest integer."""
    return max(1, int(round(p * math.sqrt(SOPT_COEF[tiling] * ratio))))


def leaf_cells(tiling: str, L: int) -> dict:
    """Every leaf cell of the full tree of depth L.

    Returns centres, polygon shape (sides, circumradius, first-vertex angle
    per cell), the explicit plan geometry and the root centre:
      quad  root square [0, 1]^2, leaves of side 2^-L;
      sept  leaf hexagons of circumradius r = 7^(-L/2) (first vertex at
            angle 0), hexagon 0 at the origin, lattice point (a, b) at
            (3 r a / 2, sqrt3 r (a + 2 b) / 2); the leaves are the values
            sum_k d_k beta^k, d_k in {0, the six units}, beta = 1 + 2w;
      tri   root triangle with centroid 0, circumradius 1, apex up; leaf
            triangles of circumradius 2^-L, alternately up and down.
    """
    if tiling == "quad":
        h = 2.0 ** -L
        i, j = np.meshgrid(np.arange(1 << L), np.arange(1 << L), indexing="ij")
        cx, cy = (i.ravel() + 0.5) * h, (j.ravel() + 0.5) * h
        return dict(cx=cx, cy=cy, sides=4, radius=h / math.sqrt(2.0), rotation=math.pi / 4,
                    geometry=(0.0, 0.0, 1.0), centre=(0.5, 0.5))
    if tiling == "sept":
        r = 7.0 ** (-0.5 * L)
        units = np.array([(0, 0), (1, 0), (0, 1), (-1, 1), (-1, 0), (0, -1), (1, -1)], dtype=np.int64)
        a = np.zeros(1, dtype=np.int64)
        b = np.zeros(1, dtype=np.int64)
        for _ in range(L):
            # (a + b w) beta = (a - 2b) + (2a + 3b) w, then add each digit
            na, nb = a - 2 * b, 2 * a + 3 * b
            a = (na[None, :] + units[:, 0:1]).ravel()
            b = (nb[None, :] + units[:, 1:2]).ravel()
        cx = 1.5 * r * a
        cy = 0.5 * math.sqrt(3.0) * r * (a + 2 * b)
        return dict(cx=cx, cy=cy, sides=6, radius=r, rotation=0.0, geometry=(0.0, 0.0, r), centre=(0.0, 0.0))
    if tiling == "tri":
        r = 2.0 ** -L
        # centroids in units (U, V): x = U sqrt3 r / 2, y = V r / 2
        U = np.zeros(1, dtype=np.int64)
        V = np.zeros(1, dtype=np.int64)
        up = np.ones(1, dtype=np.int64)
        for i in range(1, L + 1):
            R = 1 << (L - i)
            U = np.concatenate([U, U, U - R, U + R])
            V = np.concatenate([V, V + 2 * up * R, V - up * R, V - up * R])
            up = np.concatenate([-up, up, up, up])
        cx = U * (math.sqrt(3.0) * r / 2.0)
        cy = V * (r / 2.0)
        rot = np.where(up > 0, math.pi / 2, -math.pi / 2)
        return dict(cx=cx, cy=cy, sides=3, radius=r, rotation=rot, geometry=(0.0, 0.0, r), centre=(0.0, 0.0))
    raise ValueError("tiling must be quad, sept or tri")


def nearest_cells(cells: dict, k: int) -> np.ndarray:
    """Indices of the k cells nearest the root's centre (ties by index)."""
    d = np.hypot(cells["cx"] - cells["centre"][0], cells["cy"] - cells["centre"][1])
    return np.argsort(d, kind="stable")[:k]


def cell_workload(tiling: str, L: int, n_cells: int, per_cell, seed: int) -> dict:
    """Sources and separate targets, per_cell of each in each of the n_cells
    leaves nearest the centre (per_cell: an int, or one count per cell)."""
    cells = leaf_cells(tiling, L)
    sel = nearest_cells(cells, n_cells)
    g = inputs.rng(seed)
    shape = {}
    for key in ("sides", "radius", "rotation"):
        v = np.broadcast_to(np.asarray(cells[key]), cells["cx"].shape)
        shape[key] = v[sel]
    counts = np.broadcast_to(np.asarray(per_cell, dtype=np.int64), sel.shape)
    xs, ys = inputs.polygon_points(g, cells["cx"][sel], cells["cy"][sel], shape["sides"], shape["radius"],
                                   shape["rotation"], counts)
    u = g.uniform(-1.0, 1.0, len(xs))
    xt, yt = inputs.polygon_points(g, cells["cx"][sel], cells["cy"][sel], shape["sides"], shape["radius"],
                                   shape["rotation"], counts)
    return dict(xs=xs, ys=ys, u=u, xt=xt, yt=yt, geometry=cells["geometry"], L=L, cells=sel)


def _median_ms(fn, reps: int) -> float:
    import torch
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(1e3 * (time.perf_counter() - t0))
    return float(np.median(ts))


def run_case(tiling: str, w: dict, p: int, reps: int = 5, direct_reps: int = 3, precision: str = "fp64") -> dict:
    """FMM (plan + evaluate) and direct-sum times and the max error of Re Phi."""
    import torch
    dev = torch.device("cuda:0")
    src = torch.tensor(w["xs"] + 1j * w["ys"], dtype=torch.complex128, device=dev)
    tgt = torch.tensor(w["xt"] + 1j * w["yt"], dtype=torch.complex128, device=dev)
    u = torch.tensor(w["u"], dtype=torch.float64, device=dev)
    out = torch.empty(len(w["xt"]), dtype=torch.complex128, device=dev)
    kw = dict(src=src, tgt=tgt, p=p, lmax=w["L"], geometry=w["geometry"], precision=precision)

    def fmm_once():
        with fmm.Plan(tiling, **kw) as plan:
            plan.eval(u, out=out)

    fmm_once()   # warm-up (first launches, pool)
    t_fmm = _median_ms(fmm_once, reps)
    with fmm.Plan(tiling, **kw) as plan:
        plan.eval(u, out=out)
        torch.cuda.synchronize()
        info = plan.info()
    phi = out.cpu().numpy()
    ref_dev = torch.empty_like(out)
    fmm.direct(None, None, u, src=src, tgt=tgt, out=ref_dev)
    t_dir = _median_ms(lambda: fmm.direct(None, None, u, src=src, tgt=tgt, out=ref_dev), direct_reps)
    ref = ref_dev.cpu().numpy()
    err = float(np.max(np.abs(phi.real - ref.real))) if len(ref) else 0.0
    return dict(tiling=tiling, N=len(w["xs"]), M=len(w["xt"]), p=p, lmax=w["L"], cells=int(len(w["cells"])),
                occupied=int(info["n_cells"][w["L"]]), fmm_ms=t_fmm, plan_ms=info["plan_ms"],
                eval_ms=info["eval_ms"], direct_ms=t_dir, max_abs_err=err)


def sweep_n(p: int = 12, seed: int = 11, emit=print) -> list:
    rows = []
    for tiling in TILINGS:
        S = s_opt(tiling, p)
        for L in N_SWEEP_LEVELS[tiling]:
            full = len(leaf_cells(tiling, L)["cx"])
            ks = sorted({max(1, int(round(full * 2.0 ** (-j / 2.0)))) for j in range(0, 40)})
            ks = [k for k in ks if k * S >= 300]
            for k in ks:
                w = cell_workload(tiling, L, k, S, seed)
                row = run_case(tiling, w, p)
                row["S"] = S
                emit(json.dumps(row))
                rows.append(row)
    return rows


def fixed_n_workload(tiling: str, n: int, seed: int, p_ref: int = 12) -> dict:
    """N = M = n points over round(n / S_opt(p_ref)) cells at the shallowest
    leaf level that has that many (n spread as evenly as possible)."""
    k = max(1, int(round(n / s_opt(tiling, p_ref))))
    L = 0
    while len(leaf_cells(tiling, L)["cx"]) < k:
        L += 1
    counts = np.full(k, n // k, dtype=np.int64)
    counts[: n - int(counts.sum())] += 1
    return cell_workload(tiling, L, k, counts, seed)


def sweep_p(n: int = 5120, seed: int = 12, ps=range(2, 31, 2), emit=print) -> list:
    """N = M = n fixed (fixed_n_workload), p varied."""
    rows = []
    for tiling in TILINGS:
        w = fixed_n_workload(tiling, n, seed)
        for p in ps:
            row = run_case(tiling, w, int(p))
            emit(json.dumps(row))
            rows.append(row)
    return rows


def crossover(rows: list) -> dict:
    """Per tiling and leaf level: the smallest N at which the FMM is faster
    than the direct sum, interpolated on log N between sweep points."""
    out = {}
    for key in sorted({(r["tiling"], r["lmax"]) for r in rows}):
        rs = sorted((r for r in rows if (r["tiling"], r["lmax"]) == key), key=lambda r: r["N"])
        hit = None
        for a, b in zip(rs, rs[1:]):
            da = math.log(a["direct_ms"] / a["fmm_ms"])
            db = math.log(b["direct_ms"] / b["fmm_ms"])
            if da < 0 <= db:
                t = -da / (db - da)
                hit = math.exp(math.log(a["N"]) + t * (math.log(b["N"]) - math.log(a["N"])))
                break
        if hit is None and rs and rs[0]["direct_ms"] >= rs[0]["fmm_ms"]:
            hit = float(rs[0]["N"])
        out["%s L=%d" % key] = hit
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--sweep", choices=("n", "p"), required=True)
    ap.add_argument("--out", default=None, help="also write the rows as JSON lines here")
    a = ap.parse_args(argv)
    f = open(a.out, "w") if a.out else None

    def emit(line):
        print(line, flush=True)
        if f:
            f.write(line + "\n")
            f.flush()

    rows = sweep_n(emit=emit) if a.sweep == "n" else sweep_p(emit=emit)
    if a.sweep == "n":
        emit(json.dumps({"crossover_N": crossover(rows)}))
    if f:
        f.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
