#!/usr/bin/env python
"""Benchmark: targets/sec of full FMM solves (plan + eval) at eps = 1e-6.

Workload: N = M = 2^20 sources = targets uniform in the unit square, strengths
U[-1,1] (seed 2), one solve per tiling (quadtree, septree, triangle-quadtree)
per step, leaf size 64, p from eps and each tiling's separation ratio.  A step
is plan + eval for all three tilings with the points already resident in HBM.

Prints one JSON line.  `value` is the plain FP64 form (every step in FP64,
the paper's arithmetic): 3 * M * steps / wall time of the timed steps.
`roofline` covers its dominant kernel (the FP64 P2P near field), timed with
HIP events on the stream it runs on, as VALU lane-operations per second
against the chip's VALU rate.  `cpu_baseline` is the CPU oracle on this
host's cores on the same workload (and on one core, on a sample).  `extra`
holds the mixed-precision form on the same workload, each tiling's solve
alone, FP64 at eps 1e-10, M2L against the MFMA peaks, the clustered and
16M unit-disk workloads, and the serving stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU lane-operations per second of one MI355X: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz for FP64 instructions (a wave64 FP64 instruction holds a SIMD for
# four cycles: 78.6 TFLOP/s counting an FMA as two), twice that for 32-bit
# ones (two cycles: 157.3 TFLOP/s FP32), which the mixed near field is
# measured against.
LANE_OPS = 256 * 4 * 16 * 2.4e9
LANE_OPS_32 = 2 * LANE_OPS
# VALU instructions per source-target pair in the near-field inner loops of
# the gfx950 code (counted in the kernels' AMD assembly as the compiler emits
# it): the one-sided kernels (FP64, and mixed with separate targets), and the
# symmetric kernels (targets = sources), where one evaluation of a neighbour
# pair serves both of its sides and the leaf itself is one-sided.  The FP64
# symmetric figures are the per-evaluation slopes printed by
# paper_1204_3105_amd/csrc/count_valu.py (per-round work excluded).
VALU_PER_PAIR = {"fp64": 84.0, "mixed": 31.0}
VALU_SYM_EVAL = {"mixed": 30.5, "fp64": 73.2}
VALU_SYM_ONE_SIDED = {"mixed": 30.0, "fp64": 72.0}
SYM_CHUNKS = 2   # a leaf of at most 2 x 64 targets evaluates its pairs with higher leaves for both sides


def near_work(lv, same, n_pairs):
    """Pair evaluations of one near-field launch, from the plan's leaf level
    (point counts and neighbour lists): (symmetric evaluations, one-sided
    evaluations).  With targets = sources a neighbour pair of leaves whose
    lower leaf has at most SYM_CHUNKS chunks is evaluated once for both
    sides; the leaf itself and the other pairs one-sided; otherwise every
    pair is one-sided."""
    if not same:
        return 0.0, float(n_pairs)
    keys = lv["keys"]
    n = (lv["src_range"][:, 1] - lv["src_range"][:, 0]).astype(np.float64)
    near = lv["near"]
    a = np.repeat(np.arange(len(keys)), near.shape[1])
    kb = near.ravel()
    ok = kb >= 0
    a, b = a[ok], np.searchsorted(keys, kb[ok])
    upper = b > a
    a, b = a[upper], b[upper]
    sym = np.ceil(n[a] / 64.0) <= SYM_CHUNKS
    prod = n[a] * n[b]
    self_pairs = float(np.sum(n * n))
    return float(np.sum(prod[sym])), self_pairs + 2.0 * float(np.sum(prod[~sym]))


def near_valu_ops(lv, prec, same, n_pairs):
    """VALU lane-operations of one near-field launch: its evaluations times
    the per-evaluation instruction counts."""
    if not same:
        return n_pairs * VALU_PER_PAIR[prec]
    sym, one = near_work(lv, same, n_pairs)
    return VALU_SYM_EVAL[prec] * sym + VALU_SYM_ONE_SIDED[prec] * one


HBM_PEAK = 8.0e12
MFMA_BF16_PEAK = 2.5e15
FP64_PEAK = 78.6e12


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summaries
    (the machine-readable block of a file under profiles/), or None when none
    covers it or the kernel's source changed since the counters were taken."""
    import glob
    import hashlib
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        try:
            text = open(path).read()
            m = re.search(r"```json\n(.*?)\n```", text, re.S)
            if not m:
                continue
            rec = json.loads(m.group(1))
            if rec.get("kernel") != kernel:
                continue
            src = open(os.path.join(ROOT, rec["source"]), "rb").read()
        except (OSError, ValueError, KeyError):
            continue
        if hashlib.sha256(src).hexdigest() == rec.get("sha256"):
            return float(rec["bytes_per_launch"])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--tilings", default="quad,sept,tri")
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--check", type=int, default=2048, help="targets sampled for the error check")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20,
                    help="targets per tiling the CPU oracle evaluates on all host cores (default: all)")
    ap.add_argument("--cpu-sample-1core", type=int, default=1 << 14,
                    help="targets per tiling the CPU oracle evaluates on one core (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", dest="mixed", action="store_false",
                    help="skip the mixed-precision form (reported under extra by default)")
    ap.add_argument("--no-eps10", dest="eps10", action="store_false", help="skip the eps 1e-10 leg")
    ap.add_argument("--alone-reps", type=int, default=10,
                    help="solves per tiling and form timed one at a time (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests in the serving stream (0 = skip the serving leg)")
    ap.add_argument("--serve-loads", default="0.5,0.7,0.9",
                    help="Poisson arrival rates as fractions of the saturated request rate")
    ap.add_argument("--clustered-n", type=int, default=4 << 20,
                    help="points per side of the clustered workload (0 = skip)")
    ap.add_argument("--disk-n", type=int, default=16 << 20,
                    help="points of the unit-disk workload (0 = skip)")
    ap.add_argument("--disk-cases", default="quad:1e-4,quad:1e-6,sept:1e-4,sept:1e-6",
                    help="tiling:eps cases of the unit-disk workload")
    ap.add_argument("--disk-check", type=int, default=32,
                    help="targets of the unit-disk workload checked against the oracle (0 = none)")
    ap.add_argument("--streams", type=int, default=3,
                    help="streams that consecutive solves take turns on (1 = all on one stream)")
    ap.add_argument("--host-threads", type=int, default=0, choices=[0, 1],
                    help="1: each stream's solves are issued by a host thread of its own")
    ap.add_argument("--near-stream", default="own", choices=["own", "side"],
                    help="near field on each solve's own stream (own) or beside its far field (side)")
    ap.add_argument("--probe-rounds", type=int, default=2000,
                    help="rounds of the pair-rate probe kernel (0 = skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 512 MiB device copy first (HBM counter calibration)")
    return ap.parse_args()


def run_steps(F, torch, pts, u, tilings, eps, prec, leaf, steps, outs, streams, near_stream="own",
              threads=False):
    """`steps` passes of plan + evaluate per tiling.  Consecutive solves take
    turns on the given streams, so one solve's plan (short, latency-bound
    kernels and two host read-backs) runs while the previous solve's
    evaluation occupies the GPU.  With `threads`, each stream's solves are
    issued by a host thread of its own (the library calls release the
    interpreter lock), so one solve's read-backs do not hold back the
    others' launches.  Plans are released without a host wait; the last
    pass's plans are returned open so their event timings can be read after
    the clock."""
    solves = [(step, t, streams[j % len(streams)])
              for j, (step, t) in enumerate((s, t) for s in range(steps) for t in tilings)]
    kept = {}

    def issue(mine):
        for step, t, st in mine:
            plan = F.Plan(t, src=pts, tgt=pts, eps=eps, precision=prec, leaf_size=leaf, stream=st,
                          near_stream=near_stream)
            plan.eval(u, out=outs[t])
            if step == steps - 1:
                kept[t] = plan
            else:
                plan.close()

    if not threads or len(streams) == 1:
        issue(solves)
        return kept
    import threading
    errors = []

    def worker(k):
        try:
            issue([x for x in solves if x[2] is streams[k]])
        except BaseException as e:   # re-raised on the main thread
            errors.append(e)

    pool = [threading.Thread(target=worker, args=(k,)) for k in range(len(streams))]
    for th in pool:
        th.start()
    for th in pool:
        th.join()
    if errors:
        raise errors[0]
    return kept


def timed(F, torch, pts, u, tilings, eps, prec, leaf, steps, warmup, outs, n_streams=3, near_stream="own",
          threads=False):
    # torch's current stream alone, or that many new default-priority streams
    streams = ([torch.cuda.current_stream()] if n_streams <= 1 else
               [torch.cuda.Stream() for _ in range(n_streams)])
    for plan in run_steps(F, torch, pts, u, tilings, eps, prec, leaf, warmup, outs, streams, near_stream,
                          threads).values():
        plan.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kept = run_steps(F, torch, pts, u, tilings, eps, prec, leaf, steps, outs, streams, near_stream, threads)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    infos = {}
    for t, plan in kept.items():
        inf = plan.info()
        lv = plan.export_level(inf["lmax"])
        inf["near_evals"] = sum(near_work(lv, inf["targets_are_sources"], inf["n_near_pairs"]))
        inf["near_valu_ops"] = near_valu_ops(lv, inf["precision"], inf["targets_are_sources"],
                                             inf["n_near_pairs"])
        infos[t] = [inf]
    for plan in kept.values():
        plan.close()
    return t1 - t0, infos


def error_check(orc, w, outs, infos, tilings, nsample):
    from paper_1204_3105_amd import inputs
    idx = inputs.subsample(w.n_tgt, nsample, seed=99)
    res = {}
    for t in tilings:
        inf = infos[t][-1]
        g = orc.geom(t, inf["lmax"], *inf["geometry"])
        ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
        d1 = orc.direct_principal(w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
        got = outs[t].cpu().numpy()[idx]
        res[t] = {
            "rel_l2_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "rel_l2_re_vs_direct": float(np.linalg.norm(got.real - d1.real) / np.linalg.norm(d1.real)),
            "max_abs_re_vs_direct": float(np.max(np.abs(got.real - d1.real))),
            "sample": int(len(idx)),
        }
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_run(orc, w, infos, tilings, sample, threads, seed=7):
    """The oracle on all sources and all targets, or a seeded sample of the
    targets, per tiling, on `threads` threads.  A sample is scaled to
    whole-job throughput: keys + tree + upward pass are counted once, the
    per-target work (M2L chain, L2L, L2P, P2P) is scaled from the sample to
    all M targets.  A small sample overstates the per-target cost, since its
    targets share few cells."""
    from paper_1204_3105_amd import inputs
    idx = inputs.subsample(w.n_tgt, sample, seed=seed)
    total = 0.0
    detail = {}
    for t in tilings:
        inf = infos[t][-1]
        g = orc.geom(t, inf["lmax"], *inf["geometry"])
        times = [0.0] * 6
        t0 = time.perf_counter()
        orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt[idx], w.yt[idx], nthreads=threads, times=times)
        wall = time.perf_counter() - t0
        fixed = times[0] + times[1]
        per_target = (wall - fixed) / len(idx)
        est = fixed + per_target * w.n_tgt
        detail[t] = {"sample_wall_s": wall, "fixed_s": fixed, "projected_s": est}
        total += est
    value = len(tilings) * w.n_tgt / total
    if len(idx) == w.n_tgt:
        desc = ("oracle FMM (FP64, same trees and p) on the whole workload: all %d sources "
                "and all %d targets per tiling, timed, not scaled" % (w.n_src, w.n_tgt))
    else:
        desc = ("oracle FMM (FP64, same trees and p) on all %d sources and %d seeded "
                "targets per tiling; keys+tree+upward pass counted once, per-target "
                "work scaled to %d targets" % (w.n_src, len(idx), w.n_tgt))
    return {"value": value, "unit": "targets/s", "cores": int(threads), "kind": "oracle",
            "sample": desc, "detail": detail}


def cpu_baseline(orc, w, infos, tilings, sample, sample_1core):
    threads = orc.max_threads()
    res = cpu_run(orc, w, infos, tilings, sample, threads)
    res["cpu_model"] = cpu_model()
    res["host_threads_available"] = os.cpu_count()
    if sample_1core > 0:
        one = cpu_run(orc, w, infos, tilings, sample_1core, 1, seed=8)
        res["one_core"] = {k: one[k] for k in ("value", "unit", "cores", "sample", "detail")}
    return res


def near_roofline(infos, tilings, prec):
    """The dominant kernel, the P2P near-field launch, against the VALU issue
    rate (FP64 instructions for the FP64 kernels, 32-bit ones for the mixed
    kernels), from the plan's pair mix and the kernel's per-pair instruction
    count."""
    near_ms = np.mean([i["stage_ms"][3] for t in tilings for i in infos[t]])
    pairs = np.mean([i["n_near_pairs"] for t in tilings for i in infos[t]])
    evals = np.mean([i["near_evals"] for t in tilings for i in infos[t]])
    ops = np.mean([i["near_valu_ops"] for t in tilings for i in infos[t]])
    ach = ops / (near_ms * 1e-3)
    sym = all(i["targets_are_sources"] for t in tilings for i in infos[t])
    kname = ("k_near_mixed" if prec == "mixed" else "k_near_fp64") + ("_sym" if sym else "")
    traffic = committed_traffic(kname)
    peak = LANE_OPS_32 if prec == "mixed" else LANE_OPS
    return {"bound": "alu", "kernel": "near field (P2P), %s" % kname, "achieved": ach / 1e9,
            "peak": peak / 1e9, "unit": "G VALU lane-op/s", "frac": ach / peak, "traffic": traffic,
            "avg_launch_ms": float(near_ms), "pairs_per_launch": float(pairs),
            "evals_per_launch": float(evals), "valu_ops_per_launch": float(ops),
            "valu_per_pair": ({"symmetric_eval": VALU_SYM_EVAL[prec],
                               "one_sided": VALU_SYM_ONE_SIDED[prec]}
                              if sym else VALU_PER_PAIR[prec])}


def m2l_flops(prec, p, pairs):
    """Algorithmic M2L flops (8 (p+1)^2 per E4 pair: a complex (p+1) x (p+1)
    matrix-vector product) and the MFMA flops the kernel issues for them.
    Both forms apply the offset-free binomial matrix H (rows m = 0..p, columns
    k' = 0..p-1) to the pair's scaled Re and Im columns, 16 columns per MFMA
    (full tiles; a tile with fewer targets issues the same MFMAs).  FP64: rows
    in 16-row tiles, k' in 4-deep steps.  Mixed, 16 <= p <= 47: six BF16 split
    products, rows in 16-row tiles, k' in 32-deep blocks; below p = 16 the
    mixed form runs the FP64 kernel."""
    alg = 8.0 * (p + 1) ** 2 * pairs
    if prec == "fp64" or not 16 <= p <= 47:
        mt, kt = (p + 1 + 15) // 16, (p + 3) // 4
        issued = 2.0 * (16 * mt) * (4 * kt) * 2.0 * pairs
        peak = FP64_PEAK
    else:
        mt, kb = (p + 1 + 15) // 16, (p + 31) // 32
        issued = 6.0 * 2.0 * (16 * mt) * (32 * kb) * 2.0 * pairs
        peak = MFMA_BF16_PEAK
    return alg, issued, peak


def m2l_fraction(prec, p, pairs, ms):
    alg, issued, peak = m2l_flops(prec, p, pairs)
    sec = ms * 1e-3
    return {"stage_ms": ms, "pairs": pairs, "alg_tflops": alg / sec / 1e12, "issued_tflops": issued / sec / 1e12,
            "peak_tflops": peak / 1e12, "frac_alg": alg / sec / peak, "frac_issued": issued / sec / peak}


def m2l_mfma(infos, tilings, prec):
    """M2L against the dense MFMA peak of its arithmetic (FP64 78.6 TFLOP/s,
    BF16 2.5 PFLOP/s) per tiling, over the M2L stage time (events around the
    M2L launches; in the timed steps the stage runs beside other solves)."""
    out = {}
    for t in tilings:
        inf = infos[t]
        ms = float(np.mean([i["stage_ms"][1] for i in inf]))
        out[t] = m2l_fraction(prec, inf[-1]["p"], inf[-1]["n_m2l_pairs"], ms)
    return out


def solve_alone(F, torch, src, tgt, u, out, tiling, eps, prec, reps, leaf=64, depth="mean", near_stream="side"):
    """`reps` solves (plan + eval) one at a time on torch's stream, each
    waited for: median wall time and the last plan's info."""
    ts = []
    inf = None
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = F.Plan(tiling, src=src, tgt=tgt, eps=eps, precision=prec, leaf_size=leaf, depth=depth,
                      near_stream=near_stream)
        plan.eval(u, out=out)
        torch.cuda.synchronize()
        if r:
            ts.append((time.perf_counter() - t0) * 1e3)
        inf = plan.info()
        plan.close()
    return float(np.median(ts)), inf


def alone_leg(F, torch, pts, u, outs, tilings, eps, reps, leaf, forms):
    """Each tiling's solve alone (one stream, waited for): wall-clock
    targets/s of plan + eval, and the GPU times of the two."""
    res = {}
    for prec in forms:
        res[prec] = {}
        for t in tilings:
            ms, inf = solve_alone(F, torch, pts, pts, u, outs[t], t, eps, prec, reps, leaf)
            res[prec][t] = {"wall_ms": ms, "targets_per_s": inf["n_tgt"] / (ms * 1e-3),
                            "plan_ms_gpu": inf["plan_ms"], "eval_ms_gpu": inf["eval_ms"], "p": inf["p"]}
        print("bench: alone %s: %s" % (prec, ", ".join("%s %.3f ms" % (t, res[prec][t]["wall_ms"])
                                                        for t in tilings)), file=sys.stderr, flush=True)
    return res


def serve_bench(F, nreq, loads, leaf):
    """Mixed request stream: N log-uniform in [1e3, 2e6], uniform or 4-Gaussian
    sources (50/50), tiling uniform over three, eps in {1e-4, 1e-8}.  First
    all requests at once (saturated throughput), then Poisson arrivals at
    each of `loads` times the saturated request rate; latency = end - submit."""
    from paper_1204_3105_amd import inputs
    t0 = time.perf_counter()
    reqs = inputs.serving_stream(nreq, seed=5, rate=1.0)
    gen_s = time.perf_counter() - t0
    total_targets = sum(r.work.n_tgt for r in reqs)

    def run(arrivals):
        with F.Server(hbm_budget_bytes=64 << 30, max_inflight=64, leaf_size=leaf) as srv:
            t0 = time.perf_counter()
            pending = {}
            lat = []
            done = 0
            k = 0
            while done < len(reqs):
                now = time.perf_counter() - t0
                while k < len(reqs) and (arrivals is None or arrivals[k] <= now):
                    r = reqs[k]
                    w = r.work
                    pending[srv.submit(r.tiling, w.xs, w.ys, w.u, eps=r.eps)] = k
                    k += 1
                    now = time.perf_counter() - t0
                for t in list(pending):
                    res = srv.poll(t, want_phi=False)
                    if res is not None:
                        assert res[1]["status"] == "OK", res[1]
                        lat.append(res[1]["t_end"] - res[1]["t_submit"])
                        del pending[t]
                        done += 1
                if k < len(reqs) and arrivals is not None and not pending:
                    time.sleep(max(0.0, min(0.002, arrivals[k] - (time.perf_counter() - t0))))
                else:
                    time.sleep(0.0002)
            wall = time.perf_counter() - t0
        return wall, np.array(lat)

    wall_sat, lat_sat = run(None)
    sat_rate = len(reqs) / wall_sat
    out = {"requests": len(reqs), "total_targets": int(total_targets), "input_generation_s": gen_s,
           "saturated_requests_per_s": sat_rate, "saturated_targets_per_s": total_targets / wall_sat,
           "saturated_p50_ms": float(np.percentile(lat_sat, 50) * 1e3),
           "saturated_p99_ms": float(np.percentile(lat_sat, 99) * 1e3), "loads": {}}
    print("bench: serving saturated %.1f requests/s" % sat_rate, file=sys.stderr, flush=True)
    for load in loads:
        rate = load * sat_rate
        gaps = inputs.rng(55).exponential(1.0 / rate, len(reqs))
        wall, lat = run(np.cumsum(gaps))
        out["loads"]["%.1f" % load] = {
            "poisson_rate_requests_per_s": rate, "targets_per_s": total_targets / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3)}
        print("bench: serving load %.1f: p50 %.2f ms p99 %.2f ms" % (
            load, out["loads"]["%.1f" % load]["p50_ms"], out["loads"]["%.1f" % load]["p99_ms"]),
            file=sys.stderr, flush=True)
    return out


def oracle_refs(orc, w, inf, idx):
    """The oracle FMM on the plan's tree and p (all sources, sampled targets)
    and the principal direct sum there."""
    g = orc.geom(inf["tiling"], inf["lmax"], *inf["geometry"])
    ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
    d1 = orc.direct_principal(w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
    return ref, d1


def errors_against(phi, ref, d1):
    return {"rel_l2_vs_oracle": float(np.linalg.norm(phi - ref) / np.linalg.norm(ref)),
            "rel_l2_re_vs_direct": float(np.linalg.norm(phi.real - d1.real) / np.linalg.norm(d1.real)),
            "max_abs_re_vs_direct": float(np.max(np.abs(phi.real - d1.real))), "sample": int(len(ref))}


def clustered_leg(F, torch, orc, n, reps=3, nsample=64):
    """Clustered sources, separate uniform targets (n each; 8 Gaussians,
    sigma 0.02, N(0,1) strengths), eps 1e-6: both forms, the uniform-depth
    tree at the mean-occupancy level and at the cost-model level
    (depth="cost"); plan + evaluate wall time (median of reps), chosen level,
    and the error on sampled targets against the oracle."""
    from paper_1204_3105_amd import inputs
    w = inputs.gaussian_mixture(n, n, seed=3)
    dev = torch.device("cuda:0")
    src = torch.tensor(w.xs + 1j * w.ys, dtype=torch.complex128, device=dev)
    tgt = torch.tensor(w.xt + 1j * w.yt, dtype=torch.complex128, device=dev)
    u = torch.tensor(w.u, dtype=torch.float64, device=dev)
    out = torch.empty(n, dtype=torch.complex128, device=dev)
    idx = inputs.subsample(n, nsample, 5)
    res = {}
    for t in ("quad", "sept", "tri"):
        row = {"fp64": {}, "mixed": {}}
        for rule in ("mean", "cost"):
            refs = None
            for prec in ("fp64", "mixed"):
                ms, inf = solve_alone(F, torch, src, tgt, u, out, t, 1e-6, prec, reps, depth=rule)
                if refs is None:   # both forms build the same tree
                    refs = oracle_refs(orc, w, inf, idx)
                r = {"lmax": inf["lmax"], "ms": ms, "targets_per_s": n / (ms * 1e-3),
                     "n_near_pairs": inf["n_near_pairs"], "n_m2l_pairs": inf["n_m2l_pairs"]}
                r.update(errors_against(out.cpu().numpy()[idx], *refs))
                row[prec][rule] = r
        for prec in ("fp64", "mixed"):
            row[prec]["speedup_cost_rule"] = row[prec]["mean"]["ms"] / row[prec]["cost"]["ms"]
            print("bench: clustered %s %s: mean rule L=%d %.2f ms, cost rule L=%d %.2f ms" % (
                t, prec, row[prec]["mean"]["lmax"], row[prec]["mean"]["ms"], row[prec]["cost"]["lmax"],
                row[prec]["cost"]["ms"]), file=sys.stderr, flush=True)
        res[t] = row
    return res


def disk_leg(F, torch, orc, n, cases, reps=3, nsample=32):
    """n points uniform in the unit disk, targets = sources, quadtree and
    septree, eps 1e-4 and 1e-6, both forms: solve-alone wall time, M2L stage
    time (a solve with the near field after the far field, so M2L runs
    alone) against the MFMA peaks, and sampled errors against the oracle."""
    from paper_1204_3105_amd import inputs
    w = inputs.unit_disk(n, seed=4)
    dev = torch.device("cuda:0")
    pts = torch.tensor(w.xs + 1j * w.ys, dtype=torch.complex128, device=dev)
    u = torch.tensor(w.u, dtype=torch.float64, device=dev)
    out = torch.empty(n, dtype=torch.complex128, device=dev)
    idx = inputs.subsample(n, max(nsample, 1), 6)
    res = {}
    for case in cases:
        t, eps = case.split(":")
        eps = float(eps)
        row = {}
        ref = None
        for prec in ("fp64", "mixed"):
            ms, inf = solve_alone(F, torch, pts, pts, u, out, t, eps, prec, reps)
            phi = out.cpu().numpy()[idx]
            _, inf_own = solve_alone(F, torch, pts, pts, u, out, t, eps, prec, 1, near_stream="own")
            r = {"p": inf["p"], "lmax": inf["lmax"], "wall_ms": ms, "targets_per_s": n / (ms * 1e-3),
                 "m2l": m2l_fraction(prec, inf["p"], inf["n_m2l_pairs"], inf_own["stage_ms"][1]),
                 "near_ms": inf_own["stage_ms"][3]}
            if nsample > 0:
                if ref is None:   # both forms build the same tree
                    g = orc.geom(t, inf["lmax"], *inf["geometry"])
                    ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
                r["rel_l2_vs_oracle"] = float(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
                r["check_sample"] = int(len(idx))
            row[prec] = r
            print("bench: disk %s eps %g %s: %.2f ms, M2L %.3f ms (%.1f%% of MFMA peak issued), err %s" % (
                t, eps, prec, ms, r["m2l"]["stage_ms"], 100 * r["m2l"]["frac_issued"],
                "%.2e" % r["rel_l2_vs_oracle"] if nsample > 0 else "-"), file=sys.stderr, flush=True)
        res["%s_eps%g" % (t, eps)] = row
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path "
              "(requested --gpus %d)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import oracle
    from paper_1204_3105_amd import fmm as F
    from paper_1204_3105_amd import inputs

    F.lib()
    dev = torch.device("cuda:0")
    tilings = a.tilings.split(",")
    w = inputs.uniform_square(a.n, seed=2)
    pts = torch.tensor(w.xs + 1j * w.ys, dtype=torch.complex128, device=dev)
    u = torch.tensor(w.u, dtype=torch.float64, device=dev)
    outs = {t: torch.empty(a.n, dtype=torch.complex128, device=dev) for t in tilings}
    if a.calibrate_copy:
        src = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print("bench: n=%d tilings=%s steps=%d warmup=%d" % (a.n, tilings, a.steps, a.warmup),
          file=sys.stderr, flush=True)

    # Headline: the plain FP64 form.
    wall, infos = timed(F, torch, pts, u, tilings, a.eps, "fp64", a.leaf, a.steps, a.warmup, outs,
                        a.streams, a.near_stream, bool(a.host_threads))
    value = len(tilings) * a.n * a.steps / wall
    print("bench: timed %.3f s -> %.4g targets/s (fp64)" % (wall, value), file=sys.stderr, flush=True)
    roofline = near_roofline(infos, tilings, "fp64")
    # The pair function's own rate with its operands in registers: the
    # ceiling the near-field kernel's evaluation rate is measured against.
    probe = F.probe_pair_rate(a.probe_rounds) if a.probe_rounds > 0 else None
    ceiling = None
    if probe:
        kev = roofline["evals_per_launch"] / (roofline["avg_launch_ms"] * 1e-3)
        ceiling = {"probe_evals_per_s": probe, "kernel_evals_per_s": kev, "kernel_of_probe": kev / probe,
                   "probe_valu_lane_ops_per_s_at_model_count": probe * VALU_SYM_EVAL["fp64"],
                   "probe_of_peak_at_model_count": probe * VALU_SYM_EVAL["fp64"] / LANE_OPS}
        print("bench: pair-rate probe %.4g evals/s, near kernel %.4g evals/s (%.2f of the probe)" % (
            probe, kev, kev / probe), file=sys.stderr, flush=True)

    def per_tiling(infos):
        pt = {}
        for t in tilings:
            inf = infos[t]
            pt[t] = {
                "p": inf[-1]["p"], "lmax": inf[-1]["lmax"], "precision": inf[-1]["precision"],
                "plan_ms": float(np.mean([i["plan_ms"] for i in inf])),
                "eval_ms": float(np.mean([i["eval_ms"] for i in inf])),
                "stage_ms": [float(np.mean([i["stage_ms"][k] for i in inf])) for k in range(5)],
                "n_m2l_pairs": inf[-1]["n_m2l_pairs"], "n_near_pairs": inf[-1]["n_near_pairs"],
                "cells": int(sum(inf[-1]["n_cells"])),
            }
        return pt

    extra = {"per_tiling": per_tiling(infos), "m2l_mfma": m2l_mfma(infos, tilings, "fp64"),
             "pair_rate_ceiling": ceiling,
             "errors": error_check(oracle, w, outs, infos, tilings, a.check)}

    if a.mixed:
        wallm, infosm = timed(F, torch, pts, u, tilings, a.eps, "mixed", a.leaf, a.steps, a.warmup, outs,
                              a.streams, a.near_stream, bool(a.host_threads))
        extra["mixed_form"] = {
            "value": len(tilings) * a.n * a.steps / wallm, "ms_per_step": wallm / a.steps * 1e3,
            "dtype": "f64/f32/bf16x3", "roofline": near_roofline(infosm, tilings, "mixed"),
            "per_tiling": per_tiling(infosm), "m2l_mfma": m2l_mfma(infosm, tilings, "mixed"),
            "errors": error_check(oracle, w, outs, infosm, tilings, a.check)}
        print("bench: mixed form %.4g targets/s" % extra["mixed_form"]["value"], file=sys.stderr, flush=True)

    if a.alone_reps > 0:
        extra["solve_alone"] = alone_leg(F, torch, pts, u, outs, tilings, a.eps, a.alone_reps, a.leaf,
                                         ("fp64", "mixed") if a.mixed else ("fp64",))

    if a.eps10:
        # The same workload at eps 1e-10 (FP64 only: p 38 / 35 / 46).
        wall10, infos10 = timed(F, torch, pts, u, tilings, 1e-10, "fp64", a.leaf, a.steps, a.warmup, outs,
                                a.streams, a.near_stream, bool(a.host_threads))
        extra["fp64_eps1e-10"] = {
            "value": len(tilings) * a.n * a.steps / wall10, "ms_per_step": wall10 / a.steps * 1e3,
            "per_tiling": per_tiling(infos10), "m2l_mfma": m2l_mfma(infos10, tilings, "fp64"),
            "errors": error_check(oracle, w, outs, infos10, tilings, a.check // 4)}
        print("bench: FP64 form at eps 1e-10 %.4g targets/s" % extra["fp64_eps1e-10"]["value"], file=sys.stderr,
              flush=True)

    if a.clustered_n > 0:
        extra["clustered"] = clustered_leg(F, torch, oracle, a.clustered_n)
    if a.disk_n > 0:
        extra["unit_disk"] = disk_leg(F, torch, oracle, a.disk_n, a.disk_cases.split(","), nsample=a.disk_check)

    if a.serve_requests > 0:
        print("bench: serving stream (%d requests) ..." % a.serve_requests, file=sys.stderr, flush=True)
        extra["serving"] = serve_bench(F, a.serve_requests, [float(x) for x in a.serve_loads.split(",")], a.leaf)

    cpu = None
    if not a.no_cpu_baseline:
        print("bench: cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(oracle, w, infos, tilings, a.cpu_sample, a.cpu_sample_1core)

    line = {
        "metric": "targets/sec at rel err 1e-6, N=1M per tiling; p50/p99 solve latency",
        "value": value, "unit": "targets/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "N=M=2^20 uniform unit square, sources=targets, u~U[-1,1], "
                               "eps=%g, leaf %d, plain FP64, one plan+eval per tiling (%s) per step" %
                               (a.eps, a.leaf, "+".join(tilings)),
                   "precision": "fp64", "n": a.n, "streams": a.streams, "near_stream": a.near_stream,
                   "host_threads": a.host_threads},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
