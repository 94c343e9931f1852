#!/usr/bin/env python
"""Benchmark: targets/sec of full FMM solves (plan + eval) at eps = 1e-6.

Workload: N = M = 2^20 sources = targets uniform in the unit square, strengths
U[-1,1] (seed 2), one solve per tiling (quadtree, septree, triangle-quadtree)
per step, leaf size 64, p from eps and each tiling's separation ratio.  A step
is plan + eval for all three tilings with the points already resident in HBM.

Prints one JSON line.  `value` = 3 * M * steps / wall time of the timed
steps.  `roofline` covers the dominant kernel (the P2P near field), timed
with HIP events on the stream it runs on, as VALU lane-operations per second
against the chip's VALU rate.  `cpu_baseline` is
the CPU oracle timed on this host on a bounded sample of the same workload.
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
# x 2.4 GHz (FP64 and non-packed FP32 issue at the same rate).
LANE_OPS = 256 * 4 * 16 * 2.4e9
# VALU instructions per source-target pair in the near-field inner loops of
# the gfx950 code (counted in the kernels' AMD assembly as the compiler emits
# it): the one-sided kernels (FP64, and mixed with separate targets), and the
# symmetric kernels (targets = sources), where one evaluation of a neighbour
# pair serves both of its sides and the leaf itself is one-sided.
VALU_PER_PAIR = {"fp64": 104.0, "mixed": 31.0}
VALU_SYM_EVAL = {"mixed": 30.5, "fp64": 92.0}
VALU_SYM_ONE_SIDED = {"mixed": 30.0, "fp64": 104.0}
SYM_CHUNKS = 2   # a leaf of at most 2 x 64 targets evaluates its pairs with higher leaves for both sides


def near_valu_ops(lv, prec, same, n_pairs):
    """VALU lane-operations of one near-field launch, from the plan's leaf
    level (point counts and neighbour lists)."""
    if not same:
        return n_pairs * VALU_PER_PAIR[prec]
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
    return (VALU_SYM_EVAL[prec] * float(np.sum(prod[sym]))
            + VALU_SYM_ONE_SIDED[prec] * (self_pairs + 2.0 * float(np.sum(prod[~sym]))))
HBM_PEAK = 8.0e12
MFMA_BF16_PEAK = 2.5e15
FP64_PEAK = 78.6e12


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/), or None when the kernel's source changed since it was taken."""
    import hashlib
    import json
    import re
    path = os.path.join(ROOT, "profiles", "near_mixed_uniform1M_hbm_counters.md")
    try:
        text = open(path).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, AttributeError, ValueError, KeyError):
        return None
    if rec.get("kernel") != kernel or hashlib.sha256(src).hexdigest() != rec.get("sha256"):
        return None
    return float(rec["bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--precision", default="auto", choices=["auto", "fp64", "mixed"])
    ap.add_argument("--tilings", default="quad,sept,tri")
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--check", type=int, default=2048, help="targets sampled for the error check")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20,
                    help="targets per tiling the CPU oracle evaluates (default: all of them, "
                         "about 5 s on 16 cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare-fp64", dest="compare_fp64", action="store_false",
                    help="skip timing the plain FP64 form (reported under extra by default)")
    ap.add_argument("--serve-requests", type=int, default=300,
                    help="requests in the serving stream (0 = skip the serving leg)")
    ap.add_argument("--clustered-n", type=int, default=4 << 20,
                    help="points per side of the clustered-input leg (0 = skip)")
    ap.add_argument("--streams", type=int, default=3,
                    help="streams that consecutive solves take turns on (1 = all on one stream)")
    ap.add_argument("--host-threads", type=int, default=0, choices=[0, 1],
                    help="1: each stream's solves are issued by a host thread of its own")
    ap.add_argument("--near-stream", default="own", choices=["own", "side"],
                    help="near field on each solve's own stream (own) or beside its far field (side)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 512 MiB device copy first (HBM counter calibration)")
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="Poisson arrival rate as a fraction of the saturated request rate")
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


def cpu_baseline(orc, w, infos, tilings, sample):
    """The oracle on all sources and all targets, or a seeded sample of the
    targets, per tiling.  A sample is scaled to whole-job throughput: keys +
    tree + upward pass are counted once, the per-target work (M2L chain,
    L2L, L2P, P2P) is scaled from the sample to all M targets.  A small
    sample overstates the per-target cost, since its targets share few
    cells."""
    from paper_1204_3105_amd import inputs
    idx = inputs.subsample(w.n_tgt, sample, seed=7)
    threads = orc.max_threads()
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
        sample = ("oracle FMM (FP64, same trees and p) on the whole workload: all %d sources "
                  "and all %d targets per tiling, timed, not scaled" % (w.n_src, w.n_tgt))
    else:
        sample = ("oracle FMM (FP64, same trees and p) on all %d sources and %d seeded "
                  "targets per tiling; keys+tree+upward pass counted once, per-target "
                  "work scaled to %d targets" % (w.n_src, len(idx), w.n_tgt))
    return {"value": value, "unit": "targets/s", "cores": int(threads), "kind": "oracle",
            "sample": sample, "detail": detail}


def near_roofline(infos, tilings, prec):
    """The dominant kernel, the P2P near-field launch, against the VALU issue
    rate (FP64 VALU issues at the FP32 rate on this chip).  It runs beside
    the far-field passes and other solves, so its duration includes sharing
    the GPU with them."""
    near_ms = np.mean([i["stage_ms"][3] for t in tilings for i in infos[t]])
    pairs = np.mean([i["n_near_pairs"] for t in tilings for i in infos[t]])
    ops = np.mean([i["near_valu_ops"] for t in tilings for i in infos[t]])
    ach = ops / (near_ms * 1e-3)
    sym = all(i["targets_are_sources"] for t in tilings for i in infos[t])
    kname = ("k_near_mixed" if prec == "mixed" else "k_near_fp64") + ("_sym" if sym else "")
    traffic = committed_traffic(kname) if prec == "mixed" else None
    return {"bound": "alu", "kernel": "near field (P2P), %s" % kname, "achieved": ach / 1e9,
            "peak": LANE_OPS / 1e9, "unit": "G VALU lane-op/s", "frac": ach / LANE_OPS, "traffic": traffic,
            "avg_launch_ms": float(near_ms), "pairs_per_launch": float(pairs),
            "valu_ops_per_launch": float(ops),
            "valu_per_pair": ({"symmetric_eval": VALU_SYM_EVAL[prec],
                               "one_sided": VALU_SYM_ONE_SIDED[prec]}
                              if sym else VALU_PER_PAIR[prec])}


def serve_bench(F, nreq, load, leaf):
    """Mixed request stream: N log-uniform in [1e3, 2e6], uniform or 4-Gaussian
    sources (50/50), tiling uniform over three, eps in {1e-4, 1e-8}.  First
    all requests at once (saturated throughput), then Poisson arrivals at
    `load` times the saturated request rate; latency = end - submit."""
    from paper_1204_3105_amd import inputs
    reqs = inputs.serving_stream(nreq, seed=5, rate=1.0)
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
                    res = srv.poll(t)
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
    rate = load * sat_rate
    gaps = inputs.rng(55).exponential(1.0 / rate, len(reqs))
    arrivals = np.cumsum(gaps)
    wall, lat = run(arrivals)
    return {
        "requests": len(reqs), "total_targets": int(total_targets),
        "saturated_requests_per_s": sat_rate, "saturated_targets_per_s": total_targets / wall_sat,
        "poisson_rate_requests_per_s": rate, "load": load,
        "targets_per_s": total_targets / wall,
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "saturated_p50_ms": float(np.percentile(lat_sat, 50) * 1e3),
        "saturated_p99_ms": float(np.percentile(lat_sat, 99) * 1e3),
    }


def clustered_leg(F, torch, orc, n, reps=3, nsample=64):
    """Clustered sources, separate uniform targets (n each; 8 Gaussians,
    sigma 0.02, N(0,1) strengths), eps 1e-6, mixed: the uniform-depth tree at
    the mean-occupancy level and at the cost-model level (depth="cost"),
    plan + evaluate wall time (median of reps), chosen level, and for the
    cost rule the error on sampled targets against the oracle."""
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
        row = {}
        for rule in ("mean", "cost"):
            ts = []
            for r in range(reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan = F.Plan(t, src=src, tgt=tgt, eps=1e-6, precision="mixed", depth=rule)
                plan.eval(u, out=out)
                torch.cuda.synchronize()
                if r:
                    ts.append((time.perf_counter() - t0) * 1e3)
                inf = plan.info()
                plan.close()
            row[rule] = {"lmax": inf["lmax"], "ms": float(np.median(ts)), "n_near_pairs": inf["n_near_pairs"],
                         "n_m2l_pairs": inf["n_m2l_pairs"]}
            if rule == "cost":
                g = orc.geom(t, inf["lmax"], *inf["geometry"])
                ref = orc.fmm(g, inf["p"], w.xs, w.ys, w.u, w.xt[idx], w.yt[idx])
                phi = out.cpu().numpy()[idx]
                row[rule]["rel_l2_vs_oracle"] = float(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
        row["speedup"] = row["mean"]["ms"] / row["cost"]["ms"]
        res[t] = row
        print("bench: clustered %s: mean rule L=%d %.2f ms, cost rule L=%d %.2f ms" % (
            t, row["mean"]["lmax"], row["mean"]["ms"], row["cost"]["lmax"], row["cost"]["ms"]),
            file=sys.stderr, flush=True)
    return res


def m2l_mfma(infos, tilings):
    """M2L against the dense BF16 MFMA peak, per tiling: algorithmic flops
    (8 (p+1)^2 per E4 pair: a complex (p+1) x (p+1) matrix-vector product) and
    issued MFMA flops (six BF16 split products of a real 2(p+1) x 2p block per
    pair, padded to 16-row tiles and 32-deep k-blocks) over the M2L stage time
    (events around the M2L launches; the stage runs beside the near field)."""
    out = {}
    for t in tilings:
        inf = infos[t]
        p = inf[-1]["p"]
        pairs = inf[-1]["n_m2l_pairs"]
        ms = float(np.mean([i["stage_ms"][1] for i in inf]))
        mt, kb = (2 * (p + 1) + 15) // 16, (2 * p + 31) // 32
        alg = 8.0 * (p + 1) ** 2 * pairs
        issued = 6.0 * 2.0 * (16 * mt) * (32 * kb) * pairs
        out[t] = {"stage_ms": ms, "pairs": pairs, "alg_tflops": alg / (ms * 1e-3) / 1e12,
                  "issued_tflops": issued / (ms * 1e-3) / 1e12, "peak_tflops": MFMA_BF16_PEAK / 1e12,
                  "frac_issued": issued / (ms * 1e-3) / MFMA_BF16_PEAK}
    return out


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
    print("bench: n=%d tilings=%s precision=%s steps=%d warmup=%d" %
          (a.n, tilings, a.precision, a.steps, a.warmup), file=sys.stderr, flush=True)

    wall, infos = timed(F, torch, pts, u, tilings, a.eps, a.precision, a.leaf, a.steps, a.warmup, outs,
                        a.streams, a.near_stream, bool(a.host_threads))
    value = len(tilings) * a.n * a.steps / wall
    prec_used = infos[tilings[0]][-1]["precision"]
    print("bench: timed %.3f s -> %.4g targets/s (%s)" % (wall, value, prec_used), file=sys.stderr,
          flush=True)

    roofline = near_roofline(infos, tilings, prec_used)

    per_tiling = {}
    for t in tilings:
        inf = infos[t]
        per_tiling[t] = {
            "p": inf[-1]["p"], "lmax": inf[-1]["lmax"], "precision": inf[-1]["precision"],
            "plan_ms": float(np.mean([i["plan_ms"] for i in inf])),
            "eval_ms": float(np.mean([i["eval_ms"] for i in inf])),
            "stage_ms": [float(np.mean([i["stage_ms"][k] for i in inf])) for k in range(5)],
            "n_m2l_pairs": inf[-1]["n_m2l_pairs"], "n_near_pairs": inf[-1]["n_near_pairs"],
            "cells": int(sum(inf[-1]["n_cells"])),
            "targets_per_s_eval_only": a.n / (np.mean([i["eval_ms"] for i in inf]) * 1e-3),
            "targets_per_s_plan_eval_gpu": a.n / (np.mean([i["plan_ms"] + i["eval_ms"] for i in inf]) * 1e-3),
        }
    extra = {"per_tiling": per_tiling}
    if prec_used == "mixed":
        extra["m2l_mfma"] = m2l_mfma(infos, tilings)
    errs = error_check(oracle, w, outs, infos, tilings, a.check)
    extra["errors"] = errs

    if a.compare_fp64 and prec_used != "fp64":
        wall64, infos64 = timed(F, torch, pts, u, tilings, a.eps, "fp64", a.leaf, a.steps, 1, outs, a.streams,
                                a.near_stream, bool(a.host_threads))
        extra["fp64_form"] = {"value": len(tilings) * a.n * a.steps / wall64,
                              "ms_per_step": wall64 / a.steps * 1e3,
                              "near_roofline": near_roofline(infos64, tilings, "fp64"),
                              "errors": error_check(oracle, w, outs, infos64, tilings, a.check)}
        print("bench: plain FP64 form %.4g targets/s" % extra["fp64_form"]["value"], file=sys.stderr,
              flush=True)
        # The same workload at eps 1e-10 (FP64 only: p 38 / 35 / 46).
        wall10, infos10 = timed(F, torch, pts, u, tilings, 1e-10, "fp64", a.leaf, a.steps, 1, outs, a.streams,
                                a.near_stream, bool(a.host_threads))
        extra["fp64_eps1e-10"] = {
            "value": len(tilings) * a.n * a.steps / wall10, "ms_per_step": wall10 / a.steps * 1e3,
            "per_tiling": {t: {"p": infos10[t][-1]["p"],
                               "plan_ms": float(np.mean([i["plan_ms"] for i in infos10[t]])),
                               "eval_ms": float(np.mean([i["eval_ms"] for i in infos10[t]]))} for t in tilings},
            "errors": error_check(oracle, w, outs, infos10, tilings, a.check // 4)}
        print("bench: FP64 form at eps 1e-10 %.4g targets/s" % extra["fp64_eps1e-10"]["value"], file=sys.stderr,
              flush=True)

    if a.serve_requests > 0:
        print("bench: serving stream (%d requests) ..." % a.serve_requests, file=sys.stderr, flush=True)
        extra["serving"] = serve_bench(F, a.serve_requests, a.serve_load, a.leaf)
        print("bench: serving p50 %.2f ms p99 %.2f ms" % (extra["serving"]["p50_ms"],
                                                          extra["serving"]["p99_ms"]),
              file=sys.stderr, flush=True)

    if a.clustered_n > 0:
        extra["clustered"] = clustered_leg(F, torch, oracle, a.clustered_n)

    cpu = None
    if not a.no_cpu_baseline:
        print("bench: cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(oracle, w, infos, tilings, a.cpu_sample)

    dtype = {"fp64": "f64", "mixed": "f64/f32/bf16x3"}[prec_used]
    line = {
        "metric": "targets/sec at rel err 1e-6, N=1M per tiling; p50/p99 solve latency",
        "value": value, "unit": "targets/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": "N=M=2^20 uniform unit square, sources=targets, u~U[-1,1], "
                               "eps=%g, leaf %d, one plan+eval per tiling (%s) per step" %
                               (a.eps, a.leaf, "+".join(tilings)),
                   "precision": prec_used, "n": a.n, "streams": a.streams, "near_stream": a.near_stream,
                   "host_threads": a.host_threads},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
