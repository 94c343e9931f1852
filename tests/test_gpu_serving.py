"""Serving: continuous batching of independent solves.

Every result of a mixed stream (different tilings, sizes, eps, precisions,
sources = targets or not) must equal the same request solved alone with
fmm_plan + fmm_eval, bit for bit; memory exhaustion forced from the host (a
tiny budget) must only queue requests; a failing request must not disturb
the others."""
import time

import numpy as np
import pytest

from paper_1204_3105_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    from paper_1204_3105_amd import fmm
    fmm.lib()
    return fmm


def make_stream(n, seed, n_hi=60000):
    reqs = inputs.serving_stream(n, seed=seed, rate=1e9, n_lo=50, n_hi=n_hi)
    out = []
    rng = np.random.default_rng(seed)
    for k, r in enumerate(reqs):
        prec = ["auto", "fp64", "mixed"][k % 3]
        w = r.work
        if k % 4 == 3:   # separate targets
            m = max(1, w.n_src // 2)
            out.append((r.tiling, w.xs, w.ys, w.u, r.eps, prec, rng.random(m), rng.random(m)))
        else:
            out.append((r.tiling, w.xs, w.ys, w.u, r.eps, prec, None, None))
    return out


def alone(F, t, xs, ys, u, eps, prec, xt, yt):
    with F.Plan(t, xs, ys, xt, yt, eps=eps, precision=prec) as p:
        return p.eval(u)


def wait_all(srv, tickets, timeout=120):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t in tickets:
            if t in res:
                continue
            r = srv.poll(t)
            if r is not None:
                res[t] = r
        assert time.time() - t0 < timeout, "serving stream did not finish"
        time.sleep(0.001)
    return res


def test_mixed_stream_equals_alone(F):
    stream = make_stream(40, seed=5)
    with F.Server(hbm_budget_bytes=16 << 30, max_inflight=16) as srv:
        tickets = [srv.submit(*req) for req in stream]
        res = wait_all(srv, tickets)
    for t, req in zip(tickets, stream):
        phi, info = res[t]
        assert info["status"] == "OK", info
        ref = alone(F, *req)
        assert np.array_equal(phi, ref), (req[0], len(req[1]), req[4], req[5])
        assert info["t_submit"] <= info["t_admit"] <= info["t_start"] <= info["t_end"]


def test_tiny_budget_queues_and_completes(F):
    stream = make_stream(12, seed=6, n_hi=20000)
    with F.Server(hbm_budget_bytes=1, max_inflight=4) as srv:
        tickets = [srv.submit(*req) for req in stream]
        res = wait_all(srv, tickets)
    # With a budget below any request, each runs alone, in order.
    order = sorted(tickets, key=lambda t: res[t][1]["t_admit"])
    assert order == tickets
    for a, b in zip(tickets, tickets[1:]):
        assert res[a][1]["t_end"] <= res[b][1]["t_admit"] + 1e-3
    for t, req in zip(tickets, stream):
        assert np.array_equal(res[t][0], alone(F, *req))


def test_bad_request_does_not_disturb_others(F):
    stream = make_stream(6, seed=7, n_hi=10000)
    bad_x = stream[0][1].copy()
    bad_x[0] = np.nan
    with F.Server() as srv:
        with pytest.raises(F.FMMError):
            srv.submit("quad", stream[0][1], stream[0][2], stream[0][3], eps=0.0)
        tb = srv.submit("quad", bad_x, stream[0][2], stream[0][3], eps=1e-6)
        tickets = [srv.submit(*req) for req in stream]
        res = wait_all(srv, tickets + [tb])
    assert res[tb][1]["status"] == "INVALID" and res[tb][0] is None
    for t, req in zip(tickets, stream):
        assert res[t][1]["status"] == "OK"
        assert np.array_equal(res[t][0], alone(F, *req))


def test_small_request_overtakes_large_batch(F):
    # A large FP64 request is planned and launched first; a small request
    # submitted right after it is planned while the large batch runs, starts
    # on the second evaluation stream and finishes first.  Both equal their
    # solves alone.
    big = inputs.uniform_square(8 << 20, seed=21)
    small = inputs.uniform_square(3000, seed=22)
    print("serving overtake: big n=%d fp64 eps 1e-10, small n=%d" % (big.n_src, small.n_src), flush=True)
    with F.Server(hbm_budget_bytes=32 << 30, max_inflight=8) as srv:
        tb = srv.submit("tri", big.xs, big.ys, big.u, eps=1e-10, precision="fp64")
        ts = srv.submit("quad", small.xs, small.ys, small.u, eps=1e-6, precision="fp64")
        res = wait_all(srv, [tb, ts])
    rb, rs = res[tb][1], res[ts][1]
    assert rb["status"] == "OK" and rs["status"] == "OK"
    print("serving overtake: big start %.4f end %.4f, small start %.4f end %.4f" % (
        rb["t_start"] - rb["t_submit"], rb["t_end"] - rb["t_submit"], rs["t_start"] - rb["t_submit"],
        rs["t_end"] - rb["t_submit"]), flush=True)
    assert rs["t_start"] >= rb["t_start"]   # the large batch was already running
    assert rs["t_end"] < rb["t_end"]
    assert np.array_equal(res[ts][0], alone(F, "quad", small.xs, small.ys, small.u, 1e-6, "fp64", None, None))
    assert np.array_equal(res[tb][0], alone(F, "tri", big.xs, big.ys, big.u, 1e-10, "fp64", None, None))
