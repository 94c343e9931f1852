"""The benchmark's near-field work model (host logic, no GPU): VALU
operations of one launch from a plan's leaf sizes and neighbour lists,
against a count by hand on three leaves in a row."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def level():
    # leaves 0, 1, 2 with 10, 140 and 10 points; each sees itself and its
    # neighbours in the row (near lists hold cell keys, -1 = empty)
    keys = np.array([0, 1, 2])
    src_range = np.array([[0, 10], [10, 150], [150, 160]])
    near = -np.ones((3, 13), dtype=np.int64)
    near[0, :2] = [0, 1]
    near[1, :3] = [1, 0, 2]
    near[2, :2] = [2, 1]
    return {"keys": keys, "src_range": src_range, "near": near}


def test_symmetric_mix_by_hand():
    # self pairs 10^2 + 140^2 + 10^2 one-sided; pair {0, 1}: the lower leaf
    # has one chunk of 64, so 10 x 140 evaluations serve both sides; pair
    # {1, 2}: the lower leaf has three chunks, so both sides one-sided
    for prec in ("mixed", "fp64"):
        want = (bench.VALU_SYM_EVAL[prec] * 10 * 140
                + bench.VALU_SYM_ONE_SIDED[prec] * (100 + 19600 + 100 + 2 * 140 * 10))
        assert bench.near_valu_ops(level(), prec, True, 0) == want


def test_one_sided_plans_use_the_per_pair_count():
    for prec in ("mixed", "fp64"):
        assert bench.near_valu_ops(level(), prec, False, 1234) == 1234 * bench.VALU_PER_PAIR[prec]


class _FakeF:
    """Stands in for the binding: records which stream each solve was issued on."""

    def __init__(self):
        import threading
        self.log = []
        self.mu = threading.Lock()
        F = self

        class Plan:
            def __init__(self, t, stream=None, **kw):
                self.t, self.stream, self.closed = t, stream, False

            def eval(self, u, out=None):
                with F.mu:
                    F.log.append((self.t, self.stream))

            def close(self):
                self.closed = True

        self.Plan = Plan


def test_run_steps_issue_order_with_and_without_threads():
    # every solve issued once, solve j on stream j mod S, each stream's solves
    # in step order, and the last step's plans returned open
    tilings = ["quad", "sept", "tri"]
    for threads in (False, True):
        for streams in (["s0"], ["s0", "s1"], ["s0", "s1", "s2"]):
            F = _FakeF()
            kept = bench.run_steps(F, None, None, None, tilings, 1e-6, "mixed", 64, 4,
                                   {t: None for t in tilings}, streams, threads=threads)
            want = [(t, streams[j % len(streams)])
                    for j, t in enumerate(t for _ in range(4) for t in tilings)]
            assert sorted(F.log) == sorted(want)
            for st in streams:
                assert [x for x in F.log if x[1] == st] == [x for x in want if x[1] == st]
            assert sorted(kept) == sorted(tilings)
            assert not any(p.closed for p in kept.values())


def test_near_roofline_from_plan_infos():
    # two tilings, one launch each: VALU operations over the launch time
    # against the issue rate; traffic only from a committed counter summary
    # whose kernel source is unchanged
    infos = {"quad": [{"stage_ms": [0, 0, 0, 0.5, 0], "n_near_pairs": 100, "near_valu_ops": 4e9, "near_evals": 5e7,
                       "targets_are_sources": True}],
             "tri": [{"stage_ms": [0, 0, 0, 1.5, 0], "n_near_pairs": 300, "near_valu_ops": 8e9, "near_evals": 1e8,
                      "targets_are_sources": True}]}
    r = bench.near_roofline(infos, ["quad", "tri"], "fp64")
    assert r["kernel"].endswith("k_near_fp64_sym")
    assert r["traffic"] == bench.committed_traffic("k_near_fp64_sym")
    assert abs(r["achieved"] * 1e9 - 6e9 / 1e-3) < 1.0
    assert abs(r["frac"] - 6e12 / bench.LANE_OPS) < 1e-12
    assert r["valu_per_pair"] == {"symmetric_eval": 73.2, "one_sided": 72.0}
    # the mixed kernel against the 32-bit issue rate, twice the FP64 one
    rm = bench.near_roofline(infos, ["quad", "tri"], "mixed")
    assert rm["kernel"].endswith("k_near_mixed_sym")
    assert abs(rm["frac"] - 6e12 / (2 * bench.LANE_OPS)) < 1e-12
    assert rm["peak"] == 2 * r["peak"]


def test_m2l_flop_model_by_hand():
    # p = 22: algorithmic 8 (p+1)^2 = 4232 per pair; FP64 MFMA form: rows
    # 0..22 in two 16-row tiles, k' = 0..21 in six 4-deep steps, Re and Im
    # columns: 2 x 32 x 24 x 2 = 3072 per pair; BF16x3: six products of H
    # padded to 32 rows x 32 columns with the two columns: 6 x 2 x 32 x 32 x 2
    # = 24576 per pair
    alg, issued, peak = bench.m2l_flops("fp64", 22, 10)
    assert alg == 42320 and issued == 30720 and peak == bench.FP64_PEAK
    alg, issued, peak = bench.m2l_flops("mixed", 22, 10)
    assert alg == 42320 and issued == 245760 and peak == bench.MFMA_BF16_PEAK
    # below p = 16 the mixed form runs the FP64 kernel
    assert bench.m2l_flops("mixed", 15, 1) == bench.m2l_flops("fp64", 15, 1)
    # p = 15 fills one row tile and four k-steps exactly
    assert bench.m2l_flops("fp64", 15, 1)[1] == 2 * 16 * 16 * 2
    f = bench.m2l_fraction("fp64", 22, 10, 1.0)
    assert abs(f["frac_alg"] - 42320 / 1e-3 / bench.FP64_PEAK) < 1e-15


def test_committed_traffic_checks_the_source_hash(tmp_path, monkeypatch):
    import hashlib
    import json
    (tmp_path / "profiles").mkdir()
    (tmp_path / "k.hip").write_bytes(b"kernel source")
    rec = {"kernel": "k_x", "source": "k.hip", "sha256": hashlib.sha256(b"kernel source").hexdigest(),
           "bytes_per_launch": 123.0}
    (tmp_path / "profiles" / "x.md").write_text("# x\n\n```json\n%s\n```\n" % json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.committed_traffic("k_x") == 123.0
    assert bench.committed_traffic("k_y") is None
    (tmp_path / "k.hip").write_bytes(b"kernel source, changed")
    assert bench.committed_traffic("k_x") is None
