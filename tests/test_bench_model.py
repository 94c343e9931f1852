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
