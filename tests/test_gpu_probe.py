"""The FP64 pair-rate probe (fmm_probe_pair_rate): a finite rate below the
VALU issue bound of the chip (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz over
at least 70 VALU instructions per evaluation) and above a floor no working
build falls under; bad arguments are rejected."""
import ctypes as C

import pytest

pytestmark = pytest.mark.gpu


def test_probe_pair_rate_bounds():
    from paper_1204_3105_amd import fmm
    r = fmm.probe_pair_rate(200)
    print("pair-rate probe: %.4g evaluations/s" % r, flush=True)
    assert 1e10 < r < 256 * 4 * 16 * 2.4e9 / 70


def test_probe_rejects_bad_arguments():
    from paper_1204_3105_amd import fmm
    L = fmm.lib()
    out = C.c_double(0.0)
    assert L.fmm_probe_pair_rate(0, 0, C.byref(out)) != 0
    assert L.fmm_probe_pair_rate(10, -1, C.byref(out)) != 0
