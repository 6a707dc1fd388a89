"""cch_probe_fp64, the calibration of the FP64 roofline denominators: the
three rates are positive, finite, and none exceeds the published FP64 peak
of the MI355X (78.6 TFLOP/s for the matrix and the vector units) by more
than a clock margin; a NULL output is refused."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_probe_rates_within_published_peak():
    import paper_1709_03005_amd as cc
    r = cc.probe_fp64(0)
    print(f"[peaks] FP64 TFLOP/s: {r}", flush=True)
    for name, v in r.items():
        assert np.isfinite(v) and v > 1.0, (name, v)
        assert v < 78.6 * 1.1, (name, v)


def test_probe_null_refused():
    import paper_1709_03005_amd as cc
    assert cc.lib.cch_probe_fp64(0, None, ctypes.c_void_p(0)) == cc.CCH_E_INVALID_ARG
