"""pd_probe_peak, the microbenchmarks behind the issue-rate roofline: every
unit reports a positive rate, and four FMAs per exponential run slower than
exponentials alone (the two share the vector issue)."""
import ctypes
import math

import pytest

pytestmark = pytest.mark.gpu


def test_unit_rates(pd):
    pdl, ctx = pd
    r = {k: ctx.probe_peak(k) for k in pdl.Context.PEAK_KINDS}
    for k, v in r.items():
        assert math.isfinite(v) and v > 0, (k, v)
    assert r["fp32_fma4_exp2"] < r["exp2"]
    # a 32x32x16 matrix-core product does far more flops per instruction than an FMA
    assert r["mfma_bf16"] > r["fp32_fma"]


def test_bad_kind_is_rejected(pd):
    pdl, ctx = pd
    rate = ctypes.c_double(0.0)
    st = pdl.lib().pd_probe_peak(ctx._h, 5, ctypes.byref(rate), None)
    assert st == 1  # PD_ERR_INVALID_ARG
