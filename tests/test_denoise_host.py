"""Host-side checks of the denoiser pipeline: the flat parameter layout of
psl.h matches the oracle's parameter list, and the time-to-1% summary
follows its definition on a hand-made result."""
import math

import numpy as np
import pytest


def test_flat_layout_matches_oracle_parameter_list():
    from oracle import denoiser as D
    from paper_1503_01725_amd import unet_init
    for c in (8, 16, 32):
        a = [(n, int(np.prod(s))) for n, s in D.param_shapes(c, 2)]
        b = [(n, int(np.prod(s))) for n, s in unet_init.layer_shapes(c)]
        assert a == b
    flat = unet_init.init_params(7, 8)
    total = sum(int(np.prod(s)) for _, s in D.param_shapes(8, 2))
    assert flat.dtype == np.float32 and flat.size == total


def test_time_to_one_percent_summary():
    from paper_1503_01725_amd.denoise import summarize
    row = {"plain_rms": 2.0, "denoised_rms": 0.3, "plain_gamma": 0.8, "denoised_gamma": 0.99,
           "sigma_rel": 0.05, "t_infer_s": 0.01}
    from paper_1503_01725_amd.denoise import EVAL_COUNTS
    case = {"hist_per_s": 1e8}
    case.update({f"{nl:.0e}": dict(row) for nl in EVAL_COUNTS})
    res = {"cases": [case]}
    out = summarize(res)
    n1 = 1e6 * (0.05 / 0.01) ** 2
    assert out["time_to_1pct"]["plain_histories"] == pytest.approx(n1)
    assert out["time_to_1pct"]["plain_s"] == pytest.approx(n1 / 1e8)
    rms1 = 2.0 * math.sqrt(1e6 / n1)
    assert out["time_to_1pct"]["rms_error_percent_of_dmax"] == pytest.approx(rms1)
    assert out["time_to_1pct"]["denoised_histories"] == 1e6
    assert out["time_to_1pct"]["denoised_s"] == pytest.approx(1e6 / 1e8 + 0.01)
    # equal-RMS speed-up at 1e6: plain histories (2.0 / 0.3)^2 * 1e6 against 1e6 + inference
    eq = out["equal_rms"]["1e+06"]
    assert eq["plain_histories_same_rms"] == pytest.approx(1e6 * (2.0 / 0.3) ** 2)
    assert eq["speedup"] == pytest.approx((1e6 * (2.0 / 0.3) ** 2 / 1e8) / (1e6 / 1e8 + 0.01))
    # stated RMS errors: plain (2.0 / e)^2 * 1e6 histories; the denoised 0.3 % is
    # reached at the first count for every stated error above it
    for e in (2.0, 1.0, 0.6):
        st = out["time_to_rms"][f"{e:g}"]
        assert st["plain_histories"] == pytest.approx(1e6 * (2.0 / e) ** 2)
        assert st["denoised_histories"] == 1e6
        assert st["speedup"] == pytest.approx((1e6 * (2.0 / e) ** 2 / 1e8) / (1e6 / 1e8 + 0.01))


def test_time_to_stated_rms_unreachable_is_null():
    from paper_1503_01725_amd.denoise import summarize, EVAL_COUNTS
    case = {"hist_per_s": 1e8}
    for nl in EVAL_COUNTS:
        case[f"{nl:.0e}"] = {"plain_rms": 2.0 * (1e6 / nl) ** 0.5, "denoised_rms": 0.8,
                             "plain_gamma": 0.8, "denoised_gamma": 0.9, "sigma_rel": 0.05,
                             "t_infer_s": 0.01}
    out = summarize({"cases": [case]})
    assert out["time_to_rms"]["1"]["denoised_histories"] == 1e6
    assert out["time_to_rms"]["0.6"]["denoised_histories"] is None
    assert out["time_to_rms"]["0.6"]["speedup"] is None
