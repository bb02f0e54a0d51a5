"""The paper-shaped commissioning experiment end to end at small sizes, with
and without the ring-smoothness term of the fit: every field and metric is
produced, the fit never raises the residual of the commissioning data above
the uncommissioned model's (the solver starts there and only descends), and
the corrections stay positive."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_commissioning_experiment_runs(eng):
    from paper_1503_01725_amd import commission_eval as ce
    r = ce.evaluate(hist_per_basis=2e4, hist_per_field=2e7, hist_measured=4e7, max_iter=300,
                    log=lambda m: print(m, flush=True))
    assert set(r["fields"]) == {f"{s:g}x{s:g}" for s in ce.FIELDS_EVAL}
    for f, d in r["fields"].items():
        for m in ("reference", "commissioned"):
            assert set(d[m]) == {"pdd"} | {f"{a}_{x:g}" for x in ce.DEPTHS
                                          for a in ("inline", "crossline")}
            assert all(v is None or math.isfinite(v) for v in d[m]["pdd"].values())
    n = r["nnls"]
    assert n["rel_residual"] <= n["rel_residual_uncommissioned"] * (1 + 1e-9)
    assert r["bases"] == 610 and 0 < r["bases_used"] <= 610
    assert r["output_factor_diff_pct"]["reference"]["10"] == 0.0


def test_commissioning_experiment_with_ring_smoothness(eng):
    """The smoothness term is zero at the start point (equal factors), and the
    solver only descends, so the residual of the commissioning data still
    cannot rise above the uncommissioned model's."""
    from paper_1503_01725_amd import commission_eval as ce
    r = ce.evaluate(hist_per_basis=2e4, hist_per_field=2e7, hist_measured=4e7, max_iter=300,
                    smooth=1e-4, log=lambda m: print(m, flush=True))
    assert r["smooth"] == 1e-4
    n = r["nnls"]
    assert n["rel_residual"] <= n["rel_residual_uncommissioned"] * (1 + 1e-9)
    for d in r["fields"].values():
        assert all(v is None or math.isfinite(v) for v in d["commissioned"]["pdd"].values())
