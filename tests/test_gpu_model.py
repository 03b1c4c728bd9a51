"""The step-model sweep on the device: every measured point is consistent
with the library's own counts, and the fit and prediction run on it."""
import numpy as np
import pytest

from paper_1907_02290_amd import model

pytestmark = pytest.mark.gpu


def test_sweep_fit_predict_small():
    print("case model sweep plummer 2^16", flush=True)
    pts = model.sweep("plummer_1m", [0.5, 1.0], [32, 128], n=1 << 16,
                      reuse=2, cycles=1)
    assert len(pts) == 4
    for p in pts:
        assert p["n"] == 1 << 16
        assert p["n_i"] == pytest.approx(p["n"] / p["n_groups"])
        assert p["n_list"] == pytest.approx(p["n_inter"] / p["n"])
        assert p["t_int"] > 0 and p["force_ms"] > 0 and p["ms_per_step"] > 0
        # the walk's entries per group cannot be fewer than its own particles
        assert p["n_epj"] >= p["n"]
        assert set(p["phase_ms"]) >= {"force", "walk", "moments", "kick"}
    coef = model.fit(pts)
    assert np.isfinite(coef["alpha_calc"]) and np.isfinite(coef["alpha_transfer"])
    for p in pts:
        ms, total = model.predict(p, coef)
        assert total > 0 and np.isfinite(total)
