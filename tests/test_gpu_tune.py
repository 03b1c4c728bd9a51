"""The n_grp / n_leaf autotuner times real reuse cycles on the device and
returns the fastest candidate."""
import pytest

pytestmark = pytest.mark.gpu


def test_tuner_picks_the_fastest_candidate():
    from paper_1907_02290_amd import tune
    res = tune.tune("plummer_4k", n=20000, n_grps=(16, 64, 256),
                    n_leafs=(4, 8), cycles=1)
    assert len(res["results"]) == 6
    best = min(res["results"], key=lambda r: r["ms_per_step"])
    assert res["best"] == dict(n_grp=best["n_grp"], n_leaf=best["n_leaf"])
    for r in res["results"]:
        assert r["ms_per_step"] > 0 and r["interactions"] > 0
    # smaller groups mean more groups
    g = {(r["n_grp"], r["n_leaf"]): r["groups"] for r in res["results"]}
    assert g[(16, 8)] > g[(64, 8)] > g[(256, 8)]
