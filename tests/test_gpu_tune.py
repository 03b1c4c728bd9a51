"""The autotuner times real reuse cycles on the device: stage 1 over the
group and leaf sizes, stage 2 over the force kernel's tile shapes at the
stage-1 choice, with an optional accuracy guard supplied by the caller."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_tuner_picks_the_fastest_candidate():
    from paper_1907_02290_amd import tune
    res = tune.tune("plummer_4k", n=20000, n_grps=(16, 64, 256),
                    n_leafs=(4, 8), tiles=(64, 192), waves=(4, 6), cycles=1)
    s1 = [r for r in res["results"] if r["stage"] == 1]
    s2 = [r for r in res["results"] if r["stage"] == 2]
    assert len(s1) == 6 and len(s2) == 4
    b1 = min(s1, key=lambda r: r["ms_per_step"])
    assert all((r["n_grp"], r["n_leaf"]) == (b1["n_grp"], b1["n_leaf"])
               for r in s2)
    best = min(s2 + [b1], key=lambda r: r["ms_per_step"])
    assert res["best"] == dict(n_grp=best["n_grp"], n_leaf=best["n_leaf"],
                               tile_j=best["tile_j"],
                               waves_per_simd=best["waves_per_simd"])
    for r in res["results"]:
        assert r["ms_per_step"] > 0 and r["interactions"] > 0
    # smaller groups mean more groups
    g = {(r["n_grp"], r["n_leaf"]): r["groups"] for r in s1}
    assert g[(16, 8)] > g[(64, 8)] > g[(256, 8)]
    # the tile shape does not change the lists
    assert len({r["interactions"] for r in s2}) == 1


def test_tuner_accuracy_guard_drops_inaccurate_candidates():
    """Candidates whose error exceeds the bound are not chosen, however
    fast.  The error function here is a stand-in that scores the k-th
    candidate -k, so that with the bound -3 only the third stage-1
    candidate (n_grp 256) and the stage-2 candidates are admissible."""
    from paper_1907_02290_amd import tune
    calls = []

    def err(forces):
        assert len(forces) == 4 and np.all(np.isfinite(forces[0]))
        calls.append(1)
        return -float(len(calls))

    res = tune.tune("plummer_4k", n=20000, n_grps=(16, 64, 256),
                    tiles=(192,), waves=(6,), cycles=1, error=err,
                    max_err=-3.0)
    assert res["best"]["n_grp"] == 256
    s1 = [r for r in res["results"] if r["stage"] == 1]
    assert [r["admissible"] for r in s1] == [False, False, True]
    assert res["error_bound"] == -3.0
