"""Host-side helpers of the learned-refresh driver (no GPU)."""
import numpy as np

from paper_1907_02290_amd import learn, nbody


def test_threshold_keeps_the_target_recall():
    rng = np.random.default_rng(0)
    y = rng.uniform(size=5000) < 0.2
    p = np.where(y, rng.uniform(0.3, 1.0, y.size), rng.uniform(0.0, 0.7, y.size))
    for r in (0.9, 0.98, 1.0):
        ps = learn.choose_threshold(p, y, r)
        st = learn.classify(p, y, ps)
        assert st["recall"] >= r
        # the next larger positive score as threshold would lose recall
        higher = np.sort(p[y])
        k = np.searchsorted(higher, ps, side="right")
        if k < higher.size:
            assert learn.classify(p, y, higher[k])["recall"] < r or r == 0
    assert learn.choose_threshold(p, np.zeros_like(y), 0.98) == 1.0


def test_classify_counts():
    p = np.array([0.9, 0.1, 0.6, 0.4])
    y = np.array([1, 1, 0, 0])
    st = learn.classify(p, y, 0.5)
    assert st == dict(recall=0.5, flagged=0.5, positives=0.5, precision=0.5)


def test_initial_weights_layout():
    w = learn.init_weights(3)
    assert w.dtype == np.float32 and w.size == nbody.MLP_NPARAM
    b1 = w[768:832]
    b2 = w[832 + 4096:832 + 4096 + 64]
    b3 = w[-1]
    assert np.all(b1 == 0) and np.all(b2 == 0) and b3 == 0
    assert np.std(w[:768]) < 0.5 and np.std(w[832:832 + 4096]) < 0.2
    np.testing.assert_array_equal(w, learn.init_weights(3))


def test_force_error_metric():
    ref = (np.array([1.0, 0.0]), np.array([0.0, 2.0]), np.zeros(2))
    got = (np.array([1.1, 0.0]), np.array([0.0, 2.0]), np.zeros(2))
    np.testing.assert_allclose(learn.force_error(got, ref), [0.1, 0.0])
