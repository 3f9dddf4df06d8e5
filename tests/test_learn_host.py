"""Host-side logic of the learned classifier: the working-point search and
the seeded initialisation (no GPU)."""
import numpy as np

from paper_1912_09161_amd import learn


def test_choose_threshold_counts_best_logit_per_particle():
    # particles 1..4 reconstructible; particle 5 is not; -1 = ghost
    particle = np.array([1, 1, 2, 3, -1, 5, 4])
    logit = np.array([0.2, 0.9, 0.5, -0.3, 2.0, 3.0, 0.1])
    reco = np.array([1, 2, 3, 4])
    # best logits of the reconstructible particles: 0.9, 0.5, 0.1, -0.3
    assert learn.choose_threshold(logit, particle, reco, 0.25) == np.float32(0.9)
    assert learn.choose_threshold(logit, particle, reco, 0.5) == np.float32(0.5)
    assert learn.choose_threshold(logit, particle, reco, 0.51) == np.float32(0.1)
    assert learn.choose_threshold(logit, particle, reco, 1.0) == np.float32(-0.3)


def test_choose_threshold_is_always_finite():
    particle = np.array([1, -1])
    logit = np.array([0.4, 1.0])
    reco = np.array([1, 2])  # particle 2 has no track: 100 % is unreachable
    thr = learn.choose_threshold(logit, particle, reco, 1.0)
    assert thr == np.float32(0.4)  # highest reachable efficiency (50 %)
    assert np.isfinite(learn.choose_threshold(logit, particle, reco, 0.0))
    assert np.isfinite(learn.choose_threshold(logit, np.array([-1, -1]), reco, 0.5))


def test_he_uniform_bounds_and_seed():
    p = learn.he_uniform(3)
    assert p.shape == (1377,) and p.dtype == np.float32
    assert np.all(np.abs(p[0:256]) <= np.sqrt(6 / 8))
    assert np.all(np.abs(p[288:1312]) <= np.sqrt(6 / 32))
    assert np.all(p[256:288] == 0) and np.all(p[1312:1344] == 0) and p[1376] == 0
    assert np.array_equal(p, learn.he_uniform(3)) and not np.array_equal(p, learn.he_uniform(4))
