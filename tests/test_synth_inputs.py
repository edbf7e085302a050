"""Properties of the seeded input generators (synth) that the workloads rely on."""
import numpy as np

import synth
from synth.problems import _ring_nearest


def test_ring_window_selects_the_nearest_cameras():
    """Ranking only the window around the closest camera gives exactly the full
    ranking's cameras, nearest first."""
    rng = np.random.default_rng(0)
    for n, c_hi in ((50, 8), (60, 20), (300, 20), (47, 20)):
        th = 2 * np.pi * np.arange(n) / n
        phi = rng.uniform(-np.pi, np.pi, 5000)
        c = rng.integers(2, min(c_hi, n) + 1, 5000)
        assert np.array_equal(_ring_nearest(phi, th, c, c_hi), _ring_nearest(phi, th, c, c_hi, full=True))


def test_batch_workload_shape():
    """64 problems, cameras in [50, 800], 200 landmarks per camera, 2-20 observers."""
    sizes = synth.problems.config4_sizes(seed=0)
    assert len(sizes) == 64 and sizes.min() >= 50 and sizes.max() <= 800
    p = synth.config4(seed=0, count=2, lo=50, hi=60)[0]
    cnt = np.bincount(p.obs_lm)
    assert p.n_lms == 200 * p.n_cams and cnt.min() >= 2 and cnt.max() <= 20


def test_batch_workload_parallel_generation_is_identical():
    a = synth.config4(seed=1, count=3, lo=50, hi=70)
    b = synth.config4(seed=1, count=3, lo=50, hi=70, workers=2)
    for p, q in zip(a, b):
        assert p.name == q.name and np.array_equal(p.obs_cam, q.obs_cam) and np.array_equal(p.J_p, q.J_p)
