"""Host-side pieces of the serving loop (no GPU): the arrival process."""
import numpy as np

from paper_2509_22857_amd.serving import poisson_arrivals


def test_poisson_arrivals_seeded_increasing_and_rate():
    a = poisson_arrivals(10.0, 4000, 7)
    b = poisson_arrivals(10.0, 4000, 7)
    assert np.array_equal(a, b)
    assert np.all(np.diff(a) > 0)
    gaps = np.diff(np.concatenate([[0.0], a]))
    # exponential gaps: mean 1/rate, coefficient of variation 1
    assert abs(gaps.mean() - 0.1) < 0.01
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.06
