"""Quantisation-aware polynomial fitting (Section 3.2): the bounded integer
least-squares solution, pinned by exhaustive search over the whole
coefficient box at small b, and by local optimality at the paper's setting
d = 2, b = 10, c = 2."""
import itertools

import numpy as np
import pytest

from paper_2509_22857_amd import qafit


def brute_force(d, b, c):
    """Every A in the box; the objective ||B A - Y||^2 in exact integers
    (x = k / 2^b, Y = 2^b ReLU(x), everything scaled by 2^(2 b d)); the
    lexicographically smallest among the minimisers."""
    ks = np.arange(-int(c * 2 ** b), int(c * 2 ** b) + 1, dtype=np.int64)
    lo, hi = -2 ** (b - 1), 2 ** (b - 1) - 1
    box = np.array(list(itertools.product(range(lo, hi + 1), repeat=d + 1)), dtype=np.int64)
    cols = np.stack([ks ** e * 2 ** (b * (d - e)) for e in range(d + 1)], axis=0)  # [d+1][points]
    res = box @ cols - np.maximum(ks, 0) * 2 ** (b * d)
    obj = (res * res).sum(axis=1)
    best = obj.min()
    return min(tuple(int(v) for v in a) for a in box[obj == best])


@pytest.mark.parametrize("d,b,c", [(2, 3, 2.0), (2, 4, 2.0), (2, 5, 2.0), (2, 4, 1.0), (3, 3, 2.0), (1, 5, 2.0)])
def test_matches_exhaustive_search(d, b, c):
    assert tuple(qafit.qa_fit(d, b, c)) == brute_force(d, b, c)


def test_paper_setting():
    A = qafit.qa_fit(2, 10, 2.0)
    lo, hi = -512, 511
    assert all(lo <= a <= hi for a in A)
    assert all(a != 0 for a in A)  # no monomial truncated
    best = qafit.objective_exact(A, 10, 2.0)
    # no integer point within 2 of it in every coordinate does better
    for delta in itertools.product(range(-2, 3), repeat=3):
        B = [min(max(a + e, lo), hi) for a, e in zip(A, delta)]
        assert qafit.objective_exact(B, 10, 2.0) >= best
    # at least as good as rounding the real fit and clipping to the box
    ks = qafit.grid(10, 2.0)
    x = ks / 1024.0
    real = np.linalg.lstsq(np.vander(x, 3, increasing=True), np.maximum(ks, 0).astype(float), rcond=None)[0]
    rounded = [int(min(max(round(v), lo), hi)) for v in real]
    assert best <= qafit.objective_exact(rounded, 10, 2.0)
    # the fitted polynomial follows ReLU on [-c, c] (within a quadratic's reach)
    p = np.polynomial.polynomial.polyval(x, qafit.coefficients())
    assert np.max(np.abs(p - np.maximum(x, 0))) < 0.2
