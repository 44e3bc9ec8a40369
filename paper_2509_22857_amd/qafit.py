"""Quantisation-aware polynomial fitting of ReLU (Section 3.2 of the paper,
after PILLAR): the activation polynomial's coefficients are integers at b
fractional bits, found as the exact solution of a bounded integer
least-squares problem rather than by rounding a real fit, so no monomial is
truncated to zero.

On the grid X = {k 2^-b : k integer, |k 2^-b| <= c} the targets are
Y_i = 2^b ReLU(x_i) (integers) and B_ik = x_i^k (0 <= k <= d).  The
coefficients A in Z^(d+1), each in [-2^(b-1), 2^(b-1) - 1], minimise
||B A - Y||^2, and the polynomial is p(x) = sum_k (a_k / 2^b) x^k.  The
paper's setting is d = 2, b = 10, c = 2.

The minimiser is found by Fincke-Pohst enumeration: with G = B^T B = R^T R
(R upper triangular) and A* the real least-squares solution,
||B A - Y||^2 = ||R (A - A*)||^2 + ||B A* - Y||^2, so the integer points
inside the ellipsoid ||R (A - A*)||^2 <= r^2 can be listed coordinate by
coordinate from a_d down to a_0, every coordinate's interval cut to the box.
r^2 starts at the objective of the rounded, clipped real solution (a
feasible point) and shrinks to each better point found.  Candidates are
compared on the objective in exact integer arithmetic (scaled by 2^(2 b d),
which makes every residual an integer); among equal objectives the
lexicographically smallest A wins.
"""
from __future__ import annotations

import math

import numpy as np


def grid(b: int, c: float) -> np.ndarray:
    """The integers k with |k 2^-b| <= c."""
    kmax = int(math.floor(c * (1 << b)))
    return np.arange(-kmax, kmax + 1, dtype=np.int64)


def objective_exact(A, b: int, c: float) -> int:
    """||B A - Y||^2 scaled by 2^(2 b d), as an exact integer: with x = k 2^-b
    the residual times 2^(b d) is sum_k a_k k^k' 2^(b (d - k')) - ReLU(k) 2^(b d)."""
    d = len(A) - 1
    tot = 0
    for k in grid(b, c).tolist():
        r = sum(int(a) * k ** e * (1 << (b * (d - e))) for e, a in enumerate(A)) - max(k, 0) * (1 << (b * d))
        tot += r * r
    return tot


def qa_fit(d: int = 2, b: int = 10, c: float = 2.0):
    """Integer coefficients (a_0 .. a_d) of the bounded integer least-squares
    fit of 2^b ReLU on the b-bit grid of [-c, c]."""
    ks = grid(b, c)
    x = ks.astype(np.float64) / (1 << b)
    B = np.vander(x, d + 1, increasing=True)
    Y = np.maximum(ks, 0).astype(np.float64)
    lo, hi = -(1 << (b - 1)), (1 << (b - 1)) - 1
    G = B.T @ B
    a_star = np.linalg.solve(G, B.T @ Y)
    R = np.linalg.cholesky(G).T  # upper triangular, G = R^T R

    def quad(A):
        v = R @ (np.asarray(A, dtype=np.float64) - a_star)
        return float(v @ v)

    start = [int(min(max(round(v), lo), hi)) for v in a_star]
    best = (objective_exact(start, b, c), start)
    r2 = quad(start) * (1 + 1e-9) + 1e-9
    A = [0] * (d + 1)

    def visit(k, partial):
        nonlocal best, r2
        # row k of R (A - A*) = R_kk (a_k - a*_k) + sum_{j > k} R_kj (a_j - a*_j)
        off = sum(R[k, j] * (A[j] - a_star[j]) for j in range(k + 1, d + 1))
        room = r2 - partial
        if room < 0:
            return
        half = math.sqrt(room) / abs(R[k, k])
        centre = a_star[k] - off / R[k, k]
        for v in range(max(lo, math.ceil(centre - half)), min(hi, math.floor(centre + half)) + 1):
            A[k] = v
            t = R[k, k] * (v - a_star[k]) + off
            p = partial + t * t
            if p > r2:
                continue
            if k == 0:
                cand = (objective_exact(A, b, c), list(A))
                if cand < best:
                    best = cand
                    r2 = quad(A) * (1 + 1e-9) + 1e-9
            else:
                visit(k - 1, p)

    visit(d, 0.0)
    return best[1]


def coefficients(d: int = 2, b: int = 10, c: float = 2.0) -> np.ndarray:
    """The fitted polynomial's real coefficients a_k / 2^b, k = 0 .. d."""
    return np.array(qa_fit(d, b, c), dtype=np.float64) / (1 << b)
