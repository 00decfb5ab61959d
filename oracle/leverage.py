"""Leverage scores and the per-core sampling tables (oracle; test infrastructure).

* Definition 4: the i-th leverage score of A is the squared norm of row i of
  the matrix of left singular vectors of A (rank(A) columns).
* eq. (3): p^(n)(i_n) = l_{i_n}(G^(n)_(2)) / rank(G^(n)_(2)).
* The paper computes these with an economic SVD (Appendix B.2, "compute
  distributions").  Its tolerance for the numerical rank is not stated; we
  use numpy's default, tol = max(rows, cols) * eps * sigma_max.  When the
  unfolding has full row rank (rank equals its number of rows) every row of
  U is a unit vector and we set the scores to exactly 1.

Integer table (how a draw from p^(n) is made reproducible bit for bit): each
probability is turned into an integer weight Q_i = floor(p_i * 2^52) (the
FP64 product is exact, being a power-of-two scaling), C is the inclusive
prefix sum of Q and T = C[-1].  A draw then uses the exact sampling
probabilities Q_i / T; entries with Q_i = 0 are never drawn.
"""
from __future__ import annotations

import numpy as np

from .ring import core_unfolding

SCALE = 2.0 ** 52


def numerical_rank(s, shape):
    if s.size == 0 or s[0] == 0.0:
        return 0
    tol = s[0] * max(shape) * np.finfo(np.float64).eps
    return int(np.sum(s > tol))


def leverage_scores(A):
    """(scores, rank) of a matrix A via its economic SVD (Definition 4)."""
    A = np.asarray(A, dtype=np.float64)
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    r = numerical_rank(s, A.shape)
    if r == A.shape[0]:
        return np.ones(A.shape[0]), r
    return np.sum(U[:, :r] ** 2, axis=1), r


def mode_distribution(G):
    """p^(n) of eq. (3) for core G (R_{n-1} x I_n x R_n)."""
    ell, r = leverage_scores(core_unfolding(G))
    if r == 0:
        raise ZeroDivisionError("core is zero: its distribution is undefined")
    return ell / r


def integer_table(p):
    """(Q, C, T): integer weights floor(p * 2^52), inclusive prefix sums, total."""
    p = np.asarray(p, dtype=np.float64)
    Q = np.floor(p * SCALE).astype(np.uint64)
    C = np.cumsum(Q, dtype=np.uint64)
    return Q, C, int(C[-1])


def core_table(G):
    """Integer sampling table of one core: integer_table(mode_distribution(G))."""
    return integer_table(mode_distribution(G))


def uniform_table(I):
    """Integer table of the uniform distribution over I indices (the uniform-sampling
    comparison of Section 4: p_i = 1/I)."""
    return integer_table(np.full(int(I), 1.0 / int(I)))
