"""Pins of leverage scores, per-core distributions and integer tables."""
import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import leverage, ring
from oracle.leverage import integer_table, leverage_scores, mode_distribution, SCALE
from synth import random_cores, rng_for


def qr_scores(A):
    """Leverage scores as squared row norms of an orthonormal basis of range(A)
    from a column-pivoted QR (library routine), independent of the SVD path."""
    Q, R, _ = scipy.linalg.qr(A, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    r = int(np.sum(d > d[0] * max(A.shape) * np.finfo(float).eps * 10)) if d.size else 0
    return np.sum(Q[:, :r] ** 2, axis=1), r


@pytest.mark.parametrize("shape", [(50, 6), (200, 25), (9, 9)])
def test_leverage_matches_qr_row_norms(shape):
    A = rng_for(21, shape[0]).standard_normal(shape)
    ell, r = leverage_scores(A)
    ref, rr = qr_scores(A)
    assert r == rr == min(shape)
    np.testing.assert_allclose(ell, ref, atol=1e-12)


def test_leverage_rank_deficient():
    rng = rng_for(22, 0)
    A = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 8))  # rank 3
    ell, r = leverage_scores(A)
    ref, rr = qr_scores(A)
    assert r == rr == 3
    np.testing.assert_allclose(ell, ref, atol=1e-10)
    assert abs(ell.sum() - 3) < 1e-10


@pytest.mark.parametrize("shape", [(30, 4), (7, 20), (100, 100)])
def test_leverage_sum_is_rank_and_bounded(shape):
    # Section 2.2: sum of leverage scores = rank; each score in [0, 1]
    A = rng_for(23, shape[1]).standard_normal(shape)
    ell, r = leverage_scores(A)
    assert abs(ell.sum() - r) < 1e-10
    assert np.all(ell >= -1e-15) and np.all(ell <= 1 + 1e-12)


def test_wide_full_rank_is_uniform_exactly():
    A = rng_for(24, 0).standard_normal((12, 40))
    ell, r = leverage_scores(A)
    assert r == 12 and np.all(ell == 1.0)


def test_leverage_of_kronecker_is_product():
    # proof of Lemma 6: scores of a Kronecker product are products of scores
    rng = rng_for(25, 0)
    A = rng.standard_normal((6, 2))
    B = rng.standard_normal((5, 3))
    ell_k, _ = leverage_scores(np.kron(A, B))
    ea, _ = leverage_scores(A)
    eb, _ = leverage_scores(B)
    np.testing.assert_allclose(ell_k, np.kron(ea, eb), atol=1e-12)


def product_distribution(cores, n):
    """q^{!=n} (eq. (4)) over rows lin(i_{n+1}..i_{n-1}) of G^{!=n}_[2]."""
    N = len(cores)
    modes = [(n + 1 + k) % N for k in range(N - 1)]
    ps = [mode_distribution(cores[m]) for m in modes]
    q = ps[0]
    for p in ps[1:]:
        q = np.kron(p, q)  # first index fastest
    return q


@pytest.mark.parametrize("n", [0, 1, 2])
def test_lemma6_product_distribution_dominates_leverage(n):
    # Lemma 6: q^{!=n} is a distribution and q(i) >= beta_n * l_i(G^{!=n}_[2]) / rank
    dims, ranks = (6, 7, 5), (2, 3, 2)
    cores = random_cores(dims, ranks, rng_for(26, n))
    N = 3
    q = product_distribution(cores, n)
    assert abs(q.sum() - 1) < 1e-12
    A = ring.subchain_unfolding(cores, n)
    ell, r = qr_scores(A)
    Rp, Rn = ranks[(n - 1) % N], ranks[n]
    beta = 1.0 / (Rp * Rn * np.prod([ranks[j] ** 2 for j in range(N) if j not in ((n - 1) % N, n)]))
    assert np.all(q >= beta * ell / r - 1e-15)
    # the sharper per-row bound in the proof: l_i(G^{!=n}_[2]) <= prod_j l_{i_j}(G^(j)_(2))
    modes = [(n + 1 + k) % N for k in range(N - 1)]
    ells = [leverage_scores(ring.core_unfolding(cores[m]))[0] for m in modes]
    prod = ells[0]
    for e in ells[1:]:
        prod = np.kron(e, prod)
    assert np.all(ell <= prod + 1e-12)


def test_subchain_range_in_kronecker_range():
    # supplementary lemma: range(G^{!=n}_[2]) within range of the Kronecker product of core unfoldings
    dims, ranks = (5, 6, 4), (2, 2, 3)
    cores = random_cores(dims, ranks, rng_for(27, 0))
    n = 1
    N = 3
    modes = [(n + 1 + k) % N for k in range(N - 1)]
    K = ring.core_unfolding(cores[modes[0]])
    for m in modes[1:]:
        K = np.kron(ring.core_unfolding(cores[m]), K)
    A = ring.subchain_unfolding(cores, n)
    Qk, _ = np.linalg.qr(K)
    resid = A - Qk @ (Qk.T @ A)
    assert np.linalg.norm(resid) < 1e-10 * np.linalg.norm(A)


def test_integer_table():
    p = mode_distribution(rng_for(28, 0).standard_normal((3, 50, 4)))
    Q, C, T = integer_table(p)
    # Q = floor(p * 2^52), checked in exact rational arithmetic
    for pi, qi in zip(p, Q):
        f = Fraction(pi) * (1 << 52)
        assert int(qi) <= f < int(qi) + 1
    assert np.all(np.diff(C.astype(object)) == Q[1:].astype(object))
    assert T == sum(int(v) for v in Q)
    assert abs(T - SCALE) <= len(p) + SCALE * 1e-14


def test_uniform_table_for_wide_core():
    G = rng_for(29, 0).standard_normal((5, 12, 6))  # I=12 < P=30: full row rank
    Q, C, T = leverage.core_table(G)
    assert np.all(Q == Q[0]) and int(Q[0]) == int(np.floor((1.0 / 12) * SCALE))
