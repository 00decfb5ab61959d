"""Pins of the Philox generator and the sampler (Algorithm 3, Definition 5)."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import philox, sampler
from oracle.leverage import integer_table, uniform_table
from synth import rng_for


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((123, 456), (7, 1, 2, 3)),
                                     ((2 ** 64 - 1, 2 ** 63), (2 ** 64 - 2, 2 ** 64 - 1, 5, 2 ** 60))])
def test_philox_matches_numpy_library(key, ctr):
    # numpy.random.Philox is Philox4x64-10 and increments its counter before each block
    c = sum(int(v) << (64 * k) for k, v in enumerate(ctr))  # 256-bit counter, word 0 lowest
    c = (c - 1) % (1 << 256)
    prev = [(c >> (64 * k)) & (2 ** 64 - 1) for k in range(4)]
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(prev, dtype=np.uint64))
    lib = [int(g.random_raw()) for _ in range(4)]
    assert list(philox.philox4x64_10(ctr, key)) == lib


def test_philox_vectorised_equals_scalar():
    rng = rng_for(31, 0)
    cs = rng.integers(0, 2 ** 63, (64, 4), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    k0, k1 = 0xDEADBEEF12345678, 0x0F0F0F0F0F0F0F0F
    vec = philox.philox4x64_10_np(cs[:, 0], cs[:, 1], cs[:, 2], cs[:, 3], k0, k1)
    for r in range(64):
        assert tuple(int(v[r]) for v in vec) == philox.philox4x64_10(cs[r], (k0, k1))


def test_mulhilo_exact():
    rng = rng_for(32, 0)
    a = rng.integers(0, 2 ** 63, 1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2 ** 63, 1000, dtype=np.uint64)
    hi, lo = philox.mulhilo64_np(a, b)
    for x, y, h, l in zip(a, b, hi, lo):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & (2 ** 64 - 1)


def test_draw_boundaries_and_zero_mass():
    # table with a zero-weight entry: C = [2, 2, 5], T = 5
    Q = np.array([2, 0, 3], dtype=np.uint64)
    C = np.cumsum(Q, dtype=np.uint64)
    T = 5
    for t, want in [(0, 0), (1, 0), (2, 2), (3, 2), (4, 2)]:
        r = -(-(t << 64) // T)  # smallest r with floor(r T / 2^64) = t
        got = sampler.draw_index(C, T, np.array([r], dtype=np.uint64))
        assert int(got[0]) == want


def test_draws_follow_table_chi2():
    p = np.array([0.05, 0.0, 0.2, 0.1, 0.3, 0.15, 0.2])
    Q, C, T = integer_table(p)
    r = sampler.philox_words(200000, 1, 5, 0, 0)[:, 0]
    idx = sampler.draw_index(C, T, r)
    counts = np.bincount(idx, minlength=len(p))
    assert counts[1] == 0
    nz = p > 0
    exp = len(idx) * Q[nz].astype(float) / T
    chi2 = float(np.sum((counts[nz] - exp) ** 2 / exp))
    assert chi2 < 22.5  # 5 dof, p ~ 4e-4


def test_product_distribution_sums_to_one_exactly():
    # Lemma 6 (first part): q^{!=n} sums to 1; in exact rational arithmetic over integer tables
    rng = rng_for(33, 0)
    tabs = []
    for I in (3, 4, 2):
        p = rng.random(I)
        p /= p.sum()
        Q, C, T = integer_table(p)
        tabs.append([Fraction(int(v), T) for v in Q])
    tot = sum(a * b * c for a, b, c in itertools.product(*tabs))
    assert tot == 1


def test_update_streams_are_distinct_and_weights_definition5():
    rng = rng_for(34, 0)
    tables = []
    for I in (7, 5, 6):
        p = rng.random(I)
        tables.append(integer_table(p / p.sum()))
    J = 64
    i0, w0 = sampler.draw_update(tables, 0, J, seed=9, stream_id=0, u=0)
    i1, w1 = sampler.draw_update(tables, 0, J, seed=9, stream_id=0, u=3)
    i2, _ = sampler.draw_update(tables, 0, J, seed=9, stream_id=1, u=0)
    assert not np.array_equal(i0, i1) and not np.array_equal(i0, i2)
    # the same key and counter give the same draws
    i3, w3 = sampler.draw_update(tables, 0, J, seed=9, stream_id=0, u=0)
    assert np.array_equal(i0, i3) and np.array_equal(w0, w3)
    # Definition 5 rescaling: w = 1/sqrt(J q), q the exact probability of the drawn tuple
    for j in range(J):
        q = Fraction(1)
        for k, m in enumerate((1, 2)):
            Q, C, T = tables[m]
            q *= Fraction(int(Q[i0[j, k]]), T)
        assert abs(w0[j] ** -2 / J - float(q)) <= 1e-14 * float(q)


@pytest.mark.parametrize("I", [1, 3, 7, 40, 500, 2000])
def test_uniform_table_is_exactly_uniform(I):
    Q, C, T = uniform_table(I)
    assert len(set(int(v) for v in Q)) == 1
    assert T == I * int(Q[0])
    assert Fraction(int(Q[0]), T) == Fraction(1, I)


def test_uniform_draws_weights_closed_form_and_chi2():
    dims = (5, 9, 6)
    tables = [uniform_table(I) for I in dims]
    J = 30000
    idx, w = sampler.draw_update(tables, 0, J, seed=4, stream_id=2, u=1)
    # Definition 5 with q = prod_k 1/I_k: w = sqrt(I_1 I_2 / J) for every sample
    np.testing.assert_allclose(w, np.sqrt(9 * 6 / J), rtol=1e-15)
    for k, I in enumerate((9, 6)):
        counts = np.bincount(idx[:, k], minlength=I)
        exp = J / I
        chi2 = float(np.sum((counts - exp) ** 2 / exp))
        assert chi2 < {9: 26.1, 6: 20.5}[I]  # I-1 dof, p ~ 1e-3
