"""Pins of the sampled relative-error estimate (Section 3.1, Termination Criteria): the entry
evaluation against the dense ring contraction, the draws against numpy's own Philox4x64-10,
the estimator against exact values it must reproduce, and its statistical error against the
exact fit."""
import numpy as np
import pytest

from oracle import als, estimate, ring
from synth import random_cores, ring_tensor, rng_for


def test_entries_match_dense_ring():
    dims, ranks = (4, 3, 5, 2), (2, 3, 1, 4)
    cores = random_cores(dims, ranks, rng_for(51, 1))
    full = ring.tr_full(cores)
    idx = np.stack(np.unravel_index(np.arange(full.size), dims), axis=1)
    np.testing.assert_allclose(estimate.tr_entries(cores, idx), full.ravel(), rtol=1e-12, atol=1e-13)


def test_draws_are_the_library_philox_words():
    # word 0 of the block with counter (s, tag, 0, 1); numpy.random.Philox increments its
    # 256-bit counter before each block, so it starts one below
    dims, S, key, tag = (7, 11, 13), 50, (12345, 678), 3
    E = 7 * 11 * 13
    want = []
    for s in range(S):
        c = s + (tag << 64) + (1 << 192) - 1
        g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                             counter=np.array([(c >> (64 * k)) & (2 ** 64 - 1) for k in range(4)], dtype=np.uint64))
        r = int(g.random_raw())
        want.append((r * E) >> 64)
    got = estimate.estimate_indices(dims, S, key[0], key[1], tag)
    assert [int(np.ravel_multi_index(tuple(i), dims)) for i in got] == want


def test_exact_ring_data_estimate_zero():
    dims, ranks = (9, 8, 7), (3, 2, 4)
    cores = random_cores(dims, ranks, rng_for(52, 1))
    X = ring_tensor(cores)
    assert estimate.sampled_fit_estimate(cores, X, 4000, seed=1) < 1e-12


def test_single_entry_residual_scales_with_its_hit_count():
    # one entry off by delta: est^2 ||X||^2 = (E / S) h delta^2, h = number of draws of that entry
    dims, ranks, S = (5, 6, 4), (2, 2, 2), 3000
    cores = random_cores(dims, ranks, rng_for(53, 1))
    X = ring_tensor(cores)
    idx = estimate.estimate_indices(dims, S, 9, 0)
    lin = np.ravel_multi_index(tuple(idx.T), dims)
    e_star = int(np.bincount(lin).argmax())
    h = int(np.sum(lin == e_star))
    delta = 0.75
    Xp = X.copy().ravel()
    Xp[e_star] += delta
    Xp = Xp.reshape(dims)
    est = estimate.sampled_fit_estimate(cores, Xp, S, seed=9)
    want = (X.size / S) * h * delta ** 2 / float(np.sum(Xp * Xp))
    assert abs(est ** 2 - want) <= 1e-12 * want


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_estimate_within_five_standard_errors_of_exact_fit(seed):
    # E[est^2] = fit^2; the standard error of the mean of S draws of d^2 (E / ||X||^2) from the
    # exact distribution of squared residuals bounds the deviation
    dims, ranks, S = (14, 12, 13), (3, 3, 3), 20000
    true = random_cores(dims, ranks, rng_for(54, 1))
    X = ring_tensor(true) + 0.3 * rng_for(54, 2).standard_normal(dims)
    cores = random_cores(dims, ranks, rng_for(54, 3))
    d2 = (ring.tr_full(cores) - X).ravel() ** 2
    x2 = float(np.sum(X * X))
    fit2 = float(np.sum(d2)) / x2
    se = X.size * float(np.std(d2)) / np.sqrt(S) / x2
    est = estimate.sampled_fit_estimate(cores, X, S, seed=seed)
    assert abs(est ** 2 - fit2) <= 5 * se
    assert abs(np.sqrt(fit2) - als.fit_error(cores, X)) <= 1e-12


def test_draws_uniform_over_entries():
    dims, S = (3, 4, 5), 60000
    idx = estimate.estimate_indices(dims, S, 5, 2)
    counts = np.bincount(np.ravel_multi_index(tuple(idx.T), dims), minlength=60)
    chi2 = float(np.sum((counts - S / 60) ** 2 / (S / 60)))
    assert chi2 < 59 + 5 * np.sqrt(2 * 59)  # 59 degrees of freedom, 5 sigma
