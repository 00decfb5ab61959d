"""Pins of the sampled update (Algorithms 2-4) and of whole ALS runs."""
import itertools

import numpy as np
import pytest

from oracle import als, ring, sampler
from oracle.leverage import core_table
from synth import make_config, random_cores, ring_tensor, rng_for


def tables_for(cores, n):
    return [None if m == n else core_table(cores[m]) for m in range(len(cores))]


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_sketch_rows_are_weighted_design_rows(n):
    # Algorithm 4 row j = w_j * row lin(i_{n+1}..i_{n-1}) of G^{!=n}_[2] (Definition 3)
    dims, ranks = (3, 4, 2, 3), (2, 3, 1, 2)
    cores = random_cores(dims, ranks, rng_for(41, n))
    N = 4
    modes = [(n + 1 + k) % N for k in range(N - 1)]
    idx, w = sampler.draw_update(tables_for(cores, n), n, 40, 3, 0, n)
    A = als.sketch_subchain(cores, n, idx, w)
    full = ring.subchain_unfolding(cores, n)
    for j in range(40):
        row = ring.lin_index(idx[j], [dims[m] for m in modes])
        np.testing.assert_allclose(A[j], w[j] * full[row], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("n", [0, 2, 3])
def test_sketch_fibers_are_weighted_data_rows(n):
    dims = (3, 4, 2, 3)
    X = rng_for(42, n).standard_normal(dims)
    N = 4
    modes = [(n + 1 + k) % N for k in range(N - 1)]
    idx = np.stack([rng_for(43, k).integers(0, dims[m], 25) for k, m in enumerate(modes)], axis=1)
    w = rng_for(44, n).random(25) + 0.5
    B = als.sketch_fibers(X, n, idx, w)
    XnT = ring.unfold_cyclic(X, n).T
    for j in range(25):
        row = ring.lin_index(idx[j], [dims[m] for m in modes])
        np.testing.assert_allclose(B[j], w[j] * XnT[row], rtol=1e-14)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_exact_recovery_from_consistent_system(n):
    # noise-free TR data, every other core at the truth: one sampled update recovers core n
    dims, ranks = (14, 12, 16), (3, 2, 4)
    true = random_cores(dims, ranks, rng_for(45, n))
    X = ring_tensor(true)
    cores = [c.copy() for c in true]
    cores[n] = rng_for(46, n).standard_normal(cores[n].shape)
    new, _, _ = als.sampled_update(X, cores, tables_for(cores, n), n, 60, 0, 0, n)
    np.testing.assert_allclose(new, true[n], rtol=0, atol=1e-10 * np.abs(true[n]).max())


def test_noise_free_als_reaches_zero_error():
    dims, ranks = (20, 22, 18), (2, 3, 2)
    X = ring_tensor(random_cores(dims, ranks, rng_for(1, 1)))
    init = random_cores(dims, ranks, rng_for(1, 3))
    cores = als.tr_als_sampled(X, init, 300, 40, seed=0)
    assert als.fit_error(cores, X) < 1e-8


def test_c1_recipe_reaches_noise_floor():
    # 60^3, ranks 3, sigma = 1e-3 noise: the error floor is sigma / RMS(X) (up to the fitted dof)
    X, _, _ = make_config("c1", dtype=np.float64)
    init = random_cores(X.shape, (3, 3, 3), rng_for(1, 3))
    cores = als.tr_als_sampled(X, init, 2000, 10, seed=0)
    floor = 1e-3 / np.sqrt(np.mean(X ** 2))
    assert 0.97 * floor < als.fit_error(cores, X) < 1.03 * floor


def test_sketched_gram_is_unbiased():
    # S^T S is unbiased (Definition 5 rescaling): E[A~^T A~] = G^{!=n T}_[2] G^{!=n}_[2],
    # E[A~^T X~] = G^{!=n T}_[2] X_[n]^T
    dims, ranks = (4, 5, 3), (2, 2, 3)
    cores = random_cores(dims, ranks, rng_for(47, 0))
    X = rng_for(48, 0).standard_normal(dims)
    n = 1
    A = ring.subchain_unfolding(cores, n)
    F = A.T @ A
    Fx = A.T @ ring.unfold_cyclic(X, n).T
    tabs = tables_for(cores, n)
    accH = np.zeros_like(F)
    accB = np.zeros_like(Fx)
    trials = 400
    for u in range(trials):
        idx, w = sampler.draw_update(tabs, n, 50, 7, 0, u)
        As = als.sketch_subchain(cores, n, idx, w)
        Bs = als.sketch_fibers(X, n, idx, w)
        accH += As.T @ As
        accB += As.T @ Bs
    assert np.linalg.norm(accH / trials - F) < 0.05 * np.linalg.norm(F)
    assert np.linalg.norm(accB / trials - Fx) < 0.08 * np.linalg.norm(Fx)


def test_theorem7_relative_error_guarantee():
    # Theorem 7: with J above eq. (7)'s bound, the sampled solution is (1+eps)-optimal w.p. >= 1-delta
    dims, ranks = (30, 6, 25), (1, 2, 1)
    cores = random_cores(dims, ranks, rng_for(49, 0))
    X = ring_tensor(cores) + 0.5 * rng_for(50, 0).standard_normal(dims)
    n = 1
    eps, delta = 0.5, 0.2
    prodR2 = np.prod([r ** 2 for r in ranks])
    Pn = ranks[0] * ranks[1]
    bound = prodR2 * max(16 / (3 * (np.sqrt(2) - 1) ** 2) * np.log(4 * Pn / delta), 4 / (eps * delta))
    J = int(bound) + 1
    A = ring.subchain_unfolding(cores, n)
    B = ring.unfold_cyclic(X, n).T
    Z, *_ = np.linalg.lstsq(A, B, rcond=None)
    opt = np.linalg.norm(A @ Z - B)
    tabs = tables_for(cores, n)
    ok = 0
    trials = 40
    for u in range(trials):
        new, _, _ = als.sampled_update(X, cores, tabs, n, J, 11, 0, u)
        res = np.linalg.norm(A @ ring.core_unfolding(new).T - B)
        ok += res <= (1 + eps) * opt
    assert ok >= (1 - delta) * trials


def test_solution_invariant_to_global_weight_scale():
    rng = rng_for(51, 0)
    A = rng.standard_normal((80, 6))
    B = rng.standard_normal((80, 5))
    np.testing.assert_allclose(als.solve_core(3.7 * A, 3.7 * B, 2, 3), als.solve_core(A, B, 2, 3), rtol=1e-12)


def test_rank_deficient_sketch_is_flagged():
    A = np.zeros((30, 4))
    A[:, :2] = rng_for(52, 0).standard_normal((30, 2))
    with pytest.raises(als.SingularSystem):
        als.solve_core(A, np.ones((30, 3)), 2, 2)


def test_fit_error_termwise():
    dims, ranks = (3, 4, 2), (2, 2, 2)
    cores = random_cores(dims, ranks, rng_for(53, 0))
    X = rng_for(54, 0).standard_normal(dims)
    num = 0.0
    for i in itertools.product(*[range(d) for d in dims]):
        v = np.trace(cores[0][:, i[0], :] @ cores[1][:, i[1], :] @ cores[2][:, i[2], :])
        num += (v - X[i]) ** 2
    assert abs(als.fit_error(cores, X) - np.sqrt(num / np.sum(X ** 2))) < 1e-13


def test_exact_als_and_sampled_agree_on_noisy_data():
    # Section 4.1 protocol: the sampled method reaches the exact method's error within a small factor
    dims, ranks = (25, 24, 26), (2, 2, 2)
    X = ring_tensor(random_cores(dims, ranks, rng_for(55, 0)))
    X = X + 0.01 * np.linalg.norm(X) / np.sqrt(X.size) * rng_for(56, 0).standard_normal(dims)
    init = random_cores(dims, ranks, rng_for(57, 0))
    e_ex = als.fit_error(als.tr_als_exact(X, init, 15), X)
    e_s = als.fit_error(als.tr_als_sampled(X, init, 400, 15, seed=0), X)
    assert e_s <= 1.2 * e_ex


@pytest.mark.parametrize("n", [0, 2])
def test_uniform_sampled_and_exact_updates_recover_consistent_core(n):
    # noise-free TR data with the other cores at the truth: any full-rank row subset (uniform
    # draws) and the full design (Algorithm 1) both return the true core
    dims, ranks = (11, 13, 12), (2, 3, 2)
    true = random_cores(dims, ranks, rng_for(58, n))
    X = ring_tensor(true)
    cores = [c.copy() for c in true]
    cores[n] = rng_for(59, n).standard_normal(cores[n].shape)
    tol = 1e-10 * np.abs(true[n]).max()
    new_u, idx, w = als.lockstep_update(X, cores, n, 80, 0, 0, n, uniform=True)
    np.testing.assert_allclose(new_u, true[n], rtol=0, atol=tol)
    N = 3
    others = [dims[(n + 1 + k) % N] for k in range(N - 1)]
    np.testing.assert_allclose(w, np.sqrt(np.prod(others) / 80), rtol=1e-15)
    np.testing.assert_allclose(als.exact_update(X, cores, n), true[n], rtol=0, atol=tol)


def test_sample_count_may_change_between_updates():
    dims, ranks = (9, 10, 11), (2, 2, 2)
    X = rng_for(60, 0).standard_normal(dims)
    init = random_cores(dims, ranks, rng_for(60, 3))
    rec = []
    Js = {0: 50, 1: 50, 2: 50, 3: 20, 4: 20, 5: 90}
    als.tr_als_sampled(X, init, lambda u: Js[u], 2, seed=0, record=rec)
    assert [r[2].shape[0] for r in rec] == [Js[u] for u in range(6)]
    # the first updates are those of a run with a fixed J (same counters, same tables)
    rec2 = []
    als.tr_als_sampled(X, init, 50, 1, seed=0, record=rec2)
    for a, b in zip(rec[:3], rec2):
        assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("n", [0, 1, 3])
def test_normalize_core_is_a_gauge_change(n):
    # QR with positive diagonal: Q orthonormal, R upper, TR and both cores' leverage unchanged
    from oracle.leverage import leverage_scores
    dims, ranks = (5, 6, 4, 7), (2, 3, 4, 2)
    cores = random_cores(dims, ranks, rng_for(61, n))
    cores[n] = cores[n] * 1e3  # scales drifted apart
    out = als.normalize_core(cores, n)
    Rp, I, Rn = cores[n].shape
    Q = out[n].reshape(Rp * I, Rn)
    np.testing.assert_allclose(Q.T @ Q, np.eye(Rn), atol=1e-13)
    T0, T1 = ring.tr_full(cores), ring.tr_full(out)
    assert np.linalg.norm(T1 - T0) <= 1e-12 * np.linalg.norm(T0)
    nx = (n + 1) % 4
    for m in (n, nx):
        a, _ = leverage_scores(ring.core_unfolding(cores[m]))
        b, _ = leverage_scores(ring.core_unfolding(out[m]))
        np.testing.assert_allclose(b, a, atol=1e-12)
    # R = Q^T G_n is upper triangular with a positive diagonal
    R = Q.T @ cores[n].reshape(Rp * I, Rn)
    assert np.all(np.diag(R) > 0) and np.allclose(np.tril(R, -1), 0, atol=1e-9 * np.abs(R).max())


def test_normalized_als_follows_the_same_iterates():
    # a gauge change leaves the LS optimum, the draws and hence TR(G) after every update unchanged
    dims, ranks = (18, 20, 22), (2, 3, 2)
    X = rng_for(62, 0).standard_normal(dims)
    init = random_cores(dims, ranks, rng_for(62, 3))
    a = als.tr_als_sampled(X, init, 120, 3, seed=1)
    b = als.tr_als_sampled(X, init, 120, 3, seed=1, normalize=True)
    Ta, Tb = ring.tr_full(a), ring.tr_full(b)
    assert np.linalg.norm(Ta - Tb) <= 1e-9 * np.linalg.norm(Ta)
    e = als.tr_als_exact(X, init, 2)
    f = als.tr_als_exact(X, init, 2, normalize=True)
    assert np.linalg.norm(ring.tr_full(e) - ring.tr_full(f)) <= 1e-9 * np.linalg.norm(ring.tr_full(e))
