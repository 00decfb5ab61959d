"""Pins of the oracle's TR format code against definitions and the paper's worked example."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import ring
from synth import random_cores, rng_for

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_tr(cores):
    """eq. (1) summed term by term over every bond-index tuple."""
    N = len(cores)
    dims = [c.shape[1] for c in cores]
    ranks = [c.shape[2] for c in cores]
    X = np.zeros(dims)
    for i in itertools.product(*[range(d) for d in dims]):
        tot = 0.0
        for r in itertools.product(*[range(R) for R in ranks]):
            prod = 1.0
            for n in range(N):
                prod *= cores[n][r[n - 1], i[n], r[n]]
            tot += prod
        X[i] = tot
    return X


@pytest.mark.parametrize("dims,ranks", [((2, 3, 2), (2, 3, 1)), ((2, 2, 3, 2), (2, 1, 3, 2)),
                                        ((3, 2), (2, 3))])
def test_tr_full_matches_termwise_sum(dims, ranks):
    cores = random_cores(dims, ranks, rng_for(11, 0))
    np.testing.assert_allclose(ring.tr_full(cores), brute_tr(cores), rtol=1e-12, atol=1e-12)


def test_worked_example_remark1():
    with open(os.path.join(GOLDEN, "remark1_worked_example.json")) as f:
        g = json.load(f)
    G = np.array(g["core_values_column_major"], dtype=np.float64).reshape(g["core_shape"], order="F")
    X = ring.tr_full([G, G, G, G])
    assert 4 * G.size == g["tr_parameters"]
    # TT ranks are the ranks of the sequential unfoldings (first k modes vs rest)
    tt = [np.linalg.matrix_rank(X.reshape(2 ** k, -1)) for k in (1, 2, 3)]
    assert tt == g["tt_ranks"]
    r = [1] + tt + [1]
    assert sum(r[k] * 2 * r[k + 1] for k in range(4)) == g["tt_parameters"]


def test_cyclic_shift_invariance():
    dims, ranks = (3, 4, 2, 3), (2, 3, 2, 1)
    cores = random_cores(dims, ranks, rng_for(12, 0))
    X = ring.tr_full(cores)
    N = len(cores)
    for s in range(1, N):
        Xs = ring.tr_full(cores[s:] + cores[:s])
        np.testing.assert_allclose(Xs, np.transpose(X, [(s + k) % N for k in range(N)]), rtol=1e-12,
                                   atol=1e-12)


def test_rank_one_ring_is_outer_product():
    dims = (3, 4, 5)
    cores = random_cores(dims, (1, 1, 1), rng_for(13, 0))
    v = [c[0, :, 0] for c in cores]
    np.testing.assert_allclose(ring.tr_full(cores), np.einsum("i,j,k->ijk", *v), rtol=1e-13)


def test_tensor_train_special_case():
    # R_0 = R_N = 1 (Section 2.1): the ring is a train; X(i) = g0(i0)^T G1(i1) g2(i2)
    rng = rng_for(14, 0)
    G0 = rng.standard_normal((1, 3, 2))
    G1 = rng.standard_normal((2, 4, 3))
    G2 = rng.standard_normal((3, 2, 1))
    X = ring.tr_full([G0, G1, G2])
    for i in itertools.product(range(3), range(4), range(2)):
        val = G0[0, i[0], :] @ G1[:, i[1], :] @ G2[:, i[2], 0]
        assert abs(X[i] - val) < 1e-12


def test_unfoldings_follow_definition2():
    rng = rng_for(15, 0)
    X = rng.standard_normal((2, 3, 4, 2))
    N = X.ndim
    for n in range(N):
        Xc = ring.unfold_classical(X, n)
        Xk = ring.unfold_cyclic(X, n)
        rest_c = [k for k in range(N) if k != n]
        rest_k = [(n + 1 + k) % N for k in range(N - 1)]
        for i in itertools.product(*[range(d) for d in X.shape]):
            col_c = ring.lin_index([i[k] for k in rest_c], [X.shape[k] for k in rest_c])
            col_k = ring.lin_index([i[k] for k in rest_k], [X.shape[k] for k in rest_k])
            assert Xc[i[n], col_c] == X[i]
            assert Xk[i[n], col_k] == X[i]


def test_subchain_follows_definition3():
    dims, ranks = (2, 3, 2, 2), (2, 1, 3, 2)
    cores = random_cores(dims, ranks, rng_for(16, 0))
    N = len(cores)
    for n in range(N):
        S = ring.subchain_tensor(cores, n)
        modes = [(n + 1 + k) % N for k in range(N - 1)]
        for i in itertools.product(*[range(dims[m]) for m in modes]):
            full_i = [None] * N
            for k, m in enumerate(modes):
                full_i[m] = i[k]
            col = ring.lin_index(i, [dims[m] for m in modes])
            for rn in range(ranks[n]):
                for rp in range(ranks[(n - 1) % N]):
                    # sum over all bonds except r_{n-1}, r_n
                    tot = 0.0
                    for r in itertools.product(*[range(R) for R in ranks]):
                        if r[n] != rn or r[(n - 1) % N] != rp:
                            continue
                        prod = 1.0
                        for j in range(N):
                            if j != n:
                                prod *= cores[j][r[j - 1], full_i[j], r[j]]
                        tot += prod
                    assert abs(S[rn, col, rp] - tot) < 1e-12


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_ls_reformulation_is_exact(n):
    # Section 2.1: TR(G) unfolded at mode n equals G^{!=n}_[2] G^(n)_(2)^T, transposed
    dims, ranks = (3, 2, 4, 3), (2, 3, 2, 2)
    cores = random_cores(dims, ranks, rng_for(17, n))
    X = ring.tr_full(cores)
    lhs = ring.subchain_unfolding(cores, n) @ ring.core_unfolding(cores[n]).T
    np.testing.assert_allclose(lhs, ring.unfold_cyclic(X, n).T, rtol=1e-12, atol=1e-12)
    # and the residual identity with a different tensor
    Y = rng_for(18, n).standard_normal(dims)
    a = np.linalg.norm((X - Y).ravel())
    b = np.linalg.norm(lhs - ring.unfold_cyclic(Y, n).T)
    assert abs(a - b) < 1e-12 * max(1.0, a)


def test_core_unfolding_roundtrip():
    G = rng_for(19, 0).standard_normal((3, 5, 2))
    Z2 = ring.core_unfolding(G)
    assert Z2.shape == (5, 6)
    assert Z2[4, 1 + 3 * 1] == G[1, 4, 1]
    np.testing.assert_array_equal(ring.core_from_unfolding(Z2, 3, 2), G)
