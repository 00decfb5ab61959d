"""Pins of the oracle's dense reference of a generated data source (oracle/generated.py)."""
import math

import numpy as np
from scipy import stats

from oracle.generated import clean_fit, dense_generated, philox_normals
from oracle.philox import philox4x64_10
from oracle.ring import tr_full
from synth import random_cores, rng_for


def test_normals_match_scalar_philox_and_box_muller():
    # vectorised generator vs the scalar Philox block and the textbook transform (math module)
    z = philox_normals(40, 11, 7)
    for e in (0, 1, 17, 39):
        w = philox4x64_10([e, 2 ** 64 - 1, 2 ** 64 - 1, 0], [11, 7])
        u1 = ((w[0] >> 11) + 1) * 2.0 ** -53
        u2 = (w[1] >> 11) * 2.0 ** -53
        assert z[e] == math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def test_normals_are_standard_normal():
    z = philox_normals(200_000, 3, 1)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    # different keys give independent streams
    z2 = philox_normals(200_000, 3, 2)
    assert abs(np.corrcoef(z, z2)[0, 1]) < 0.01


def test_dense_generated_noise_level_and_zero_noise():
    dims, ranks = (9, 10, 11), (3, 2, 4)
    G = random_cores(dims, ranks, rng_for(5, 1))
    X0, s0 = dense_generated(G, 0.0, 1, 0)
    assert s0 == 0.0 and np.array_equal(X0, tr_full(G))
    X, s = dense_generated(G, 0.05, 1, 0)
    clean = tr_full(G)
    assert np.isclose(s, 0.05 * np.linalg.norm(clean) / np.sqrt(clean.size))
    # the realised noise is within a few percent of the requested level
    assert abs(np.linalg.norm(X - clean) / np.linalg.norm(clean) / 0.05 - 1.0) < 0.1


def test_clean_fit_reference_values():
    dims, ranks = (6, 7, 5, 4), (2, 3, 2, 2)
    G = random_cores(dims, ranks, rng_for(6, 1))
    assert clean_fit(G, G) == 0.0
    # scaling one core scales the ring (eq. (1) is multilinear in the cores)
    G2 = [2.0 * G[0]] + G[1:]
    assert np.isclose(clean_fit(G2, G), 1.0)
    Gneg = [-G[0]] + G[1:]
    assert np.isclose(clean_fit(Gneg, G), 2.0)
