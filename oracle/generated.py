"""Dense reference of a generated data source (oracle; test infrastructure only).

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's CPU baseline use
this module.  A generated source describes the data tensor as

    X = TR(G*) + sigma * Z,

a tensor ring of given "true" cores G* (eq. (1)) plus iid standard normal noise,
with sigma = noise_rel * ||TR(G*)||_F / sqrt(prod_n I_n).  Noise entry Z[e] at the
C-order linear index e is the Box-Muller transform of the first two 64-bit words
(w0, w1) of the Philox4x64-10 block with key (noise_seed, noise_stream) and
counter (e, 2^64 - 1, 2^64 - 1, 0):

    u1 = (floor(w0 / 2^11) + 1) * 2^-53,   u2 = floor(w1 / 2^11) * 2^-53,
    Z[e] = sqrt(-2 ln u1) * cos(2 pi u2).

Here the whole tensor is formed densely (small tensors only) from those
definitions, so that the oracle's ALS can run on it and be compared with a
GPU handle that generates only the sampled fibers.
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x64_10_np
from .ring import tr_full

ALL_ONES = np.uint64(0xFFFFFFFFFFFFFFFF)


def philox_normals(count: int, key0: int, key1: int) -> np.ndarray:
    """Z[e] for e = 0 .. count-1 (FP64)."""
    e = np.arange(count, dtype=np.uint64)
    w = philox4x64_10_np(e, ALL_ONES, ALL_ONES, np.uint64(0), np.uint64(key0), np.uint64(key1))
    u1 = ((w[0] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (w[1] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def dense_generated(true_cores, noise_rel: float, noise_seed: int, noise_stream: int):
    """(X, sigma): the dense FP64 tensor of a generated source."""
    clean = tr_full([np.asarray(c, dtype=np.float64) for c in true_cores])
    sigma = noise_rel * np.linalg.norm(clean) / np.sqrt(clean.size)
    Z = philox_normals(clean.size, noise_seed, noise_stream).reshape(clean.shape)
    return clean + sigma * Z, sigma


def clean_fit(cores, true_cores) -> float:
    """||TR(G) - TR(G*)||_F / ||TR(G*)||_F by dense contraction (small tensors)."""
    a = tr_full([np.asarray(c, dtype=np.float64) for c in cores])
    b = tr_full([np.asarray(c, dtype=np.float64) for c in true_cores])
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
