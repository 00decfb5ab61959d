"""Sampled estimate of the relative fit error (oracle; test infrastructure).

Section 3.1 (Termination Criteria): computing ||TR(G) - X||_F exactly costs a pass over every
entry of X, which defeats the sublinear cost of the method; instead the relative error can be
estimated from sampled entries (the approach of Battaglino et al. for CP).  Here S entries are
drawn uniformly with replacement from the E = prod_n I_n entries, and

    est^2 = (E / S) sum_s (TR(G)(i_s) - X(i_s))^2 / ||X||_F^2

so that E/S times the sum is an unbiased estimate of ||TR(G) - X||_F^2; est is its square
root over ||X||_F.  TR(G)(i) is the trace of the product of the lateral slices G^(n)(:, i_n, :)
(eq. (1)).

Draws (a reading; the paper names no generator or sampling scheme): entry s takes word 0 of
the Philox4x64-10 block with key (seed, stream_id) and counter (s, tag, 0, 1), and its C-order
linear index is t = floor(r E / 2^64) (the high word of the 128-bit product), uniform over
[0, E) up to a relative bias below E / 2^64.  The fourth counter word 1 keeps these blocks
apart from the sample draws of Algorithm 3 (counter (j, k/4, u, 0)).
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x64_10_np, mulhilo64_np


def estimate_indices(dims, S, seed, stream_id, tag=0):
    """(S, N) int64 multi-indices of the sampled entries, C order."""
    E = int(np.prod([int(d) for d in dims]))
    s = np.arange(int(S), dtype=np.uint64)
    r = philox4x64_10_np(s, np.uint64(tag), np.uint64(0), np.uint64(1), seed, stream_id)[0]
    t, _ = mulhilo64_np(r, np.uint64(E))
    return np.stack(np.unravel_index(t.astype(np.int64), tuple(int(d) for d in dims)), axis=1)


def tr_entries(cores, idx):
    """TR(G) at the multi-indices idx (S x N): trace of the product of lateral slices (eq. (1))."""
    idx = np.asarray(idx)
    M = np.transpose(np.asarray(cores[0], dtype=np.float64)[:, idx[:, 0], :], (1, 0, 2))
    for n in range(1, len(cores)):
        M = M @ np.transpose(np.asarray(cores[n], dtype=np.float64)[:, idx[:, n], :], (1, 0, 2))
    return np.einsum("sii->s", M)


def sampled_fit_estimate(cores, X, S, seed=0, stream_id=0, tag=0):
    """The sampled relative-error estimate est of Section 3.1 (see above)."""
    X = np.asarray(X, dtype=np.float64)
    idx = estimate_indices(X.shape, S, seed, stream_id, tag)
    d = tr_entries(cores, idx) - X[tuple(idx.T)]
    est2 = (X.size / float(S)) * float(np.sum(d * d)) / float(np.sum(X * X))
    return float(np.sqrt(est2))
