"""Drawing the sample index tuples of one ALS update (oracle; test infrastructure).

Algorithm 3: a draw from q^{!=n} (eq. (4)) is a tuple of independent draws
i_j ~ p^(j), one per mode j != n; the sampling matrix of Definition 5 is never
formed, only the index tuples are kept (Section 3).  Draws are with
replacement and duplicates are kept (Definition 5: J independent draws).

Randomness (a reading; the paper names no generator): the k-th mode draw of
sample j in update number u (u = sweep * N + n counts updates from the first
one) uses word (k mod 4) of the Philox4x64-10 block with

    key     = (seed, stream_id)
    counter = (j, k // 4, u, 0).

From a 64-bit word r and the integer table (C, T) of mode m = (n+1+k) mod N,
the draw is t = floor(r * T / 2^64) (exact 128-bit product) and
i = min{ i : t < C_i }.  The rescaling of Definition 5 uses the exact
sampling probability of the tuple, q = prod_k Q_{i_k} / T_k, evaluated in
FP64 in the order k = 0, 1, ..., N-2, and w = 1 / sqrt(J * q).
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x64_10_np, mulhilo64_np
from .ring import cyclic_modes


def philox_words(J, n_words, seed, stream_id, u):
    """uint64 array (J, n_words): word k of sample j (counter (j, k//4, u, 0))."""
    j = np.arange(J, dtype=np.uint64)
    out = np.empty((J, n_words), dtype=np.uint64)
    for blk in range((n_words + 3) // 4):
        x = philox4x64_10_np(j, np.uint64(blk), np.uint64(u), np.uint64(0), seed, stream_id)
        for w in range(4):
            k = 4 * blk + w
            if k < n_words:
                out[:, k] = x[w]
    return out


def draw_index(C, T, r):
    """i = min{i : t < C_i} with t = floor(r * T / 2^64) (uint64 arrays)."""
    t, _ = mulhilo64_np(r, np.uint64(T))
    return np.searchsorted(C, t, side="right")


def draw_update(tables, n, J, seed, stream_id, u):
    """Sample tuples for the update of core n.

    tables[m] = (Q, C, T) for every mode m != n.  Returns
    idx (J, N-1) int64 with idx[:, k] the index drawn in mode (n+1+k) mod N,
    and w (J,) float64, the Definition 5 rescaling 1/sqrt(J q).
    """
    N = len(tables)
    modes = cyclic_modes(n, N)
    r = philox_words(J, N - 1, seed, stream_id, u)
    idx = np.empty((J, N - 1), dtype=np.int64)
    q = np.ones(J)
    for k, m in enumerate(modes):
        Q, C, T = tables[m]
        idx[:, k] = draw_index(C, T, r[:, k])
        q = q * (Q[idx[:, k]].astype(np.float64) / float(T))
    w = 1.0 / np.sqrt(float(J) * q)
    return idx, w
