"""Tensor-ring format, unfoldings and subchains (oracle; test infrastructure).

Index conventions (the paper's readings are listed with the design notes):

* Indices are 0-based.  A tensor is a C-order numpy array ``X[i_0..i_{N-1}]``.
* Core ``n`` has shape ``(R_{n-1}, I_n, R_n)`` with ``R_{-1} = R_{N-1}``
  (Section 2.1: ``R_0 = R_N`` in the paper's 1-based numbering).
* The paper's multi-index linearisation (Section 2, "Preliminaries") puts
  the *first* index fastest: ``lin(i_1..i_N) = sum_n i_n prod_{j<n} I_j``.
  With 0-based indices this is ``sum_k i_k prod_{l<k} I_l``; the printed
  formula mixes 1-based indices with a 0-based offset, so we take the 0-based
  reading.  This order only fixes the *row order* of the unfolded design
  matrix and of the data matrix, which the least-squares solution does not
  depend on.
"""
from __future__ import annotations

import numpy as np


def lin_index(idx, dims):
    """Paper's linear index of a multi-index, first index fastest (0-based)."""
    out = 0
    stride = 1
    for i, d in zip(idx, dims):
        out += int(i) * stride
        stride *= int(d)
    return out


def cyclic_modes(n, N):
    """Modes other than n in the cyclic order n+1, ..., N-1, 0, ..., n-1.

    This is the order of the indices in the mode-n unfolding (Definition 2),
    in the subchain (Definition 3) and in the sampler (Algorithm 3).
    """
    return [(n + 1 + k) % N for k in range(N - 1)]


def tr_full(cores):
    """Dense tensor of a tensor ring: X(i) = trace(prod_n G^(n)(:, i_n, :)).

    Eq. (1): X(i_1..i_N) = sum_{r_1..r_N} prod_n G^(n)(r_{n-1}, i_n, r_n) with
    r_0 = r_N, i.e. the trace of the product of the lateral slices.  Computed
    by multiplying the slices left to right for all index tuples at once and
    taking the trace at the end.
    """
    N = len(cores)
    cores = [np.asarray(c, dtype=np.float64) for c in cores]
    # P[a, i_0, ..., i_k, b] = (G^(0)(:, i_0, :) ... G^(k)(:, i_k, :))[a, b]
    P = cores[0]
    for k in range(1, N):
        P = np.tensordot(P, cores[k], axes=([P.ndim - 1], [0]))
    # close the ring: trace over the first and the last bond index
    return np.trace(P, axis1=0, axis2=P.ndim - 1)


def unfold_classical(X, n):
    """Classical mode-n unfolding X_(n) (Definition 2): rows i_n, columns
    lin(i_0..i_{n-1} i_{n+1}..i_{N-1}) with the first index fastest."""
    N = X.ndim
    order = [n] + [k for k in range(N) if k != n]
    return np.transpose(X, order).reshape(X.shape[n], -1, order="F")


def unfold_cyclic(X, n):
    """Mode-n unfolding X_[n] (Definition 2): rows i_n, columns
    lin(i_{n+1}..i_{N-1} i_0..i_{n-1}) with the first index fastest."""
    N = X.ndim
    order = [n] + cyclic_modes(n, N)
    return np.transpose(X, order).reshape(X.shape[n], -1, order="F")


def core_unfolding(G):
    """G_(2) of a core (R_{n-1} x I_n x R_n): classical mode-2 unfolding,
    rows i_n, column a + R_{n-1} * b holds G(a, i_n, b)."""
    return unfold_classical(np.asarray(G), 1)


def subchain_tensor(cores, n):
    """Subchain tensor G^{!=n} (Definition 3), shape R_n x prod_{j!=n} I_j x R_{n-1}.

    Element (r_n, lin(i_{n+1}..i_{n-1}), r_{n-1}) is the sum over the inner
    bond indices of the product of the cores other than n, taken in the
    cyclic order n+1, ..., N-1, 0, ..., n-1.
    """
    N = len(cores)
    modes = cyclic_modes(n, N)
    S = np.asarray(cores[modes[0]], dtype=np.float64)  # (R_n, I_{m0}, R_{m0})
    for m in modes[1:]:
        S = np.tensordot(S, np.asarray(cores[m], dtype=np.float64), axes=([S.ndim - 1], [0]))
    # S: (R_n, I_{m0}, ..., I_{m_{N-2}}, R_{n-1}); merge the middle, first fastest
    Rn, Rp = S.shape[0], S.shape[-1]
    mid = S.shape[1:-1]
    K = int(np.prod(mid))
    out = np.empty((Rn, K, Rp))
    for b in range(Rn):
        for a in range(Rp):
            out[b, :, a] = S[(b, Ellipsis, a)].reshape(-1, order="F")
    return out


def subchain_unfolding(cores, n):
    """G^{!=n}_[2]: mode-2 unfolding of the subchain (Definition 2 applied to
    the 3-way subchain), rows lin(i_{n+1}..i_{n-1}), column a + R_{n-1} * b
    holds G^{!=n}(b, row, a).  This is the design matrix of the ALS update
    of core n (Section 2.1)."""
    return unfold_cyclic(subchain_tensor(cores, n), 1)


def core_from_unfolding(Z2, Rp, Rn):
    """Inverse of ``core_unfolding``: Z_(2) (I x Rp*Rn) -> core (Rp, I, Rn)."""
    I = Z2.shape[0]
    return np.transpose(np.asarray(Z2).reshape(I, Rp, Rn, order="F"), (1, 0, 2))
