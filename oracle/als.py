"""Sampled and exact TR-ALS (oracle; test infrastructure).

Follows the paper's Algorithm 2 (TR-ALS-Sampled) step by step in FP64:

  init cores 1..N-1 (0-based; core 0 is overwritten by the first update)
  p^(m) for m = 1..N-1                                   (eq. (3))
  repeat for a fixed number of sweeps:
    for n = 0..N-1:
      draw the J index tuples                            (Algorithm 3)
      sketch the design matrix from the cores            (Algorithm 4)
      sketch the data: J sampled mode-n fibers of X      (Algorithm 2, "sample X")
      core n = argmin || G~ Z_(2)^T - X~ ||_F            (Algorithm 2, LS solve)
      recompute p^(n)                                    (Algorithm 2, last step)

The sampled least-squares problem is solved with ``numpy.linalg.lstsq``
(an orthogonal-factorisation solver, as the paper's QR-based solve,
Appendix B.1).  Rows of the sketched data are rescaled by the same factor
as the rows of the sketched design matrix (Definition 5 applies S = R Omega
to both sides).  No normalisation of cores is done (Section 2.1 says it may
be omitted).
"""
from __future__ import annotations

import numpy as np

from .leverage import core_table, uniform_table
from .ring import core_from_unfolding, cyclic_modes, subchain_unfolding, unfold_cyclic, tr_full
from .sampler import draw_update


class SingularSystem(ArithmeticError):
    """The sketched design matrix does not have full column rank."""


def sketch_subchain(cores, n, idx, w):
    """Algorithm 4: rows of S G^{!=n}_[2] built from lateral slices.

    Row j is the product G^(m_0)(:, i_{m_0}, :) ... G^(m_{N-2})(:, i_{m_{N-2}}, :)
    (an R_n x R_{n-1} matrix M_j, eq. (5)) in the column order of
    G^{!=n}_[2], i.e. column a + R_{n-1} b holds M_j(b, a), times w_j.
    """
    N = len(cores)
    modes = cyclic_modes(n, N)
    Rn = cores[n].shape[2]
    Rp = cores[n].shape[0]
    J = idx.shape[0]
    A = np.empty((J, Rp * Rn))
    for j in range(J):
        M = np.asarray(cores[modes[0]][:, idx[j, 0], :], dtype=np.float64)
        for k in range(1, N - 1):
            M = M @ np.asarray(cores[modes[k]][:, idx[j, k], :], dtype=np.float64)
        A[j] = w[j] * M.T.reshape(-1, order="F")
    return A


def sketch_fibers(X, n, idx, w):
    """Algorithm 2, "sample X": row j is w_j X(i_0, .., i_n = :, .., i_{N-1})."""
    N = X.ndim
    modes = cyclic_modes(n, N)
    pos = {m: k for k, m in enumerate(modes)}
    # mode-n axis moved last; the other axes keep their natural order
    Xn = np.moveaxis(np.asarray(X, dtype=np.float64), n, -1)
    sel = tuple(idx[:, pos[m]] for m in range(N) if m != n)
    Xs = Xn[sel]  # (J, I_n): the index arrays are adjacent and lead
    return w[:, None] * Xs


def solve_core(A, B, Rp, Rn):
    """Sampled LS solve (Algorithm 2): Z_(2)^T = argmin ||A Z_(2)^T - B||_F,
    returned as the core (Rp, I_n, Rn)."""
    P = A.shape[1]
    if np.linalg.matrix_rank(A) < P:
        raise SingularSystem("sketched design matrix is rank deficient")
    Zt, *_ = np.linalg.lstsq(A, B, rcond=None)
    return core_from_unfolding(Zt.T, Rp, Rn)


def normalize_core(cores, n):
    """Normalisation step after the update of core n (Section 2.1 allows such steps):
    G_n = Q R with Q from the (R_{n-1} I_n) x R_n unfolding (Householder QR, R's diagonal made
    positive), core n <- Q and core n+1 <- R G_{n+1} (product over its first index).  TR is
    unchanged, and so are the leverage scores of both cores.  Returns a new list."""
    N = len(cores)
    Rp, I, Rn = cores[n].shape
    Q, R = np.linalg.qr(np.asarray(cores[n], dtype=np.float64).reshape(Rp * I, Rn))
    d = np.abs(np.diag(R))
    if d.size and d.min() <= max(Q.shape) * np.finfo(np.float64).eps * d.max():
        raise SingularSystem("core is rank deficient along its bond to the next core")
    sgn = np.sign(np.diag(R))
    Q, R = Q * sgn, sgn[:, None] * R
    out = list(cores)
    out[n] = Q.reshape(Rp, I, Rn)
    nx = (n + 1) % N
    out[nx] = np.einsum("ab,bic->aic", R, np.asarray(cores[nx], dtype=np.float64))
    return out


def sampled_update(X, cores, tables, n, J, seed, stream_id, u):
    """One inner iteration of Algorithm 2 for core n (update number u).

    Returns (new core n, idx, w).  ``tables[m]`` is the integer table of
    p^(m) for every m != n.
    """
    idx, w = draw_update(tables, n, J, seed, stream_id, u)
    A = sketch_subchain(cores, n, idx, w)
    B = sketch_fibers(X, n, idx, w)
    Rp, _, Rn = cores[n].shape
    return solve_core(A, B, Rp, Rn), idx, w


def table_of(G, uniform=False):
    """Sampling table of core G: leverage scores (eq. (3)) or uniform."""
    return uniform_table(G.shape[1]) if uniform else core_table(G)


def lockstep_update(X, cores, n, J, seed, stream_id, u, uniform=False):
    """Sampled update of core n taking every table from ``cores`` afresh.

    Used to compare against a GPU run one update at a time: the GPU's cores
    before the update are passed in, so both sides draw from the same
    distributions.  Returns (new core n, idx, w).
    """
    N = len(cores)
    tables = [None] * N
    for m in range(N):
        if m != n:
            tables[m] = table_of(cores[m], uniform)
    return sampled_update(X, cores, tables, n, J, seed, stream_id, u)


def tr_als_sampled(X, init_cores, J, sweeps, seed=0, stream_id=0, record=None, u0=0, uniform=False,
                   normalize=False):
    """Algorithm 2 with a fixed number of sweeps (the paper's experiments fix
    the iteration count, Section 4.1).  ``record`` (a list) receives
    (u, n, idx, w) for every update.  ``J`` may be a function of the update
    number u (the sample size can change between updates, Section 3.2).
    ``uniform`` draws from uniform distributions instead of eq. (3);
    ``normalize`` applies ``normalize_core`` after every update.
    Returns the list of cores."""
    X = np.asarray(X, dtype=np.float64)
    N = X.ndim
    cores = [np.array(c, dtype=np.float64) for c in init_cores]
    tables = [None] * N
    for m in range(N):
        if m != (u0 % N):
            tables[m] = table_of(cores[m], uniform)
    for u in range(u0, u0 + sweeps * N):
        n = u % N
        Ju = J(u) if callable(J) else J
        cores[n], idx, w = sampled_update(X, cores, tables, n, Ju, seed, stream_id, u)
        if normalize:
            cores = normalize_core(cores, n)
        tables[n] = table_of(cores[n], uniform)
        if record is not None:
            record.append((u, n, idx, w))
    return cores


def exact_update(X, cores, n):
    """One inner iteration of Algorithm 1: core n refit against the full design
    matrix G^{!=n}_[2] and the full unfolding X_[n]^T."""
    A = subchain_unfolding(cores, n)
    B = unfold_cyclic(np.asarray(X, dtype=np.float64), n).T
    Rp, _, Rn = cores[n].shape
    return solve_core(A, B, Rp, Rn)


def tr_als_exact(X, init_cores, sweeps, normalize=False):
    """Algorithm 1 (TR-ALS) with a fixed number of sweeps.  For small tensors only."""
    X = np.asarray(X, dtype=np.float64)
    N = X.ndim
    cores = [np.array(c, dtype=np.float64) for c in init_cores]
    for _ in range(sweeps):
        for n in range(N):
            cores[n] = exact_update(X, cores, n)
            if normalize:
                cores = normalize_core(cores, n)
    return cores


def fit_error(cores, X):
    """Relative error ||TR(cores) - X||_F / ||X||_F (Section 3.1, Section 4.1)."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.linalg.norm((tr_full(cores) - X).ravel()) / np.linalg.norm(X.ravel()))
