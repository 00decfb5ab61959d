"""Shared helpers of the GPU tests: run the library and the oracle side by side."""
import sys

import numpy as np

from oracle import als as oals


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    """Frobenius-norm ratio ||a - b|| / ||b|| (reported beside the element-wise check)."""
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def slice_diff(got, want):
    """Worst lateral slice of a core (R_{n-1}, I_n, R_n): the largest over i of
    max|got[:, i, :] - want[:, i, :]| / max|want[:, i, :]|, and that slice's index.  Every
    entry of a slice is held to a fraction of the slice's own largest entry, so one wrong slice
    cannot hide in the norm of the whole core."""
    g = np.asarray(got, dtype=np.float64)
    o = np.asarray(want, dtype=np.float64)
    if g.shape != o.shape:
        raise AssertionError(f"core shapes differ: {g.shape} vs {o.shape}")
    d = np.abs(g - o).max(axis=(0, 2))
    s = np.abs(o).max(axis=(0, 2))
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(s > 0, d / np.where(s > 0, s, 1.0), np.where(d > 0, np.inf, 0.0))
    i = int(np.argmax(ratio))
    return float(ratio[i]), i


def assert_core_close(got, want, tol, what="core"):
    """Element-wise core parity: every lateral slice within tol of its own largest entry."""
    worst, i = slice_diff(got, want)
    assert worst <= tol, (f"{what}: lateral slice {i} differs by {worst:.3e} of its largest entry "
                          f"(bar {tol:.1e}; Frobenius ratio of the core {rel(got, want):.3e})")
    return worst


def to_np(cores):
    return [c.detach().cpu().numpy().astype(np.float64) for c in cores]


def lockstep(t, X64, n_updates, J, seed=0, stream_id=0, core_tol=1e-4, start=0, w_rtol=1e-6):
    """Compare n_updates single updates of handle t with the oracle, each from
    the GPU's cores before the update: sampled indices bit for bit, weights to w_rtol,
    the new core slice by slice to core_tol.  Returns the worst slice difference."""
    N = X64.ndim
    worst = 0.0
    for k in range(n_updates):
        u = start + k
        n = u % N
        before = to_np(t.get_cores())
        t.step(1)
        idx_g, w_g = t.last_samples()
        core_o, idx_o, w_o = oals.lockstep_update(X64, before, n, J, seed, stream_id, u)
        assert np.array_equal(idx_g, idx_o), f"update {u}: sampled indices differ " \
                                             f"({int(np.sum(idx_g != idx_o))} entries)"
        # w_j = 1/sqrt(J q_j): the GPU takes leverage from the inverse Gram of each core (or a
        # pivoted QR), the oracle from its SVD; they agree to ~cond(G_(2))^2 eps at worst
        np.testing.assert_allclose(w_g, w_o, rtol=w_rtol)
        core_g = to_np(t.get_cores())[n]
        r = assert_core_close(core_g, core_o, core_tol, f"update {u} (core {n})")
        say(f"  update {u} core {n}: worst slice {r:.3e}, Frobenius ratio {rel(core_g, core_o):.3e}")
        worst = max(worst, r)
    return worst
