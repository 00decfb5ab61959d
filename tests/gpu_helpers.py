"""Shared helpers of the GPU tests: run the library and the oracle side by side."""
import sys

import numpy as np

from oracle import als as oals


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def to_np(cores):
    return [c.detach().cpu().numpy().astype(np.float64) for c in cores]


def lockstep(t, X64, n_updates, J, seed=0, stream_id=0, core_tol=1e-4, start=0):
    """Compare n_updates single updates of handle t with the oracle, each from
    the GPU's cores before the update.  Returns the worst core difference."""
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
        # w_j = 1/sqrt(J q_j): the GPU takes leverage from the inverse Gram of each core, the
        # oracle from its SVD; they agree to ~cond(G_(2))^2 eps (1e-8 for the worst cores here)
        np.testing.assert_allclose(w_g, w_o, rtol=1e-6)
        core_g = to_np(t.get_cores())[n]
        r = rel(core_g, core_o)
        worst = max(worst, r)
        assert r <= core_tol, f"update {u} (core {n}): rel diff {r:.3e} > {core_tol:.1e}"
    return worst
