"""The paper's comparison protocol between exact and sampled TR-ALS (Section 4.1 and the
supplement's experiment details), run on the GPU.

1. Exact TR-ALS (Algorithm 1) from given initial cores, sweep by sweep, until the relative
   error changes by less than ``tol`` of its value between two sweeps (|e_k - e_{k-1}| < tol
   e_k), or ``max_sweeps`` sweeps have run.  The sweep count S and the final error E fix the
   reference.
2. Sampled TR-ALS (Algorithm 2) from the same initial cores for S sweeps, with J starting at
   ``J0`` and increased by ``step`` until its error is below ``factor`` * E.  A J whose sampled
   system turns out rank deficient (too few rows for the design's coherence) counts as not
   reaching the target.
3. Both are timed over their S sweeps (fit evaluations excluded); the speedup is the ratio.

Everything runs through the library's handles; the sampled runs reuse one handle (the sample
count, cores and update counter are reset between candidates).
"""
from __future__ import annotations

import time

from . import TRALS
from ._lib import TRALS_ESINGULAR, TralsError


def _timed_sweeps(h, sweeps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.sweep(sweeps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def exact_reference(X, ranks, init_cores, precision="f64", tol=1e-3, max_sweeps=100):
    """(sweeps S, error E, seconds of the S sweeps) of exact TR-ALS."""
    h = TRALS(X, ranks, 0, precision=precision, init_cores=init_cores, method="exact")
    prev = h.fit_error()
    secs = 0.0
    for s in range(1, max_sweeps + 1):
        secs += _timed_sweeps(h, 1)
        e = h.fit_error()
        if abs(prev - e) < tol * e:
            break
        prev = e
    h.close()
    return s, e, secs


def find_sample_size(X, ranks, init_cores, sweeps, target, J0, step, J_max, precision="f64", seed=0,
                     method="leverage"):
    """Smallest J = J0 + k * step (<= J_max) whose S-sweep error is below target.

    Returns (J, error, seconds of the S sweeps), or (None, best error, None) if no J up to
    J_max reaches the target."""
    h = TRALS(X, ranks, J_max, seed=seed, precision=precision, init_cores=init_cores, method=method)
    best = float("inf")
    J = J0
    try:
        while J <= J_max:
            h.update_counter = 0  # first: the tables of modes 1..N-1 are then rebuilt
            h.set_cores(init_cores)
            h.set_samples(J)
            try:
                secs = _timed_sweeps(h, sweeps)
            except TralsError as err:
                if err.code != TRALS_ESINGULAR:
                    raise
                J += step  # rank-deficient sample; set_cores clears the failed state
                continue
            e = h.fit_error()
            best = min(best, e)
            if e < target:
                return J, e, secs
            J += step
        return None, best, None
    finally:
        h.close()


def compare(X, ranks, init_cores, precision="f64", tol=1e-3, max_sweeps=100, factor=1.1, J0=None, step=100,
            J_max=None, seed=0, method="leverage"):
    """The full protocol; returns a dict of the reference, the J found and the speedup."""
    N = len(ranks)
    P = max(ranks[(n - 1) % N] * ranks[n] for n in range(N))
    J0 = 2 * P if J0 is None else J0
    J_max = 100 * P if J_max is None else J_max
    S, E, t_ex = exact_reference(X, ranks, init_cores, precision, tol, max_sweeps)
    J, e, t_s = find_sample_size(X, ranks, init_cores, S, factor * E, J0, step, J_max, precision, seed, method)
    return {
        "sweeps": S, "exact_error": E, "exact_s": t_ex,
        "samples": J, "sampled_error": e, "sampled_s": t_s,
        "speedup": (t_ex / t_s) if t_s else None, "factor": factor,
    }
