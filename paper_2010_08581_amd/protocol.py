"""The paper's comparison protocol between exact and sampled TR-ALS (Section 4.1 and the
supplement's experiment details), run on the GPU.

1. Exact TR-ALS (Algorithm 1) from given initial cores, sweep by sweep, until the relative
   error changes by less than ``tol`` of its value between two sweeps (|e_k - e_{k-1}| < tol
   e_k), or ``max_sweeps`` sweeps have run: S sweeps.
2. Every method then runs again from the same initial cores for 2 S sweeps without checking
   convergence.  E is the error of exact TR-ALS after its 2 S sweeps.
3. TR-ALS-Sampled (Algorithm 2): the sample size J starts at J0 (2 R^2 in the paper) and grows
   by ``step`` until the error after 2 S sweeps is below ``factor`` * E; the first such J is
   reported with its error and time.  J_max bounds the walk.  A J whose sampled system turns
   out rank deficient counts as not reaching the target.
4. The speedup is the ratio of the two 2 S-sweep times (fit evaluations excluded).

``search="bisect"`` replaces the walk by doubling and bisection on the same grid (far fewer
runs, but it assumes the error falls with J, which the sampled error after a fixed number of
sweeps need not do); it is not the paper's rule.

Everything runs through the library's handles; the sampled runs reuse one handle (the sample
count, cores and update counter are reset between candidates).  ``normalize`` applies the
optional normalisation step to both methods.
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


def exact_reference(X, ranks, init_cores, precision="f64", tol=1e-3, max_sweeps=100, normalize=False):
    """Sweeps S of the convergence run of exact TR-ALS, then its rerun for 2 S sweeps from the
    same cores: (S, error E after the 2 S sweeps, seconds of the 2 S sweeps)."""
    h = TRALS(X, ranks, 0, precision=precision, init_cores=init_cores, method="exact", normalize=normalize)
    prev = h.fit_error()
    for s in range(1, max_sweeps + 1):
        h.sweep(1)
        e = h.fit_error()
        if abs(prev - e) < tol * e:
            break
        prev = e
    h.update_counter = 0
    h.set_cores(init_cores)
    secs = _timed_sweeps(h, 2 * s)
    E = h.fit_error()
    h.close()
    return s, E, secs


def find_sample_size(X, ranks, init_cores, sweeps, target, J0, step, J_max, precision="f64", seed=0,
                     method="leverage", normalize=False, search="walk"):
    """First J = J0 + k * step (<= J_max) whose error after ``sweeps`` sweeps is below target:
    walking the grid upwards (search="walk", the paper's rule), or by doubling then bisection
    (search="bisect", equal to the walk when the error falls with J).

    Returns (J, error, seconds of the sweeps, runs), or (None, best error, None, runs) if no
    J up to J_max reaches the target."""
    if search not in ("walk", "bisect"):
        raise ValueError("search: 'walk' or 'bisect'")
    h = TRALS(X, ranks, J_max, seed=seed, precision=precision, init_cores=init_cores, method=method,
              normalize=normalize)
    tried = {}

    def run(J):
        if J not in tried:
            h.update_counter = 0  # first: the tables of modes 1..N-1 are then rebuilt
            h.set_cores(init_cores)
            h.set_samples(J)
            try:
                secs = _timed_sweeps(h, sweeps)
                tried[J] = (h.fit_error(), secs)
            except TralsError as err:
                if err.code != TRALS_ESINGULAR:
                    raise
                tried[J] = (float("inf"), None)  # rank-deficient sample; set_cores clears the state
        return tried[J]

    try:
        k_max = (J_max - J0) // step
        if search == "walk":
            for k in range(k_max + 1):
                J = J0 + k * step
                e, secs = run(J)
                if e < target:
                    return J, e, secs, len(tried)
            best = min(e for e, _ in tried.values())
            return None, best, None, len(tried)
        k_lo, k = -1, 0  # grid index k <-> J0 + k * step; k_lo: largest index known to fail
        while True:
            if run(J0 + k * step)[0] < target:
                break
            k_lo = k
            if k == k_max:
                best = min(e for e, _ in tried.values())
                return None, best, None, len(tried)
            k = min(2 * k + 1, k_max)
        k_hi = k
        while k_hi - k_lo > 1:
            mid = (k_lo + k_hi) // 2
            if run(J0 + mid * step)[0] < target:
                k_hi = mid
            else:
                k_lo = mid
        J = J0 + k_hi * step
        e, secs = tried[J]
        return J, e, secs, len(tried)
    finally:
        h.close()


def compare(X, ranks, init_cores, precision="f64", tol=1e-3, max_sweeps=100, factor=1.1, J0=None, step=100,
            J_max=None, seed=0, method="leverage", normalize=False, search="walk"):
    """The full protocol; returns a dict of the reference, the J found and the speedup."""
    N = len(ranks)
    P = max(ranks[(n - 1) % N] * ranks[n] for n in range(N))
    J0 = 2 * P if J0 is None else J0
    J_max = 100 * P if J_max is None else J_max
    S, E, t_ex = exact_reference(X, ranks, init_cores, precision, tol, max_sweeps, normalize)
    J, e, t_s, runs = find_sample_size(X, ranks, init_cores, 2 * S, factor * E, J0, step, J_max, precision, seed,
                                       method, normalize, search)
    return {
        "convergence_sweeps": S, "sweeps": 2 * S, "exact_error": E, "exact_s": t_ex,
        "samples": J, "sampled_error": e, "sampled_s": t_s,
        "speedup": (t_ex / t_s) if t_s else None, "factor": factor, "J0": J0, "step": step, "J_max": J_max,
        "search": search, "runs": runs, "normalize": bool(normalize),
        "outcome": (f"J = {J}: error {e:.4g} < {factor} x {E:.4g} after {2 * S} sweeps" if J is not None else
                    f"no J in [{J0}, {J_max}] (step {step}) reaches {factor} x the exact error {E:.4g} after "
                    f"{2 * S} sweeps (best {e:.4g})"),
    }
