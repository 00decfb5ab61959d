"""FP64 CPU oracle for leverage-score-sampled tensor-ring ALS.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
numpy implementation of what the GPU path computes, written from Malik &
Becker, "A Sampling-Based Method for Tensor Ring Decomposition" (ICML 2021):

* ``ring``     -- TR format (eq. (1)), unfoldings (Definition 2), subchain
                  tensor (Definition 3) and the least-squares reformulation
                  (Section 2.1).
* ``leverage`` -- leverage scores (Definition 4), per-core distributions
                  p^(n) (eq. (3)) and their integer cumulative tables.
* ``philox``   -- Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11), the
                  counter-based generator both sides implement.
* ``sampler``  -- Algorithm 3: independent draws i_j ~ p^(j) per mode j != n.
* ``als``      -- Algorithm 4 (sketched subchain), line "sample X" of
                  Algorithm 2, the sampled LS solve, Algorithm 2 itself,
                  Algorithm 1 (exact TR-ALS) and the relative fit error.
* ``estimate`` -- the relative error estimated from sampled entries
                  (Section 3.1, Termination Criteria).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and never imports it; the product path never calls into it.
"""
from . import ring, leverage, philox, sampler, als, estimate  # noqa: F401
from .ring import tr_full, unfold_classical, unfold_cyclic, core_unfolding, subchain_tensor, \
    subchain_unfolding, lin_index  # noqa: F401
from .leverage import leverage_scores, mode_distribution, integer_table  # noqa: F401
from .philox import philox4x64_10, philox4x64_10_np  # noqa: F401
from .sampler import draw_update  # noqa: F401
from .als import sketch_subchain, sketch_fibers, solve_core, sampled_update, tr_als_sampled, \
    tr_als_exact, fit_error, SingularSystem  # noqa: F401
