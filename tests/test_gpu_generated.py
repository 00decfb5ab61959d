"""GPU parity of the generated data source (X = TR(G*) + sigma Z, fibers made per update)
against the oracle run on the dense tensor built from the same definition."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import als as oals  # noqa: E402
from oracle.generated import clean_fit, dense_generated  # noqa: E402
from synth import random_cores, rng_for  # noqa: E402
from tests.gpu_helpers import assert_core_close, lockstep, rel, say, to_np  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_08581_amd import _lib
    _lib.load()


def gen_handle(true, ranks, J, noise, key, precision, init):
    from paper_2010_08581_amd import TRALS
    return TRALS.generated(true, ranks, J, noise_rel=noise, noise_seed=key[0], noise_stream=key[1],
                           precision=precision, init_cores=init)


def test_generated_fp64_free_running_matches_dense_oracle():
    say("case: generated 3-way 18x20x22 true ranks (2,3,2), fit ranks (2,3,2), fp64, 4 sweeps")
    dims, ranks = (18, 20, 22), (2, 3, 2)
    true = random_cores(dims, ranks, rng_for(21, 1))
    init = random_cores(dims, ranks, rng_for(21, 3))
    X, _ = dense_generated(true, 0.01, 5, 9)
    rec = []
    ref = oals.tr_als_sampled(X, init, 300, 4, seed=0, record=rec)
    t = gen_handle(true, ranks, 300, 0.01, (5, 9), "f64", init)
    for u, n, idx_o, w_o in rec:
        t.step(1)
        idx_g, w_g = t.last_samples()
        assert np.array_equal(idx_g, idx_o), f"update {u}: indices differ"
        np.testing.assert_allclose(w_g, w_o, rtol=1e-10)
    got = to_np(t.get_cores())
    for n in range(3):
        assert_core_close(got[n], ref[n], 1e-9, f"core {n}")
    fg = t.fit_error()
    fo = clean_fit(got, true)
    say(f"clean fit gpu={fg:.9e} oracle={fo:.9e}")
    assert abs(fg - fo) <= 1e-9 * max(fo, 1e-12)


def test_generated_fp32_lockstep_4way_rank_mismatch():
    say("case: generated 4-way 14x16x15x13 true ranks (3,2,4,3), fit ranks (2,2,3,2), fp32 lockstep")
    dims = (14, 16, 15, 13)
    true = random_cores(dims, (3, 2, 4, 3), rng_for(22, 1))
    ranks = (2, 2, 3, 2)
    init = random_cores(dims, ranks, rng_for(22, 3))
    X, _ = dense_generated(true, 0.02, 7, 1)
    t = gen_handle(true, ranks, 400, 0.02, (7, 1), "f32", init)
    worst = lockstep(t, X, 8, 400)
    say(f"worst core rel diff {worst:.3e}")
    fg = t.fit_error()
    fo = clean_fit(to_np(t.get_cores()), true)
    assert abs(fg - fo) <= 1e-9 * fo


def test_generated_5way_serving_shape_converges():
    say("case: generated 5-way 40x52x36x48x44 ranks (3,4,5,3,4), fp32, J=2048, 5 sweeps")
    dims, ranks = (40, 52, 36, 48, 44), (3, 4, 5, 3, 4)
    true = random_cores(dims, ranks, rng_for(23, 1))
    init = random_cores(dims, ranks, rng_for(23, 3))
    t = gen_handle(true, ranks, 2048, 0.01, (1, 23), "f32", init)
    f0 = t.fit_error()
    t.sweep(5)
    f5 = t.fit_error()
    say(f"clean fit {f0:.4e} -> {f5:.4e}")
    assert np.isfinite(f5) and f5 < 0.2 * f0


@pytest.mark.parametrize("dims,ranks,prec,J", [
    ((26, 30, 28), (12, 11, 12), "f64", 1200),   # P = 144, 132, 132: the generated fibers' three
    ((26, 30, 28), (12, 11, 12), "f32", 1200),   # 48-wide k-rounds; FP32 takes the three-slice path
    ((9, 8, 10, 7, 8), (12, 5, 12, 4, 12), "f32", 1500),  # order 5, P up to 144
])
def test_generated_serving_ranks_lockstep(dims, ranks, prec, J):
    # serving ranks reach 12 (P = R_{n-1} R_n up to 144): the generated fibers and the rest of
    # the update against the oracle on the dense tensor of the same definition
    say(f"case: generated {dims} ranks {ranks} {prec} J={J} lockstep")
    true = random_cores(dims, ranks, rng_for(24, 1))
    init = random_cores(dims, ranks, rng_for(24, 3))
    X, _ = dense_generated(true, 0.01, 3, 17)
    t = gen_handle(true, ranks, J, 0.01, (3, 17), prec, init)
    worst = lockstep(t, X, 2 * len(dims), J, core_tol=1e-9 if prec == "f64" else 1e-4)
    say(f"worst slice {worst:.3e}")
    fg = t.fit_error()
    fo = clean_fit(to_np(t.get_cores()), true)
    assert abs(fg - fo) <= 1e-9 * fo
