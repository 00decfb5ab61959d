"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar: sampled indices bit-exact; FP64 cores within 1e-9 relative (free-running),
FP32 cores within 1e-4 relative per update (lockstep: before every update the
oracle starts from the GPU's current cores, so both sides draw from the same
tables).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import als as oals  # noqa: E402
from synth import make_config, random_cores, ring_tensor, rng_for, video_tensor  # noqa: E402
from tests.gpu_helpers import assert_core_close, lockstep, rel, say, to_np  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_08581_amd import _lib
    _lib.load()


def TR(*a, **k):
    from paper_2010_08581_amd import TRALS
    return TRALS(*a, **k)


def test_c1_free_running_fp64_full_config():
    say("case: c1 60^3 R=3 J=2000 fp64, 10 sweeps free-running")
    X, _, init = make_config("c1", dtype=np.float64)
    rec = []
    ref = oals.tr_als_sampled(X, init, 2000, 10, seed=0, record=rec)
    t = TR(torch.tensor(X, device="cuda"), (3, 3, 3), 2000, seed=0, precision="f64", init_cores=init)
    for u, n, idx_o, w_o in rec:
        t.step(1)
        idx_g, w_g = t.last_samples()
        assert np.array_equal(idx_g, idx_o), f"update {u}: indices differ"
        np.testing.assert_allclose(w_g, w_o, rtol=1e-10)
    got = to_np(t.get_cores())
    for n in range(3):
        assert_core_close(got[n], ref[n], 1e-9, f"core {n}")
    fg = t.fit_error()
    fo = oals.fit_error(ref, X)
    say(f"c1 fit gpu={fg:.9e} oracle={fo:.9e}")
    assert abs(fg - fo) <= 1e-9 * fo


def test_fp32_lockstep_3way_ragged():
    say("case: fp32 120x136x150 R=10 J=1000 lockstep 6 updates")
    X, _, init = make_config("c2", dims=(120, 136, 150), dtype=np.float32)
    t = TR(torch.tensor(X, device="cuda"), (10, 10, 10), 1000, precision="f32", init_cores=init)
    worst = lockstep(t, X.astype(np.float64), 6, 1000)
    say(f"worst core rel diff {worst:.3e}")


def test_fp32_lockstep_5way():
    say("case: fp32 5-way 21x22x20x23x19 R=5 J=4096 lockstep 5 updates")
    X, _, init = make_config("c3", dims=(21, 22, 20, 23, 19), dtype=np.float32)
    t = TR(torch.tensor(X, device="cuda"), (5,) * 5, 4096, precision="f32", init_cores=init)
    worst = lockstep(t, X.astype(np.float64), 5, 4096)
    say(f"worst core rel diff {worst:.3e}")


def test_fp32_lockstep_video_shape_small():
    say("case: fp32 video 24x32x3x200 R=4 J=700 lockstep 8 updates")
    X = video_tensor(24, 32, 3, 200, K=4, seed=0)
    init = random_cores(X.shape, (4, 4, 4, 4), rng_for(0, 3))
    t = TR(torch.tensor(X, device="cuda"), (4, 4, 4, 4), 700, precision="f32", init_cores=init)
    worst = lockstep(t, X.astype(np.float64), 8, 700)
    say(f"worst core rel diff {worst:.3e}")


def test_order2_rank1_fp64():
    say("case: fp64 order 2, ranks (1,3), J=40")
    rng = rng_for(61, 0)
    X = rng.standard_normal((50, 70))
    init = random_cores(X.shape, (1, 3), rng_for(61, 3))
    t = TR(torch.tensor(X, device="cuda"), (1, 3), 40, precision="f64", init_cores=init)
    lockstep(t, X, 4, 40, core_tol=1e-10)


def test_wide_and_square_cores_fp64():
    # I_n < P_n and I_n == P_n take the uniform table, I_n > P_n the Cholesky path
    say("case: fp64 8x9x10 R=3 J=64")
    X = rng_for(62, 0).standard_normal((8, 9, 10))
    init = random_cores(X.shape, (3, 3, 3), rng_for(62, 3))
    t = TR(torch.tensor(X, device="cuda"), (3, 3, 3), 64, precision="f64", init_cores=init)
    lockstep(t, X, 6, 64, core_tol=1e-10)


def test_large_scale_cores_ragged_P_fp64():
    # Gram and core-Gram diagonals far above 1 / (P eps) with P = 15, 27, 45 (not multiples
    # of the 16-wide Cholesky blocks): the padded unit pivots must not count as breakdown
    say("case: fp64 40x50x60 R=(3,9,5) cores scaled by 1e7, J=200")
    X = rng_for(65, 0).standard_normal((40, 50, 60))
    init = [1e7 * c for c in random_cores(X.shape, (3, 9, 5), rng_for(65, 3))]
    t = TR(torch.tensor(X, device="cuda"), (3, 9, 5), 200, precision="f64", init_cores=init)
    lockstep(t, X, 6, 200, core_tol=1e-9)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_fit_error_matches_oracle(prec, tol):
    say(f"case: fit error {prec}")
    dims, ranks = (33, 41, 29, 7), (3, 4, 2, 5)
    X = rng_for(63, 0).standard_normal(dims).astype(np.float32 if prec == "f32" else np.float64)
    cores = random_cores(dims, ranks, rng_for(63, 1))
    t = TR(torch.tensor(X, device="cuda"), ranks, 200, precision=prec, init_cores=cores)
    got = to_np(t.get_cores())
    want = oals.fit_error(got, X.astype(np.float64))
    assert abs(t.fit_error() - want) <= tol * want


def test_nan_in_x_rejected():
    say("case: NaN in X")
    from paper_2010_08581_amd import TralsError
    X = np.ones((10, 11, 12), dtype=np.float32)
    X[3, 4, 5] = np.nan
    with pytest.raises(TralsError) as e:
        TR(torch.tensor(X, device="cuda"), (2, 2, 2), 50, precision="f32")
    assert e.value.code == -1


def test_zero_core_is_singular_and_recoverable():
    say("case: all-zero core")
    from paper_2010_08581_amd import TralsError
    X = rng_for(64, 0).standard_normal((20, 21, 22))
    init = random_cores(X.shape, (2, 2, 2), rng_for(64, 3))
    t = TR(torch.tensor(X, device="cuda"), (2, 2, 2), 100, precision="f64", init_cores=init)
    bad = [c.copy() for c in init]
    bad[1][:] = 0.0
    with pytest.raises(TralsError) as e:
        t.set_cores(bad)
    assert e.value.code == -3
    with pytest.raises(TralsError):
        t.step(1)  # failed state
    t.set_cores(init)  # reset
    t.step(3)


def test_resume_and_determinism():
    # A run is deterministic bit for bit.  A run resumed from saved cores takes its first
    # tables from those cores, where the uninterrupted run took them from the right-hand sides
    # of the updates (the same leverage scores up to rounding): its draws are the same and its
    # cores agree to rounding.
    say("case: resume 2+2 sweeps vs 4 sweeps")
    X, _, init = make_config("c1", dims=(30, 31, 32), dtype=np.float64)
    Xt = torch.tensor(X, device="cuda")
    a = TR(Xt, (3, 3, 3), 300, precision="f64", init_cores=init)
    a.sweep(3)
    a.step(2)
    ia = a.last_samples()[0].copy()
    a.step(1)
    ca = to_np(a.get_cores())
    b = TR(Xt, (3, 3, 3), 300, precision="f64", init_cores=init)
    b.sweep(2)
    mid = to_np(b.get_cores())
    c = TR(Xt, (3, 3, 3), 300, precision="f64", init_cores=mid)
    c.update_counter = 2 * 3
    c.sweep(1)
    c.step(2)
    ic = c.last_samples()[0].copy()
    c.step(1)
    cc = to_np(c.get_cores())
    assert np.array_equal(ia, ic)
    for n in range(3):
        assert_core_close(cc[n], ca[n], 1e-10)
    d = TR(Xt, (3, 3, 3), 300, precision="f64", init_cores=init)
    d.sweep(4)
    for n, cd in enumerate(to_np(d.get_cores())):
        assert np.array_equal(ca[n], cd)


def test_c2_full_size_lockstep():
    say("case: c2 full size 500^3 R=10 J=8192 fp32 lockstep 3 updates")
    X, _, init = make_config("c2", dtype=np.float32)
    t = TR(torch.tensor(X, device="cuda"), (10, 10, 10), 8192, precision="f32", init_cores=init)
    X64 = X.astype(np.float64)
    del X
    worst = lockstep(t, X64, 3, 8192)
    say(f"c2 worst core rel diff {worst:.3e}")


def test_c3_full_size_lockstep():
    say("case: c3 full size 40^5 R=5 J=4096 fp32 lockstep 5 updates")
    X, _, init = make_config("c3", dtype=np.float32)
    t = TR(torch.tensor(X, device="cuda"), (5,) * 5, 4096, precision="f32", init_cores=init)
    X64 = X.astype(np.float64)
    del X
    worst = lockstep(t, X64, 5, 4096)
    say(f"c3 worst core rel diff {worst:.3e}")


def test_c4_full_size_video_lockstep():
    # 240x320x3x2000 video-shaped tensor, ranks 20 (P = 400), J = 16384: one update per mode
    say("case: c4 full size video 240x320x3x2000 R=20 J=16384 fp32 lockstep 4 updates")
    X = video_tensor()
    init = random_cores(X.shape, (20,) * 4, rng_for(0, 3))
    t = TR(torch.tensor(X, device="cuda"), (20,) * 4, 16384, precision="f32", init_cores=init)
    worst = lockstep(t, X, 4, 16384)
    say(f"c4 worst core rel diff {worst:.3e}")


def test_rank32_instances_fp64():
    # ranks 26-30 (the 32-rank draw instance), P = 728-840 (the blocked factorisation over 46-53
    # blocks, the widest triangular-solve instance) and a tall mode-0 core (800 x 728: its table
    # from the blocked factorisation of the core Gram); the other cores are wide (uniform tables)
    say("case: fp64 800x40x40 R=(26,30,28) J=3000 lockstep 3 updates (ranks up to 32)")
    dims, ranks = (800, 40, 40), (26, 30, 28)
    X = ring_tensor(random_cores(dims, ranks, rng_for(67, 1)))
    X = X + 0.01 * np.linalg.norm(X) / np.sqrt(X.size) * rng_for(67, 2).standard_normal(dims)
    init = random_cores(dims, ranks, rng_for(67, 3))
    t = TR(torch.tensor(X, device="cuda"), ranks, 3000, precision="f64", init_cores=init)
    worst = lockstep(t, X, 3, 3000, core_tol=1e-8)
    say(f"worst core rel diff {worst:.3e}")


def test_large_P_blocked_cholesky_fp64():
    # P = 168, 156, 182 (11-12 blocks of 16): the blocked multi-workgroup factorisation, with a
    # partial last 64-column step, for the normal equations and the (tall) core Grams
    say("case: fp64 200x190x180 R=(12,13,14) J=600 lockstep 4 updates (large P)")
    dims, ranks = (200, 190, 180), (12, 13, 14)
    X = ring_tensor(random_cores(dims, ranks, rng_for(66, 1)))
    X = X + 0.01 * np.linalg.norm(X) / np.sqrt(X.size) * rng_for(66, 2).standard_normal(dims)
    init = random_cores(dims, ranks, rng_for(66, 3))
    t = TR(torch.tensor(X, device="cuda"), ranks, 600, precision="f64", init_cores=init)
    worst = lockstep(t, X, 4, 600, core_tol=1e-8)
    say(f"worst core rel diff {worst:.3e}")


def test_single_workgroup_limit_fp64():
    # P = 132, 144, 132 (9 blocks of 16): the largest factorisations held whole in one
    # workgroup's LDS, with the right-hand-side reduction run beside them in the same launch
    say("case: fp64 150x140x130 R=(12,12,11) J=700 lockstep 3 updates (P up to 144)")
    dims, ranks = (150, 140, 130), (12, 12, 11)
    X = ring_tensor(random_cores(dims, ranks, rng_for(68, 1)))
    X = X + 0.01 * np.linalg.norm(X) / np.sqrt(X.size) * rng_for(68, 2).standard_normal(dims)
    init = random_cores(dims, ranks, rng_for(68, 3))
    t = TR(torch.tensor(X, device="cuda"), ranks, 700, precision="f64", init_cores=init)
    worst = lockstep(t, X, 3, 700, core_tol=1e-8)
    say(f"worst core rel diff {worst:.3e}")


def test_fp32_three_slice_lockstep():
    # P = 132, 144, 132 > 128: the FP32 path multiplies three 8-bit slices of the sketch and of
    # the weighted fibers on the BF16 matrix cores (48-row tiles, exponent blocks of 64 samples,
    # a ragged last block)
    say("case: fp32 150x140x130 R=(12,12,11) J=1500 lockstep 4 updates (three-slice contraction)")
    dims, ranks = (150, 140, 130), (12, 12, 11)
    X = ring_tensor(random_cores(dims, ranks, rng_for(69, 1)))
    X = (X + 0.01 * np.linalg.norm(X) / np.sqrt(X.size) * rng_for(69, 2).standard_normal(dims)).astype(np.float32)
    init = random_cores(dims, ranks, rng_for(69, 3))
    t = TR(torch.tensor(X, device="cuda"), ranks, 1500, precision="f32", init_cores=init)
    worst = lockstep(t, X.astype(np.float64), 4, 1500)
    say(f"worst slice {worst:.3e}")


def test_fp32_three_slice_few_samples():
    # P = 110, 130, 143 (one above 128: the handle takes the three-slice path for every mode) with
    # J = 300: the split pass and the contraction on five 64-sample blocks, the last holding 44
    # samples, few splits per tile; I_n = 70, 5, 129 (ragged column tiles, a wide core)
    say("case: fp32 70x5x129 R=(10,13,11) J=300 lockstep 3 updates (three-slice, few samples)")
    dims, ranks = (70, 5, 129), (10, 13, 11)
    X = ring_tensor(random_cores(dims, ranks, rng_for(71, 1)))
    X = (X + 0.01 * np.linalg.norm(X) / np.sqrt(X.size) * rng_for(71, 2).standard_normal(dims)).astype(np.float32)
    init = random_cores(dims, ranks, rng_for(71, 3))
    t = TR(torch.tensor(X, device="cuda"), ranks, 300, precision="f32", init_cores=init)
    worst = lockstep(t, X.astype(np.float64), 3, 300)
    say(f"worst slice {worst:.3e}")
