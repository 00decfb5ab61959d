"""GPU parity of the BF16 form (BF16 data panels and sketch on matrix cores, FP32
accumulation, FP64 Cholesky and leverage tables) against the FP64 oracle.

Tolerances: BF16 rounds each operand to 8 significant bits (unit roundoff 2^-9 ~ 2e-3), so a
sampled LS solution from BF16 operands differs from the FP64 one by a few times 2^-9 for the
well-conditioned systems used here (measured 2-3e-3): per-update cores must agree within 1e-2
in lockstep.  The sampling never sees BF16 (tables come from the FP32 cores in FP64), so the
indices stay bit-exact.  The fit error at convergence must be within 1e-2 relative of the
oracle's.  Each case runs for the default BF16 form (subchain rows formed in FP64, rounded once
to BF16) and for "bf16c", whose subchain products also run on BF16 matrix cores (each operand a
pair of BF16 values, FP32 accumulation).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import als as oals  # noqa: E402
from synth import make_config  # noqa: E402
from tests.gpu_helpers import lockstep, say  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def TR(*a, **k):
    from paper_2010_08581_amd import TRALS
    return TRALS(*a, **k)


@pytest.mark.parametrize("prec", ["bf16", "bf16c"])
@pytest.mark.parametrize("cfg,dims,ranks,J", [
    ("c2", (120, 136, 150), (10, 10, 10), 2000),
    ("c3", (21, 22, 20, 23, 19), (5,) * 5, 4096),
])
def test_bf16_lockstep(cfg, dims, ranks, J, prec):
    # "bf16c": the subchain products on BF16 matrix cores too (pairs of BF16 operands, FP32
    # accumulation: about 16 bits per product, below the BF16 rounding of the sketch)
    say(f"case: {prec} lockstep {cfg} {dims} ranks {ranks} J={J}")
    X, _, init = make_config(cfg, dims=dims, dtype=np.float32, ranks=ranks)
    t = TR(torch.tensor(X, device="cuda"), ranks, J, precision=prec, init_cores=init)
    worst = lockstep(t, X.astype(np.float64), 2 * len(dims), J, core_tol=1e-2)
    say(f"bf16 worst core rel diff {worst:.3e}")


@pytest.mark.parametrize("prec", ["bf16", "bf16c"])
@pytest.mark.parametrize("cfg,dims,ranks,J,sweeps", [
    ("c3", (21, 22, 20, 23, 19), (5,) * 5, 4096, 6),
    ("c3", (30, 26, 28, 24), (5,) * 4, 3000, 8),
])
def test_bf16_converged_fit_within_1e2_of_oracle(cfg, dims, ranks, J, sweeps, prec):
    say(f"case: {prec} converged fit {cfg} {dims} ranks {ranks} J={J} sweeps={sweeps}")
    X, _, init = make_config(cfg, dims=dims, dtype=np.float32, ranks=ranks)
    t = TR(torch.tensor(X, device="cuda"), ranks, J, precision=prec, init_cores=init)
    t.sweep(sweeps)
    fb = t.fit_error()
    ref = oals.tr_als_sampled(X.astype(np.float64), init, J, sweeps, seed=0)
    fo = oals.fit_error(ref, X.astype(np.float64))
    say(f"fit bf16={fb:.6e} oracle={fo:.6e} rel={abs(fb - fo) / fo:.2e}")
    assert abs(fb - fo) <= 1e-2 * fo


@pytest.mark.parametrize("prec", ["bf16", "bf16c"])
def test_bf16_lockstep_rank20(prec):
    # P = 400 (the BF16 contraction's 80-row tiles, the blocked factorisation, the 24-rank draw
    # instance writing the transposed BF16 pair) on a 4-way tensor with a C = 3 mode like the
    # video workload, built from rank-20 cores plus 1% noise; every core unfolding is wide
    # (uniform tables).  Lockstep keeps each system at the oracle's conditioning: an
    # over-parameterised free run (rank 20 on a small tensor of four blobs) drives the sampled
    # systems to cond(A)^2 2^-9 > 1, beyond what BF16 operands resolve.
    from synth import random_cores, ring_tensor, rng_for
    say(f"case: {prec} lockstep 30x32x3x36 R=20 J=1500, 4 updates")
    dims, ranks = (30, 32, 3, 36), (20,) * 4
    X = ring_tensor(random_cores(dims, ranks, rng_for(68, 1)))
    X = (X + 0.01 * np.linalg.norm(X) / np.sqrt(X.size) * rng_for(68, 2).standard_normal(dims)).astype(np.float32)
    init = random_cores(dims, ranks, rng_for(68, 3))
    t = TR(torch.tensor(X, device="cuda"), ranks, 1500, precision=prec, init_cores=init)
    worst = lockstep(t, X.astype(np.float64), 4, 1500, core_tol=1e-2)
    say(f"bf16 worst core rel diff {worst:.3e}")


def test_bf16_fit_is_measured_against_fp32_x():
    # the BF16 form keeps an FP32 copy of X for the fit: with the same cores the fit equals the FP32 path's
    say("case: bf16 fit uses fp32 X")
    X, _, init = make_config("c3", dims=(12, 13, 11, 10, 9), dtype=np.float32)
    a = TR(torch.tensor(X, device="cuda"), (5,) * 5, 400, precision="bf16", init_cores=init)
    b = TR(torch.tensor(X, device="cuda"), (5,) * 5, 400, precision="f32", init_cores=init)
    assert abs(a.fit_error() - b.fit_error()) <= 1e-12 * b.fit_error()
