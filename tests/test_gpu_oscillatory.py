"""10-way 4 x ... x 4 oscillatory-function tensors with ranks 10 (Section 4.1.2): deep subchains
(eight slice products per sampled row), 4-element fibers, every core unfolding wide (uniform
leverage); and the exact-vs-sampled protocol driver."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import als as oals  # noqa: E402
from synth import oscillatory_tensor, random_cores, ring_tensor, rng_for  # noqa: E402
from tests.gpu_helpers import assert_core_close, lockstep, rel, say, to_np  # noqa: E402

pytestmark = pytest.mark.gpu

R10 = (10,) * 10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_08581_amd import _lib
    _lib.load()


def TR(*a, **k):
    from paper_2010_08581_amd import TRALS
    return TRALS(*a, **k)


def test_linear_growth_fp64_lockstep():
    say("case: linear growth 4^10 R=10 fp64 J=300, lockstep 12 updates")
    X = oscillatory_tensor("linear_growth")
    init = random_cores(X.shape, R10, rng_for(80, 3))
    t = TR(torch.tensor(X, device="cuda"), R10, 300, seed=1, precision="f64", init_cores=init)
    worst = lockstep(t, X, 12, 300, seed=1, core_tol=1e-8)
    say(f"worst core rel diff {worst:.3e}")


def test_airy_fp32_lockstep():
    say("case: airy 4^10 R=10 fp32 J=500, lockstep 10 updates")
    X = oscillatory_tensor("airy", dtype=np.float32)
    init = random_cores(X.shape, R10, rng_for(81, 3))
    t = TR(torch.tensor(X, device="cuda"), R10, 500, seed=2, precision="f32", init_cores=init)
    worst = lockstep(t, X.astype(np.float64), 10, 500, seed=2, core_tol=1e-4)
    say(f"worst core rel diff {worst:.3e}")


def test_chirp_exact_update_matches_oracle():
    say("case: chirp 4^10 R=10 exact fp64, 2 updates (262144-row designs)")
    X = oscillatory_tensor("chirp")
    init = random_cores(X.shape, R10, rng_for(82, 3))
    t = TR(torch.tensor(X, device="cuda"), R10, 0, precision="f64", init_cores=init, method="exact")
    cores = [c.copy() for c in init]
    for u in range(2):
        t.step(1)
        cores[u] = oals.exact_update(X, cores, u)
        r = assert_core_close(to_np(t.get_cores())[u], cores[u], 1e-8, f"update {u}")
        say(f"update {u}: worst slice {r:.3e}")


def test_protocol_finds_sample_size():
    from paper_2010_08581_amd import protocol
    say("case: protocol on 40x42x44 R=3 fp64")
    dims, ranks = (40, 42, 44), (3, 3, 3)
    X = ring_tensor(random_cores(dims, ranks, rng_for(83, 1)))
    X = X + 0.05 * np.linalg.norm(X) / np.sqrt(X.size) * rng_for(83, 2).standard_normal(dims)
    init = random_cores(dims, ranks, rng_for(83, 3))
    Xt = torch.tensor(X, device="cuda")
    res = protocol.compare(Xt, ranks, init, tol=1e-4, max_sweeps=30, factor=1.1, step=50)
    say(str(res))
    assert 1 <= res["convergence_sweeps"] <= 30 and res["sweeps"] == 2 * res["convergence_sweeps"]
    assert res["samples"] is not None and res["samples"] >= 18
    assert res["sampled_error"] < 1.1 * res["exact_error"]
    # the reported error is reproduced by a fresh handle with the J found
    t = TR(Xt, ranks, res["samples"], precision="f64", init_cores=init)
    t.sweep(res["sweeps"])
    assert t.fit_error() == res["sampled_error"]
