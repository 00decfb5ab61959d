"""The exact-vs-sampled protocol (Section 4.1; supplement, experiment details) on the CPU with
fake handles: the sample-size search and the sweep counts of the two runs."""
import pytest

from paper_2010_08581_amd import protocol
from paper_2010_08581_amd._lib import TRALS_ESINGULAR, TralsError


class FakeHandle:
    """Sampled handle: the error after a run is err(J, sweeps run since the last reset); J in
    `singular` raises like a rank-deficient sample."""

    def __init__(self, err, singular=()):
        self.err, self.singular, self.J, self.runs = err, set(singular), None, []
        self.update_counter = 0
        self.swept = 0

    def set_cores(self, cores):
        self.swept = 0

    def set_samples(self, J):
        self.J = J

    def sweep(self, n):
        self.runs.append(self.J)
        self.swept += n
        if self.J in self.singular:
            raise TralsError(TRALS_ESINGULAR, "trals_sweep")

    def fit_error(self):
        return self.err(self.J, self.swept)

    def close(self):
        pass


class FakeExact(FakeHandle):
    """Exact handle: the error after k sweeps is err(k)."""

    def __init__(self, err):
        super().__init__(lambda J, k: err(k))


@pytest.fixture
def fake(monkeypatch):
    made = {}

    def factory(err, singular=(), exact_err=None):
        def ctor(*a, **k):
            if k.get("method") == "exact":
                made["exact"] = FakeExact(exact_err)
                return made["exact"]
            made["h"] = FakeHandle(err, singular)
            return made["h"]
        monkeypatch.setattr(protocol, "TRALS", ctor)
        monkeypatch.setattr(protocol, "_timed_sweeps", lambda h, s: h.sweep(s) or 0.01 * s)
        return made
    return factory


def linear_scan(err, target, J0, step, J_max, singular=()):
    J = J0
    while J <= J_max:
        if J not in singular and err(J) < target:
            return J
        J += step
    return None


@pytest.mark.parametrize("J_true", [200, 300, 1700, 4900, 5000])
@pytest.mark.parametrize("search", ["walk", "bisect"])
def test_search_matches_linear_scan_on_a_step(fake, J_true, search):
    err = lambda J, k: 1.0 if J < J_true else 0.5  # noqa: E731
    made = fake(err)
    J, e, secs, runs = protocol.find_sample_size(None, (2, 2), None, 3, 0.9, 200, 100, 5000, search=search)
    assert J == linear_scan(lambda J: err(J, 3), 0.9, 200, 100, 5000) == J_true
    assert e == 0.5 and secs == pytest.approx(0.03)
    if search == "walk":
        assert runs == (J_true - 200) // 100 + 1  # every grid point up to the first success
    else:
        assert runs <= 2 * 6 + 2  # doubling then bisection over 49 grid points
    assert len(made["h"].runs) == runs


def test_walk_finds_the_first_J_of_a_non_monotone_curve(fake):
    # the sampled error after a fixed number of sweeps need not fall with J: here J = 600 reaches
    # the target, 700 .. 2900 do not, 3000 and above do.  The paper's rule (walk up from J0) takes
    # 600; doubling + bisection steps over the dip and lands on the later band.
    def err(J, k):
        return 0.5 if J == 600 or J >= 3000 else 1.0
    fake(err)
    J, e, _, runs = protocol.find_sample_size(None, (2, 2), None, 3, 0.9, 200, 100, 5000, search="walk")
    assert J == 600 and runs == 5
    fake(err)
    Jb, _, _, _ = protocol.find_sample_size(None, (2, 2), None, 3, 0.9, 200, 100, 5000, search="bisect")
    assert Jb == 3000


def test_search_reports_failure_and_skips_singular(fake):
    made = fake(lambda J, k: 2.0, singular={200, 300})
    J, e, secs, runs = protocol.find_sample_size(None, (2, 2), None, 3, 0.9, 200, 100, 1000)
    assert J is None and secs is None and e == 2.0 and runs == 9
    made = fake(lambda J, k: 0.1, singular={200})
    J, e, secs, runs = protocol.find_sample_size(None, (2, 2), None, 3, 0.9, 200, 100, 1000)
    assert J == 300
    assert made["h"].runs == [200, 300]


def test_compare_runs_every_method_for_twice_the_convergence_sweeps(fake):
    # exact error after k sweeps: 0.1 + 1/(k+1)^2; it changes by less than 1e-3 of itself first
    # after sweep S, then both methods run 2 S sweeps from the initial cores; E = exact error
    # at 2 S, target 1.1 E; the sampled error reaches it from J = 900 on
    def exact_err(k):
        return 0.1 + 1.0 / (k + 1) ** 2
    S = next(k for k in range(1, 200) if abs(exact_err(k) - exact_err(k - 1)) < 1e-3 * exact_err(k))
    E = exact_err(2 * S)
    seen = []

    def err(J, k):
        seen.append(k)
        return 1.05 * E if J >= 900 else 1.5 * E
    made = fake(err, exact_err=exact_err)
    res = protocol.compare(None, (10, 10), None, tol=1e-3, max_sweeps=100, factor=1.1, step=100)
    assert res["convergence_sweeps"] == S and res["sweeps"] == 2 * S
    assert res["exact_error"] == E and res["exact_s"] == pytest.approx(0.01 * 2 * S)
    assert res["J0"] == 200 and res["samples"] == 900 and res["runs"] == 8
    assert set(seen) == {2 * S}  # every sampled error read after exactly 2 S sweeps
    assert res["speedup"] == pytest.approx(1.0)
    assert made["exact"].swept == 2 * S
