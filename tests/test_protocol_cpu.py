"""The exact-vs-sampled protocol's J search, on the CPU with a fake handle."""
import pytest

from paper_2010_08581_amd import protocol
from paper_2010_08581_amd._lib import TRALS_ESINGULAR, TralsError


class FakeHandle:
    """Error of a run = err(J); J in `singular` raises like a rank-deficient sample."""

    def __init__(self, err, singular=()):
        self.err, self.singular, self.J, self.runs = err, set(singular), None, []
        self.update_counter = 0

    def set_cores(self, cores):
        pass

    def set_samples(self, J):
        self.J = J

    def sweep(self, n):
        self.runs.append(self.J)
        if self.J in self.singular:
            raise TralsError(TRALS_ESINGULAR, "trals_sweep")

    def fit_error(self):
        return self.err(self.J)

    def close(self):
        pass


@pytest.fixture
def fake(monkeypatch):
    made = {}

    def factory(err, singular=()):
        def ctor(*a, **k):
            made["h"] = FakeHandle(err, singular)
            return made["h"]
        monkeypatch.setattr(protocol, "TRALS", ctor)
        monkeypatch.setattr(protocol, "_timed_sweeps", lambda h, s: h.sweep(s) or 0.01)
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
def test_search_matches_linear_scan(fake, J_true):
    err = lambda J: 1.0 if J < J_true else 0.5  # noqa: E731
    made = fake(err)
    J, e, secs, runs = protocol.find_sample_size(None, (2, 2), None, 3, 0.9, 200, 100, 5000)
    assert J == linear_scan(err, 0.9, 200, 100, 5000) == J_true
    assert e == 0.5 and secs == 0.01
    assert runs <= 2 * 6 + 2  # doubling then bisection over 49 grid points
    assert len(made["h"].runs) == runs


def test_search_reports_failure_and_skips_singular(fake):
    made = fake(lambda J: 2.0, singular={200, 300})
    J, e, secs, runs = protocol.find_sample_size(None, (2, 2), None, 3, 0.9, 200, 100, 1000)
    assert J is None and secs is None and e == 2.0
    made = fake(lambda J: 0.1, singular={200})
    J, e, secs, runs = protocol.find_sample_size(None, (2, 2), None, 3, 0.9, 200, 100, 1000)
    assert J == 300
