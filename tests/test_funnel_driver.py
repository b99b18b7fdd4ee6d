"""Host logic of the funnel-inference driver (paper_2509_14185_amd.funnel)
with a stand-in problem (no GPU): the lam sequence is the oracle's secant
sequence (oracle/funnel.py) for the same proxies, training continues across
lam values, each problem is closed, and the run stops when a secant step
leaves the allowed range."""
import pytest

from oracle import funnel as fo
from paper_2509_14185_amd import funnel as fn


class FakeProblem:
    """r_hat = a (lam - lam*) + b theta[0]; each step adds 1 to theta[0]."""
    made, closed = [], []

    def __init__(self, lam, a, lam_star, b):
        self.lam, self.a, self.lam_star, self.b = lam, a, lam_star, b
        FakeProblem.made.append(lam)

    def step(self, theta, mu, stats=True):
        theta[0] += 1.0

    def funnel_residual(self, theta, y_max):
        return self.a * (self.lam - self.lam_star) + self.b * theta[0], 0.25 * y_max

    def close(self):
        FakeProblem.closed.append(self.lam)


@pytest.mark.parametrize("b", [0.0, 1e-3])
def test_sequence_matches_oracle(b):
    FakeProblem.made, FakeProblem.closed = [], []
    theta = [0.0]
    lams, rs, ys = fn.funnel_inference(lambda l: FakeProblem(l, 2.0, 0.6057, b), theta, 0.55, 0.01, 5, 3, 1e-3,
                                       y_max=0.8)
    assert theta[0] == 15.0                      # 5 trainings of 3 steps, continued
    assert FakeProblem.closed == FakeProblem.made == lams
    assert ys == [0.2] * 5
    for n in range(1, 5):
        assert lams[n] == pytest.approx(fo.secant_next(lams[:n], rs[:n], 0.01), rel=1e-15)
    if b == 0.0:
        assert lams[2] == pytest.approx(0.6057, rel=1e-14)


def test_stops_outside_the_range():
    theta = [0.0]
    # r = lam - 2 with lam_0 = 0.5, dlam = 0.1 -> the secant proposes lam = 2, outside (0, 1)
    lams, rs, ys = fn.funnel_inference(lambda l: FakeProblem(l, 1.0, 2.0, 0.0), theta, 0.5, 0.1, 6, 1, 1e-3,
                                       lam_range=(0.0, 1.0))
    assert lams == [0.5, 0.6]
    assert len(rs) == len(ys) == 2
