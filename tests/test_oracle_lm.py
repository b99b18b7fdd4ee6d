"""Pins of the oracle's Levenberg-Marquardt step (oracle/gn.py, lm_step):
a linear least-squares problem, where the Gauss-Newton model is exact (gain
ratio 1) and the iteration must reach numpy's lstsq solution; Rosenbrock's
function as residuals (More, Garbow and Hillstrom, problem 1), whose
minimiser (1, 1) is known; rejection sequences checked by brute force
(independent 2x2 solves); the stop at mu_max at a stationary point; a failed
factorisation handled as a rejection.  CPU only."""
import numpy as np
import pytest

import workloads
from oracle import gn as ogn
from oracle import profile1d as p1


class Linear:
    """r(theta) = A theta - b."""

    def __init__(self, A, b):
        self.A, self.b = A, b

    def residual_rows(self, theta):
        return self.A @ theta - self.b

    def jacobian(self, theta):
        return self.A.copy()


class Rosenbrock:
    """r = (10 (t2 - t1^2), 1 - t1); h = |r|^2 / 2 has its minimum 0 at (1, 1)."""

    def residual_rows(self, t):
        return np.array([10.0 * (t[1] - t[0] ** 2), 1.0 - t[0]])

    def jacobian(self, t):
        return np.array([[-20.0 * t[0], 10.0], [-1.0, 0.0]])


def test_linear_problem_has_unit_gain_and_reaches_lstsq():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((40, 7))
    b = rng.standard_normal(40)
    prob = Linear(A, b)
    theta, mu = np.zeros(7), 1.0
    for k in range(40):
        th1, out = ogn.lm_step(prob, theta, mu)
        if out["status"] != "ok":
            # at the floor no trial decreases h by more than rounding
            assert out["half_sq_norm"] - 0.5 * float((A @ theta - b) @ (A @ theta - b)) == 0.0
            break
        if out["half_sq_norm"] - out["half_sq_norm_new"] > 1e-8 * out["half_sq_norm"]:
            # the model is exact: accepted at once, actual and predicted decrease agree
            assert out["tries"] == 1
            assert abs(out["rho"] - 1.0) < 1e-8
            assert out["mu"] == max(mu / 3.0, 1e-12)
        theta, mu = th1, out["mu"]
    assert k >= 3
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.linalg.norm(theta - ref) < 1e-10 * np.linalg.norm(ref)


def test_rosenbrock_reaches_the_minimiser_monotonically():
    prob = Rosenbrock()
    theta, mu = np.array([-1.2, 1.0]), 1e-3
    h = 0.5 * float(prob.residual_rows(theta) @ prob.residual_rows(theta))
    for k in range(200):
        theta, out = ogn.lm_step(prob, theta, mu)
        if out["status"] != "ok":
            break
        assert out["half_sq_norm_new"] <= h
        h, mu = out["half_sq_norm_new"], out["mu"]
    assert np.linalg.norm(theta - np.array([1.0, 1.0])) < 1e-10


def _brute_h(prob, theta, mu):
    r, J = prob.residual_rows(theta), prob.jacobian(theta)
    d = np.linalg.solve(J.T @ J + mu * np.eye(2), -J.T @ r)
    r1 = prob.residual_rows(theta + d)
    return 0.5 * float(r1 @ r1), d


@pytest.mark.parametrize("up", [2.0, 10.0])
def test_rejections_follow_the_objective(up):
    # from (-1.2, 1) the undamped GN step lands at (1, -3.84), h = 1171 > 12.1
    prob = Rosenbrock()
    theta = np.array([-1.2, 1.0])
    r0 = prob.residual_rows(theta)
    h0 = 0.5 * float(r0 @ r0)
    th1, out = ogn.lm_step(prob, theta, 1e-3, up=up)
    assert out["status"] == "ok" and out["tries"] == {2.0: 10, 10.0: 4}[up]
    for k, mu in enumerate(out["mus"]):
        assert mu == pytest.approx(1e-3 * up ** k, rel=1e-15)
        hk, dk = _brute_h(prob, theta, mu)
        if k < out["tries"] - 1:
            assert hk >= h0          # rejected trials did not decrease h
        else:
            assert hk < h0           # the accepted one did
            np.testing.assert_allclose(th1, theta + dk, rtol=1e-12, atol=1e-14)


def test_damping_update_follows_the_gain_ratio():
    prob = Rosenbrock()
    theta, mu = np.array([-1.2, 1.0]), 1.0
    seen = set()
    for k in range(60):
        th1, out = ogn.lm_step(prob, theta, mu)
        assert out["status"] == "ok"
        mu_try, rho = out["mus"][-1], out["rho"]
        if rho > 0.75:
            assert out["mu"] == max(mu_try / 3.0, 1e-12); seen.add("down")
        elif rho < 0.25:
            assert out["mu"] == min(mu_try * 2.0, 1e12); seen.add("up")
        else:
            assert out["mu"] == mu_try; seen.add("keep")
        theta, mu = th1, out["mu"]
        if np.linalg.norm(theta - 1.0) < 1e-12:
            break
    assert "down" in seen


def test_stationary_point_is_rejected_until_mu_max():
    prob = Rosenbrock()
    theta = np.array([1.0, 1.0])          # r = 0, g = 0: no decrease is possible
    th1, out = ogn.lm_step(prob, theta, 1e-2, up=10.0, mu_max=1.0)
    assert out["status"] == "rejected"
    assert out["mus"] == pytest.approx([1e-2, 1e-1, 1.0])
    assert np.array_equal(th1, theta)


def test_failed_factorisation_is_a_rejection():
    rng = np.random.default_rng(6)
    A = rng.standard_normal((20, 5))
    A[:, 2] = 0.0                         # G has an exact zero pivot at column 3
    prob = Linear(A, rng.standard_normal(20))
    th1, out = ogn.lm_step(prob, np.zeros(5), 0.0, mu_min=1e-3)
    assert out["infos"][0] == 3 and out["infos"][1] == 0
    assert out["mus"] == [0.0, 1e-3]
    assert out["status"] == "ok" and out["tries"] == 2
    assert th1[2] == 0.0                  # the damped solution leaves the null direction alone


def test_max_tries_bounds_the_factorisations():
    prob = Rosenbrock()
    th1, out = ogn.lm_step(prob, np.array([-1.2, 1.0]), 1e-3, up=2.0, max_tries=3)
    assert out["tries"] == 3 and out["status"] == "rejected"
    assert out["mu"] == pytest.approx(1e-3 * 8)


def test_lm_decreases_the_ccf_objective():
    inp = workloads.make_inputs("ccf_small", n=200, m_quad=64, widths=[1, 12, 12, 1])
    prob = p1.Problem.from_inputs(inp)
    theta, mu = inp["theta0"], 1e-3
    h = None
    for k in range(4):
        theta, out = ogn.lm_step(prob, theta, mu)
        assert out["status"] == "ok"
        assert h is None or out["half_sq_norm"] == pytest.approx(h, rel=1e-14)
        assert out["half_sq_norm_new"] < out["half_sq_norm"]
        h, mu = out["half_sq_norm_new"], out["mu"]
