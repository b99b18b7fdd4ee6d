"""Pins of the oracle's stochastic full-matrix Gauss-Newton step
(oracle/rank1.py): the exact expectation of the rank-1 estimate over every
sign vector equals J^T J; the moving average reaches (1 - beta^k) u u^T for a
constant estimate; with an exact curvature estimate the closed-form
learning rate is 1 and the momentum 0 (the paper's remark that a step length
of 1 is viable when G is exact), which on a linear problem is the ridge
solution; the coefficients minimise the quadratic model over the plane they
span (checked against perturbations and a brute-force least-squares fit of
the model's values).  CPU only."""
import itertools

import numpy as np
import pytest

import workloads
from oracle import profile1d as p1
from oracle import rank1


class Linear:
    def __init__(self, A, b):
        self.A, self.b = A, b

    def residual_rows(self, theta):
        return self.A @ theta - self.b

    def jacobian(self, theta):
        return self.A.copy()


def test_rank1_estimate_is_unbiased_exactly():
    rng = np.random.default_rng(3)
    J = rng.integers(-9, 10, size=(6, 4)).astype(np.float64)
    acc = np.zeros((4, 4))
    for signs in itertools.product((-1.0, 1.0), repeat=6):
        u = rank1.estimate(J, np.array(signs))
        acc += np.outer(u, u)
    np.testing.assert_array_equal(acc / 64.0, J.T @ J)


def test_rademacher_signs():
    v = workloads.rademacher(10000, 5)
    assert set(np.unique(v)) == {-1.0, 1.0}
    assert abs(v.mean()) < 0.05


def test_moving_average_of_a_constant_estimate():
    u = np.array([1.0, -2.0, 0.5])
    G = np.zeros((3, 3))
    beta = 0.9
    for k in range(1, 8):
        G = rank1.ema(G, u, beta)
        np.testing.assert_allclose(G, (1 - beta ** k) * np.outer(u, u), rtol=1e-14)


@pytest.mark.parametrize("gamma", [1e-3, 0.5])
def test_exact_curvature_gives_unit_step_and_ridge_solution(gamma):
    rng = np.random.default_rng(4)
    A = rng.standard_normal((30, 6))
    b = rng.standard_normal(30)
    prob = Linear(A, b)
    st = rank1.State(6)
    st.prev = rng.standard_normal(6)        # an arbitrary previous update
    # beta = 1 keeps the injected estimate: G_ema = J^T J exactly
    st.G = A.T @ A
    th, info = rank1.step(prob, np.zeros(6), st, np.ones(30), 1.0, gamma, True)
    assert info["alpha"] == pytest.approx(1.0, abs=1e-10)
    assert info["mu"] == pytest.approx(0.0, abs=1e-10)
    ridge = np.linalg.solve(A.T @ A + gamma * np.eye(6), A.T @ b)
    np.testing.assert_allclose(th, ridge, rtol=1e-10, atol=1e-12)


def _model(J, g, gamma, d):
    return float(g @ d + 0.5 * ((J @ d) @ (J @ d) + gamma * d @ d))


def test_coefficients_minimise_the_model_on_their_plane():
    inp = workloads.make_inputs("ccf_small", n=120, m_quad=40, widths=[1, 8, 8, 1])
    prob = p1.Problem.from_inputs(inp)
    theta = inp["theta0"]
    J = p1.jacobian(prob, theta)
    r = p1.residual_rows(prob, theta)
    g = J.T @ r
    rng = np.random.default_rng(8)
    Delta, d0 = rng.standard_normal(theta.size), rng.standard_normal(theta.size)
    gamma = 1e-2
    a, m, model, used = rank1.mg_coefficients(J, g, gamma, Delta, d0)
    assert used
    assert model == pytest.approx(_model(J, g, gamma, a * Delta + m * d0), rel=1e-12)
    for ea, em in itertools.product((-1e-3, 0.0, 1e-3), repeat=2):
        if ea or em:
            assert _model(J, g, gamma, (a + ea) * Delta + (m + em) * d0) > model
    # brute force: fit the quadratic q(x, y) = M(x Delta + y d0) on a grid and
    # locate its stationary point
    pts = [(x, y) for x in (-1.0, 0.0, 1.0, 2.0) for y in (-1.0, 0.0, 1.0, 2.0)]
    X = np.array([[1, x, y, x * x, x * y, y * y] for x, y in pts])
    c = np.linalg.lstsq(X, np.array([_model(J, g, gamma, x * Delta + y * d0) for x, y in pts]), rcond=None)[0]
    H = np.array([[2 * c[3], c[4]], [c[4], 2 * c[5]]])
    xy = np.linalg.solve(H, -c[1:3])
    assert xy == pytest.approx([a, m], rel=1e-8, abs=1e-10)


def test_without_previous_update_only_the_learning_rate():
    inp = workloads.make_inputs("ccf_small", n=120, m_quad=40, widths=[1, 8, 8, 1])
    prob = p1.Problem.from_inputs(inp)
    st = rank1.State(inp["P"] if "P" in inp else inp["theta0"].size)
    th, info = rank1.step(prob, inp["theta0"], st, workloads.rademacher(121, 1), 0.9, 1e-2, True)
    assert not info["used_momentum"] and info["mu"] == 0.0
    assert info["model"] < 0.0
    np.testing.assert_allclose(st.prev, info["alpha"] * info["Delta"], rtol=0, atol=0)
    np.testing.assert_allclose(st.G, 0.1 * np.outer(info["u"], info["u"]), rtol=1e-15)


def test_stochastic_steps_decrease_the_ccf_objective():
    inp = workloads.make_inputs("ccf_small", n=200, m_quad=64, widths=[1, 12, 12, 1])
    prob = p1.Problem.from_inputs(inp)
    theta = inp["theta0"]
    st = rank1.State(theta.size)
    h0 = 0.5 * float(p1.residual_rows(prob, theta) @ p1.residual_rows(prob, theta))
    for k in range(40):
        theta, info = rank1.step(prob, theta, st, workloads.rademacher(201, 100 + k), 0.95, 1e-3, k % 5 == 0)
        assert info["model"] <= 0.0
    h1 = 0.5 * float(p1.residual_rows(prob, theta) @ p1.residual_rows(prob, theta))
    assert h1 < 0.5 * h0
