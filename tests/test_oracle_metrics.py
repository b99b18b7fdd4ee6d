"""Pins of the oracle's validation metric and of the solve checker.

validation_max (paper: Methods, "Validation Metrics for Solutions": the
largest raw residual |R| over a dense validation grid) is compared with a
reference computed here point by point from the definitions, sharing nothing
with oracle/profile1d.py:
  - y from s by y = sqrt((1 - s)^(-2(1+lam)) - 1), written out;
  - a hand-written tanh network and the envelope in closed form;
  - Theta' by the complex-step derivative of that field;
  - the Hilbert transform of the even field by adaptive quadrature with a
    Cauchy weight (scipy.integrate.quad), not the oracle's fixed nodes:
      (H f)(y) = (1/pi) p.v. int_0^inf f(t) (1/(y - t) + 1/(y + t)) dt.
The oracle's own error is then its node rule's quadrature error, which the
tolerance allows.  A validation_max taken over the collocation points, or
with the collocation points' Hilbert weights, fails (the tests show the
collocation maximum differs by far more than the tolerance).

backward_error (the checker of every solve) is pinned by a hand-evaluated
2 x 2 case and by a negative test: a solution perturbed by 1e-10 must fail
the 5e-14 bar that the exact one passes.
"""
import numpy as np
import pytest
from scipy import integrate

import workloads
from oracle import gn as ogn
from oracle import profile1d as p1


def y_of_s(s, lam):
    return np.sqrt((1.0 - s) ** (-2.0 * (1.0 + lam)) - 1.0)


class Field:
    """Theta(y) = E(y) NN(q(y)) for a one-hidden-layer tanh network."""

    def __init__(self, lam, equation, seed, width=3):
        rng = np.random.default_rng(seed)
        self.W1 = rng.uniform(-1.5, 1.5, width)
        self.b1 = rng.uniform(-0.5, 0.5, width)
        self.W2 = rng.uniform(-1.0, 1.0, width)
        self.b2 = 0.7
        self.lam, self.eq = lam, equation

    def theta_vector(self):
        # oracle layout: W1 (3 x 1) row-major, b1, W2 (1 x 3), b2
        return np.concatenate([self.W1, self.b1, self.W2, [self.b2]])

    def __call__(self, y):
        lam = self.lam
        e = lam / (2.0 * (1.0 + lam))
        w = 1.0 + y * y
        q = w ** (-1.0 / (2.0 * (1.0 + lam)))
        nn = sum(self.W2[k] * np.tanh(self.W1[k] * q + self.b1[k]) for k in range(len(self.W1))) + self.b2
        env = y * y * w ** (e - 1.0) if self.eq == p1.CCF else y * w ** (e - 0.5)
        return env * nn

    def deriv(self, y):
        h = 1e-30
        return float(np.imag(self(complex(y, h))) / h)


def hilbert_quad(f, y):
    """(1/pi) p.v. int_0^inf f(t) 2y/(y^2 - t^2) dt for even f, by adaptive quadrature."""
    if y == 0.0:
        return 0.0
    B = 2.0 * y + 4.0
    kw = dict(epsabs=1e-14, epsrel=1e-13, limit=400)
    # p.v. int_0^B f(t)/(y - t) dt = -p.v. int_0^B f(t)/(t - y) dt
    pv, _ = integrate.quad(f, 0.0, B, weight="cauchy", wvar=y, **kw)
    reg, _ = integrate.quad(lambda t: f(t) / (y + t), 0.0, B, **kw)
    tail, _ = integrate.quad(lambda t: f(t) * 2.0 * y / (y * y - t * t), B, np.inf, **kw)
    return (-pv + reg + tail) / np.pi


def reference_R(field, y):
    lam = field.lam
    Th = float(field(y))
    Thy = field.deriv(y)
    U = hilbert_quad(lambda t: float(field(t)), y) if field.eq == p1.CCF else Th
    return -lam * Th + ((1.0 + lam) * y + U) * Thy


def oracle_problem(field, n, m_quad, sval):
    inp = workloads.make_inputs("ccf_small", n=n, m_quad=m_quad, widths=[1, 3, 1])
    return p1.Problem(field.eq, [1, 3, 1], field.lam, inp["s"], sq=inp["sq"], wq=inp["wq"], sval=sval)


@pytest.mark.parametrize("equation,lam,seed", [(p1.CCF, 0.6057, 3), (p1.CCF, 0.4703, 8), (p1.BURGERS, 0.5, 4)])
def test_validation_max_against_pointwise_definition(equation, lam, seed):
    fld = Field(lam, equation, seed)
    n = 8
    sval = workloads.validation_grid(n)            # origin + 4n midpoints
    prob = oracle_problem(fld, n, 2048, sval)
    theta = fld.theta_vector()
    yv = y_of_s(sval, lam)
    Rref = np.array([reference_R(fld, y) for y in yv])
    got = p1.validation_max(prob, theta)
    ref = float(np.max(np.abs(Rref)))
    tol = 1e-9 if equation == p1.CCF else 1e-13
    assert abs(got - ref) <= tol * ref
    # the residual at the origin is zero for these envelopes (Theta(0) = 0 and
    # Theta'(0) = 0 for the even field, U(0) = 0 for the odd one), and a grid
    # holding only the origin gives exactly zero
    assert Rref[0] == 0.0
    only0 = oracle_problem(fld, n, 2048, np.zeros(1))
    assert p1.validation_max(only0, theta) == 0.0
    # the collocation maximum is a different number: an implementation that
    # took it would fail the comparison above
    R_coll, _ = p1.raw_residual(prob, theta)
    assert abs(float(np.max(np.abs(R_coll))) - ref) > 1e3 * tol * ref


def test_validation_max_follows_the_grid_it_is_given():
    """Every point of the grid counts: dropping the point where |R| peaks
    lowers the maximum to the next largest reference value."""
    fld = Field(0.6057, p1.CCF, 3)
    sval = workloads.validation_grid(8)
    yv = y_of_s(sval, fld.lam)
    Rref = np.abs([reference_R(fld, y) for y in yv])
    k = int(np.argmax(Rref))
    keep = np.delete(np.arange(sval.size), k)
    prob = oracle_problem(fld, 8, 2048, sval[keep])
    got = p1.validation_max(prob, fld.theta_vector())
    ref = float(np.max(Rref[keep]))
    assert abs(got - ref) <= 1e-9 * ref and ref < Rref[k]


def test_backward_error_hand_evaluated():
    # (G + mu I) = diag(2, 1), g = (-2, -1): the solution is (1, 1)
    G = np.diag([2.0, 1.0])
    g = np.array([-2.0, -1.0])
    assert ogn.backward_error(G, 0.0, g, np.array([1.0, 1.0])) == 0.0
    eps = 1e-6
    d = np.array([1.0, 1.0 + eps])
    # residual (0, eps); |A|_F = sqrt(5), |d| = sqrt(1 + (1+eps)^2), |g| = sqrt(5)
    ref = eps / (np.sqrt(5.0) * np.sqrt(1.0 + (1.0 + eps) ** 2) + np.sqrt(5.0))
    assert ogn.backward_error(G, 0.0, g, d) == pytest.approx(ref, rel=1e-9)
    # mu enters the diagonal: diag(1, 0) + 1 I, same system
    assert ogn.backward_error(np.diag([1.0, 0.0]), 1.0, g, np.array([1.0, 1.0])) == 0.0


def test_backward_error_rejects_a_perturbed_solution():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((300, 120))
    G = A.T @ A
    g = rng.standard_normal(120)
    mu = 1e-3
    d, info = ogn.damped_solve(G, g, mu)
    assert info == 0
    assert ogn.backward_error(G, mu, g, d) < 5e-15
    for seed in range(3):
        v = np.random.default_rng(100 + seed).standard_normal(120)
        bad = d + 1e-10 * np.linalg.norm(d) * v / np.linalg.norm(v)
        assert ogn.backward_error(G, mu, g, bad) > 5e-14
    # a sign error in the right-hand side is caught at once
    assert ogn.backward_error(G, mu, -g, d) > 1e-3


# ---- projected normal-equation residual (the step checker at sizes where
#      the oracle cannot form J): pinned against the full-matrix formula

PROJ_CASES = {
    "bouss2d": dict(n=40, ne=6, widths=[2, 8, 8, 3], nval=8),
    "ipm2d": dict(n=48, n1=12, ne=6, widths=[2, 10, 9, 1], nval=8),
}


@pytest.mark.parametrize("name", list(PROJ_CASES))
def test_projected_normal_residuals_against_full_matrices(name):
    from oracle import profile2d as p2

    inp = workloads.make_inputs_2d(name, **PROJ_CASES[name])
    po = p2.Problem.from_inputs(inp)
    theta = inp["theta0"] + 0.05 * np.random.default_rng(5).standard_normal(po.P)
    r = po.residual_rows(theta)
    J = po.jacobian(theta)
    G, g = ogn.gram_and_gradient(J, r)
    mu = 1e-3
    d, info = ogn.damped_solve(G, g, mu)
    assert info == 0
    k = 8
    W = np.random.default_rng(1).standard_normal((k, po.P))
    # formula: for a delta that is not the solution, w^T v equals the
    # projection of (G + mu I) delta + g formed from the full J
    dd = d + 0.3 * np.linalg.norm(d) * W[0] / np.linalg.norm(W[0])
    pr = ogn.projected_normal_residuals(po.residual_rows, theta, dd, mu, k=k, seed=1)
    ref = W @ (J.T @ (J @ dd + r) + mu * dd)
    assert np.all(np.abs(pr["proj"] - ref) <= 1e-12 * np.abs(W) @ (np.abs(J.T) @ (np.abs(J @ dd) + np.abs(r)) + mu * np.abs(dd)))
    # the Hutchinson estimate of |J|_F^2
    F2 = float(np.sum(J * J))
    assert 0.2 * F2 < pr["F2"] < 5.0 * F2
    # the exact solution passes the bound of a 5e-14 backward error ...
    pr = ogn.projected_normal_residuals(po.residual_rows, theta, d, mu, k=k, seed=1)
    assert np.all(np.abs(pr["proj"]) <= ogn.projected_bound(pr, mu))
    # ... a perturbation of 1e-7 |d| in a random direction does not, nor a
    # step from the wrong sign of the gradient
    v = np.random.default_rng(9).standard_normal(po.P)
    bad = d + 1e-7 * np.linalg.norm(d) * v / np.linalg.norm(v)
    pr = ogn.projected_normal_residuals(po.residual_rows, theta, bad, mu, k=k, seed=1)
    assert np.any(np.abs(pr["proj"]) > ogn.projected_bound(pr, mu))
    pr = ogn.projected_normal_residuals(po.residual_rows, theta, -d, mu, k=k, seed=1)
    assert np.any(np.abs(pr["proj"]) > 1e3 * ogn.projected_bound(pr, mu))
