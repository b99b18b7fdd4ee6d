"""Oracle of the stochastic full-matrix Gauss-Newton step (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper: Methods, "Second-order Optimizer".  Instead of forming G = J^T J each
step, the paper estimates it by an exponential moving average, across
iterations, of an unbiased rank-1 estimator that needs one product with the
Jacobian, and sets the learning rate and momentum in closed form each
iteration by the scheme of Martens and Grosse (2015, K-FAC, section 7).
The steps, in the paper's order:

1. u = J^T v with a random v, E[v v^T] = I (here Rademacher signs passed in
   as data), so E[u u^T] = J^T J;
2. G_ema <- beta G_ema + (1 - beta) u u^T (G_ema starts at 0);
3. Delta = -(G_ema + gamma I)^{-1} g, g = J^T r = grad h for h = |r|^2 / 2,
   with the factor of G_ema + gamma I refreshed only on the steps the caller
   chooses (the inversion is amortised);
4. (alpha, mu) minimise the damped quadratic model
   M(d) = g^T d + d^T (J^T J + gamma I) d / 2 over d = alpha Delta + mu d0,
   d0 the previous update, with the exact J^T J through products with J;
   without a usable previous update only alpha;
5. theta <- theta + d, d0 <- d.

Readings (not fixed by the paper): beta, gamma and the refresh period are
inputs; the model uses the damping gamma of step 3; momentum is dropped when
d0 = 0 or when the 2x2 system is numerically singular (its determinant at
most 1e-12 of the product of its diagonal).
"""
from __future__ import annotations

import numpy as np

from . import dense
from . import gn as ogn


def estimate(J, v):
    """u = J^T v (the rank-1 estimate of J^T J is u u^T)."""
    return np.asarray(J, dtype=np.float64).T @ np.asarray(v, dtype=np.float64)


def ema(G, u, beta):
    """beta G + (1 - beta) u u^T."""
    return beta * G + (1.0 - beta) * np.outer(u, u)


def mg_coefficients(J, g, gamma, Delta, d0):
    """(alpha, mu, model value, used_momentum) minimising
    M(a Delta + m d0) = (a, m) g-terms + quadratic form with C = J^T J + gamma I."""
    JD = J @ Delta
    a11 = float(JD @ JD + gamma * Delta @ Delta)
    b1 = float(g @ Delta)
    if d0 is not None and np.any(d0 != 0):
        Jd = J @ d0
        a12 = float(JD @ Jd + gamma * Delta @ d0)
        a22 = float(Jd @ Jd + gamma * d0 @ d0)
        b2 = float(g @ d0)
        det = a11 * a22 - a12 * a12
        if det > 1e-12 * a11 * a22:
            alpha = (-b1 * a22 + b2 * a12) / det
            mu = (-b2 * a11 + b1 * a12) / det
            model = 0.5 * (alpha * alpha * a11 + 2 * alpha * mu * a12 + mu * mu * a22) + alpha * b1 + mu * b2
            return alpha, mu, model, True
    alpha = -b1 / a11
    return alpha, 0.0, 0.5 * alpha * alpha * a11 + alpha * b1, False


class State:
    """Optimizer state carried across steps: G_ema, the factor of
    G_ema + gamma I, the previous update."""

    def __init__(self, P):
        self.G = np.zeros((P, P))
        self.L = None
        self.prev = np.zeros(P)


def step(prob, theta, state, v, beta, gamma, refactor, momentum=True):
    """One stochastic GN step; updates state in place.  Returns
    (theta_next, info) with info: alpha, mu, model, used_momentum, half_sq_norm,
    u, g, Delta, delta, chol_info."""
    theta = np.asarray(theta, dtype=np.float64)
    r = ogn._residual(prob, theta)
    J = ogn._jacobian(prob, theta)
    g = dense.gradient(J, r)
    u = estimate(J, v)
    state.G = ema(state.G, u, beta)
    info = dict(half_sq_norm=0.5 * float(r @ r), u=u, g=g, chol_info=0)
    if refactor or state.L is None:
        A = state.G.copy()
        A[np.diag_indices_from(A)] += gamma
        L, ci = dense.cholesky(A)
        info["chol_info"] = ci
        if ci != 0:
            return theta.copy(), info
        state.L = L
    z = dense.solve_lower(state.L, -g)
    Delta = dense.solve_lower_t(state.L, z)
    alpha, mu, model, used = mg_coefficients(J, g, gamma, Delta, state.prev if momentum else None)
    delta = alpha * Delta + mu * state.prev
    state.prev = delta
    info.update(alpha=alpha, mu=mu, model=model, used_momentum=used, Delta=Delta, delta=delta)
    return theta + delta, info
