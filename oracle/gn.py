"""Oracle damped Gauss-Newton step (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper: Methods, "Second-order Optimizer".  The objective is a weighted sum of
squares h = sum_i c_i |f_i|^2 and the update is
theta_{t+1} = theta_t - (G + gamma I)^{-1} grad h with the full Gauss-Newton
matrix G (no structural approximation).  With h = |r|^2/2 (weights folded into
the rows) this is G = J^T J, grad h = J^T r; the step length is 1, which the
paper notes is viable when G is computed exactly.  mu below is the damping.
"""
from __future__ import annotations

import numpy as np

from . import dense
from . import profile1d as p1


def gram_and_gradient(J, r):
    """G = J^T J and g = J^T r, compensated dot products (dense.c)."""
    return dense.gram(J), dense.gradient(J, r)


def damped_solve(G, g, mu):
    """delta = -(G + mu I)^{-1} g by Cholesky and two substitutions.

    Returns (delta, info); info is the 1-based failing pivot or 0.
    """
    A = np.array(G, dtype=np.float64, copy=True)
    A[np.diag_indices_from(A)] += mu
    L, info = dense.cholesky(A)
    if info != 0:
        return None, info
    z = dense.solve_lower(L, -np.asarray(g, dtype=np.float64))
    return dense.solve_lower_t(L, z), 0


def step(prob, theta, mu):
    """One damped GN step.  Returns (theta_next, info dict).  prob is a 1D
    profile problem (profile1d.Problem) or any problem with residual_rows and
    jacobian methods (profile2d.Problem)."""
    if hasattr(prob, "residual_rows"):
        r = prob.residual_rows(theta)
        J = prob.jacobian(theta)
    else:
        r = p1.residual_rows(prob, theta)
        J = p1.jacobian(prob, theta)
    G, g = gram_and_gradient(J, r)
    delta, info = damped_solve(G, g, mu)
    stats = dict(half_sq_norm=0.5 * float(r @ r), r=r, J=J, G=G, g=g, delta=delta, chol_info=info)
    if delta is None or not np.all(np.isfinite(delta)):
        return np.array(theta, copy=True), stats
    return theta + delta, stats


def backward_error(G, mu, g, delta):
    """Normwise backward error |(G+mu I) d + g| / (|G+mu I| |d| + |g|) (2-norms; |A| by Frobenius)."""
    A = np.array(G, copy=True)
    A[np.diag_indices_from(A)] += mu
    res = dense.symv_lower(np.tril(A), delta) + g
    return float(np.linalg.norm(res) / (np.linalg.norm(A) * np.linalg.norm(delta) + np.linalg.norm(g)))
