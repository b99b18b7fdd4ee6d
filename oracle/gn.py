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

import math

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


def projected_normal_residuals(residual, theta, delta, mu, k=8, seed=0, h=1e-30):
    """Projections of the normal-equation residual
    v = (J^T J + mu I) delta + J^T r on k Gaussian directions w, for problems
    whose J is too large to form (checker; parity of a step at full size).

    residual(t) returns r(t) for a real or complex parameter vector t.  J w
    and J delta are complex-step directional derivatives (one evaluation
    each, exact up to rounding), so that
        w^T v = (J w)^T (J delta + r) + mu w^T delta,
    the last dot products summed exactly (math.fsum of the rounded terms).
    Also returned: F2 = mean |J w|^2, the unbiased (Hutchinson) estimate of
    |J|_F^2, |delta|, |r|, and per direction the rounding bound of the
    evaluation itself, eps (|J w|^T (|J delta| + |r|) + mu |w|^T |delta|).
    A step whose normwise backward error is b satisfies
    |v| <= b ((|J|_F^2 + sqrt(P) mu) |delta| + |J|_F |r|), and |w^T v| is at
    most 6 |v| for a Gaussian w with probability 1 - 2e-9."""
    theta = np.asarray(theta, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)

    def jdir(d):
        t = theta.astype(np.complex128) + 1j * h * np.asarray(d, dtype=np.float64)
        return np.asarray(residual(t)).imag / h

    r = np.asarray(residual(theta), dtype=np.float64)
    Jd = jdir(delta)
    u = Jd + r
    W = np.random.default_rng(seed).standard_normal((k, theta.size))
    proj, err, sq = [], [], []
    eps = np.finfo(np.float64).eps
    for w in W:
        Jw = jdir(w)
        sq.append(float(Jw @ Jw))
        proj.append(math.fsum(np.concatenate([Jw * u, [mu * math.fsum(w * delta)]])))
        err.append(eps * (float(np.abs(Jw) @ (np.abs(Jd) + np.abs(r))) + mu * float(np.abs(w) @ np.abs(delta))))
    return dict(proj=np.array(proj), F2=float(np.mean(sq)), dnorm=float(np.linalg.norm(delta)),
                rnorm=float(np.linalg.norm(r)), eval_err=np.array(err), P=theta.size)


def projected_bound(pr, mu, b=5e-14):
    """Largest |w^T v| allowed for a step of backward error b (see
    projected_normal_residuals): 6 b ((F2 + sqrt(P) mu) |delta| + sqrt(F2) |r|)
    plus the evaluation's rounding bound."""
    F2 = pr["F2"]
    return 6.0 * b * ((F2 + math.sqrt(pr["P"]) * mu) * pr["dnorm"] + math.sqrt(F2) * pr["rnorm"]) + pr["eval_err"]


LM_DEFAULTS = dict(mu_min=1e-12, mu_max=1e12, up=2.0, down=3.0, rho_lo=0.25, rho_hi=0.75, max_tries=20)


def _residual(prob, theta):
    if hasattr(prob, "residual_rows"):
        return np.asarray(prob.residual_rows(theta), dtype=np.float64)
    return p1.residual_rows(prob, theta)


def _jacobian(prob, theta):
    if hasattr(prob, "jacobian"):
        return np.asarray(prob.jacobian(theta), dtype=np.float64)
    return p1.jacobian(prob, theta)


def lm_step(prob, theta, mu, **kw):
    """One step with Levenberg-Marquardt damping.

    Paper: Methods, "Second-order Optimizer": the damping decides how far the
    local quadratic model of the objective is trusted and is adjusted during
    training, by the classical Levenberg-Marquardt method for some problems.
    The rule is the one stated in the literature the paper cites (Levenberg
    1944, Marquardt 1963), in gain-ratio form:

    - delta(mu) = -(G + mu I)^{-1} g with G = J^T J, g = J^T r at theta
      (formed once; only the damped system is solved again);
    - rho = (h(theta) - h(theta + delta)) / (h(theta) - |r + J delta|^2 / 2),
      h = |r|^2 / 2: the actual decrease over the decrease of the
      Gauss-Newton (linear) model;
    - a trial is accepted iff h(theta + delta) is finite and rho > 0.  Then
      mu <- max(mu / down, mu_min) if rho > rho_hi, mu <- min(mu * up, mu_max)
      if rho < rho_lo;
    - otherwise (including a failed factorisation) the trial is rejected;
      if mu already equals mu_max the step ends with theta unchanged, else
      mu <- min(max(mu * up, mu_min), mu_max) and the solve is repeated, at
      most max_tries factorisations in all.

    rho_lo = rho_hi = 0 with up = down is Marquardt's rule (decrease: mu / nu,
    increase: mu nu and retry).  Returns (theta_next, out) with out: status
    ("ok", "rejected" or "nonfinite"), mu (damping for the next step), tries,
    rho (of the last trial), mus (the damping of each trial), infos (Cholesky
    info of each trial), half_sq_norm (at theta), half_sq_norm_new (at
    theta_next), delta (the accepted update or None).
    """
    o = dict(LM_DEFAULTS)
    o.update(kw)
    theta = np.asarray(theta, dtype=np.float64)
    r = _residual(prob, theta)
    h0 = 0.5 * float(r @ r)
    out = dict(status="rejected", mu=mu, tries=0, rho=float("nan"), mus=[], infos=[], half_sq_norm=h0,
               half_sq_norm_new=h0, delta=None)
    if not np.isfinite(h0):
        out["status"] = "nonfinite"
        return theta.copy(), out
    J = _jacobian(prob, theta)
    G, g = gram_and_gradient(J, r)
    while out["tries"] < o["max_tries"]:
        out["tries"] += 1
        out["mus"].append(mu)
        delta, info = damped_solve(G, g, mu)
        out["infos"].append(info)
        rho, h1 = float("-inf"), float("nan")
        if delta is not None and np.all(np.isfinite(delta)):
            trial = theta + delta
            r1 = _residual(prob, trial)
            h1 = 0.5 * float(r1 @ r1)
            lin = r + J @ delta
            pred = h0 - 0.5 * float(lin @ lin)
            rho = (h0 - h1) / pred if pred > 0 else float("-inf")
        out["rho"] = rho
        if np.isfinite(h1) and rho > 0:
            if rho > o["rho_hi"]:
                mu = max(mu / o["down"], o["mu_min"])
            elif rho < o["rho_lo"]:
                mu = min(mu * o["up"], o["mu_max"])
            out.update(status="ok", mu=mu, half_sq_norm_new=h1, delta=delta)
            return trial, out
        if mu >= o["mu_max"]:
            break
        mu = min(max(mu * o["up"], o["mu_min"]), o["mu_max"])
        out["mu"] = mu
    return theta.copy(), out
