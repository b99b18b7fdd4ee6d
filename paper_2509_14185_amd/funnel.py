"""Funnel inference of the blow-up rate lam (paper: Methods, "Identifying
Admissible lambda Values").

Near an admissible lam* the smallest residual reachable at a fixed lam,
taken with its sign, is about linear in lam with a zero at lam*.  Each
outer iteration trains at a fixed lam with damped Gauss-Newton steps on the
GPU (gn.Problem.step), measures the proxy r_hat(lam) on the GPU
(gn.Problem.funnel_residual: the validation residual of largest magnitude,
with its sign, over y <= y_max) and moves lam by the secant method:
lam_1 = lam_0 + dlam, then the zero of the line through the last two
(lam, r_hat) pairs.  The secant is the line's zero,
lam_{n+1} = lam_n - r_n (lam_n - lam_{n-1}) / (r_n - r_{n-1}); with equal
proxies lam stays.  Training continues from the previous lam's parameters;
the run stops when a secant step leaves the allowed range of lam (the
equations need lam > 0).  Only this scalar recurrence runs on the host.
"""
from __future__ import annotations


def next_lambda(lams, rs, dlam):
    """The next lam from the history (lam_0..lam_n, r_0..r_n)."""
    if len(lams) == 1:
        return lams[0] + dlam
    a, b = lams[-2], lams[-1]
    ra, rb = rs[-2], rs[-1]
    if ra == rb:
        return b
    return b - rb * (b - a) / (rb - ra)


def funnel_inference(make_problem, theta, lam0, dlam, outer, steps, mu, y_max=1.0, on_iter=None,
                     lam_range=(0.0, float("inf"))):
    """Run up to `outer` trainings of `steps` GN steps (damping mu) each.

    make_problem(lam) -> gn.Problem with its points set (closed here after
    use); theta: device parameters, updated in place (training continues
    across lam values).  on_iter(n, lam, r_hat, y_at), if given, is called
    after each training.  The run stops early when the next lam is not
    finite or leaves the open interval lam_range.  Returns (lams, r_hats,
    y_ats)."""
    lams, rs, ys = [], [], []
    lam = float(lam0)
    lo, hi = lam_range
    for n in range(outer):
        if not (lo < lam < hi):
            break
        prob = make_problem(lam)
        try:
            for _ in range(steps):
                prob.step(theta, mu, stats=False)
            r, y = prob.funnel_residual(theta, y_max)
        finally:
            prob.close()
        lams.append(lam)
        rs.append(r)
        ys.append(y)
        if on_iter is not None:
            on_iter(n, lam, r, y)
        lam = next_lambda(lams, rs, dlam)
    return lams, rs, ys
