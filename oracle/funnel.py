"""Oracle: funnel inference of the blow-up rate lam (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper: Methods, "Identifying Admissible lambda Values", funnel inference.
Only at an admissible lam* can the equation be satisfied exactly, so the
smallest residual reachable by training at a fixed lam, taken with its sign,
r(lam), is about linear near lam* with a zero there.  Its proxy r_hat(lam):
train at the fixed lam until the solution has relaxed, then take the
residual of largest magnitude (with its sign) over a small neighbourhood of
the origin.  lam is moved by the secant method on the history of
(lam_n, r_hat_n): lam_1 = lam_0 + dlam, then the zero of the line through the
last two points.

Readings (not fixed by the paper):
- The secant formula as printed combines lam_n with r_hat_{n-1}; the zero of
  the line through (lam_{n-1}, r_{n-1}) and (lam_n, r_n) is
  lam_{n+1} = lam_n - r_n (lam_n - lam_{n-1}) / (r_n - r_{n-1}), the
  standard secant step, which is taken here (the printed combination does
  not return the zero even for an exactly linear r).
- The neighbourhood is the validation points with y <= y_max; ties in |R|
  go to the smallest index; a NaN residual counts as the largest.
- Training at each lam continues from the previous lam's parameters.
- When the last two proxies are equal there is no secant; lam stays.
"""
from __future__ import annotations

import numpy as np


def proxy(R, y, y_max):
    """(r_hat, y_at): the R_i of largest |R_i| over y_i <= y_max."""
    R = np.asarray(R, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    best, bi = -1.0, -1
    for i in range(R.size):
        if not (y[i] <= y_max):
            continue
        a = np.inf if np.isnan(R[i]) else abs(R[i])
        if a > best:
            best, bi = a, i
    if bi < 0:
        raise ValueError("no point with y <= y_max")
    return float(R[bi]), float(y[bi])


def secant_next(lams, rs, dlam):
    """lam_{n+1} from the history lam_0..lam_n, r_0..r_n."""
    if len(lams) == 1:
        return lams[0] + dlam
    l0, l1 = lams[-2], lams[-1]
    r0, r1 = rs[-2], rs[-1]
    if r1 == r0:  # no secant through two equal values: lam stays
        return l1
    return l1 - r1 * (l1 - l0) / (r1 - r0)


def funnel(r_of_lam, lam0, dlam, n):
    """n evaluations of r_of_lam along the secant sequence from lam0."""
    lams, rs = [], []
    lam = lam0
    for _ in range(n):
        lams.append(lam)
        rs.append(r_of_lam(lam))
        lam = secant_next(lams, rs, dlam)
    return lams, rs
