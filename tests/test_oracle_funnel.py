"""Pins of the funnel-inference oracle (oracle/funnel.py), CPU only:
- the secant update returns the exact zero of a linear r after two
  evaluations, wherever the two points lie, and takes lam_0 + dlam first;
- on a smooth nonlinear r with a simple zero it converges superlinearly to
  the zero (a library root finder gives the reference);
- the proxy picks the signed value of largest magnitude inside the
  neighbourhood only, the smallest index on ties, and a NaN over any number;
  brute force over random inputs."""
import math

import numpy as np
import pytest
import scipy.optimize

from oracle import funnel as fo


def test_first_step_is_the_perturbation():
    assert fo.secant_next([0.6], [0.3], 0.01) == pytest.approx(0.61, abs=0.0)


@pytest.mark.parametrize("lam_star,slope,lam0,dlam", [(0.6057, 2.0, 0.5, 0.02), (0.4703, -0.7, 0.9, -0.1),
                                                     (1.5, 1e-3, 1.49, 1e-4)])
def test_linear_zero_in_one_secant_step(lam_star, slope, lam0, dlam):
    lams, rs = fo.funnel(lambda l: slope * (l - lam_star), lam0, dlam, 3)
    assert lams[1] == lam0 + dlam
    assert lams[2] == pytest.approx(lam_star, rel=1e-13, abs=1e-15)
    assert abs(rs[2]) < 1e-13 * abs(slope)


def test_printed_combination_is_not_the_zero():
    # the printed form lam_n - r_{n-1} (lam_{n-1} - lam_n) / (r_{n-1} - r_n)
    # misses the zero of an exactly linear r; the standard step does not
    r = lambda l: 3.0 * (l - 0.6)
    l0, l1 = 0.5, 0.52
    printed = l1 - r(l0) * (l0 - l1) / (r(l0) - r(l1))
    assert abs(printed - 0.6) > 1e-3
    assert fo.secant_next([l0, l1], [r(l0), r(l1)], 0.0) == pytest.approx(0.6, rel=1e-14)


def test_superlinear_on_a_smooth_zero():
    r = lambda l: math.tanh(3.0 * (l - 0.6057)) + 0.4 * (l - 0.6057) ** 2
    ref = scipy.optimize.brentq(r, 0.0, 1.0, xtol=1e-15)
    lams, rs = fo.funnel(r, 0.55, 0.01, 8)
    err = [abs(l - ref) for l in lams]
    assert err[-1] < 1e-13
    # order > 1: e_{k+1} / e_k -> 0 while the errors are resolved
    ratios = [err[k + 1] / err[k] for k in range(2, 5) if err[k] > 1e-12]
    assert ratios and all(q2 < q1 for q1, q2 in zip(ratios, ratios[1:]))
    assert ratios[-1] < 0.05


def test_proxy_neighbourhood_sign_and_ties():
    R = np.array([0.1, -0.5, 0.4, 0.5, -2.0, 9.0])
    y = np.array([0.0, 0.1, 0.2, 0.3, 0.9, 1.5])
    assert fo.proxy(R, y, 1.0) == (-2.0, 0.9)          # sign kept, y = 1.5 outside
    assert fo.proxy(R, y, 0.35) == (-0.5, 0.1)         # |-0.5| = |0.5|: smallest index
    assert fo.proxy(R, y, 0.0) == (0.1, 0.0)           # a single point
    Rn = R.copy()
    Rn[2] = np.nan
    r, yy = fo.proxy(Rn, y, 1.0)
    assert np.isnan(r) and yy == 0.2
    with pytest.raises(ValueError):
        fo.proxy(R, y + 2.0, 1.0)


def test_proxy_brute_force():
    rng = np.random.default_rng(4)
    for _ in range(50):
        n = int(rng.integers(1, 40))
        R = rng.standard_normal(n)
        y = rng.uniform(0, 2, n)
        ym = float(rng.uniform(0.2, 2.0))
        inside = np.flatnonzero(y <= ym)
        if inside.size == 0:
            continue
        i = inside[np.argmax(np.abs(R[inside]))]
        assert fo.proxy(R, y, ym) == (R[i], y[i])


def test_equal_proxies_keep_lam():
    assert fo.secant_next([0.5, 0.6], [0.2, 0.2], 0.01) == 0.6
